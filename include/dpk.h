/*
 * dpk.h -- C ABI of libdpk.so: MI355X (gfx950) evaluation of the smooth two-body-embedding
 * Deep Potential (se_e2_a): energy, forces and virial of one frame.
 *
 * The operation follows DeePMD-kit v2 (arXiv 2304.09409):
 *   Sec. II.A        E = sum_i E_i with E_i = F_0(D^i); neighbour lists padded to N_c.
 *   Sec. II.A.1      D^i = N_c^-2 (G^i)^T R^i (R^i)^T G^i_<, environment rows
 *                    (s, s x/r, s y/r, s z/r) with r_ij = r_j - r_i and the C^2 switching function
 *                    s(r) (eq. switch); G_j = N^{a_i,a_j}(s(r_ij)) (eq. G2); per-species nets.
 *   Sec. II.A.2      E_i = F_0(D^i) (eq. fitting_energy); F_i = -dE/dr_i;
 *                    Xi_ab = -sum_g dE/dh_ga h_gb.
 *   Sec. II.A.6      layers y = w_hat * tanh(x W + b) (+ x or + {x,x}) (eq. NN); tabulated
 *                    embedding by quintic pieces (eq. compress).
 *   Sec. III.B.1     neighbour formatting by (type, distance, index).
 *
 * Conventions shared by every entry point:
 *   - Units: Angstrom and eV; the virial is in eV with Xi_ab stored at [3a + b].
 *   - coord is [natoms][3] row-major; atype is [natoms] with values in [0, ntypes);
 *     box is the 3x3 cell h row-major, rows are the lattice vectors (h_ab = component b of
 *     lattice vector a), or NULL for an open (non-periodic) cluster.
 *   - Outputs are in the caller's atom order.
 *   - Every function returns DPK_OK (0) or a negative code; dpk_last_error() returns a
 *     thread-local description of the last failure on the calling thread.
 *   - No function keeps a caller pointer after it returns, except as stated for the device
 *     entry point's stream-ordered completion.
 *
 * Model parameter blob (FP64, flat, owned by the caller during dpk_model_create only):
 *   embedding nets first, net index e = a_i * ntypes + a_j (or e = a_j when type_one_side; for
 *   se_e3 e = a_j * ntypes + a_k), each with layers 1 -> emb[0] -> emb[1] -> emb[2]; then one
 *   fitting net per type a_i with layers (emb[2] * axis, or emb[2] for se_e2_r and se_e3) ->
 *   fit[0] -> fit[1] -> fit[2] -> 1. Every layer stores
 *   W [n_in][n_out] row-major, then b [n_out], then w_hat [n_out]. Hidden layers use tanh with a
 *   skip connection +x when n_out == n_in and +{x,x} when n_out == 2 n_in; the fitting output
 *   layer is linear without skip.
 */
#ifndef DPK_H
#define DPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DPK_OK = 0,
    DPK_E_INVALID_ARG = -1,   /* NULL pointer, natoms < 1, bad model description            */
    DPK_E_TYPE_RANGE = -2,    /* an atom type outside [0, ntypes)                            */
    DPK_E_BOX = -3,           /* det(h) <= 0                                                  */
    DPK_E_NBR_OVERFLOW = -4,  /* more candidates within r_c than the selection buffer holds,
                                 or (strict mode) a neighbour cut by sel                      */
    DPK_E_BUDGET = -5,        /* the frame's device workspace exceeds the context's budget    */
    DPK_E_OOM = -6,           /* device allocation failed                                     */
    DPK_E_DEVICE = -7,        /* a HIP call failed                                            */
    DPK_E_UNIMPLEMENTED = -8, /* combination not supported (e.g. table in FP64 with ntypes>4) */
    DPK_E_TIMEOUT = -9,       /* dpk_server_wait_for: the frame is not done yet               */
    DPK_E_CANCELLED = -10     /* a served frame withdrawn by dpk_server_cancel before it ran  */
};

enum {
    DPK_FP64 = 0,   /* every GEMM and activation in FP64 (FP64 MFMA)                          */
    DPK_MIXED = 1,  /* embedding and fitting GEMMs as three BF16 MFMA products (hi*hi + hi*lo +
                       lo*hi) with FP32 accumulation; FP32 activations; FP64 geometry, switching
                       function, force chain rule, force and virial accumulation, energy sum  */
    DPK_BF16 = 2,   /* as DPK_MIXED with one BF16 product per GEMM (fast, about 1e-2 relative) */
    DPK_FP32 = 3    /* the paper's FP32 inference (Sec. IV): embedding and fitting GEMMs on FP32 MFMA
                       (v_mfma_f32_16x16x4f32), FP32 activations and an FP32 table; FP64 geometry,
                       switching function, force chain rule, force and virial accumulation, and
                       energy sum, as in DPK_MIXED                                              */
};

#define DPK_MAX_TYPES 8

/* Descriptor kinds (Sec. II.A.1, the DeepPot-SE family):
 *   DPK_SE_E2_A  two-body embedding, full information: D = N_c^-2 G^T R R^T G_< (M x M_<);
 *   DPK_SE_E2_R  two-body embedding, radial-only: the environment row is s alone and
 *                D = N_c^-1 sum_j s_j G_j (M values; the printed radial-only form omits the s
 *                factor, which with zero padding would make D jump at r_c);
 *   DPK_SE_E3    three-body embedding (eq. descrpt-e3): D = N_c^-2 (R R^T) : G with
 *                G_jk = N^{a_j, a_k}(theta_jk), theta_jk = R_j . R_k, over every ordered pair of
 *                kept neighbours (M values); one net per ordered pair of neighbour types. */
enum { DPK_SE_E2_A = 0, DPK_SE_E2_R = 1, DPK_SE_E3 = 2 };

/* Model description. sel[] are the per-type neighbour capacities (N_c = sum of sel);
 * emb[] the embedding widths, axis = M_< (se_e2_a only), fit[] the fitting hidden widths; the
 * fitting input is M x M_< for se_e2_a and M for the other two. This build's kernels require
 * emb = {25, 50, 100}, axis = 16, fit = {240, 240, 240}; se_e3 also N_c <= 128. */
typedef struct {
    int32_t ntypes;
    int32_t sel[DPK_MAX_TYPES];
    double rcut;
    double rcut_smth;
    int32_t emb[3];
    int32_t axis;
    int32_t fit[3];
    int32_t type_one_side;   /* se_e2_a / se_e2_r: one net per neighbour type (not per pair)    */
    int32_t descriptor;      /* DPK_SE_E2_A (0), DPK_SE_E2_R or DPK_SE_E3                       */
} dpk_model_desc;

typedef struct dpk_model dpk_model;   /* immutable after creation; shareable across contexts  */
typedef struct dpk_ctx dpk_ctx;       /* one device + workspace; not thread-safe             */

typedef struct {
    int64_t nbr_dropped;          /* neighbours cut by sel in the last computed frame          */
    int64_t table_out_of_range;   /* tabulated inputs outside [0, table range] (last frame)    */
    int64_t max_candidates;       /* largest number of atoms within r_c of one atom            */
    int64_t workspace_bytes;      /* device bytes held by the context                          */
} dpk_stats;

/* Last error message of the calling thread ("" if none). Never NULL; valid until the next
 * failing call on the same thread. */
const char *dpk_last_error(void);

/* Create a model (Sec. II.A: E = sum_i F_0(D^i); Sec. II.A.1: the se_e2_a, se_e2_r or se_e3
 * descriptor with per-species embedding nets; Sec. II.A.2: per-species fitting nets; Sec. II.A.6,
 * eq. NN: the layer form) from a description and its FP64 parameter blob of nparams values in the
 * layout above. The blob is copied; the caller keeps ownership of desc and params.
 * DPK_E_INVALID_ARG for a NULL pointer, a bad description (ntypes outside 1..8, negative sel, sum
 * of sel outside 1..4096, not 0 < rcut_smth < rcut, an unknown descriptor) or a blob of the wrong
 * size; DPK_E_UNIMPLEMENTED for widths other than emb (25, 50, 100), axis 16, fit (240, 240, 240),
 * or an se_e3 model with N_c > 128. *out is NULL on failure. */
int dpk_model_create(const dpk_model_desc *desc, const double *params, int64_t nparams,
                     dpk_model **out);

/* Number of FP64 values the blob of desc must hold (the layer sizes of Sec. II.A.1 and II.A.2
 * with the layout above), or -1 for a NULL desc or ntypes outside 1..8. */
int64_t dpk_model_param_count(const dpk_model_desc *desc);

/* Read a model file (the frozen model the paper's C API loads, Sec. III.A): the magic
 * "DPKMODEL", a uint64 little-endian header length, a versioned JSON header (format
 * "dpk-se_e2_a", version 1: ntypes, sel, rcut, rcut_smth, embedding, axis, fitting,
 * type_one_side, descriptor ("se_e2_a" if absent, "se_e2_r", "se_e3"), nparams, compression =
 * null or {stride, x_max}), zero padding to a multiple of 8
 * bytes, then the FP64 blob (little-endian binary64, layout above). A compressed model's table is
 * rebuilt from the parameters at load (Sec. II.A.6), exactly as dpk_model_tabulate builds it.
 * DPK_E_INVALID_ARG for an unreadable, truncated or malformed file (the message says which key);
 * the checks of dpk_model_create apply. The caller frees *out with dpk_model_free. */
int dpk_model_load(const char *path, dpk_model **out);

/* Write m to path in the format dpk_model_load reads (for a compressed model, its stride and
 * range; the table itself is not stored). DPK_E_INVALID_ARG if the file cannot be written. */
int dpk_model_save(const dpk_model *m, const char *path);

/* Copy out a model's description (desc, if not NULL), its FP64 blob (params, if not NULL:
 * dpk_model_param_count(desc) values, caller-owned) and its table stride and range (0 for a model
 * without table). */
int dpk_model_describe(const dpk_model *m, dpk_model_desc *desc, double *params,
                       double *tab_stride, double *tab_xmax);

/* Replace the embedding nets by quintic tables (Sec. II.A.6, eq. compress): nodes at
 * x_l = l * stride, l = 0..L_c with L_c = ceil(x_max / stride), values and first and second
 * derivatives of each net at the nodes, and the paper's coefficient formulas. The table
 * variable is the net input: x = s(r), or theta = R_j . R_k (in [0, 2 s_max^2]) for se_e3.
 * Contexts created afterwards use the table. */
int dpk_model_tabulate(dpk_model *m, double stride, double x_max);

/* Free a model (NULL is ignored). Contexts created from it must be freed first. */
void dpk_model_free(dpk_model *m);

/* Create a context on HIP device `device` with precision DPK_FP64, DPK_MIXED, DPK_BF16 or DPK_FP32 (the
 * paper's FP64 and reduced-precision inference, Sec. IV; the precision of each step is listed at
 * the precision enum). The model's weights (and table, if the model is compressed at this point)
 * are packed for the precision and copied to the device; the model must outlive the context.
 * hbm_budget_bytes bounds model + workspace (0 = no bound; DPK_E_BUDGET if the model alone
 * exceeds it). strict_sel != 0 makes a neighbour cut by sel (reading R6 of the design notes: the
 * nearest sel[t] are kept) an error, DPK_E_NBR_OVERFLOW, instead of a counted truncation.
 * DPK_E_INVALID_ARG for a NULL pointer, an unknown precision or a missing device. */
int dpk_ctx_create(const dpk_model *m, int device, int precision, size_t hbm_budget_bytes,
                   int strict_sel, dpk_ctx **out);

/* Wait for the context's work, free its device memory and streams (NULL is ignored). */
void dpk_ctx_free(dpk_ctx *c);

/* Device bytes of the model plus the workspace of a frame of natoms atoms (neighbour list of N_c
 * entries per atom, Sec. II.A; descriptor and fitting scratch; the cell grid counted at one bin
 * per atom, an upper bound at liquid densities); -1 for a NULL context or natoms < 1. */
int64_t dpk_ctx_workspace_bytes(const dpk_ctx *c, int64_t natoms);

/* Host-pointer entry point: E, F and the virial of one frame (Sec. II.A.2: E = sum_i E_i,
 * F_i = -dE/dr_i, Xi_ab = -sum_g dE/dh_ga h_gb; atom_energy receives E_i). Copies the frame to the
 * device, evaluates it and copies the results back; returns after the results are in the
 * caller's buffers (all host pointers, caller-owned; energy: 1 double; force: natoms*3; virial: 9;
 * atom_energy: natoms or NULL). A frame that overflows the candidate buffer sized from its mean
 * density is rerun once with the largest buffer. Errors: DPK_E_INVALID_ARG (NULL, natoms < 1),
 * DPK_E_TYPE_RANGE, DPK_E_BOX (det h <= 0, or a cell thinner than r_c / 3), DPK_E_NBR_OVERFLOW
 * (more than 1024 atoms within r_c of one atom, or strict mode and a neighbour cut by sel),
 * DPK_E_BUDGET, DPK_E_OOM, DPK_E_DEVICE. */
int dpk_compute(dpk_ctx *c, int64_t natoms, const double *coord, const int32_t *atype,
                const double *box, double *energy, double *force, double *virial,
                double *atom_energy);

/* Device-pointer entry point, the same evaluation as dpk_compute (Sec. II.A.2): d_coord,
 * d_atype and the outputs are device pointers; box is a HOST pointer (9 doubles) or NULL. All work is enqueued on hip_stream (a hipStream_t, NULL for
 * the default stream) and the call returns without waiting, except with box == NULL, where it
 * waits once for the cluster's bounding box. The outputs are valid once the stream reaches this
 * point. The call itself returns only argument, box, budget and launch errors: errors found on
 * the device (an atom type out of range, DPK_E_TYPE_RANGE; a candidate-buffer overflow,
 * DPK_E_NBR_OVERFLOW, after which that frame's E, F and virial are not valid) are reported by the
 * next dpk_ctx_check(). The per-atom candidate buffer of the neighbour search is sized from the
 * frame's mean density (twice the expected count within r_c, at least 256, at most 1024) unless
 * dpk_ctx_set_candidate_capacity fixed it; after an overflow the caller reruns the frame with
 * the 1024-entry buffer, as dpk_compute does by itself. */
int dpk_compute_device(dpk_ctx *c, int64_t natoms, const double *d_coord,
                       const int32_t *d_atype, const double *box, double *d_energy,
                       double *d_force, double *d_virial, double *d_atom_energy,
                       void *hip_stream);

/* One domain's share of a spatially decomposed frame (the MD code's domain decomposition, Sec.
 * III.B.2; third-party MD interfaces, Sec. III.D): atoms 0.. nlocal - 1 are owned, atoms nlocal..
 * nlocal + nghost - 1 are ghost copies of atoms owned elsewhere (or periodic images), each at the
 * position its owner's domain sent. There is no cell: every atom within r_c of an owned atom must be
 * among the owned and ghost atoms. Neighbour lists are built for owned atoms only, over all atoms,
 * ordered and truncated as Sec. II.A.1 and III.B.1 (the internal search), or (ext_start and
 * ext_list not NULL) from the caller's candidate lists: owned atom i's candidates are ext_list
 * [ext_start[i] .. ext_start[i + 1]) (caller indices in [0, nlocal + nghost), any order, no
 * duplicates, e.g. an MD code's list with a skin), of which those within r_c are ordered and
 * truncated the same way. E = sum of E_i over owned atoms (atom_energy: nlocal values or NULL);
 * force: (nlocal + nghost) * 3, the forces on owned atoms and on ghosts from this domain's pairs
 * (the caller adds each ghost's force to its owner: the reverse exchange); virial = -sum over
 * pairs with an owned centre of g_ij (x) r_ij, so the domains' virials add up to the frame's. Host
 * buffers, caller-owned, synchronous. Errors as dpk_compute; DPK_E_INVALID_ARG also for an
 * ext_start that does not start at 0 or decreases, an index outside [0, nlocal + nghost), or only
 * one of ext_start/ext_list; DPK_E_UNIMPLEMENTED with ghosts and 8 atom types. */
int dpk_compute_ghost(dpk_ctx *c, int64_t nlocal, int64_t nghost, const double *coord,
                      const int32_t *atype, const int32_t *ext_start, const int32_t *ext_list,
                      double *energy, double *force, double *virial, double *atom_energy);

/* As dpk_compute_device with the cell h (Sec. II.A.2: h_ab = component b of lattice vector a) in
 * DEVICE memory: d_box points to 9 doubles on the context's device, or is NULL (open cluster).
 * The box is read back to the host in stream order (one wait on hip_stream), since the cell list
 * and the image stencil are set up on the host; everything else is as dpk_compute_device. */
int dpk_compute_device_dbox(dpk_ctx *c, int64_t natoms, const double *d_coord,
                            const int32_t *d_atype, const double *d_box, double *d_energy,
                            double *d_force, double *d_virial, double *d_atom_energy,
                            void *hip_stream);

/* The device-pointer entry point for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation. Same arguments, layout,
 * results and stream semantics as dpk_compute_device, with a periodic box required (box == NULL
 * is DPK_E_INVALID_ARG: an open cluster's bounding box is read back to the host). The call makes
 * no device allocation and no hipMalloc/hipFree: the frame's workspace (cell list, neighbour
 * list, descriptor, fitting scratch, block partials, statistics) lives in one fixed region of
 * 256 MiB per device, part of the library's image and held until the process ends. A frame whose
 * workspace exceeds it is rejected with DPK_E_BUDGET (with the water model of cfg. sel [46, 92]:
 * about 24,000 atoms in DPK_MIXED, 11,000 in DPK_FP64). Every call on a device shares that
 * region, which keeps the last call's contents (the library clears what must start at zero):
 * calls that overlap on one device, from any context or thread, race and give wrong results, so
 * the caller serialises them (one stream, or events). dpk_ctx_check, dpk_ctx_stats and the debug
 * dumps after such a call read the region; the context's own workspace is left as it was. The
 * stage profiler records nothing for these calls. */
int dpk_compute_device_noalloc(dpk_ctx *c, int64_t natoms, const double *d_coord,
                               const int32_t *d_atype, const double *box, double *d_energy,
                               double *d_force, double *d_virial, double *d_atom_energy,
                               void *hip_stream);

/* Wait for the context's last stream and report device-side errors of the last frame:
 * DPK_E_TYPE_RANGE, DPK_E_NBR_OVERFLOW (candidate buffer, or a cut by sel in strict mode), or a
 * failed HIP call (DPK_E_DEVICE); DPK_OK before any frame. */
int dpk_ctx_check(dpk_ctx *c);

/* Candidate-buffer entries per atom of the neighbour search for the frames that follow: 0 (sized
 * from each frame's mean density, the default), 256, 512 or 1024 (the largest; a frame that
 * overflows it has more than 1024 atoms within r_c of one atom). Any other value is
 * DPK_E_INVALID_ARG. Open clusters always use 1024. */
int dpk_ctx_set_candidate_capacity(dpk_ctx *c, int entries);

/* Statistics of the last frame (waits for it): neighbours cut by sel (reading R6; Sec. II.A pads
 * lists to N_c), table inputs outside the table's range (Sec. II.A.6; reading R9: the nearest
 * piece is extrapolated), the largest number of atoms within r_c of one atom, and the device
 * bytes the context holds. */
int dpk_ctx_stats(dpk_ctx *c, dpk_stats *out);

/* Stage profiler. While enabled, every frame records HIP events on its stream around each stage
 * below; dpk_ctx_profile_read waits for the context's last stream and returns the summed stage
 * durations (milliseconds, one per stage) and the number of frames since profiling was enabled.
 * Enabling resets the sums. For timing tools (no effect on results). */
enum {
    DPK_STAGE_PREP = 0,      /* type partition, wrap into the cell, bins, candidate records */
    DPK_STAGE_NLIST = 1,     /* candidate search, sorted per-type selection                 */
    DPK_STAGE_EMBED_FWD = 2, /* environment rows, embedding net, contraction T              */
    DPK_STAGE_FIT = 3,       /* descriptor, fitting net forward and input gradient           */
    DPK_STAGE_EMBED_BWD = 4, /* embedding re-evaluation, adjoint, forces, block E and virial */
    DPK_STAGE_FINAL = 5,     /* energy and virial sums over the blocks                       */
    DPK_NSTAGES = 6
};
/* Enable (1) or disable (0) the profiler; waits for the context's last frame. */
int dpk_ctx_profile(dpk_ctx *c, int enable);
/* stage_ms: DPK_NSTAGES doubles (host, caller-owned); frames: 1 int64 or NULL. */
int dpk_ctx_profile_read(dpk_ctx *c, double *stage_ms, int64_t *frames);

/* Stage dumps of the last computed frame (host buffers, caller-owned, caller order), for parity
 * tests; DPK_E_INVALID_ARG before any frame. nlist: natoms * N_c neighbour indices (caller
 * numbering, -1 padding), the per-type blocks of Sec. II.A.1 (N_c padding, Sec. II.A), each
 * sorted by (distance, index, image) as Sec. III.B.1 orders them. */
int dpk_debug_nlist(dpk_ctx *c, int32_t *nlist);
/* The descriptor factor T = N_c^-1 G^T R of Sec. II.A.1 (natoms * M * 4: atom, feature m,
 * component k) and dE/dT (same layout), as FP64. */
int dpk_debug_descriptor(dpk_ctx *c, double *T, double *dT);

/* ---------------------------------------------------------------------------------------------
 * Model deviation (Sec. II.C): an ensemble of n_m models of one description (same types, sel,
 * cut-offs, widths, type_one_side and table, different parameters) evaluated on one frame. The
 * types, cell list and neighbour list are built once for all models; embedding, fitting and
 * adjoint run for all models together (one launch per stage). With ensemble averages
 * <y> = n_m^-1 sum_k y_k:
 *   eps_F,i = sqrt(< |F_i - <F_i>|^2 >),   eps_Xi,ab = N^-1 sqrt(< (Xi_ab - <Xi_ab>)^2 >),
 * and, for nu >= 0, the relative forms eps_F,i / (|<F_i>| + nu) and eps_Xi,ab / (|<Xi_ab>| + nu)
 * (the paper's |<Xi>| read per component). Statistics: max, average and min of eps_F,i over the
 * atoms and of eps_Xi,ab over the nine components.
 * -------------------------------------------------------------------------------------------- */
#define DPK_MAX_MODELS 16
typedef struct dpk_devi dpk_devi;

typedef struct {
    double f_max, f_avg, f_min;   /* of eps_F,i over the atoms                 */
    double v_max, v_avg, v_min;   /* of eps_Xi,ab over the nine components     */
} dpk_devi_stats;

/* Create an ensemble on `device` in `precision` (as dpk_ctx_create) from n_models models in
 * 1..DPK_MAX_MODELS, each packed and copied to the device (the models must outlive the ensemble).
 * Every descriptor kind (se_e2_a, se_e2_r, se_e3), network or compressed. DPK_E_INVALID_ARG for
 * NULL pointers, a bad count, or models whose descriptions or tables differ from model 0's. */
int dpk_devi_create(const dpk_model *const *models, int n_models, int device, int precision,
                    dpk_devi **out);
void dpk_devi_free(dpk_devi *d);

/* Evaluate every model on one frame (host buffers as dpk_compute; synchronous) and the deviations.
 * nu < 0: absolute deviations; nu >= 0: the relative forms. Outputs (host, caller-owned, any may be
 * NULL): energy [n_models]; force [n_models][natoms][3] (caller atom order); virial
 * [n_models][9]; eps_f [natoms]; eps_v [9] (Xi_ab at [3a + b]); stats. Errors as dpk_compute. */
int dpk_devi_compute(dpk_devi *d, int64_t natoms, const double *coord, const int32_t *atype,
                     const double *box, double nu, double *energy, double *force, double *virial,
                     double *eps_f, double *eps_v, dpk_devi_stats *stats);

/* ---------------------------------------------------------------------------------------------
 * Serving: continuous admission of frames of uneven size from many concurrent simulations (the
 * paper's inference interfaces serve MD codes frame by frame, Sec. III.A and III.D; here frames of
 * many simulations share the device).
 * A server owns nslots device slots on one GPU (each a context with its own stream and workspace,
 * sharing one copy of the model). A scheduler thread admits queued frames in arrival order as
 * soon as a slot is idle and the HBM budget (model + every slot's workspace) allows, freeing idle
 * slots' workspaces when that makes room; admitted work runs concurrently on the slots' streams.
 * A free slot takes the longest prefix of the queue that the budget admits (up to 64 frames of at
 * most 8192 atoms each) as one batch: one launch per stage for all of its frames, atoms of all
 * frames sorted by type together, each frame with its own cell, bins and results. The head of
 * the queue is never overtaken. A frame with an atom type out of range fails at submission
 * (DPK_E_TYPE_RANGE on its ticket); if a batch reports another data error, its frames run again
 * one by one so that only the faulty frame fails. Batches go back to the slot that ran the
 * previous frame of their first frame's simulation when it is idle, reusing its device buffers.
 * -------------------------------------------------------------------------------------------- */
typedef struct dpk_server dpk_server;

typedef struct {
    int64_t natoms;
    const double *coord;      /* host, [natoms][3]; caller keeps it alive until the frame is done */
    const int32_t *atype;     /* host, [natoms]                                                     */
    const double *box;        /* host, 9 doubles, or NULL                                           */
    double *energy;           /* host outputs, written when the frame completes                     */
    double *force;            /* [natoms][3]                                                        */
    double *virial;           /* [9]                                                                */
    double *atom_energy;      /* [natoms] or NULL                                                   */
    int64_t simulation;       /* id of the simulation the frame belongs to, or -1                   */
} dpk_frame;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t peak_bytes;        /* largest device footprint (model + slot workspaces) reached     */
    int64_t budget_waits;      /* frames whose admission waited for the budget (each counted once) */
    int64_t slot_reuse;        /* batches that ran on the slot of their simulation's previous frame */
    int64_t launches;          /* batches launched (frames completed / launches = mean batch size) */
} dpk_server_counters;

/* Create a server for model m (which must outlive it) on `device` with a precision as for
 * dpk_ctx_create. hbm_budget_bytes bounds model + all slot workspaces (0: no bound); nslots in
 * 1..64, else DPK_E_INVALID_ARG. Starts the scheduler thread. */
int dpk_server_create(const dpk_model *m, int device, int precision, int nslots,
                      size_t hbm_budget_bytes, dpk_server **out);
/* Queue a frame (E, F, virial as dpk_compute; host buffers, caller-owned); returns at once with a
 * ticket. DPK_E_INVALID_ARG for a NULL pointer or natoms < 1, DPK_E_BOX for a bad cell,
 * DPK_E_BUDGET if the frame alone exceeds the budget. The server reads coord, atype and box and
 * writes the outputs until the frame is done: the caller keeps them valid until dpk_server_poll or
 * dpk_server_wait reports it done. */
int dpk_server_submit(dpk_server *s, const dpk_frame *f, uint64_t *ticket);
/* *done = 0 while queued or running, 1 when finished successfully, or the frame's (negative)
 * error code. Never blocks. */
int dpk_server_poll(dpk_server *s, uint64_t ticket, int *done);
/* Block until the frame finishes; returns its result code (error text via dpk_last_error). */
int dpk_server_wait(dpk_server *s, uint64_t ticket);
/* As dpk_server_wait for at most timeout_us microseconds (>= 0): DPK_E_TIMEOUT if the frame is
 * still queued or running then (it stays in the server; wait, poll or cancel it later). For callers
 * that keep a per-request deadline. */
int dpk_server_wait_for(dpk_server *s, uint64_t ticket, int64_t timeout_us);
/* Withdraw a frame that is still queued: it finishes at once with DPK_E_CANCELLED (its outputs
 * untouched) and the server no longer reads its inputs. A frame already admitted to a slot runs to
 * completion: DPK_E_INVALID_ARG (as for an unknown or finished ticket), the frame unaffected. */
int dpk_server_cancel(dpk_server *s, uint64_t ticket);
/* Forget a finished frame's record (its result code and times); the ticket is unknown afterwards.
 * DPK_E_INVALID_ARG if the frame is still queued or running. Records of finished frames are kept
 * until released (or until dpk_server_free). */
int dpk_server_release(dpk_server *s, uint64_t ticket);
/* Host steady-clock nanoseconds of the frame's submission, start on the device and completion
 * (times[3]); valid once the frame is done. */
int dpk_server_times(dpk_server *s, uint64_t ticket, int64_t *times);
/* Counters since creation (a consistent snapshot). */
int dpk_server_stats(dpk_server *s, dpk_server_counters *out);
/* Waits for every queued frame, then frees the server and its slots. */
void dpk_server_free(dpk_server *s);

/* The server's admission rule as a pure function (no device work): choose a slot for a frame
 * needing need_bytes of workspace, given each slot's busy flag, workspace bytes and last
 * simulation id. Returns 1 (admit into *slot; if *release_idle, the other idle slots' workspaces
 * are freed and the chosen one resized to need_bytes first), 0 (wait), or DPK_E_BUDGET (the frame
 * cannot fit even on an empty device). budget_bytes = 0 means unbounded. */
int dpk_admit_plan(int nslots, const int32_t *busy, const int64_t *slot_bytes,
                   const int64_t *slot_sim, int64_t need_bytes, int64_t simulation,
                   int64_t budget_bytes, int64_t model_bytes, int32_t *slot,
                   int32_t *release_idle);

/* ------------------------------------------------------------------------------------------
 * Training (Sec. II.B, "Trainer"): the loss of eq. loss for one frame and its gradient with
 * respect to every model parameter, in FP64 on the device, including the force and virial terms
 * (derivatives of the forces with respect to the parameters: second derivatives of E). The
 * learning-rate schedule (eq. learning_rate), the prefactor schedule p(tau) and Adam steps on a
 * device copy of the parameters. se_e2_a models.
 * ---------------------------------------------------------------------------------------- */
typedef struct dpk_trainer dpk_trainer;

/* Labels and prefactors of one frame's loss, L = p_e L_E + p_f L_F + p_v L_Xi with
 * L_E = (E - E*)^2 / N, L_F = sum_k q_k |F_k - F*_k|^2 / (3N), L_Xi = sum_ab (Xi - Xi*)_ab^2 / (9N)
 * (eq. loss and the per-atom prefactor form L_F^p; q_k = 1/|F*_k|^2 gives the relative form L_F^r).
 * A NULL label leaves its term out; every pointer is read during the call only. */
typedef struct {
    const double *energy;      /* E*, one value, or NULL                                   */
    const double *force;       /* F* [natoms][3] (caller order), or NULL                   */
    const double *virial;      /* Xi* [9], or NULL                                         */
    const double *atom_pref;   /* q_k [natoms], or NULL (all 1)                            */
    double pe, pf, pv;         /* prefactors p_E, p_F, p_Xi                                */
} dpk_loss_spec;

/* Copy the model's parameters to `device` (FP64) with zero gradient and Adam moments. The model
 * is copied; the caller may free it afterwards. DPK_E_UNIMPLEMENTED for se_e2_r and se_e3 models,
 * DPK_E_INVALID_ARG for NULL pointers, DPK_E_DEVICE / DPK_E_OOM on device failures. */
int dpk_trainer_create(const dpk_model *m, int device, dpk_trainer **out);
void dpk_trainer_free(dpk_trainer *t);

/* One frame (host buffers, caller order; box as dpk_compute): evaluate E, F and Xi with the
 * current parameters, the loss (loss[4] = {L, L_E, L_F, L_Xi}, the terms unweighted), and add
 * weight * dL/dtheta to the trainer's gradient (weight = 1/B averages a mini-batch of B frames,
 * eq. loss). energy/force/virial receive the prediction if not NULL. The gradient stays on the
 * device. Errors as dpk_compute. */
int dpk_trainer_accumulate(dpk_trainer *t, int64_t natoms, const double *coord, const int32_t *atype,
                           const double *box, const dpk_loss_spec *spec, double weight, double *loss,
                           double *energy, double *force, double *virial);

/* Host copy of the accumulated gradient (dpk_model_param_count values, blob layout). */
int dpk_trainer_gradient(dpk_trainer *t, double *grad);
/* Clear the accumulated gradient. */
int dpk_trainer_zero_grad(dpk_trainer *t);
/* One Adam step (Kingma and Ba) with the accumulated gradient and learning rate lr (moments
 * beta1, beta2, eps; bias corrections from the trainer's step count), then clear the gradient. */
int dpk_trainer_adam_step(dpk_trainer *t, double lr, double beta1, double beta2, double eps);
/* Host copy of the current parameters (blob layout), or replace them (moments and step kept). */
int dpk_trainer_params(dpk_trainer *t, double *params);
int dpk_trainer_set_params(dpk_trainer *t, const double *params);

/* eq. learning_rate: lr0 * r^floor(step / decay_steps), r = (lr_stop / lr0)^(decay_steps / stop_steps). */
double dpk_learning_rate(double lr0, double lr_stop, int64_t step, int64_t stop_steps, int64_t decay_steps);
/* The prefactor schedule p = p_limit (1 - lr / lr0) + p_start lr / lr0. */
double dpk_loss_prefactor(double p_start, double p_limit, double lr, double lr0);

#ifdef __cplusplus
}
#endif
#endif /* DPK_H */
