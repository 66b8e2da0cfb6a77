// dpk_launch.h -- host-side launchers of the libdpk kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "dpk_internal.h"

namespace dpk {

// Set the calling thread's error message (dpk_last_error) and return code.
int set_error(int code, const char* msg);

void launch_zero(void* p, size_t bytes, hipStream_t s);
// Bytes of the per-device workspace of the allocation-free entry point, and the number of devices
// it is tracked for.
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;
constexpr int MAX_DEVICES = 64;
// Device address of that workspace on `device`, which must be the current device (looked up once
// per device, then cached); 0 on success, -1 if the lookup failed.
int scratch_region(int device, void** ptr);
// Preparation of a frame of any size in three launches; cell_count is zero on entry and on exit
// (the caller clears it once after allocating it); cell_tmp holds n ints of scratch.
void launch_prep_large(int n, const double* coord, const int* atype, int ntypes, const GeomParams& gp, int* tcount,
                       int* toff, int* bcount, int* boff, int* perm, int* inv_perm, int* itype, DevStats* st,
                       double* pos, int* cell_of, int* cell_count, int* cell_start, int* cursor, int* cell_tmp,
                       double4* cand, double* f_int, hipStream_t s, int nlocal = -1);
void launch_bbox(int n, const double* coord, double* out, hipStream_t s);
// All preparation phases in one workgroup; false (nothing launched) when the frame is too large.
// nlocal (both preparations): atoms nlocal.. n - 1 are ghosts, placed after the owned atoms in
// the internal order (class ntypes, so ntypes < MAXT); -1: no ghosts.
bool launch_prep_small(int n, const double* coord, const int* atype, int ntypes, const GeomParams& gp, int* tcount,
                       int* toff, int* perm, int* inv_perm, int* itype, DevStats* st, double* pos, int* cell_of,
                       int* cell_start, double4* cand, double* f_int, hipStream_t s, int nlocal = -1);
// Single frame: gp by value, gps == nullptr. Batch: gps/fd/frame_of on the device and the largest
// stencil and candidate buffer of the batch's frames.
void launch_nlist(int n, const double* pos, const int* perm, const int* inv_perm, const int* cell_of,
                  const int* cell_start, const double4* cand, const GeomParams& gp, int* nl_j, double* nl_r,
                  int* nnei, DevStats* st, hipStream_t s, const GeomParams* gps = nullptr,
                  const FrameDesc* fd = nullptr, const int* frame_of = nullptr, int max_stencil = 0, int max_cap = 0);
// Batched frames (each at most prep_small_max_atoms() atoms and prep_small_max_cells() bins).
void launch_batch_prep(int nframes, int ntypes, const double* coord, const int* atype, const GeomParams* gps,
                       FrameDesc* fd, int* tcount, int* toff, int* perm, int* inv_perm, int* itype, int* frame_of,
                       DevStats* st, double* pos, int* cell_of, int* cell_start, double4* cand, double* f_int,
                       double* vir_atom, hipStream_t s);
void launch_finalize_batch(int nframes, const FrameDesc* fd, const int* inv_perm, const double* ei,
                           const double* vir_atom, const double* f_int, double* out, DevStats* st, hipStream_t s);
int prep_small_max_atoms();
int prep_small_max_cells();
void launch_debug_nlist(int n, int ncentre, int nc, const int* perm, const int* nl_j, int* out, hipStream_t s);
// Neighbour lists of the nlocal owned atoms from external candidate lists (CSR by caller index over
// the owned atoms: ext_start [nlocal + 1], ext [ext_start[nlocal]] caller indices < ntot).
void launch_nlist_ext(int nlocal, int ntot, const double* pos, const int* perm, const int* inv_perm, const int* itype,
                      const int* ext_start, const int* ext, const GeomParams& gp, int* nl_j, double* nl_r, int* nnei,
                      DevStats* st, hipStream_t s);
// Per-atom force deviation of an ensemble of nm models (model k's forces at F + k * stride doubles).
void launch_force_devi(int n, int nm, const double* F, int64_t stride, double nu, double* eps, hipStream_t s);

// precision: 0 = FP64, 1 = split-BF16 (three products), 2 = BF16 (one product), 3 = FP32
// blocks of the embedding backward for a frame on the network or the table path (one [E, virial]
// partial each; the two paths have their own launch shapes), and their maximum over launch shapes
// (workspace sizing)
int embed_bwd_blocks(int precision, bool table, int64_t natoms, int ncu, bool e3 = false);
int64_t embed_bwd_max_blocks(int precision, int64_t natoms);
// E and the virial of a single frame from the backward pass's nb partials [E, virial[9]], and the
// frame's dropped-neighbour count into st
void launch_finalize(int nb, const double* part, double* energy, double* virial, DevStats* st, hipStream_t s);
int fit_atoms_per_block(int precision);
void launch_embed_fwd(int precision, bool table, const EmbArgs& a, hipStream_t s, bool e3 = false);
void launch_embed_bwd(int precision, bool table, const EmbArgs& a, hipStream_t s, bool e3 = false);
void launch_e3_env(int precision, const EmbArgs& a, hipStream_t s);
// Tabulated embedding of the two-body descriptors as products with the table (forward or
// backward), its block count (one [E, virial] partial each) and its smallest block in atoms.
void launch_tab(bool fwd, int precision, const EmbArgs& a, hipStream_t s);
// order[k] = internal index of candidate record k (records in bin order, one per atom; n records);
// *cnt (zero on entry) += the number of internal atoms i < n - 1 in the bin of atom i + 1
void launch_spatial_order(int n, const double4* cand, const int* cell_of, int* order, int* cnt, hipStream_t s);
int tab_blocks(int64_t natoms, int ncu);
int tab_atoms_per_block_min();
void launch_fit(int precision, const FitArgs& a, hipStream_t s);
// BF16 fitting kernel (split = three products); 16-atom tiles per block for a frame of natoms
void launch_fitx(bool split, const FitArgs& a, hipStream_t s);
int fitx_tiles_per_block(int natoms, int ncu);

}  // namespace dpk
