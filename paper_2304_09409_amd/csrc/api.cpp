// api.cpp -- host side of libdpk: the C ABI declared in include/dpk.h.
//
// Model packing (per precision), the quintic table build (Sec. II.A.6, eq. compress), device
// workspace management, frame geometry set-up and the launch sequence of one evaluation:
//   types -> cell list -> neighbour list -> embedding + contraction (T) -> fitting (E_i, dE/dT)
//   -> adjoint (F, virial) -> reductions.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dpk.h"
#include "arena.h"
#include "dpk_internal.h"
#include "dpk_launch.h"
#include "dpk_train.h"

using namespace dpk;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(DPK_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_float(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Embedding nets: one per (a_i, a_j), one per a_j (type_one_side), or, for the three-body
// descriptor, one per ordered pair of neighbour types (a_j, a_k) (Sec. II.A.1).
int emb_nets(const dpk_model_desc* d)
{
    return (d->type_one_side && d->descriptor != DPK_SE_E3) ? d->ntypes : d->ntypes * d->ntypes;
}

// Width of the descriptor, the fitting net's input: M x M_< (se_e2_a) or M (se_e2_r, se_e3).
int fit_width(const dpk_model_desc* d) { return d->descriptor == DPK_SE_E2_A ? d->emb[2] * d->axis : d->emb[2]; }

int64_t count_params(const dpk_model_desc* d)
{
    int e[4] = {1, d->emb[0], d->emb[1], d->emb[2]};
    int f[5] = {fit_width(d), d->fit[0], d->fit[1], d->fit[2], 1};
    int64_t nets = emb_nets(d);
    int64_t c = 0;
    for (int k = 0; k < 3; ++k) c += nets * ((int64_t)e[k] * e[k + 1] + 2 * e[k + 1]);
    for (int k = 0; k < 4; ++k) c += (int64_t)d->ntypes * ((int64_t)f[k] * f[k + 1] + 2 * f[k + 1]);
    return c;
}

struct Layer {
    int nin, nout;
    const double *W, *b, *wh;
};

}  // namespace

struct dpk_model {
    dpk_model_desc desc;
    std::vector<double> params;
    int nets = 0, nc = 0;
    std::vector<Layer> emb;   // [nets][3]
    std::vector<Layer> fit;   // [ntypes][4]
    bool tabulated = false;
    double tab_dx = 0.0;
    double tab_xmax = 0.0;
    int tab_nint = 0;
    std::vector<double> table;   // [nets][nint][100][6]
};

namespace {

void index_layers(dpk_model* m)
{
    const dpk_model_desc& d = m->desc;
    int e[4] = {1, d.emb[0], d.emb[1], d.emb[2]};
    int f[5] = {fit_width(&d), d.fit[0], d.fit[1], d.fit[2], 1};
    const double* p = m->params.data();
    auto take = [&](int nin, int nout) {
        Layer L{nin, nout, p, p + (int64_t)nin * nout, p + (int64_t)nin * nout + nout};
        p += (int64_t)nin * nout + 2 * nout;
        return L;
    };
    m->emb.clear();
    m->fit.clear();
    for (int n = 0; n < m->nets; ++n)
        for (int k = 0; k < 3; ++k) m->emb.push_back(take(e[k], e[k + 1]));
    for (int t = 0; t < d.ntypes; ++t)
        for (int k = 0; k < 4; ++k) m->fit.push_back(take(f[k], f[k + 1]));
}

// Value and first two derivatives (d/dx) of embedding net `net` at x, carried forward through
// the layers of eq. NN (tanh, skip by size).
void embed_derivs(const dpk_model* m, int net, double x, double* y, double* y1, double* y2)
{
    std::vector<double> z{x}, z1{1.0}, z2{0.0};
    for (int k = 0; k < 3; ++k) {
        const Layer& L = m->emb[(size_t)net * 3 + k];
        std::vector<double> a(L.nout), n0(L.nout), n1(L.nout), n2(L.nout);
        for (int o = 0; o < L.nout; ++o) {
            double v = L.b[o], v1 = 0.0, v2 = 0.0;
            for (int i = 0; i < L.nin; ++i) {
                const double w = L.W[(int64_t)i * L.nout + o];
                v += z[i] * w;
                v1 += z1[i] * w;
                v2 += z2[i] * w;
            }
            const double t = std::tanh(v), gp = 1.0 - t * t;
            const double t1 = gp * v1, t2 = gp * v2 - 2.0 * t * gp * v1 * v1;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            if (L.nout == L.nin) { s0 = z[o]; s1 = z1[o]; s2 = z2[o]; }
            else if (L.nout == 2 * L.nin) { s0 = z[o % L.nin]; s1 = z1[o % L.nin]; s2 = z2[o % L.nin]; }
            n0[o] = L.wh[o] * t + s0;
            n1[o] = L.wh[o] * t1 + s1;
            n2[o] = L.wh[o] * t2 + s2;
        }
        z.swap(n0);
        z1.swap(n1);
        z2.swap(n2);
    }
    for (int o = 0; o < E2; ++o) { y[o] = z[o]; y1[o] = z1[o]; y2[o] = z2[o]; }
}

// Physical position of logical K index k in the packed embedding weights, so that each lane's
// operands of one MFMA fragment are contiguous. FP64 (16-wide chunks): lanes of group g supply
// k = 16c + g + 4v (v = 0..3). BF16 paths (32-wide chunks of v_mfma_f32_16x16x32_bf16): lanes
// of group g supply positions 8g..8g+7, holding k = 32c + 4g + v (v < 4) and 32c + 16 + 4g + v - 4
// (v >= 4), i.e. rows 4g..4g+3 of the previous layer's output tiles 2c and 2c + 1.
inline int kphys(int precision, int k)
{
    if (precision == DPK_FP32) return k;   // lane group g holds K values 16c + 4g + v: already contiguous
    if (precision != DPK_FP64) {
        const int c = k >> 5, r = k & 31;
        return 32 * c + 8 * ((r & 15) >> 2) + (r >> 4) * 4 + (r & 3);
    }
    const int c = k >> 4, r = k & 15;
    return 16 * c + 4 * (r & 3) + (r >> 2);
}

// K index held by value j (0..7) of lane group g in K-chunk c of a fragment-major BF16 matrix:
// the 16x16x32 BF16 MFMA reads k = 8g + j of the chunk; values 0..3 are rows 4g..4g+3 of the
// previous layer's output tile 2c and values 4..7 the same rows of tile 2c + 1.
inline int kidx32(int c, int g, int j) { return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4)); }

// Row position of register u of lane group g in embedding layer l (the K position of layer 1, the
// output row of layers 2 and 3) for the precision's MFMA layout: FP64 lanes of group g hold K
// values 16c + g + 4v and output rows g + 4r of each tile, FP32 K values 16c + 4g + v and output
// rows 4g + r, the BF16 paths K values kidx32(c, g, v) and output rows 4g + r.
inline int emb_pos(int precision, int l, int g, int u)
{
    const bool f64 = precision == DPK_FP64;
    if (l == 1) {
        if (precision == DPK_FP32) return 16 * (u / 4) + 4 * g + u % 4;
        const int vpl = f64 ? 4 : 8, c = u / vpl, v = u % vpl;
        return f64 ? 16 * c + g + 4 * v : kidx32(c, g, v);
    }
    const int r = u & 3;
    return 16 * (u >> 2) + (f64 ? g + 4 * r : 4 * g + r);
}

// Pack one matrix of `rows` x `kdim` (zero-padded to the tiles and chunks) in fragment-major
// order: fragment (c, t) at frag0 + c * ntiles + t, lane 16g + i holding row 16t + i.
template <class Fn>
void pack_frags(std::vector<uint16_t>& out, size_t frag0, int ntiles, int nch, int rows, int kdim, bool split,
                Fn&& w)
{
    for (int c = 0; c < nch; ++c)
        for (int t = 0; t < ntiles; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int row = 16 * t + (lane & 15), k = kidx32(c, lane >> 4, j);
                    const double v = (row < rows && k < kdim) ? w(row, k) : 0.0;
                    const uint16_t hb = bf16_bits((float)v);
                    const size_t i = (frag0 + (size_t)c * ntiles + t) * XF_ELEMS + lane * 8 + j;
                    out[i] = hb;
                    out[i + 512] = split ? bf16_bits((float)(v - (double)bf16_float(hb))) : 0;
                }
}

// Dense matrix (row-major, `rows` x `cols`) in each plane's element type.
struct Planes {
    int precision;
    std::vector<double> d;     // FP64
    std::vector<float> f;      // FP32
    std::vector<uint16_t> h, l;
    void init(int prec, size_t n) {
        precision = prec;
        if (prec == DPK_FP64) d.assign(n, 0.0);
        else if (prec == DPK_FP32) f.assign(n, 0.0f);
        else { h.assign(n, 0); if (prec == DPK_MIXED) l.assign(n, 0); }
    }
    void set(size_t i, double v) {
        if (precision == DPK_FP64) { d[i] = v; return; }
        if (precision == DPK_FP32) { f[i] = (float)v; return; }
        const uint16_t hb = bf16_bits((float)v);
        h[i] = hb;
        if (precision == DPK_MIXED) l[i] = bf16_bits((float)(v - (double)bf16_float(hb)));
    }
};

}  // namespace

struct dpk_ctx {
    const dpk_model* model = nullptr;
    int device = 0, precision = 0, strict = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;        // own stream for the host entry point
    hipStream_t last_stream = nullptr;   // stream of the last frame
    size_t acc_size = 8;
    int ncu = 256;                       // compute units of the device
    // device model
    void* evec = nullptr;
    void* emat = nullptr;
    void* fvec = nullptr;
    void* fmat = nullptr;
    void* table = nullptr;
    // the table as uploaded when the context was created (a later dpk_model_tabulate does not
    // change what this context evaluates)
    bool tab = false;
    double tab_dx = 0.0;
    int tab_nint = 0;
    size_t model_bytes = 0;
    size_t evec_b = 0, emat_b = 0, fvec_b = 0, fmat_b = 0, table_b = 0;   // bytes of each packed buffer
    bool owns_model = true;              // false for server slots sharing the first slot's copy
    // workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    Arena* arena = nullptr;              // server slot under a budget: the workspace is carved from it
    int64_t cap_atoms = 0;
    int64_t cap_cells = 0;
    bool cells_clear = false;            // cell_count is all zero (the multi-block preparation keeps it so)
    bool views_scratch = false;          // the views below point into the device's shared scratch
    void* scratch = nullptr;             // that scratch (allocation-free entry point), this device's copy
    int* ext_buf = nullptr;              // external neighbour candidates (ghost-atom entry point)
    size_t ext_cap = 0;                  // ints it holds
    // views of the workspace (valid for the capacity)
    int *perm, *inv_perm, *itype, *tcount, *toff, *cell_of, *cell_tmp, *cell_count, *cell_start, *cursor;
    int *nl_j, *nnei, *h_atype, *bcount, *boff;
    double *pos, *nl_r, *Ei, *F, *vir_part, *bbox, *h_coord, *h_out;
    double4* cand;
    int* frame_of;                       // batched frames: frame of each internal atom
    double* vir_atom;                    // batched frames: virial per centre atom [N][9]
    FrameDesc* fd;                       // batched frames: [BATCH_MAX_FRAMES]
    GeomParams* gps;                     // batched frames: [BATCH_MAX_FRAMES]
    void* pin_desc = nullptr;            // pinned staging of fd and gps
    hipEvent_t desc_copied = nullptr;    // recorded after the last copy out of pin_desc
    bool desc_pending = false;
    void *T, *dT, *act;
    void* env;                           // three-body descriptor: environment rows [N][nc][4]
    DevStats* stats;
    int64_t vir_blocks = 0;
    // frame being set up (for the candidate-buffer estimate) and the overflow retry switch
    int64_t cur_natoms = 0;
    bool force_big_cap = false;
    int cap_fixed = 0;                   // candidate-buffer entries set by the caller (0: estimated)
    // last frame: atoms, and the centre atoms among them (fewer with ghost atoms)
    int64_t last_n = 0;
    int64_t last_centres = 0;
    // stage profiler: one set of DPK_NSTAGES + 1 events per profiled frame
    bool profiling = false;
    std::vector<std::vector<hipEvent_t>> prof_events;
    size_t prof_used = 0;
};

namespace {

int check_stats(const dpk_ctx* c, const DevStats& st);

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool is_e3(const dpk_ctx* c) { return c->model->desc.descriptor == DPK_SE_E3; }
// The fitting net runs on the dense kernel (FP64 or FP32 weights, a scratch row of 6 x 240 per
// atom) for FP64 and FP32, and for every precision when the descriptor has M values.
bool dense_fitting(const dpk_ctx* c)
{
    return c->precision == DPK_FP64 || c->precision == DPK_FP32 || c->model->desc.descriptor != DPK_SE_E2_A;
}

// Atom slots of the fitting grid for n atoms: the dense kernel's 64-atom blocks leave at most 63
// padding slots; the BF16-path kernel tiles each species separately (at most 64 per species).
int64_t fit_slots(int64_t n, bool dense)
{
    return (n + FIT_AF - 1) / FIT_AF * FIT_AF + FIT_AF * (dense ? 1 : MAXT + 1);
}

// Byte layout of the workspace for n atoms and ncell bins; if base != nullptr, assign views.
size_t layout_ws(dpk_ctx* c, int64_t n, int64_t ncell, char* base)
{
    const dpk_model* m = c->model;
    const int nt = m->desc.ntypes, nc = m->nc;
    const int64_t nvb = embed_bwd_max_blocks(c->precision, n);
    const bool e3 = c->model->desc.descriptor == DPK_SE_E3;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    char* p;
    p = take(sizeof(int) * n); if (base) c->perm = (int*)p;
    p = take(sizeof(int) * n); if (base) c->inv_perm = (int*)p;
    p = take(sizeof(int) * n); if (base) c->itype = (int*)p;
    p = take(sizeof(int) * MAXT); if (base) c->tcount = (int*)p;
    p = take(sizeof(int) * (MAXT + 1)); if (base) c->toff = (int*)p;
    p = take(sizeof(int) * MAXT * ((n + PREP_BLOCK - 1) / PREP_BLOCK)); if (base) c->bcount = (int*)p;
    p = take(sizeof(int) * MAXT * ((n + PREP_BLOCK - 1) / PREP_BLOCK)); if (base) c->boff = (int*)p;
    p = take(sizeof(int) * STATS_WORDS); if (base) c->stats = (DevStats*)p;   // with the drop counters
    p = take(sizeof(double) * 3 * n); if (base) c->pos = (double*)p;
    p = take(sizeof(int) * n); if (base) c->cell_of = (int*)p;
    p = take(sizeof(int) * n); if (base) c->cell_tmp = (int*)p;
    p = take(sizeof(double4) * n); if (base) c->cand = (double4*)p;
    p = take(sizeof(int) * ncell); if (base) c->cell_count = (int*)p;
    p = take(sizeof(int) * (ncell + 1)); if (base) c->cell_start = (int*)p;
    p = take(sizeof(int) * ncell); if (base) c->cursor = (int*)p;
    p = take(sizeof(int) * n * nc); if (base) c->nl_j = (int*)p;
    p = take(sizeof(int) * n * nt); if (base) c->nnei = (int*)p;
    p = take(sizeof(double) * 3 * n * nc); if (base) c->nl_r = (double*)p;
    p = take(c->acc_size * n * E2 * 4); if (base) c->T = p;
    p = take(c->acc_size * n * E2 * 4); if (base) c->dT = p;
    // fitting scratch, for every atom slot of the fitting grid (padding lanes get their own rows):
    // FP64 [slots][6][240] with at most 63 padding slots; BF16 paths [blocks][3][16][tiles][64][4]
    // (XF_ACT floats per 16 slots), species-aligned tiles: at most 64 padding slots per species
    const bool dense_fit = dense_fitting(c);
    const int64_t nfit = fit_slots(n, dense_fit);
    p = take(dense_fit ? c->acc_size * nfit * 6 * FW : sizeof(float) * (nfit / 16) * XF_ACT);
    if (base) c->act = p;
    p = take(e3 ? c->acc_size * n * nc * 4 : 0); if (base) c->env = e3 ? p : nullptr;
    p = take(sizeof(double) * n); if (base) c->Ei = (double*)p;
    p = take(sizeof(double) * 3 * n); if (base) c->F = (double*)p;
    p = take(sizeof(double) * 10 * nvb); if (base) { c->vir_part = (double*)p; c->vir_blocks = nvb; }
    p = take(sizeof(double) * 8); if (base) c->bbox = (double*)p;
    p = take(sizeof(double) * 3 * n); if (base) c->h_coord = (double*)p;
    p = take(sizeof(int) * n); if (base) c->h_atype = (int*)p;
    p = take(sizeof(double) * (10 * BATCH_MAX_FRAMES + 4 * n)); if (base) c->h_out = (double*)p;
    p = take(sizeof(int) * n); if (base) c->frame_of = (int*)p;
    p = take(sizeof(double) * 9 * n); if (base) c->vir_atom = (double*)p;
    p = take(sizeof(FrameDesc) * BATCH_MAX_FRAMES); if (base) c->fd = (FrameDesc*)p;
    p = take(sizeof(GeomParams) * BATCH_MAX_FRAMES); if (base) c->gps = (GeomParams*)p;
    return off;
}

// Returns the event set of this frame (nullptr when not profiling).
std::vector<hipEvent_t>* prof_frame(dpk_ctx* c)
{
    if (!c->profiling) return nullptr;
    if (c->prof_used == c->prof_events.size()) {
        std::vector<hipEvent_t> ev(DPK_NSTAGES + 1);
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->prof_events.push_back(ev);
    }
    return &c->prof_events[c->prof_used++];
}

inline void prof_mark(std::vector<hipEvent_t>* ev, int k, hipStream_t s)
{
    if (ev) hipEventRecord((*ev)[k], s);
}

// The workspace's memory goes back where it came from: the server's arena, or the device.
void free_ws_mem(dpk_ctx* c)
{
    if (c->arena && c->arena->owns(c->ws)) c->arena->give_back((char*)c->ws - c->arena->base, (int64_t)c->ws_bytes);
    else hipFree(c->ws);
    c->ws = nullptr;
}

// arena_only (a server slot's admission): carve from the arena or report DPK_E_BUDGET, without
// falling back to a device allocation
int ensure_ws(dpk_ctx* c, int64_t n, int64_t ncell, bool arena_only = false)
{
    if (n <= c->cap_atoms && ncell <= c->cap_cells && c->ws) {
        if (c->views_scratch) {
            // the last frame ran in the shared scratch: point the views back at this workspace
            layout_ws(c, c->cap_atoms, c->cap_cells, (char*)c->ws);
            c->views_scratch = false;
        }
        return DPK_OK;
    }
    int64_t nn = std::max<int64_t>(n, c->cap_atoms), ncl = std::max<int64_t>(ncell, c->cap_cells);
    size_t bytes = layout_ws(c, nn, ncl, nullptr);
    if (c->budget && bytes + c->model_bytes > c->budget)
        return fail(DPK_E_BUDGET, "frame of %lld atoms needs %zu workspace bytes + %zu model bytes, budget %zu",
                    (long long)n, bytes, c->model_bytes, c->budget);
    if (c->ws) {
        // the old buffers may still be used by work queued on this context's streams
        if (c->last_stream) HIPCHK(hipStreamSynchronize(c->last_stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        free_ws_mem(c);
    }
    void* p = nullptr;
    const int64_t off = c->arena ? c->arena->carve((int64_t)bytes) : -1;
    if (off >= 0) {
        p = c->arena->base + off;
    } else if (arena_only) {
        c->ws_bytes = 0;
        c->cap_atoms = c->cap_cells = 0;
        return DPK_E_BUDGET;
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        // (a slot's admission carves its workspace from the arena beforehand; only a launch that
        // needs more than was admitted comes here)
        hipGetLastError();
        return fail(DPK_E_OOM, "hipMalloc of %zu workspace bytes failed", bytes);
    }
    c->ws = p;
    c->ws_bytes = bytes;
    c->cap_atoms = nn;
    c->cap_cells = ncl;
    c->cells_clear = false;
    c->views_scratch = false;
    layout_ws(c, nn, ncl, (char*)p);
    return DPK_OK;
}

// Cell geometry (Sec. II.A: coordinates under PBC or in vacuum). Rows of h are the lattice
// vectors; fractional s = r h^-1; perpendicular width d_k = det h / |a_l x a_m|.
int setup_geometry(dpk_ctx* c, const double* box, const double* bbox, GeomParams& gp)
{
    const dpk_model* m = c->model;
    const double rc = m->desc.rcut;
    std::memset(&gp, 0, sizeof(gp));
    gp.rc2 = rc * rc;
    gp.ntypes = m->desc.ntypes;
    gp.nc = m->nc;
    int acc = 0;
    for (int t = 0; t < m->desc.ntypes; ++t) {
        gp.sel[t] = m->desc.sel[t];
        gp.off[t] = acc;
        acc += m->desc.sel[t];
    }
    if (box) {
        const double* h = box;
        const double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                           h[2] * (h[3] * h[7] - h[4] * h[6]);
        if (!(det > 0.0)) return fail(DPK_E_BOX, "det(box) = %g is not positive", det);
        gp.periodic = 1;
        for (int k = 0; k < 9; ++k) gp.h[k] = h[k];
        gp.hinv[0] = (h[4] * h[8] - h[5] * h[7]) / det;
        gp.hinv[1] = (h[2] * h[7] - h[1] * h[8]) / det;
        gp.hinv[2] = (h[1] * h[5] - h[2] * h[4]) / det;
        gp.hinv[3] = (h[5] * h[6] - h[3] * h[8]) / det;
        gp.hinv[4] = (h[0] * h[8] - h[2] * h[6]) / det;
        gp.hinv[5] = (h[2] * h[3] - h[0] * h[5]) / det;
        gp.hinv[6] = (h[3] * h[7] - h[4] * h[6]) / det;
        gp.hinv[7] = (h[1] * h[6] - h[0] * h[7]) / det;
        gp.hinv[8] = (h[0] * h[4] - h[1] * h[3]) / det;
        for (int k = 0; k < 3; ++k) {
            const double* a = h + 3 * ((k + 1) % 3);
            const double* b = h + 3 * ((k + 2) % 3);
            const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
            const double width = det / std::sqrt(cx * cx + cy * cy + cz * cz);
            // bins of at least r_c (a 3 x 3 x 3 stencil; bins of r_c / 2 visit less volume, 15.6 r_c^3
            // against 27 r_c^3, but their 125-bin stencil set-up cost more than that saved on the
            // water and fcc boxes)
            int nb = (int)std::floor(width / rc);
            if (nb < 1) nb = 1;
            if (nb > 256) nb = 256;
            gp.nb[k] = nb;
            gp.K[k] = (int)std::ceil(rc / (width / nb));
        }
        // expected atoms within r_c at the frame's mean density, doubled plus a margin
        const double expect = (double)c->cur_natoms / det * 4.18879020478639 * rc * rc * rc;
        const double want = 2.0 * expect + 64.0;
        gp.cap = c->force_big_cap ? NL_CAP
                 : c->cap_fixed     ? c->cap_fixed
                                    : (want <= 256.0 ? 256 : (want <= 512.0 ? 512 : NL_CAP));
        if ((2 * gp.K[0] + 1) * (2 * gp.K[1] + 1) * (2 * gp.K[2] + 1) > NL_STENCIL)
            return fail(DPK_E_BOX, "cell too thin for r_c: a width below r_c/3 needs more than %d image bins", NL_STENCIL);
    } else {
        gp.periodic = 0;
        for (int k = 0; k < 3; ++k) {
            const double lo = bbox[k], hi = bbox[3 + k];
            double ext = hi - lo;
            int nb = (int)std::floor(ext / rc);
            if (nb < 1) nb = 1;
            if (nb > 256) nb = 256;
            gp.nb[k] = nb;
            gp.origin[k] = lo;
            gp.binw[k] = (ext > 0.0 ? ext : 1.0) / nb;
            if (nb * gp.binw[k] < ext) gp.binw[k] = std::nextafter(gp.binw[k], 1e300);
            gp.K[k] = (int)std::ceil(rc / gp.binw[k]);
            if (gp.K[k] > nb) gp.K[k] = nb;
        }
        gp.cap = NL_CAP;   // clusters can be locally dense: largest buffer
    }
    return DPK_OK;
}

template <class T>
int upload(void** dst, const T* src, size_t n)
{
    HIPCHK(hipMalloc(dst, sizeof(T) * n));
    HIPCHK(hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice));
    return DPK_OK;
}

int upload_planes(void** dst, const Planes& P)
{
    if (P.precision == DPK_FP64) return upload(dst, P.d.data(), P.d.size());
    if (P.precision == DPK_FP32) return upload(dst, P.f.data(), P.f.size());
    std::vector<uint16_t> all(P.h);
    all.insert(all.end(), P.l.begin(), P.l.end());
    return upload(dst, all.data(), all.size());
}

// Pack and upload the model for one precision.
int upload_model(dpk_ctx* c)
{
    const dpk_model* m = c->model;
    const int prec = c->precision, nets = m->nets, nt = m->desc.ntypes;
    const bool f64 = prec == DPK_FP64;
    // FP64 and FP32 fit on the 16x16x4 MFMA with dense row-major weights (k_fit_dense); the BF16
    // paths use fragment-major weights (k_fitx), except for a descriptor of M values, which every
    // precision other than FP64 fits on the dense FP32 kernel
    const bool radial = m->desc.descriptor != DPK_SE_E2_A;
    const bool dense = dense_fitting(c);
    const int fprec = f64 ? DPK_FP64 : DPK_FP32;   // precision of the dense fitting weights
    std::vector<double> ev((size_t)nets * EVEC, 0.0), fv((size_t)nt * FVEC, 0.0);
    Planes em, fm;
    em.init(prec, (size_t)nets * EM_SIZE);
    if (dense) fm.init(fprec, (size_t)nt * FM_SIZE);
    std::vector<uint16_t> fx;
    if (!dense) fx.assign((size_t)nt * XF_NFRAG * XF_ELEMS, 0);
    // feature at each row position of the embedding layers in the skip-aligned order (-1: padding,
    // zero weights)
    int f1[K2P], f2[N2P], f3[N3P];
    for (int g = 0; g < 4; ++g) {
        for (int u = 0; u < K2P / 4; ++u) f1[emb_pos(prec, 1, g, u)] = emb_feat(1, g, u);
        for (int u = 0; u < N2P / 4; ++u) f2[emb_pos(prec, 2, g, u)] = emb_feat(2, g, u);
        for (int u = 0; u < N3P / 4; ++u) f3[emb_pos(prec, 3, g, u)] = emb_feat(3, g, u);
    }
    for (int n = 0; n < nets; ++n) {
        const Layer* L = &m->emb[(size_t)n * 3];
        double* v = &ev[(size_t)n * EVEC];
        for (int k = 0; k < K2P; ++k)
            if (f1[k] >= 0) {
                v[EV_W1 + k] = L[0].W[f1[k]];
                v[EV_B1 + k] = L[0].b[f1[k]];
                v[EV_WH1 + k] = L[0].wh[f1[k]];
            }
        for (int k = 0; k < N2P; ++k)
            if (f2[k] >= 0) { v[EV_B2 + k] = L[1].b[f2[k]]; v[EV_WH2 + k] = L[1].wh[f2[k]]; }
        for (int k = 0; k < N3P; ++k)
            if (f3[k] >= 0) { v[EV_B3 + k] = L[2].b[f3[k]]; v[EV_WH3 + k] = L[2].wh[f3[k]]; }
        const size_t base = (size_t)n * EM_SIZE;
        for (int k = 0; k < K2P; ++k)
            for (int o = 0; o < N2P; ++o)
                if (f1[k] >= 0 && f2[o] >= 0)
                    em.set(base + EM_W2T + (size_t)o * K2P + kphys(prec, k), L[1].W[f1[k] * E1 + f2[o]]);
        for (int k = 0; k < N2P; ++k)
            for (int o = 0; o < N3P; ++o)
                if (f2[k] >= 0 && f3[o] >= 0)
                    em.set(base + EM_W3T + (size_t)o * N2P + kphys(prec, k), L[2].W[f2[k] * E2 + f3[o]]);
    }
    for (int t = 0; t < nt; ++t) {
        const Layer* L = &m->fit[(size_t)t * 4];
        double* v = &fv[(size_t)t * FVEC];
        for (int k = 0; k < FW; ++k) {
            v[FV_B1 + k] = L[0].b[k]; v[FV_WH1 + k] = L[0].wh[k];
            v[FV_B2 + k] = L[1].b[k]; v[FV_WH2 + k] = L[1].wh[k];
            v[FV_B3 + k] = L[2].b[k]; v[FV_WH3 + k] = L[2].wh[k];
            v[FV_W4 + k] = L[3].W[k];
        }
        v[FV_B4] = L[3].b[0];
        v[FV_WH4] = L[3].wh[0];
        if (!dense) {
            // fragment-major BF16 packing: W[in][out] of each layer, read as W^T (forward) or W (backward)
            const bool split = prec == DPK_MIXED;
            const size_t f0 = (size_t)t * XF_NFRAG;
            const double *W1 = L[0].W, *W2 = L[1].W, *W3 = L[2].W;
            pack_frags(fx, f0 + XF_W1F, 15, XF_NCH1, FW, DD, split, [&](int o, int f) { return W1[(size_t)f * FW + o]; });
            pack_frags(fx, f0 + XF_W2F, 15, XF_NCH2, FW, FW, split, [&](int o, int i) { return W2[(size_t)i * FW + o]; });
            pack_frags(fx, f0 + XF_W3F, 15, XF_NCH2, FW, FW, split, [&](int o, int i) { return W3[(size_t)i * FW + o]; });
            pack_frags(fx, f0 + XF_W3B, 15, XF_NCH2, FW, FW, split, [&](int i, int o) { return W3[(size_t)i * FW + o]; });
            pack_frags(fx, f0 + XF_W2B, 15, XF_NCH2, FW, FW, split, [&](int i, int o) { return W2[(size_t)i * FW + o]; });
            pack_frags(fx, f0 + XF_W1B, E2, XF_NCH2, DD, FW, split, [&](int f, int o) { return W1[(size_t)f * FW + o]; });
            continue;
        }
        const size_t base = (size_t)t * FM_SIZE;
        // layer 1: W1^T [240][K] and W1 [K][240], K = 1600 (M x M_<) or 112 (M, zero-padded)
        const int nin = radial ? E2 : DD, kw = radial ? N3P : DD;
        for (int f = 0; f < nin; ++f)
            for (int o = 0; o < FW; ++o) {
                const double w = L[0].W[(int64_t)f * FW + o];
                fm.set(base + FM_W1T + (size_t)o * kw + kphys(fprec, f), w);
                fm.set(base + FM_W1 + (size_t)f * FW + kphys(fprec, o), w);
            }
        for (int li = 1; li <= 2; ++li) {
            const int64_t mt = li == 1 ? FM_W2T : FM_W3T, mw = li == 1 ? FM_W2 : FM_W3;
            for (int i = 0; i < FW; ++i)
                for (int o = 0; o < FW; ++o) {
                    const double w = L[li].W[(int64_t)i * FW + o];
                    fm.set(base + mt + (size_t)o * FW + kphys(fprec, i), w);
                    fm.set(base + mw + (size_t)i * FW + kphys(fprec, o), w);
                }
        }
    }
    int rc;
    if (f64) {
        if ((rc = upload(&c->evec, ev.data(), ev.size()))) return rc;
        if ((rc = upload(&c->fvec, fv.data(), fv.size()))) return rc;
    } else {
        std::vector<float> evf(ev.begin(), ev.end()), fvf(fv.begin(), fv.end());
        if ((rc = upload(&c->evec, evf.data(), evf.size()))) return rc;
        if ((rc = upload(&c->fvec, fvf.data(), fvf.size()))) return rc;
    }
    if ((rc = upload_planes(&c->emat, em))) return rc;
    if (dense) {
        if ((rc = upload_planes(&c->fmat, fm))) return rc;
    } else if ((rc = upload(&c->fmat, fx.data(), fx.size()))) {
        return rc;
    }
    c->evec_b = ev.size() * c->acc_size;
    c->fvec_b = fv.size() * c->acc_size;
    c->emat_b = f64 ? em.d.size() * 8 : prec == DPK_FP32 ? em.f.size() * 4 : (em.h.size() + em.l.size()) * 2;
    c->fmat_b = f64 ? fm.d.size() * 8 : dense ? fm.f.size() * 4 : fx.size() * 2;
    c->model_bytes = c->evec_b + c->fvec_b + c->emat_b + c->fmat_b;
    if (m->tabulated) {
        // the per-interval layout, then the table as the row-major matrix C[6 l + j][m] and its
        // transpose (the two-body descriptors' product kernels read whole 16-wide rows of both)
        const int nint = m->tab_nint, kp = tab_kp(nint);
        const size_t nets = (size_t)m->nets, prod = nets * kp * N3P;
        std::vector<double> tab(m->table.size() + 2 * prod, 0.0);
        std::copy(m->table.begin(), m->table.end(), tab.begin());
        double* tk = tab.data() + m->table.size();
        double* tm = tk + prod;
        for (size_t net = 0; net < nets; ++net)
            for (int l = 0; l < nint; ++l)
                for (int o = 0; o < E2; ++o)
                    for (int j = 0; j < 6; ++j) {
                        const double v = m->table[((net * nint + l) * E2 + o) * 6 + j];
                        tk[(net * kp + 6 * l + j) * N3P + o] = v;
                        tm[(net * N3P + o) * kp + 6 * l + j] = v;
                    }
        if (f64) {
            if ((rc = upload(&c->table, tab.data(), tab.size()))) return rc;
        } else {
            std::vector<float> tf(tab.begin(), tab.end());
            if ((rc = upload(&c->table, tf.data(), tf.size()))) return rc;
        }
        c->table_b = tab.size() * c->acc_size;
        c->model_bytes += c->table_b;
        c->tab = true;
        c->tab_dx = m->tab_dx;
        c->tab_nint = m->tab_nint;
    }
    return DPK_OK;
}

// Embedding, fitting and adjoint over n atoms (internal order), after the neighbour list.
// vir_atom == nullptr: virial as per-block partials; else per centre atom (batched frames).
// Embedding, fitting and the backward pass. F: force accumulator in caller order (zeroed by the
// preparation). Single frame (single = true): per-block partials [E, virial] and E_i in caller
// order (atom_energy, if not nullptr); batch: per-atom virials (vir_atom).
// spatial: the candidate records hold exactly the n centres (no ghosts), so the tabulated
// backward may take its atoms in their bin order
void run_network(dpk_ctx* c, int n, const GeomParams& gp, double* F, double* vir_atom, bool single,
                 double* atom_energy, std::vector<hipEvent_t>* ev, hipStream_t s, bool spatial = true)
{
    const dpk_model* m = c->model;
    const int nt = m->desc.ntypes;
    EmbArgs ea;
    std::memset(&ea, 0, sizeof(ea));
    ea.natoms = n;
    ea.ntypes = nt;
    ea.nc = m->nc;
    ea.type_one_side = m->desc.type_one_side;
    ea.ncu = c->ncu;
    ea.apw = 1;
    for (int t = 0; t < nt; ++t) ea.off[t] = gp.off[t];
    ea.itype = c->itype;
    ea.nnei = c->nnei;
    ea.nl_j = c->nl_j;
    ea.nl_r = c->nl_r;
    ea.rs = m->desc.rcut_smth;
    ea.rc = m->desc.rcut;
    // se_e3: D = N_c^-2 sum over neighbour pairs; its nets are indexed by the pair's types
    const bool e3 = is_e3(c);
    ea.inv_nc = e3 ? 1.0 / ((double)m->nc * m->nc) : 1.0 / m->nc;
    if (e3) ea.type_one_side = 0;
    ea.env = c->env;
    ea.evec = c->evec;
    ea.emat = c->emat;
    ea.table = c->table;
    ea.tab_dx = c->tab_dx;
    ea.tab_nint = c->tab_nint;
    ea.T = c->T;
    ea.dT = c->dT;
    ea.perm = c->perm;
    ea.F = F;
    ea.vir_part = c->vir_part;
    ea.vir_atom = vir_atom;
    ea.stats = c->stats;
    if (single) {
        ea.Ei = c->Ei;
        ea.atom_energy = atom_energy;
    }
    const bool tab = c->tab;
    prof_mark(ev, DPK_STAGE_EMBED_FWD, s);
    if (e3) launch_e3_env(c->precision, ea, s);
    launch_embed_fwd(c->precision, tab, ea, s, e3);

    FitArgs fa;
    std::memset(&fa, 0, sizeof(fa));   // one model: nmodels and the per-model strides zero
    fa.natoms = n;
    fa.ntypes = nt;
    fa.ncu = c->ncu;
    fa.itype = c->itype;
    fa.toff = c->toff;
    fa.fvec = c->fvec;
    fa.fmat = c->fmat;
    fa.T = c->T;
    fa.dT = c->dT;
    fa.act = c->act;
    fa.Ei = c->Ei;
    fa.radial = m->desc.descriptor != DPK_SE_E2_A;
    prof_mark(ev, DPK_STAGE_FIT, s);
    launch_fit(c->precision, fa, s);

    prof_mark(ev, DPK_STAGE_EMBED_BWD, s);
    if (tab && !e3 && spatial) {
        // the preparation's bin-sort scratch (cell_tmp) is free once the lists are built
        // (its count goes to the statistics block, which the preparation cleared)
        launch_spatial_order(n, c->cand, c->cell_of, c->cell_tmp, &c->stats->order_local, s);
        ea.order = c->cell_tmp;
        ea.order_cnt = &c->stats->order_local;
    }
    launch_embed_bwd(c->precision, tab, ea, s, e3);
}

// The launches of one frame on the views laid out for it. shared: the views point into the
// device's shared scratch, which keeps whatever the last call left, so the bin counts are cleared
// every time, and no profiler event is recorded.
// Preparation (partition, wrap, bin; d_force zeroed) and neighbour search of one frame.
void enqueue_geometry(dpk_ctx* c, int n, const double* d_coord, const int* d_atype, const GeomParams& gp,
                      double* d_force, hipStream_t s, bool shared, std::vector<hipEvent_t>* ev)
{
    const int nt = c->model->desc.ntypes;
    prof_mark(ev, DPK_STAGE_PREP, s);
    if (!launch_prep_small(n, d_coord, d_atype, nt, gp, c->tcount, c->toff, c->perm, c->inv_perm, c->itype, c->stats,
                           c->pos, c->cell_of, c->cell_start, c->cand, d_force, s)) {
        if (shared) {
            launch_zero(c->cell_count, sizeof(int) * (size_t)gp.nb[0] * gp.nb[1] * gp.nb[2], s);
        } else {
            if (!c->cells_clear) launch_zero(c->cell_count, sizeof(int) * (size_t)c->cap_cells, s);
            c->cells_clear = false;
        }
        launch_prep_large(n, d_coord, d_atype, nt, gp, c->tcount, c->toff, c->bcount, c->boff, c->perm, c->inv_perm,
                          c->itype, c->stats, c->pos, c->cell_of, c->cell_count, c->cell_start, c->cursor, c->cell_tmp,
                          c->cand, d_force, s);
        if (!shared) c->cells_clear = true;   // its scan clears the counts it read
    }
    prof_mark(ev, DPK_STAGE_NLIST, s);
    launch_nlist(n, c->pos, c->perm, c->inv_perm, c->cell_of, c->cell_start, c->cand, gp, c->nl_j, c->nl_r, c->nnei,
                 c->stats, s);
}

void enqueue_frame(dpk_ctx* c, int n, const double* d_coord, const int* d_atype, const GeomParams& gp,
                   double* d_energy, double* d_force, double* d_virial, double* d_atom_energy, hipStream_t s,
                   bool shared)
{
    // the forces accumulate straight into d_force (caller order), which the preparation zeroes
    std::vector<hipEvent_t>* ev = shared ? nullptr : prof_frame(c);
    enqueue_geometry(c, n, d_coord, d_atype, gp, d_force, s, shared, ev);
    run_network(c, n, gp, d_force, nullptr, true, d_atom_energy, ev, s);
    prof_mark(ev, DPK_STAGE_FINAL, s);
    launch_finalize(embed_bwd_blocks(c->precision, c->tab, n, c->ncu, is_e3(c)), c->vir_part, d_energy, d_virial,
                    c->stats, s);
    prof_mark(ev, DPK_NSTAGES, s);
}

// One frame of a batch: host copies of the coordinates (for an open cluster's bounding box) and
// of the cell.
struct BatchFrame {
    int64_t natoms;
    const double* coord;
    const double* box;
    bool want_ei;
};

int frame_geometry(dpk_ctx* c, const BatchFrame& f, GeomParams& gp)
{
    c->cur_natoms = f.natoms;
    if (f.box) return setup_geometry(c, f.box, nullptr, gp);
    double bb[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
    for (int64_t i = 0; i < f.natoms; ++i)
        for (int k = 0; k < 3; ++k) {
            bb[k] = std::min(bb[k], f.coord[3 * i + k]);
            bb[3 + k] = std::max(bb[3 + k], f.coord[3 * i + k]);
        }
    return setup_geometry(c, nullptr, bb, gp);
}

// Layout of a batch: per-frame geometry and offsets, total atoms and concatenated bins (ncell + 1
// entries per frame), the largest stencil and candidate buffer. Outputs of frame f start at
// fd[f].out_off doubles: E, virial[9], F[3n] and, if asked for, E_i[n].
int batch_plan(dpk_ctx* c, int nf, const BatchFrame* fr, GeomParams* gps, FrameDesc* fd, int64_t* natoms,
               int64_t* ncells, int* max_stencil, int* max_cap, int64_t* out_doubles)
{
    if (nf < 1 || nf > BATCH_MAX_FRAMES) return fail(DPK_E_INVALID_ARG, "batch of %d frames", nf);
    int64_t n = 0, nc = 0, out = 0;
    int ms = 0, mc = 0;
    for (int f = 0; f < nf; ++f) {
        int rc = frame_geometry(c, fr[f], gps[f]);
        if (rc) return rc;
        const int64_t ncell = (int64_t)gps[f].nb[0] * gps[f].nb[1] * gps[f].nb[2];
        if (fr[f].natoms > prep_small_max_atoms() || ncell > prep_small_max_cells())
            return fail(DPK_E_INVALID_ARG, "frame of %lld atoms / %lld bins is too large for a batch",
                        (long long)fr[f].natoms, (long long)ncell);
        std::memset(&fd[f], 0, sizeof(FrameDesc));
        fd[f].atom_off = (int)n;
        fd[f].natoms = (int)fr[f].natoms;
        fd[f].cell_off = (int)nc;
        fd[f].ncell = (int)ncell;
        fd[f].out_off = (int)out;
        fd[f].want_ei = fr[f].want_ei ? 1 : 0;
        n += fr[f].natoms;
        nc += ncell + 1;
        out += 10 + (fr[f].want_ei ? 4 : 3) * fr[f].natoms;
        ms = std::max(ms, (2 * gps[f].K[0] + 1) * (2 * gps[f].K[1] + 1) * (2 * gps[f].K[2] + 1));
        mc = std::max(mc, gps[f].cap);
    }
    *natoms = n;
    *ncells = nc;
    *max_stencil = ms;
    *max_cap = mc;
    *out_doubles = out;
    return DPK_OK;
}

// Pinned staging of a batch's frame descriptors and geometries (allocated once per context).
int ensure_pin_desc(dpk_ctx* c)
{
    if (c->pin_desc) return DPK_OK;
    if (hipHostMalloc(&c->pin_desc, (sizeof(FrameDesc) + sizeof(GeomParams)) * BATCH_MAX_FRAMES) != hipSuccess) {
        c->pin_desc = nullptr;
        return fail(DPK_E_OOM, "pinned staging of the batch descriptors failed");
    }
    if (hipEventCreateWithFlags(&c->desc_copied, hipEventDisableTiming) != hipSuccess) {
        hipHostFree(c->pin_desc);
        c->pin_desc = nullptr;
        c->desc_copied = nullptr;
        return fail(DPK_E_DEVICE, "event for the batch descriptors' staging failed");
    }
    return DPK_OK;
}

// Several frames in one launch per stage (serving): coordinates and types of all frames
// concatenated in caller order on the device; results of frame f at d_out + fd[f].out_off.
int compute_batch(dpk_ctx* c, int nf, const BatchFrame* fr, const double* d_coord, const int* d_atype,
                  double* d_out, hipStream_t s)
{
    GeomParams gps[BATCH_MAX_FRAMES];
    FrameDesc fd[BATCH_MAX_FRAMES];
    int64_t n, ncells, outd;
    int ms, mc, rc;
    if ((rc = batch_plan(c, nf, fr, gps, fd, &n, &ncells, &ms, &mc, &outd))) return rc;
    if ((rc = ensure_ws(c, n, ncells))) return rc;
    if ((rc = ensure_pin_desc(c))) return rc;
    // the staging is rewritten once the previous batch's copies out of it have completed (an
    // event on exactly those copies: a wait on the stream would also wait for the coordinates
    // just queued on it)
    if (c->desc_pending) HIPCHK(hipEventSynchronize(c->desc_copied));
    FrameDesc* pfd = (FrameDesc*)c->pin_desc;
    GeomParams* pgp = (GeomParams*)(pfd + BATCH_MAX_FRAMES);
    std::memcpy(pfd, fd, sizeof(FrameDesc) * nf);
    std::memcpy(pgp, gps, sizeof(GeomParams) * nf);
    HIPCHK(hipMemcpyAsync(c->fd, pfd, sizeof(FrameDesc) * nf, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->gps, pgp, sizeof(GeomParams) * nf, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(c->desc_copied, s));
    c->desc_pending = true;
    const int nt = c->model->desc.ntypes;
    launch_batch_prep(nf, nt, d_coord, d_atype, c->gps, c->fd, c->tcount, c->toff, c->perm, c->inv_perm, c->itype,
                      c->frame_of, c->stats, c->pos, c->cell_of, c->cell_start, c->cand, c->F, c->vir_atom, s);
    launch_nlist((int)n, c->pos, c->perm, c->inv_perm, c->cell_of, c->cell_start, c->cand, gps[0], c->nl_j, c->nl_r,
                 c->nnei, c->stats, s, c->gps, c->fd, c->frame_of, ms, mc);
    run_network(c, (int)n, gps[0], c->F, c->vir_atom, false, nullptr, nullptr, s);
    launch_finalize_batch(nf, c->fd, c->inv_perm, c->Ei, c->vir_atom, c->F, d_out, c->stats, s);
    HIPCHK(hipGetLastError());
    c->last_stream = s;
    c->last_n = n;
    c->last_centres = n;
    return DPK_OK;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

const char* dpk_last_error(void) { return g_err.c_str(); }

int64_t dpk_model_param_count(const dpk_model_desc* desc)
{
    if (!desc || desc->ntypes < 1 || desc->ntypes > DPK_MAX_TYPES) return -1;
    return count_params(desc);
}

int dpk_model_create(const dpk_model_desc* desc, const double* params, int64_t nparams, dpk_model** out)
{
    if (!desc || !params || !out) return fail(DPK_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (desc->ntypes < 1 || desc->ntypes > DPK_MAX_TYPES) return fail(DPK_E_INVALID_ARG, "ntypes must be in 1..8");
    if (desc->emb[0] != E0 || desc->emb[1] != E1 || desc->emb[2] != E2 || desc->axis != AX ||
        desc->fit[0] != FW || desc->fit[1] != FW || desc->fit[2] != FW)
        return fail(DPK_E_UNIMPLEMENTED, "kernels are built for emb (25,50,100), axis 16, fit (240,240,240)");
    if (!(desc->rcut > desc->rcut_smth) || !(desc->rcut_smth > 0.0))
        return fail(DPK_E_INVALID_ARG, "need 0 < rcut_smth < rcut");
    int nc = 0;
    for (int t = 0; t < desc->ntypes; ++t) {
        if (desc->sel[t] < 0) return fail(DPK_E_INVALID_ARG, "negative sel");
        nc += desc->sel[t];
    }
    if (nc < 1 || nc > 4096) return fail(DPK_E_INVALID_ARG, "sum of sel must be in 1..4096");
    if (desc->descriptor < DPK_SE_E2_A || desc->descriptor > DPK_SE_E3)
        return fail(DPK_E_INVALID_ARG, "descriptor must be DPK_SE_E2_A, DPK_SE_E2_R or DPK_SE_E3");
    if (desc->descriptor == DPK_SE_E3 && nc > E3_MAXN)
        return fail(DPK_E_UNIMPLEMENTED, "the three-body kernels take a sum of sel up to %d", E3_MAXN);
    const int64_t need = count_params(desc);
    if (nparams != need) return fail(DPK_E_INVALID_ARG, "parameter blob has %lld values, model needs %lld",
                                     (long long)nparams, (long long)need);
    dpk_model* m = new dpk_model;
    m->desc = *desc;
    m->params.assign(params, params + nparams);
    m->nets = emb_nets(desc);
    m->nc = nc;
    index_layers(m);
    *out = m;
    return DPK_OK;
}

int dpk_model_tabulate(dpk_model* m, double stride, double x_max)
{
    if (!m || !(stride > 0.0) || !(x_max > 0.0)) return fail(DPK_E_INVALID_ARG, "bad table range");
    const int nint = (int)std::ceil(x_max / stride - 1e-9);
    if (nint < 1 || nint > 100000) return fail(DPK_E_INVALID_ARG, "table would have %d intervals", nint);
    const double dx = stride;
    m->table.assign((size_t)m->nets * nint * E2 * 6, 0.0);
    std::vector<double> y((size_t)(nint + 1) * E2), y1(y.size()), y2(y.size());
    for (int net = 0; net < m->nets; ++net) {
        for (int l = 0; l <= nint; ++l)
            embed_derivs(m, net, l * dx, &y[(size_t)l * E2], &y1[(size_t)l * E2], &y2[(size_t)l * E2]);
        for (int l = 0; l < nint; ++l)
            for (int o = 0; o < E2; ++o) {
                const double f0 = y[(size_t)l * E2 + o], f1 = y[(size_t)(l + 1) * E2 + o];
                const double d0 = y1[(size_t)l * E2 + o], d1 = y1[(size_t)(l + 1) * E2 + o];
                const double s0 = y2[(size_t)l * E2 + o], s1 = y2[(size_t)(l + 1) * E2 + o];
                const double h = f1 - f0, dx2 = dx * dx, dx3 = dx2 * dx;
                double* cf = &m->table[(((size_t)net * nint + l) * E2 + o) * 6];
                cf[0] = (12.0 * h - 6.0 * (d1 + d0) * dx + (s1 - s0) * dx2) / (2.0 * dx3 * dx2);
                cf[1] = (-30.0 * h + (14.0 * d1 + 16.0 * d0) * dx + (-2.0 * s1 + 3.0 * s0) * dx2) / (2.0 * dx2 * dx2);
                cf[2] = (20.0 * h - (8.0 * d1 + 12.0 * d0) * dx + (s1 - 3.0 * s0) * dx2) / (2.0 * dx3);
                cf[3] = 0.5 * s0;
                cf[4] = d0;
                cf[5] = f0;
            }
    }
    m->tabulated = true;
    m->tab_dx = dx;
    m->tab_xmax = x_max;
    m->tab_nint = nint;
    return DPK_OK;
}

int dpk_model_describe(const dpk_model* m, dpk_model_desc* desc, double* params, double* tab_stride,
                       double* tab_xmax)
{
    if (!m) return fail(DPK_E_INVALID_ARG, "NULL model");
    if (desc) *desc = m->desc;
    if (params) std::memcpy(params, m->params.data(), sizeof(double) * m->params.size());
    if (tab_stride) *tab_stride = m->tabulated ? m->tab_dx : 0.0;
    if (tab_xmax) *tab_xmax = m->tabulated ? m->tab_xmax : 0.0;
    return DPK_OK;
}

}  // extern "C"

int dpk::set_error(int code, const char* msg)
{
    return fail(code, "%s", msg);
}

extern "C" {

void dpk_model_free(dpk_model* m) { delete m; }

int dpk_ctx_create(const dpk_model* m, int device, int precision, size_t hbm_budget_bytes, int strict_sel,
                   dpk_ctx** out)
{
    if (!m || !out) return fail(DPK_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (precision < DPK_FP64 || precision > DPK_FP32) return fail(DPK_E_INVALID_ARG, "unknown precision %d", precision);
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(DPK_E_INVALID_ARG, "device %d not present (%d devices)", device, ndev);
    HIPCHK(hipSetDevice(device));
    dpk_ctx* c = new dpk_ctx;
    c->model = m;
    c->device = device;
    c->precision = precision;
    c->budget = hbm_budget_bytes;
    c->strict = strict_sel;
    c->acc_size = precision == DPK_FP64 ? 8 : 4;
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->ncu < 1)
        c->ncu = 256;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(DPK_E_DEVICE, "hipStreamCreate failed");
    }
    int rc = upload_model(c);
    if (rc) { dpk_ctx_free(c); return rc; }
    // the allocation-free entry point's scratch on this device (looked up once per device)
    if (scratch_region(device, &c->scratch) != 0) c->scratch = nullptr;
    if (c->budget && c->model_bytes > c->budget) {
        dpk_ctx_free(c);
        return fail(DPK_E_BUDGET, "model needs %zu device bytes, budget %zu", c->model_bytes, hbm_budget_bytes);
    }
    *out = c;
    return DPK_OK;
}

void dpk_ctx_free(dpk_ctx* c)
{
    if (!c) return;
    hipSetDevice(c->device);
    if (c->last_stream) hipStreamSynchronize(c->last_stream);
    if (c->stream) hipStreamSynchronize(c->stream);
    if (c->owns_model) {
        hipFree(c->evec); hipFree(c->emat); hipFree(c->fvec); hipFree(c->fmat); hipFree(c->table);
    }
    if (c->ws) free_ws_mem(c);
    hipFree(c->ext_buf);
    hipHostFree(c->pin_desc);
    if (c->desc_copied) hipEventDestroy(c->desc_copied);
    for (auto& set : c->prof_events)
        for (auto e : set) hipEventDestroy(e);
    if (c->stream) hipStreamDestroy(c->stream);
    delete c;
}

int64_t dpk_ctx_workspace_bytes(const dpk_ctx* c, int64_t natoms)
{
    if (!c || natoms < 1) return -1;
    // bins are at least r_c wide, so a frame has at most about one bin per atom at liquid density
    return (int64_t)layout_ws(const_cast<dpk_ctx*>(c), natoms, natoms + 1, nullptr) + (int64_t)c->model_bytes;
}

int dpk_compute_device(dpk_ctx* c, int64_t natoms, const double* d_coord, const int32_t* d_atype, const double* box,
                       double* d_energy, double* d_force, double* d_virial, double* d_atom_energy, void* hip_stream)
{
    if (!c || !d_coord || !d_atype || !d_energy || !d_force || !d_virial) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (natoms < 1 || natoms > (1LL << 30)) return fail(DPK_E_INVALID_ARG, "natoms = %lld", (long long)natoms);
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = (int)natoms;
    int rc;
    GeomParams gp;
    c->cur_natoms = natoms;
    if (box) {
        if ((rc = setup_geometry(c, box, nullptr, gp))) return rc;
    } else {
        // open boundary: bounding box of the cluster (one wait on the stream)
        if ((rc = ensure_ws(c, n, 1))) return rc;
        launch_bbox(n, d_coord, c->bbox, s);
        double bb[6];
        HIPCHK(hipMemcpyAsync(bb, c->bbox, sizeof(bb), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if ((rc = setup_geometry(c, nullptr, bb, gp))) return rc;
    }
    const int64_t ncell = (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2];
    if ((rc = ensure_ws(c, n, ncell))) return rc;
    enqueue_frame(c, n, d_coord, d_atype, gp, d_energy, d_force, d_virial, d_atom_energy, s, false);
    HIPCHK(hipGetLastError());
    c->last_stream = s;
    c->last_n = n;
    c->last_centres = n;
    return DPK_OK;
}

int dpk_compute_device_dbox(dpk_ctx* c, int64_t natoms, const double* d_coord, const int32_t* d_atype,
                            const double* d_box, double* d_energy, double* d_force, double* d_virial,
                            double* d_atom_energy, void* hip_stream)
{
    if (!c) return fail(DPK_E_INVALID_ARG, "NULL context");
    double hbox[9];
    if (d_box) {
        HIPCHK(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)hip_stream;
        // in stream order, so a box written by the caller's earlier work on this stream is seen
        HIPCHK(hipMemcpyAsync(hbox, d_box, sizeof(hbox), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return dpk_compute_device(c, natoms, d_coord, d_atype, d_box ? hbox : nullptr, d_energy, d_force, d_virial,
                              d_atom_energy, hip_stream);
}

int dpk_compute_device_noalloc(dpk_ctx* c, int64_t natoms, const double* d_coord, const int32_t* d_atype,
                               const double* box, double* d_energy, double* d_force, double* d_virial,
                               double* d_atom_energy, void* hip_stream)
{
    if (!c || !d_coord || !d_atype || !d_energy || !d_force || !d_virial) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (!box)
        return fail(DPK_E_INVALID_ARG, "the allocation-free entry point needs a periodic box (an open cluster's "
                                       "bounding box is read back to the host; use dpk_compute_device)");
    if (natoms < 1 || natoms > (1LL << 30)) return fail(DPK_E_INVALID_ARG, "natoms = %lld", (long long)natoms);
    if (!c->scratch) return fail(DPK_E_DEVICE, "no scratch region on device %d", c->device);
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = (int)natoms;
    int rc;
    GeomParams gp;
    c->cur_natoms = natoms;
    if ((rc = setup_geometry(c, box, nullptr, gp))) return rc;
    const int64_t ncell = (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2];
    const size_t need = layout_ws(c, n, ncell, nullptr);
    if (need > SCRATCH_BYTES)
        return fail(DPK_E_BUDGET, "a frame of %lld atoms and %lld bins needs %zu workspace bytes; the "
                                  "allocation-free entry point holds %zu", (long long)natoms, (long long)ncell, need,
                    SCRATCH_BYTES);
    // views into the shared scratch for this frame (the context's own workspace is untouched)
    layout_ws(c, n, ncell, (char*)c->scratch);
    c->views_scratch = true;
    enqueue_frame(c, n, d_coord, d_atype, gp, d_energy, d_force, d_virial, d_atom_energy, s, true);
    HIPCHK(hipGetLastError());
    c->last_stream = s;
    c->last_n = n;
    c->last_centres = n;
    return DPK_OK;
}

int dpk_compute_ghost(dpk_ctx* c, int64_t nlocal, int64_t nghost, const double* coord, const int32_t* atype,
                      const int32_t* ext_start, const int32_t* ext_list, double* energy, double* force,
                      double* virial, double* atom_energy)
{
    if (!c || !coord || !atype || !energy || !force || !virial) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (nlocal < 1 || nghost < 0 || nlocal + nghost > (1LL << 30))
        return fail(DPK_E_INVALID_ARG, "nlocal = %lld, nghost = %lld", (long long)nlocal, (long long)nghost);
    if ((ext_start == nullptr) != (ext_list == nullptr))
        return fail(DPK_E_INVALID_ARG, "ext_start and ext_list go together");
    const dpk_model* m = c->model;
    const int nt = m->desc.ntypes;
    if (nghost > 0 && nt >= MAXT)
        return fail(DPK_E_UNIMPLEMENTED, "ghost atoms need fewer than %d atom types", MAXT);
    const int64_t ntot = nlocal + nghost;
    int64_t next = 0;
    if (ext_start) {
        if (ext_start[0] != 0) return fail(DPK_E_INVALID_ARG, "ext_start[0] must be 0");
        for (int64_t i = 0; i < nlocal; ++i)
            if (ext_start[i + 1] < ext_start[i]) return fail(DPK_E_INVALID_ARG, "ext_start decreases at %lld", (long long)i);
        next = ext_start[nlocal];
        for (int64_t q = 0; q < next; ++q)
            if (ext_list[q] < 0 || ext_list[q] >= ntot)
                return fail(DPK_E_INVALID_ARG, "ext_list[%lld] = %d is outside [0, %lld)", (long long)q, ext_list[q],
                            (long long)ntot);
    }
    HIPCHK(hipSetDevice(c->device));
    // open geometry over owned and ghost atoms (ghosts carry image positions)
    double bb[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
    for (int64_t i = 0; i < ntot; ++i)
        for (int k = 0; k < 3; ++k) {
            bb[k] = std::min(bb[k], coord[3 * i + k]);
            bb[3 + k] = std::max(bb[3 + k], coord[3 * i + k]);
        }
    GeomParams gp;
    int rc;
    c->cur_natoms = ntot;
    if ((rc = setup_geometry(c, nullptr, bb, gp))) return rc;
    if ((rc = ensure_ws(c, ntot, (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2]))) return rc;
    hipStream_t s = c->stream;
    if (ext_start) {
        const size_t need = (size_t)(nlocal + 1 + next);
        if (need > c->ext_cap) {
            HIPCHK(hipStreamSynchronize(s));
            hipFree(c->ext_buf);
            c->ext_buf = nullptr;
            c->ext_cap = 0;
            if (hipMalloc((void**)&c->ext_buf, sizeof(int) * need) != hipSuccess) {
                hipGetLastError();
                c->ext_buf = nullptr;
                return fail(DPK_E_OOM, "hipMalloc of %zu bytes for the external neighbour list failed", sizeof(int) * need);
            }
            c->ext_cap = need;
        }
        HIPCHK(hipMemcpyAsync(c->ext_buf, ext_start, sizeof(int) * (nlocal + 1), hipMemcpyHostToDevice, s));
        if (next) HIPCHK(hipMemcpyAsync(c->ext_buf + nlocal + 1, ext_list, sizeof(int) * next, hipMemcpyHostToDevice, s));
    }
    const int n = (int)ntot, nl = (int)nlocal;
    HIPCHK(hipMemcpyAsync(c->h_coord, coord, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->h_atype, atype, sizeof(int) * n, hipMemcpyHostToDevice, s));
    double* o = c->h_out;   // E, virial, F [n][3], E_i [nlocal]
    double* d_force = o + 10;
    {
        if (!launch_prep_small(n, c->h_coord, c->h_atype, nt, gp, c->tcount, c->toff, c->perm, c->inv_perm, c->itype,
                               c->stats, c->pos, c->cell_of, c->cell_start, c->cand, d_force, s, nl)) {
            if (!c->cells_clear) launch_zero(c->cell_count, sizeof(int) * (size_t)c->cap_cells, s);
            c->cells_clear = false;
            launch_prep_large(n, c->h_coord, c->h_atype, nt, gp, c->tcount, c->toff, c->bcount, c->boff, c->perm,
                              c->inv_perm, c->itype, c->stats, c->pos, c->cell_of, c->cell_count, c->cell_start,
                              c->cursor, c->cell_tmp, c->cand, d_force, s, nl);
            c->cells_clear = true;
        }
        // lists for the owned atoms only (internal positions 0.. nlocal - 1); candidates are all atoms
        if (ext_start)
            launch_nlist_ext(nl, n, c->pos, c->perm, c->inv_perm, c->itype, c->ext_buf, c->ext_buf + nl + 1, gp,
                             c->nl_j, c->nl_r, c->nnei, c->stats, s);
        else
            launch_nlist(nl, c->pos, c->perm, c->inv_perm, c->cell_of, c->cell_start, c->cand, gp, c->nl_j, c->nl_r,
                         c->nnei, c->stats, s);
        // descriptor, fitting and adjoint over the owned atoms: E_i of owned atoms only; forces land
        // on owned and ghost atoms alike (the ghosts' are the caller's to send back to their owners)
        run_network(c, nl, gp, d_force, nullptr, true, atom_energy ? o + 10 + 3 * n : nullptr, nullptr, s, nl == n);
        launch_finalize(embed_bwd_blocks(c->precision, c->tab, nl, c->ncu, is_e3(c)), c->vir_part, o, o + 1, c->stats, s);
        HIPCHK(hipGetLastError());
        c->last_stream = s;
        c->last_n = n;
        c->last_centres = nl;
        // open geometry runs with the largest candidate buffer already: an overflow is final
        rc = dpk_ctx_check(c);
    }
    if (rc) return rc;
    std::vector<double> host(10 + 3 * (size_t)n + (atom_energy ? nlocal : 0));
    HIPCHK(hipMemcpy(host.data(), o, sizeof(double) * host.size(), hipMemcpyDeviceToHost));
    *energy = host[0];
    std::memcpy(virial, &host[1], sizeof(double) * 9);
    std::memcpy(force, &host[10], sizeof(double) * 3 * n);
    if (atom_energy) std::memcpy(atom_energy, &host[10 + 3 * n], sizeof(double) * nlocal);
    return DPK_OK;
}

int dpk_ctx_set_candidate_capacity(dpk_ctx* c, int entries)
{
    if (!c) return fail(DPK_E_INVALID_ARG, "NULL context");
    if (entries != 0 && entries != 256 && entries != 512 && entries != NL_CAP)
        return fail(DPK_E_INVALID_ARG, "candidate capacity must be 0, 256, 512 or %d", NL_CAP);
    c->cap_fixed = entries;
    return DPK_OK;
}

int dpk_ctx_check(dpk_ctx* c)
{
    if (!c) return fail(DPK_E_INVALID_ARG, "NULL context");
    if (!c->last_n) return DPK_OK;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->last_stream));
    DevStats st;
    HIPCHK(hipMemcpy(&st, c->stats, sizeof(st), hipMemcpyDeviceToHost));
    return check_stats(c, st);
}

}  // extern "C"

namespace {

// Error status of a finished frame from a host copy of its statistics block.
int check_stats(const dpk_ctx* c, const DevStats& st)
{
    if (st.err_type) return fail(DPK_E_TYPE_RANGE, "an atom type is outside [0, %d)", c->model->desc.ntypes);
    if (st.err_overflow)
        return fail(DPK_E_NBR_OVERFLOW, "%d atoms within r_c of one atom exceed the selection buffer (%d)", st.max_cand,
                    NL_CAP);
    if (c->strict && st.nbr_dropped)
        return fail(DPK_E_NBR_OVERFLOW, "%llu neighbours cut by sel (strict mode)", (unsigned long long)st.nbr_dropped);
    return DPK_OK;
}

}  // namespace

extern "C" {

int dpk_compute(dpk_ctx* c, int64_t natoms, const double* coord, const int32_t* atype, const double* box, double* energy,
                double* force, double* virial, double* atom_energy)
{
    if (!c || !coord || !atype || !energy || !force || !virial) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (natoms < 1 || natoms > (1LL << 30)) return fail(DPK_E_INVALID_ARG, "natoms = %lld", (long long)natoms);
    HIPCHK(hipSetDevice(c->device));
    // Size the workspace first (geometry from the host copy of the frame), so that the device
    // entry point below never reallocates the buffers the frame is staged in.
    GeomParams gp;
    int rc;
    c->cur_natoms = natoms;
    if (box) {
        if ((rc = setup_geometry(c, box, nullptr, gp))) return rc;
    } else {
        double bb[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
        for (int64_t i = 0; i < natoms; ++i)
            for (int k = 0; k < 3; ++k) {
                bb[k] = std::min(bb[k], coord[3 * i + k]);
                bb[3 + k] = std::max(bb[3 + k], coord[3 * i + k]);
            }
        if ((rc = setup_geometry(c, nullptr, bb, gp))) return rc;
    }
    if ((rc = ensure_ws(c, natoms, (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2]))) return rc;
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->h_coord, coord, sizeof(double) * 3 * natoms, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->h_atype, atype, sizeof(int) * natoms, hipMemcpyHostToDevice, s));
    double* o = c->h_out;
    rc = dpk_compute_device(c, natoms, c->h_coord, c->h_atype, box, o, o + 10, o + 1, o + 10 + 3 * natoms, s);
    if (rc) return rc;
    rc = dpk_ctx_check(c);
    if (rc == DPK_E_NBR_OVERFLOW && !c->force_big_cap && !c->strict) {
        // a locally dense frame overflowed the estimated candidate buffer: rerun with the largest
        c->force_big_cap = true;
        rc = dpk_compute_device(c, natoms, c->h_coord, c->h_atype, box, o, o + 10, o + 1, o + 10 + 3 * natoms, s);
        if (rc == DPK_OK) rc = dpk_ctx_check(c);
        c->force_big_cap = false;
    }
    if (rc) return rc;
    std::vector<double> host(10 + 4 * natoms);
    HIPCHK(hipMemcpy(host.data(), o, sizeof(double) * host.size(), hipMemcpyDeviceToHost));
    *energy = host[0];
    std::memcpy(virial, &host[1], sizeof(double) * 9);
    std::memcpy(force, &host[10], sizeof(double) * 3 * natoms);
    if (atom_energy) std::memcpy(atom_energy, &host[10 + 3 * natoms], sizeof(double) * natoms);
    return DPK_OK;
}

int dpk_ctx_stats(dpk_ctx* c, dpk_stats* out)
{
    if (!c || !out) return fail(DPK_E_INVALID_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->workspace_bytes = (int64_t)(c->ws_bytes + c->model_bytes);
    if (!c->last_n) return DPK_OK;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->last_stream));
    DevStats st;
    HIPCHK(hipMemcpy(&st, c->stats, sizeof(st), hipMemcpyDeviceToHost));
    out->nbr_dropped = (int64_t)st.nbr_dropped;
    out->table_out_of_range = (int64_t)st.table_oor;
    out->max_candidates = st.max_cand;
    return DPK_OK;
}

int dpk_ctx_profile(dpk_ctx* c, int enable)
{
    if (!c) return fail(DPK_E_INVALID_ARG, "NULL context");
    HIPCHK(hipSetDevice(c->device));
    if (c->last_stream) HIPCHK(hipStreamSynchronize(c->last_stream));
    c->profiling = enable != 0;
    c->prof_used = 0;
    return DPK_OK;
}

int dpk_ctx_profile_read(dpk_ctx* c, double* stage_ms, int64_t* frames)
{
    if (!c || !stage_ms) return fail(DPK_E_INVALID_ARG, "NULL argument");
    HIPCHK(hipSetDevice(c->device));
    if (c->last_stream) HIPCHK(hipStreamSynchronize(c->last_stream));
    for (int k = 0; k < DPK_NSTAGES; ++k) stage_ms[k] = 0.0;
    for (size_t f = 0; f < c->prof_used; ++f)
        for (int k = 0; k < DPK_NSTAGES; ++k) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, c->prof_events[f][k], c->prof_events[f][k + 1]));
            stage_ms[k] += ms;
        }
    if (frames) *frames = (int64_t)c->prof_used;
    return DPK_OK;
}

int dpk_debug_nlist(dpk_ctx* c, int32_t* nlist)
{
    if (!c || !nlist) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (!c->last_n) return fail(DPK_E_INVALID_ARG, "no frame computed yet");
    HIPCHK(hipSetDevice(c->device));
    const int n = (int)c->last_n, nc = c->model->nc;
    int* d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(int) * (size_t)n * nc));
    launch_debug_nlist(n, (int)c->last_centres, nc, c->perm, c->nl_j, d, c->last_stream);
    hipError_t e = hipStreamSynchronize(c->last_stream);
    if (e == hipSuccess) e = hipMemcpy(nlist, d, sizeof(int) * (size_t)n * nc, hipMemcpyDeviceToHost);
    hipFree(d);
    if (e != hipSuccess) return fail(DPK_E_DEVICE, "debug nlist: %s", hipGetErrorString(e));
    return DPK_OK;
}

int dpk_debug_descriptor(dpk_ctx* c, double* T, double* dT)
{
    if (!c || !T || !dT) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (!c->last_n) return fail(DPK_E_INVALID_ARG, "no frame computed yet");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->last_stream));
    const int64_t n = c->last_n, per = E2 * 4;
    std::vector<int> perm(n);
    HIPCHK(hipMemcpy(perm.data(), c->perm, sizeof(int) * n, hipMemcpyDeviceToHost));
    std::vector<char> bt(c->acc_size * n * per), bd(c->acc_size * n * per);
    HIPCHK(hipMemcpy(bt.data(), c->T, bt.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(bd.data(), c->dT, bd.size(), hipMemcpyDeviceToHost));
    auto val = [&](const std::vector<char>& b, int64_t i) {
        return c->acc_size == 8 ? ((const double*)b.data())[i] : (double)((const float*)b.data())[i];
    };
    for (int64_t a = 0; a < n; ++a)
        for (int64_t k = 0; k < per; ++k) {
            const int64_t src = a * per + k, dst = (int64_t)perm[a] * per + k;
            const bool centre = a < c->last_centres;   // ghost atoms have no descriptor
            T[dst] = centre ? val(bt, src) : 0.0;
            dT[dst] = centre ? val(bd, src) : 0.0;
        }
    return DPK_OK;
}

}  // extern "C"

// =============================================================================================
// Model deviation (Sec. II.C): one frame, n_m models of one description. The geometry (a1-a3:
// types, cell list, neighbour list) is built once; embedding, fitting and adjoint run for all
// models in one launch per stage (blockIdx.y = model), the models' packed parameters at a fixed
// stride in one buffer per kind.
// =============================================================================================
struct dpk_devi {
    int nm = 0;
    dpk_ctx* geo = nullptr;          // model 0's context: device, precision, geometry workspace
    void *evec = nullptr, *emat = nullptr, *fvec = nullptr, *fmat = nullptr, *table = nullptr;
    void* buf = nullptr;             // per-model buffers for cap atoms
    size_t buf_bytes = 0;
    int64_t cap = 0;
    // views (model 0; model k at k times the stride)
    void *T = nullptr, *dT = nullptr, *act = nullptr;
    double *Ei = nullptr, *F = nullptr, *vir = nullptr, *ev = nullptr, *eps = nullptr;
    size_t st_T = 0, st_act = 0, st_vir = 0;
};

namespace {

bool same_desc(const dpk_model_desc& a, const dpk_model_desc& b)
{
    if (a.ntypes != b.ntypes || a.rcut != b.rcut || a.rcut_smth != b.rcut_smth || a.axis != b.axis ||
        a.type_one_side != b.type_one_side || a.descriptor != b.descriptor)
        return false;
    for (int t = 0; t < a.ntypes; ++t)
        if (a.sel[t] != b.sel[t]) return false;
    for (int k = 0; k < 3; ++k)
        if (a.emb[k] != b.emb[k] || a.fit[k] != b.fit[k]) return false;
    return true;
}

// Per-model buffers for n atoms: T, dT, fitting scratch, E_i, F (caller order), block partials,
// and the per-model [E, virial] results, then the per-atom deviation.
int devi_buffers(dpk_devi* d, int64_t n)
{
    if (n <= d->cap && d->buf) return DPK_OK;
    dpk_ctx* c = d->geo;
    const bool dense_fit = dense_fitting(c);
    const int64_t nfit = fit_slots(n, dense_fit);
    d->st_T = align256(c->acc_size * n * E2 * 4);
    d->st_act = align256(dense_fit ? c->acc_size * nfit * 6 * FW : sizeof(float) * (nfit / 16) * XF_ACT);
    d->st_vir = align256(sizeof(double) * 10 * embed_bwd_max_blocks(c->precision, n));
    const size_t per = 2 * d->st_T + d->st_act + align256(sizeof(double) * n) + align256(sizeof(double) * 3 * n) + d->st_vir;
    const size_t bytes = per * d->nm + align256(sizeof(double) * 10 * d->nm) + align256(sizeof(double) * n);
    if (d->buf) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(d->buf));
        d->buf = nullptr;
    }
    if (hipMalloc(&d->buf, bytes) != hipSuccess) {
        hipGetLastError();
        d->buf = nullptr;
        return fail(DPK_E_OOM, "hipMalloc of %zu bytes for the model ensemble failed", bytes);
    }
    char* p = (char*)d->buf;
    const size_t nm = d->nm;
    d->T = p; p += nm * d->st_T;
    d->dT = p; p += nm * d->st_T;
    d->act = p; p += nm * d->st_act;
    d->Ei = (double*)p; p += nm * align256(sizeof(double) * n);
    d->F = (double*)p; p += nm * align256(sizeof(double) * 3 * n);
    d->vir = (double*)p; p += nm * d->st_vir;
    d->ev = (double*)p; p += align256(sizeof(double) * 10 * nm);
    d->eps = (double*)p;
    d->buf_bytes = bytes;
    d->cap = n;
    return DPK_OK;
}

// The ensemble's launches of one frame on stream s: geometry once, then every model per stage.
void devi_enqueue(dpk_devi* d, int n, const GeomParams& gp, double nu, hipStream_t s)
{
    dpk_ctx* c = d->geo;
    const int nt = c->model->desc.ntypes, nm = d->nm;
    const size_t stF = align256(sizeof(double) * 3 * n), stE = align256(sizeof(double) * n);
    for (int k = 1; k < nm; ++k) launch_zero((char*)d->F + k * stF, sizeof(double) * 3 * n, s);
    if (!launch_prep_small(n, c->h_coord, c->h_atype, nt, gp, c->tcount, c->toff, c->perm, c->inv_perm, c->itype,
                           c->stats, c->pos, c->cell_of, c->cell_start, c->cand, d->F, s)) {
        if (!c->cells_clear) launch_zero(c->cell_count, sizeof(int) * (size_t)c->cap_cells, s);
        launch_prep_large(n, c->h_coord, c->h_atype, nt, gp, c->tcount, c->toff, c->bcount, c->boff, c->perm,
                          c->inv_perm, c->itype, c->stats, c->pos, c->cell_of, c->cell_count, c->cell_start, c->cursor,
                          c->cell_tmp, c->cand, d->F, s);
        c->cells_clear = true;
    }
    launch_nlist(n, c->pos, c->perm, c->inv_perm, c->cell_of, c->cell_start, c->cand, gp, c->nl_j, c->nl_r, c->nnei,
                 c->stats, s);
    EmbArgs ea;
    std::memset(&ea, 0, sizeof(ea));
    ea.natoms = n;
    ea.ntypes = nt;
    ea.nc = c->model->nc;
    // se_e3: pair nets indexed by the pair's types, N_c^-2, the environment rows staged once for
    // every model (they depend on the geometry and the shared descriptor only)
    const bool e3 = is_e3(c);
    ea.type_one_side = e3 ? 0 : c->model->desc.type_one_side;
    ea.ncu = c->ncu;
    ea.apw = 1;
    for (int t = 0; t < nt; ++t) ea.off[t] = gp.off[t];
    ea.itype = c->itype;
    ea.nnei = c->nnei;
    ea.nl_j = c->nl_j;
    ea.nl_r = c->nl_r;
    ea.rs = c->model->desc.rcut_smth;
    ea.rc = c->model->desc.rcut;
    ea.inv_nc = e3 ? 1.0 / ((double)c->model->nc * c->model->nc) : 1.0 / c->model->nc;
    ea.env = c->env;
    ea.evec = d->evec;
    ea.emat = d->emat;
    ea.table = d->table;
    ea.tab_dx = c->tab_dx;
    ea.tab_nint = c->tab_nint;
    ea.T = d->T;
    ea.dT = d->dT;
    ea.perm = c->perm;
    ea.F = d->F;
    ea.vir_part = d->vir;
    ea.stats = c->stats;
    ea.Ei = d->Ei;
    ea.nmodels = nm;
    ea.ms_evec = c->evec_b;
    ea.ms_emat = c->emat_b;
    ea.ms_table = c->table_b;
    ea.ms_T = d->st_T;
    ea.ms_F = stF;
    ea.ms_Ei = stE;
    ea.ms_vir = d->st_vir;
    if (e3) launch_e3_env(c->precision, ea, s);
    launch_embed_fwd(c->precision, c->tab, ea, s, e3);
    FitArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.natoms = n;
    fa.ntypes = nt;
    fa.ncu = c->ncu;
    fa.itype = c->itype;
    fa.toff = c->toff;
    fa.fvec = d->fvec;
    fa.fmat = d->fmat;
    fa.T = d->T;
    fa.dT = d->dT;
    fa.act = d->act;
    fa.Ei = d->Ei;
    fa.nmodels = nm;
    fa.ms_fvec = c->fvec_b;
    fa.ms_fmat = c->fmat_b;
    fa.ms_T = d->st_T;
    fa.ms_act = d->st_act;
    fa.ms_Ei = stE;
    fa.radial = c->model->desc.descriptor != DPK_SE_E2_A;
    launch_fit(c->precision, fa, s);
    launch_embed_bwd(c->precision, c->tab, ea, s, e3);
    const int nb = embed_bwd_blocks(c->precision, c->tab, n, c->ncu, e3);
    for (int k = 0; k < nm; ++k)
        launch_finalize(nb, (const double*)((const char*)d->vir + k * d->st_vir), d->ev + 10 * k, d->ev + 10 * k + 1,
                        c->stats, s);
    launch_force_devi(n, nm, d->F, (int64_t)(stF / sizeof(double)), nu, d->eps, s);
}

}  // namespace

extern "C" {

int dpk_devi_create(const dpk_model* const* models, int n_models, int device, int precision, dpk_devi** out)
{
    if (!models || !out || n_models < 1 || n_models > DPK_MAX_MODELS)
        return fail(DPK_E_INVALID_ARG, "need 1..%d models", DPK_MAX_MODELS);
    *out = nullptr;
    for (int k = 0; k < n_models; ++k) {
        if (!models[k]) return fail(DPK_E_INVALID_ARG, "NULL model %d", k);
        if (!same_desc(models[k]->desc, models[0]->desc))
            return fail(DPK_E_INVALID_ARG, "model %d has another description than model 0 (the ensemble shares "
                                           "its neighbour list)", k);
        if (models[k]->tabulated != models[0]->tabulated ||
            (models[k]->tabulated && (models[k]->tab_dx != models[0]->tab_dx || models[k]->tab_nint != models[0]->tab_nint)))
            return fail(DPK_E_INVALID_ARG, "model %d is compressed differently from model 0", k);
    }
    auto* d = new dpk_devi;
    d->nm = n_models;
    int rc = dpk_ctx_create(models[0], device, precision, 0, 0, &d->geo);
    if (rc) { delete d; return rc; }
    dpk_ctx* c = d->geo;
    struct Kind { void** all; size_t bytes; void* dpk_ctx::*src; };
    const Kind kinds[5] = {{&d->evec, c->evec_b, &dpk_ctx::evec}, {&d->emat, c->emat_b, &dpk_ctx::emat},
                           {&d->fvec, c->fvec_b, &dpk_ctx::fvec}, {&d->fmat, c->fmat_b, &dpk_ctx::fmat},
                           {&d->table, c->table_b, &dpk_ctx::table}};
    for (const Kind& kd : kinds) {
        if (!kd.bytes) continue;
        if (hipMalloc(kd.all, kd.bytes * n_models) != hipSuccess) {
            hipGetLastError();
            *kd.all = nullptr;
            dpk_devi_free(d);
            return fail(DPK_E_OOM, "hipMalloc of the ensemble's parameters failed");
        }
    }
    // pack each model as a context would and copy it into its slot of the shared buffers
    for (int k = 0; k < n_models; ++k) {
        dpk_ctx* ck = c;
        if (k > 0 && (rc = dpk_ctx_create(models[k], device, precision, 0, 0, &ck))) {
            dpk_devi_free(d);
            return rc;
        }
        for (const Kind& kd : kinds)
            if (kd.bytes && hipMemcpy((char*)*kd.all + k * kd.bytes, ck->*kd.src, kd.bytes, hipMemcpyDeviceToDevice) !=
                                hipSuccess) {
                if (ck != c) dpk_ctx_free(ck);
                dpk_devi_free(d);
                return fail(DPK_E_DEVICE, "copy of model %d's parameters failed", k);
            }
        if (ck != c) dpk_ctx_free(ck);
    }
    *out = d;
    return DPK_OK;
}

void dpk_devi_free(dpk_devi* d)
{
    if (!d) return;
    if (d->geo) {
        hipSetDevice(d->geo->device);
        hipStreamSynchronize(d->geo->stream);
        dpk_ctx_free(d->geo);
    }
    hipFree(d->evec); hipFree(d->emat); hipFree(d->fvec); hipFree(d->fmat); hipFree(d->table);
    hipFree(d->buf);
    delete d;
}

int dpk_devi_compute(dpk_devi* d, int64_t natoms, const double* coord, const int32_t* atype, const double* box,
                     double nu, double* energy, double* force, double* virial, double* eps_f, double* eps_v,
                     dpk_devi_stats* stats)
{
    if (!d || !coord || !atype) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (natoms < 1 || natoms > (1LL << 30)) return fail(DPK_E_INVALID_ARG, "natoms = %lld", (long long)natoms);
    dpk_ctx* c = d->geo;
    HIPCHK(hipSetDevice(c->device));
    GeomParams gp;
    int rc;
    c->cur_natoms = natoms;
    auto geom = [&]() {
        if (box) return setup_geometry(c, box, nullptr, gp);
        double bb[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
        for (int64_t i = 0; i < natoms; ++i)
            for (int k = 0; k < 3; ++k) {
                bb[k] = std::min(bb[k], coord[3 * i + k]);
                bb[3 + k] = std::max(bb[3 + k], coord[3 * i + k]);
            }
        return setup_geometry(c, nullptr, bb, gp);
    };
    if ((rc = geom())) return rc;
    if ((rc = ensure_ws(c, natoms, (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2]))) return rc;
    if ((rc = devi_buffers(d, natoms))) return rc;
    const int n = (int)natoms, nm = d->nm;
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->h_coord, coord, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->h_atype, atype, sizeof(int) * n, hipMemcpyHostToDevice, s));
    devi_enqueue(d, n, gp, nu, s);
    HIPCHK(hipGetLastError());
    c->last_stream = s;
    c->last_n = n;
    c->last_centres = n;
    rc = dpk_ctx_check(c);
    if (rc == DPK_E_NBR_OVERFLOW && !c->strict) {
        // a locally dense frame overflowed the estimated candidate buffer: once more with the largest
        c->force_big_cap = true;
        rc = geom();
        if (rc == DPK_OK) {
            devi_enqueue(d, n, gp, nu, s);
            rc = dpk_ctx_check(c);
        }
        c->force_big_cap = false;
    }
    if (rc) return rc;
    std::vector<double> ev(10 * (size_t)nm), eps(n);
    HIPCHK(hipMemcpy(ev.data(), d->ev, sizeof(double) * ev.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(eps.data(), d->eps, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (force) {
        const size_t stF = align256(sizeof(double) * 3 * n);
        for (int k = 0; k < nm; ++k)
            HIPCHK(hipMemcpy(force + (size_t)k * 3 * n, (const char*)d->F + k * stF, sizeof(double) * 3 * n,
                             hipMemcpyDeviceToHost));
    }
    for (int k = 0; k < nm; ++k) {
        if (energy) energy[k] = ev[10 * k];
        if (virial) std::memcpy(virial + 9 * k, &ev[10 * k + 1], sizeof(double) * 9);
    }
    if (eps_f) std::memcpy(eps_f, eps.data(), sizeof(double) * n);
    // virial deviation (nine components, FP64 on the host) and the statistics
    double ev9[9];
    for (int ab = 0; ab < 9; ++ab) {
        double mean = 0.0, var = 0.0;
        for (int k = 0; k < nm; ++k) mean += ev[10 * k + 1 + ab];
        mean /= nm;
        for (int k = 0; k < nm; ++k) var += (ev[10 * k + 1 + ab] - mean) * (ev[10 * k + 1 + ab] - mean);
        double e = std::sqrt(var / nm) / (double)n;
        if (nu >= 0.0) e /= std::fabs(mean) + nu;
        ev9[ab] = e;
    }
    if (eps_v) std::memcpy(eps_v, ev9, sizeof(ev9));
    if (stats) {
        double fmax = eps[0], fmin = eps[0], fsum = 0.0;
        for (int i = 0; i < n; ++i) {
            fmax = std::max(fmax, eps[i]);
            fmin = std::min(fmin, eps[i]);
            fsum += eps[i];
        }
        double vmax = ev9[0], vmin = ev9[0], vsum = 0.0;
        for (int ab = 0; ab < 9; ++ab) {
            vmax = std::max(vmax, ev9[ab]);
            vmin = std::min(vmin, ev9[ab]);
            vsum += ev9[ab];
        }
        stats->f_max = fmax;
        stats->f_avg = fsum / n;
        stats->f_min = fmin;
        stats->v_max = vmax;
        stats->v_avg = vsum / 9.0;
        stats->v_min = vmin;
    }
    return DPK_OK;
}

}  // extern "C"

// =============================================================================================
// Serving
// =============================================================================================
namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    dpk_frame f{};
    int64_t need = 0;          // workspace bytes of the frame alone
    int64_t ncell = 0;         // bins of the frame
    int64_t out_off = 0;       // first double of its outputs in the slot's output staging
    bool solo = false;         // run alone (after its batch reported a data error)
    bool big_cap = false;      // largest candidate buffer (after overflowing the estimated one)
    bool waited = false;       // counted once in budget_waits
    int state = 0;             // 0 queued, 1 running, 2 done
    int result = 0;
    std::string err;
    int64_t t_submit = 0, t_start = 0, t_done = 0;
};

struct Slot {
    dpk_ctx* ctx = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Request*> reqs;        // the batch in flight (empty: idle)
    int64_t sim = -1;
    double* pin_coord = nullptr;
    int* pin_type = nullptr;
    double* pin_out = nullptr;
    int64_t pin_cap = 0;
    DevStats* pin_stats = nullptr;     // host copy of the batch's statistics block
    int64_t expect = 0;                // workspace bytes once the admitted batch is launched
};

void release_ws(dpk_ctx* c)
{
    if (!c->ws) return;
    if (c->last_stream) hipStreamSynchronize(c->last_stream);
    hipStreamSynchronize(c->stream);
    free_ws_mem(c);
    c->ws_bytes = 0;
    c->cap_atoms = 0;
    c->cap_cells = 0;
}

// A batch grows to at least BATCH_TARGET_ATOMS atoms when frames queue up; the pinned staging
// reserved per slot holds such a batch plus one more frame of the largest batchable size.
constexpr int64_t BATCH_TARGET_ATOMS = 12288;
constexpr int64_t PIN_RESERVE_ATOMS = BATCH_TARGET_ATOMS + 8192;

// Host-only context with the sizes of a slot's context, for workspace planning off the slots.
void plan_ctx(const dpk_ctx* c0, dpk_ctx* p)
{
    p->model = c0->model;
    p->device = c0->device;
    p->precision = c0->precision;
    p->acc_size = c0->acc_size;
    p->ncu = c0->ncu;
}

// Workspace bytes of a frame (cell grid from the host copy of the frame); proto sizes the layout.
int frame_need(const dpk_ctx* proto, const dpk_frame& f, int64_t* need, int64_t* ncell)
{
    dpk_ctx cc;
    plan_ctx(proto, &cc);
    dpk_ctx* c = &cc;
    GeomParams gp;
    int rc;
    c->cur_natoms = f.natoms;
    if (f.box) {
        rc = setup_geometry(c, f.box, nullptr, gp);
    } else {
        double bb[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
        for (int64_t i = 0; i < f.natoms; ++i)
            for (int k = 0; k < 3; ++k) {
                bb[k] = std::min(bb[k], f.coord[3 * i + k]);
                bb[3 + k] = std::max(bb[3 + k], f.coord[3 * i + k]);
            }
        rc = setup_geometry(c, nullptr, bb, gp);
    }
    if (rc) return rc;
    *ncell = (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2];
    *need = (int64_t)layout_ws(c, f.natoms, *ncell, nullptr);
    return DPK_OK;
}

}  // namespace

struct dpk_server {
    const dpk_model* model = nullptr;
    int device = 0;
    int64_t budget = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::condition_variable wake;      // the scheduler's: a frame was queued, or the server stops
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    std::thread th;
    std::atomic<bool> stop{false};
    dpk_server_counters st{};
    int64_t model_bytes = 0;
    dpk_ctx plan;                      // host-only context for workspace sizing (never launched on)
    Arena arena;                       // under a budget: the slots' workspaces
};

namespace {

int64_t resident_bytes(dpk_server* s)
{
    int64_t b = s->model_bytes;
    for (auto& sl : s->slots) b += (int64_t)sl.ctx->ws_bytes;
    return b;
}

// Copy a finished frame's results from its slot's output staging into the caller's buffers (the
// caller reads them only after the frame is published).
void copy_result(Request* r, const double* out)
{
    const int64_t n = r->f.natoms;
    const double* o = out + r->out_off;
    *r->f.energy = o[0];
    std::memcpy(r->f.virial, o + 1, sizeof(double) * 9);
    std::memcpy(r->f.force, o + 10, sizeof(double) * 3 * n);
    if (r->f.atom_energy) std::memcpy(r->f.atom_energy, o + 10 + 3 * n, sizeof(double) * n);
}

// Mark a frame finished (server lock held).
void publish(dpk_server* s, Request* r, int rc, const std::string& msg)
{
    r->result = rc;
    r->err = msg;
    if (rc == DPK_OK) s->st.completed++;
    else s->st.failed++;
    r->t_done = now_ns();
    r->state = 2;
}

// Pinned host staging of a slot for n atoms. The server reserves PIN_RESERVE_ATOMS per slot at
// creation: pinning host memory while frames are submitted stalls the submitting threads (page
// faults wait for the pinning), so only a frame larger than the reserve grows it later.
int ensure_pinned(Slot& sl, int64_t n)
{
    if (sl.pin_cap >= n) return DPK_OK;
    hipHostFree(sl.pin_coord);
    hipHostFree(sl.pin_type);
    hipHostFree(sl.pin_out);
    sl.pin_coord = nullptr; sl.pin_type = nullptr; sl.pin_out = nullptr; sl.pin_cap = 0;
    const int64_t cap = std::max<int64_t>(n, 1024);
    if (hipHostMalloc((void**)&sl.pin_coord, sizeof(double) * 3 * cap) != hipSuccess ||
        hipHostMalloc((void**)&sl.pin_type, sizeof(int) * cap) != hipSuccess ||
        hipHostMalloc((void**)&sl.pin_out, sizeof(double) * (10 * BATCH_MAX_FRAMES + 4 * cap)) != hipSuccess)
        return fail(DPK_E_OOM, "pinned host staging of %lld atoms failed", (long long)cap);
    sl.pin_cap = cap;
    return DPK_OK;
}

bool batchable(const Request* r)
{
    return !r->solo && r->f.natoms <= prep_small_max_atoms() && r->ncell <= prep_small_max_cells();
}

// Run a batch of frames on a slot: one frame through the single-frame path, several through the
// batched launches; host staging in pinned buffers, one copy each way, the statistics block
// copied back beside the outputs. Called by the scheduler thread without the server lock: the
// slot and its context belong to that thread alone.
int launch(Slot& sl, const std::vector<Request*>& batch)
{
    dpk_ctx* c = sl.ctx;
    int64_t n = 0, outd = 0;
    for (Request* r : batch) {
        r->out_off = outd;
        n += r->f.natoms;
        outd += 10 + (r->f.atom_energy ? 4 : 3) * r->f.natoms;
    }
    int rc;
    c->force_big_cap = batch.size() == 1 && batch[0]->big_cap;
    if (batch.size() == 1) {
        if ((rc = ensure_ws(c, n, batch[0]->ncell))) return rc;
    }
    if ((rc = ensure_pinned(sl, n))) return rc;
    int64_t off = 0;
    for (Request* r : batch) {
        std::memcpy(sl.pin_coord + 3 * off, r->f.coord, sizeof(double) * 3 * r->f.natoms);
        std::memcpy(sl.pin_type + off, r->f.atype, sizeof(int) * r->f.natoms);
        off += r->f.natoms;
    }
    hipStream_t st = c->stream;
    if (batch.size() > 1) {
        std::vector<BatchFrame> fr(batch.size());
        for (size_t i = 0; i < batch.size(); ++i)
            fr[i] = BatchFrame{batch[i]->f.natoms, batch[i]->f.coord, batch[i]->f.box, batch[i]->f.atom_energy != nullptr};
        // the workspace (device coordinate buffers included) is sized by the plan before staging
        GeomParams gps[BATCH_MAX_FRAMES];
        FrameDesc fd[BATCH_MAX_FRAMES];
        int64_t nn, ncells, od;
        int ms, mc;
        if ((rc = batch_plan(c, (int)fr.size(), fr.data(), gps, fd, &nn, &ncells, &ms, &mc, &od))) return rc;
        if ((rc = ensure_ws(c, nn, ncells))) return rc;
        HIPCHK(hipMemcpyAsync(c->h_coord, sl.pin_coord, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->h_atype, sl.pin_type, sizeof(int) * n, hipMemcpyHostToDevice, st));
        if ((rc = compute_batch(c, (int)fr.size(), fr.data(), c->h_coord, c->h_atype, c->h_out, st))) return rc;
    } else {
        Request* r = batch[0];
        HIPCHK(hipMemcpyAsync(c->h_coord, sl.pin_coord, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->h_atype, sl.pin_type, sizeof(int) * n, hipMemcpyHostToDevice, st));
        double* o = c->h_out;
        rc = dpk_compute_device(c, n, c->h_coord, c->h_atype, r->f.box, o, o + 10, o + 1,
                                r->f.atom_energy ? o + 10 + 3 * n : nullptr, st);
        if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(sl.pin_out, c->h_out, sizeof(double) * outd, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sl.pin_stats, c->stats, sizeof(DevStats), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(sl.done, st));
    return DPK_OK;
}

// Scheduler thread. Each pass (1) polls the slots' events and copies the results of finished
// batches, (2) under the server lock publishes them, re-queues the frames of a batch that hit a
// data error, and admits queued frames in arrival order, (3) launches the admitted batches
// without the lock, so that submit, poll and wait never wait for a launch. A free slot takes a
// prefix of the queue as one batch (up to BATCH_MAX_FRAMES frames small enough for the batched
// launches): it grows while the admission rule accepts the combined workspace, up to
// BATCH_TARGET_ATOMS atoms and the slot's share of the budget. The head is never overtaken, so
// nothing starves; under light load batches stay short.
void scheduler(dpk_server* s)
{
    hipSetDevice(s->device);
    // short sleeps while a batch is in flight mean what they say (the default timer slack of
    // 50 us would stretch each to about 70 us, on the path of every frame's completion)
    prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    const int ns = (int)s->slots.size();
    std::vector<int32_t> busy(ns);
    std::vector<int64_t> bytes(ns), sims(ns);
    struct Finished {
        int slot, rc;
        std::string msg;
    };
    struct Admitted {
        int slot;
        std::vector<Request*> reqs;
        int rc;
        std::string msg;
    };
    std::vector<Finished> fin;
    std::vector<Admitted> adm;
    while (true) {
        // (1) finished batches: the slot state belongs to this thread
        fin.clear();
        for (int k = 0; k < ns; ++k) {
            Slot& sl = s->slots[k];
            if (sl.reqs.empty()) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            Finished f{k, DPK_OK, std::string()};
            if (q != hipSuccess) {
                f.rc = DPK_E_DEVICE;
                f.msg = hipGetErrorString(q);
            } else {
                f.rc = check_stats(sl.ctx, *sl.pin_stats);
                if (f.rc) f.msg = g_err;
            }
            if (f.rc == DPK_OK)
                for (Request* r : sl.reqs) copy_result(r, sl.pin_out);
            fin.push_back(std::move(f));
        }
        adm.clear();
        bool stop_now = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // (2) publish, or re-queue ahead of the queue
            for (Finished& f : fin) {
                Slot& sl = s->slots[f.slot];
                const bool data_err = f.rc != DPK_OK && f.rc != DPK_E_DEVICE;
                if (data_err && sl.reqs.size() > 1) {
                    // a data error of one frame fails the batch: run its frames again one by one,
                    // so that only the faulty frame reports the error
                    for (auto it = sl.reqs.rbegin(); it != sl.reqs.rend(); ++it) {
                        (*it)->solo = true;
                        (*it)->state = 0;
                        s->queue.push_front(*it);
                    }
                } else if (f.rc == DPK_E_NBR_OVERFLOW && !sl.reqs[0]->big_cap) {
                    // a locally dense frame overflowed the estimated candidate buffer: once more
                    // with the largest
                    Request* r = sl.reqs[0];
                    r->big_cap = true;
                    r->state = 0;
                    s->queue.push_front(r);
                } else {
                    for (Request* r : sl.reqs) publish(s, r, f.rc, f.msg);
                }
                sl.reqs.clear();
            }
            // admission
            while (!s->queue.empty()) {
                for (int k = 0; k < ns; ++k) {
                    // a slot admitted earlier in this pass is launched (and its workspace grown)
                    // only after the pass: count what it will hold
                    busy[k] = !s->slots[k].reqs.empty();
                    bytes[k] = (int64_t)s->slots[k].ctx->ws_bytes;
                    if (busy[k]) bytes[k] = std::max(bytes[k], s->slots[k].expect);
                    sims[k] = s->slots[k].sim;
                }
                Request* r = s->queue.front();
                int take = 1;
                int64_t need = r->need;
                int64_t batch_atoms = r->f.natoms, batch_cells = r->ncell;   // the workspace the launch sizes
                int32_t slot = -1, rel = 0;
                const int plan = dpk_admit_plan(ns, busy.data(), bytes.data(), sims.data(), r->need,
                                                r->f.simulation, s->budget, s->model_bytes, &slot, &rel);
                if (plan > 0 && batchable(r)) {
                    // longest admissible prefix of batchable frames
                    const int kmax = (int)std::min<size_t>(s->queue.size(), BATCH_MAX_FRAMES);
                    const int64_t share = s->budget ? (s->budget - s->model_bytes) / ns : INT64_MAX;
                    int64_t atoms = r->f.natoms, cells = r->ncell + 1;
                    for (int k = 2; k <= kmax && atoms < BATCH_TARGET_ATOMS; ++k) {
                        const Request* q = s->queue[k - 1];
                        if (!batchable(q)) break;
                        const int64_t nk = (int64_t)layout_ws(&s->plan, atoms + q->f.natoms, cells + q->ncell + 1,
                                                              nullptr);
                        if (nk > share) break;
                        int32_t sk = -1, rk = 0;
                        if (dpk_admit_plan(ns, busy.data(), bytes.data(), sims.data(), nk, r->f.simulation,
                                           s->budget, s->model_bytes, &sk, &rk) <= 0)
                            break;
                        atoms += q->f.natoms;
                        cells += q->ncell + 1;
                        take = k;
                        need = nk;
                        batch_atoms = atoms;
                        batch_cells = cells;
                        slot = sk;
                        rel = rk;
                    }
                }
                if (plan == 0) {
                    bool any_idle = false;
                    for (int k = 0; k < ns; ++k) any_idle |= !busy[k];
                    if (any_idle && !r->waited) {
                        r->waited = true;
                        s->st.budget_waits++;
                    }
                    break;
                }
                std::vector<Request*> batch(s->queue.begin(), s->queue.begin() + take);
                s->queue.erase(s->queue.begin(), s->queue.begin() + take);
                if (plan < 0) {
                    for (Request* b : batch) publish(s, b, plan, "frame does not fit the server's HBM budget");
                    continue;
                }
                Slot& sl = s->slots[slot];
                if (rel) {
                    for (int k = 0; k < ns; ++k)
                        if (!busy[k] && k != slot) release_ws(s->slots[k].ctx);
                    if ((int64_t)sl.ctx->ws_bytes > need) release_ws(sl.ctx);
                }
                sl.expect = need;
                if (sl.ctx->ws) {
                    // the workspace grows to the larger capacity in atoms and in bins, which can
                    // exceed both its current size and this launch's need: under a budget it starts
                    // afresh then, so that it holds what the admission counted
                    const bool fits = batch_atoms <= sl.ctx->cap_atoms && batch_cells <= sl.ctx->cap_cells;
                    const int64_t grown = fits ? (int64_t)sl.ctx->ws_bytes
                                               : (int64_t)layout_ws(&s->plan, std::max(batch_atoms, sl.ctx->cap_atoms),
                                                                    std::max(batch_cells, sl.ctx->cap_cells), nullptr);
                    if (s->budget && grown > std::max((int64_t)sl.ctx->ws_bytes, need)) release_ws(sl.ctx);
                    else sl.expect = grown;
                }
                // under a budget the workspace is carved now (the slot is idle). The budget's
                // arithmetic admitted it, but the arena's holes may be split: the idle slots'
                // workspaces are released (their holes merge) and the carve tried once more. What
                // still splits the arena then are busy slots, and the batch waits at the head of
                // the queue for one of them to finish (with every slot idle the arena is one hole).
                if (s->arena.base && ensure_ws(sl.ctx, batch_atoms, batch_cells, true) != DPK_OK) {
                    for (int k = 0; k < ns; ++k)
                        if (!busy[k] && k != slot) release_ws(s->slots[k].ctx);
                    if (ensure_ws(sl.ctx, batch_atoms, batch_cells, true) != DPK_OK) {
                        s->queue.insert(s->queue.begin(), batch.begin(), batch.end());
                        if (!r->waited) {
                            r->waited = true;
                            s->st.budget_waits++;
                        }
                        break;
                    }
                }
                // reserve the slot; its workspace grows to the batch's during the launch
                const int64_t sim = r->f.simulation;
                if (sl.sim >= 0 && sl.sim == sim) s->st.slot_reuse++;
                s->st.launches++;
                sl.sim = sim;
                sl.reqs = batch;
                const int64_t t = now_ns();
                for (Request* b : batch) {
                    b->state = 1;
                    b->t_start = t;
                }
                adm.push_back(Admitted{slot, std::move(batch), DPK_OK, std::string()});
            }
            if (!fin.empty()) s->cv.notify_all();
            bool idle = s->queue.empty();
            for (auto& sl : s->slots) idle &= sl.reqs.empty();
            stop_now = s->stop && idle;
        }
        if (stop_now) break;
        // (3) launch without the lock
        bool failed = false;
        for (Admitted& a : adm) {
            a.rc = launch(s->slots[a.slot], a.reqs);
            if (a.rc) {
                a.msg = g_err;
                failed = true;
            }
        }
        if (!adm.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Admitted& a : adm) {
                if (a.rc) {
                    for (Request* r : a.reqs) publish(s, r, a.rc, a.msg);
                    s->slots[a.slot].reqs.clear();
                }
            }
            s->st.peak_bytes = std::max(s->st.peak_bytes, resident_bytes(s));
            if (failed) s->cv.notify_all();
        }
        if (fin.empty() && adm.empty()) {
            bool inflight = false;
            for (auto& sl : s->slots) inflight |= !sl.reqs.empty();   // this thread's own state
            if (inflight) {
                // a batch is on the device: poll its event again shortly
                std::this_thread::sleep_for(std::chrono::microseconds(2));
            } else {
                // nothing on the device: sleep until a frame is queued (or the server stops)
                std::unique_lock<std::mutex> lk(s->mu);
                s->wake.wait_for(lk, std::chrono::milliseconds(1), [&] { return !s->queue.empty() || s->stop; });
            }
        }
    }
}

}  // namespace

extern "C" {

int dpk_admit_plan(int nslots, const int32_t* busy, const int64_t* slot_bytes, const int64_t* slot_sim,
                   int64_t need_bytes, int64_t simulation, int64_t budget_bytes, int64_t model_bytes, int32_t* slot,
                   int32_t* release_idle)
{
    if (nslots < 1 || !busy || !slot_bytes || !slot_sim || !slot || !release_idle || need_bytes < 0)
        return fail(DPK_E_INVALID_ARG, "bad admission query");
    *slot = -1;
    *release_idle = 0;
    if (budget_bytes > 0 && need_bytes + model_bytes > budget_bytes) return DPK_E_BUDGET;
    int pick = -1;
    // 1. the idle slot that ran this simulation's previous frame
    if (simulation >= 0)
        for (int k = 0; k < nslots; ++k)
            if (!busy[k] && slot_sim[k] == simulation) { pick = k; break; }
    // 2. the smallest idle slot that already holds enough workspace
    if (pick < 0)
        for (int k = 0; k < nslots; ++k)
            if (!busy[k] && slot_bytes[k] >= need_bytes && (pick < 0 || slot_bytes[k] < slot_bytes[pick])) pick = k;
    // 3. the idle slot with the most workspace (least growth)
    if (pick < 0)
        for (int k = 0; k < nslots; ++k)
            if (!busy[k] && (pick < 0 || slot_bytes[k] > slot_bytes[pick])) pick = k;
    if (pick < 0) return 0;
    *slot = pick;
    if (budget_bytes <= 0) return 1;
    int64_t busy_b = 0, idle_b = 0;
    for (int k = 0; k < nslots; ++k) {
        if (busy[k]) busy_b += slot_bytes[k];
        else if (k != pick) idle_b += slot_bytes[k];
    }
    const int64_t mine = std::max(slot_bytes[pick], need_bytes);
    if (model_bytes + busy_b + idle_b + mine <= budget_bytes) return 1;
    if (model_bytes + busy_b + need_bytes <= budget_bytes) {
        *release_idle = 1;
        return 1;
    }
    *slot = -1;
    return 0;
}

int dpk_server_create(const dpk_model* m, int device, int precision, int nslots, size_t hbm_budget_bytes,
                      dpk_server** out)
{
    if (!m || !out || nslots < 1 || nslots > 64) return fail(DPK_E_INVALID_ARG, "bad server arguments");
    *out = nullptr;
    auto* s = new dpk_server;
    s->model = m;
    s->device = device;
    s->budget = (int64_t)hbm_budget_bytes;
    s->slots.resize(nslots);
    for (int k = 0; k < nslots; ++k) {
        int rc;
        if (k == 0) {
            rc = dpk_ctx_create(m, device, precision, 0, 0, &s->slots[0].ctx);
        } else {
            // further slots share the first slot's device copy of the model
            dpk_ctx* c = new dpk_ctx;
            const dpk_ctx* c0 = s->slots[0].ctx;
            c->model = m;
            c->device = device;
            c->precision = precision;
            c->acc_size = c0->acc_size;
            c->ncu = c0->ncu;
            c->evec = c0->evec; c->emat = c0->emat; c->fvec = c0->fvec; c->fmat = c0->fmat; c->table = c0->table;
            c->tab = c0->tab; c->tab_dx = c0->tab_dx; c->tab_nint = c0->tab_nint;
            c->model_bytes = c0->model_bytes;
            c->owns_model = false;
            rc = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess ? DPK_OK : DPK_E_DEVICE;
            s->slots[k].ctx = c;
            if (rc) g_err = "hipStreamCreate failed";
        }
        if (!rc && hipEventCreateWithFlags(&s->slots[k].done, hipEventDisableTiming) != hipSuccess) rc = DPK_E_DEVICE;
        if (!rc && hipHostMalloc((void**)&s->slots[k].pin_stats, sizeof(DevStats)) != hipSuccess) {
            s->slots[k].pin_stats = nullptr;
            rc = fail(DPK_E_OOM, "pinned statistics staging failed");
        }
        if (!rc) rc = ensure_pinned(s->slots[k], PIN_RESERVE_ATOMS);
        if (!rc) rc = ensure_pin_desc(s->slots[k].ctx);
        if (rc) {
            for (int q = k; q >= 0; --q) {
                if (s->slots[q].done) hipEventDestroy(s->slots[q].done);
                hipHostFree(s->slots[q].pin_stats);
                hipHostFree(s->slots[q].pin_coord);
                hipHostFree(s->slots[q].pin_type);
                hipHostFree(s->slots[q].pin_out);
                if (s->slots[q].ctx) dpk_ctx_free(s->slots[q].ctx);
            }
            delete s;
            return rc;
        }
    }
    s->model_bytes = (int64_t)s->slots[0].ctx->model_bytes;
    plan_ctx(s->slots[0].ctx, &s->plan);
    if (s->budget && s->model_bytes > s->budget) {
        dpk_server_free(s);
        return fail(DPK_E_BUDGET, "model alone exceeds the server budget");
    }
    if (s->budget) {
        // whole 256-B granules, as the arena carves them
        const int64_t bytes = (s->budget - s->model_bytes + 255) & ~(int64_t)255;
        void* p = nullptr;
        if (bytes > 0 && hipMalloc(&p, (size_t)bytes) != hipSuccess) {
            hipGetLastError();
            dpk_server_free(s);
            return fail(DPK_E_OOM, "hipMalloc of the server's %lld workspace bytes failed", (long long)bytes);
        }
        s->arena.reset((char*)p, bytes);
        for (auto& sl : s->slots) sl.ctx->arena = &s->arena;
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return DPK_OK;
}

int dpk_server_submit(dpk_server* s, const dpk_frame* f, uint64_t* ticket)
{
    if (!s || !f || !ticket || !f->coord || !f->atype || !f->energy || !f->force || !f->virial || f->natoms < 1)
        return fail(DPK_E_INVALID_ARG, "bad frame");
    auto r = std::make_unique<Request>();
    r->f = *f;
    int rc = frame_need(&s->plan, *f, &r->need, &r->ncell);
    if (rc) return rc;
    const int nt = s->model->desc.ntypes;
    bool bad = false;
    for (int64_t i = 0; i < f->natoms; ++i) bad |= f->atype[i] < 0 || f->atype[i] >= nt;
    if (s->budget && r->need + s->model_bytes > s->budget)
        return fail(DPK_E_BUDGET, "frame of %lld atoms needs %lld workspace bytes; budget %lld with model %lld",
                    (long long)f->natoms, (long long)r->need, (long long)s->budget, (long long)s->model_bytes);
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = now_ns();
    *ticket = r->ticket;
    s->st.submitted++;
    if (bad) {
        // the frame fails alone, without a device launch (the ticket reports the error)
        publish(s, r.get(), DPK_E_TYPE_RANGE, "an atom type is outside [0, " + std::to_string(nt) + ")");
        s->cv.notify_all();
    } else {
        s->queue.push_back(r.get());
        s->wake.notify_one();
    }
    s->reqs[r->ticket] = std::move(r);
    return DPK_OK;
}

int dpk_server_poll(dpk_server* s, uint64_t ticket, int* done)
{
    if (!s || !done) return fail(DPK_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DPK_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    const Request* r = it->second.get();
    *done = r->state == 2 ? (r->result == DPK_OK ? 1 : r->result) : 0;
    return DPK_OK;
}

int dpk_server_wait(dpk_server* s, uint64_t ticket)
{
    if (!s) return fail(DPK_E_INVALID_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DPK_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    s->cv.wait(lk, [&] { return r->state == 2; });
    if (r->result) g_err = r->err;
    return r->result;
}

int dpk_server_wait_for(dpk_server* s, uint64_t ticket, int64_t timeout_us)
{
    if (!s || timeout_us < 0) return fail(DPK_E_INVALID_ARG, "NULL server or negative timeout");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DPK_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    if (!s->cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->state == 2; }))
        return fail(DPK_E_TIMEOUT, "frame %llu not done within %lld us", (unsigned long long)ticket,
                    (long long)timeout_us);
    if (r->result) g_err = r->err;
    return r->result;
}

int dpk_server_cancel(dpk_server* s, uint64_t ticket)
{
    if (!s) return fail(DPK_E_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DPK_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    // only a queued frame can be withdrawn (the scheduler admits under this lock, so a frame still
    // in the queue here has not been handed to a slot)
    auto q = std::find(s->queue.begin(), s->queue.end(), r);
    if (r->state != 0 || q == s->queue.end())
        return fail(DPK_E_INVALID_ARG, "frame %llu is running or done", (unsigned long long)ticket);
    s->queue.erase(q);
    publish(s, r, DPK_E_CANCELLED, "cancelled before it ran");
    s->cv.notify_all();
    return DPK_OK;
}

int dpk_server_times(dpk_server* s, uint64_t ticket, int64_t* times)
{
    if (!s || !times) return fail(DPK_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DPK_E_INVALID_ARG, "unknown ticket");
    times[0] = it->second->t_submit;
    times[1] = it->second->t_start;
    times[2] = it->second->t_done;
    return DPK_OK;
}

int dpk_server_release(dpk_server* s, uint64_t ticket)
{
    if (!s) return fail(DPK_E_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DPK_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != 2)
        return fail(DPK_E_INVALID_ARG, "ticket %llu is still queued or running", (unsigned long long)ticket);
    s->reqs.erase(it);
    return DPK_OK;
}

int dpk_server_stats(dpk_server* s, dpk_server_counters* out)
{
    if (!s || !out) return fail(DPK_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return DPK_OK;
}

void dpk_server_free(dpk_server* s)
{
    if (!s) return;
    if (s->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->wake.notify_one();
        s->th.join();
    }
    for (auto& sl : s->slots) {
        if (sl.done) hipEventDestroy(sl.done);
        hipHostFree(sl.pin_coord);
        hipHostFree(sl.pin_type);
        hipHostFree(sl.pin_out);
        hipHostFree(sl.pin_stats);
    }
    // slots past the first share its model buffers: free them first
    for (size_t k = s->slots.size(); k-- > 0;)
        if (s->slots[k].ctx) dpk_ctx_free(s->slots[k].ctx);
    if (s->arena.base) hipFree(s->arena.base);
    delete s;
}

}  // extern "C"

// Geometry of one host frame for the training path (Sec. II.B needs the same neighbour list as
// inference): partition, bin and search, with the same candidate-buffer retry as dpk_compute.
int dpk::frame_geometry(dpk_ctx* c, int64_t natoms, const double* coord, const int32_t* atype, const double* box,
                        FrameGeom* g)
{
    if (!c || !coord || !atype || !g) return fail(DPK_E_INVALID_ARG, "NULL argument");
    if (natoms < 1 || natoms > (1LL << 30)) return fail(DPK_E_INVALID_ARG, "natoms = %lld", (long long)natoms);
    HIPCHK(hipSetDevice(c->device));
    const int n = (int)natoms;
    hipStream_t s = c->stream;
    int rc = DPK_OK;
    for (int attempt = 0; attempt < 2; ++attempt) {
        GeomParams gp;
        c->cur_natoms = natoms;
        if (box) {
            rc = setup_geometry(c, box, nullptr, gp);
        } else {
            double bb[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
            for (int64_t i = 0; i < natoms; ++i)
                for (int k = 0; k < 3; ++k) {
                    bb[k] = std::min(bb[k], coord[3 * i + k]);
                    bb[3 + k] = std::max(bb[3 + k], coord[3 * i + k]);
                }
            rc = setup_geometry(c, nullptr, bb, gp);
        }
        if (rc) break;
        if ((rc = ensure_ws(c, natoms, (int64_t)gp.nb[0] * gp.nb[1] * gp.nb[2]))) break;
        HIPCHK(hipMemcpyAsync(c->h_coord, coord, sizeof(double) * 3 * natoms, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(c->h_atype, atype, sizeof(int) * natoms, hipMemcpyHostToDevice, s));
        enqueue_geometry(c, n, c->h_coord, c->h_atype, gp, c->F, s, false, nullptr);
        HIPCHK(hipGetLastError());
        c->last_stream = s;
        c->last_n = n;
        c->last_centres = n;
        rc = dpk_ctx_check(c);
        if (rc == DPK_E_NBR_OVERFLOW && !c->force_big_cap && !c->strict) {
            c->force_big_cap = true;   // a locally dense frame: once more with the largest buffer
            continue;
        }
        if (rc == DPK_OK) {
            g->n = n;
            g->nc = c->model->nc;
            g->nt = c->model->desc.ntypes;
            for (int t = 0; t < MAXT; ++t) g->off[t] = gp.off[t];
            g->itype = c->itype;
            g->nnei = c->nnei;
            g->nl_j = c->nl_j;
            g->nl_r = c->nl_r;
            g->perm = c->perm;
            g->stream = s;
        }
        break;
    }
    c->force_big_cap = false;
    return rc;
}
