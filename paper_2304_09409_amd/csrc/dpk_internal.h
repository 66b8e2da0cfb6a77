// dpk_internal.h -- shared host/device definitions of libdpk (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpk {

// Network sizes this build's kernels are written for (Sec. IV model sizes: embedding (25,50,100),
// M_< = 16, fitting (240,240,240,1)).
constexpr int E0 = 25, E1 = 50, E2 = 100, AX = 16, FW = 240, DD = E2 * AX;
constexpr int K2P = 32;    // layer-2 input width padded to whole 16-wide K-chunks
constexpr int N2P = 64;    // layer-2 output (= layer-3 input) width padded
constexpr int N3P = 112;   // layer-3 output width padded to 7 tiles of 16
constexpr int EVEC = 3 * K2P + 2 * N2P + 2 * N3P;   // W1, b1, wh1 | b2, wh2 | b3, wh3
constexpr int FVEC = 7 * FW + 8;                    // b1,wh1,b2,wh2,b3,wh3,w4 | b4, wh4, pad
constexpr int MAXT = 8;
constexpr int NL_CAP = 1024;      // candidate buffer of the neighbour-list kernel (per atom)
constexpr int NL_STENCIL = 343;   // bins visited per atom at most: (2K+1)^3 with K <= 3
constexpr int FIT_AF = 64;        // atoms per block of the fitting kernels (16 per wave)
constexpr int PREP_BLOCK = 256;   // atoms per block of the multi-block preparation

// Offsets inside one packed embedding vector block.
constexpr int EV_W1 = 0, EV_B1 = K2P, EV_WH1 = 2 * K2P, EV_B2 = 3 * K2P, EV_WH2 = 3 * K2P + N2P,
              EV_B3 = 3 * K2P + 2 * N2P, EV_WH3 = 3 * K2P + 2 * N2P + N3P;
// Offsets inside one packed fitting vector block.
constexpr int FV_B1 = 0, FV_WH1 = FW, FV_B2 = 2 * FW, FV_WH2 = 3 * FW, FV_B3 = 4 * FW,
              FV_WH3 = 5 * FW, FV_W4 = 6 * FW, FV_B4 = 7 * FW, FV_WH4 = 7 * FW + 1;
// Matrices of one fitting net, each [rows][cols] row-major, in this order.
constexpr int64_t FM_W1T = 0;                          // [240][1600]
constexpr int64_t FM_W1 = FM_W1T + (int64_t)FW * DD;   // [1600][240]
constexpr int64_t FM_W2T = FM_W1 + (int64_t)DD * FW;   // [240][240]
constexpr int64_t FM_W2 = FM_W2T + FW * FW;
constexpr int64_t FM_W3T = FM_W2 + FW * FW;
constexpr int64_t FM_W3 = FM_W3T + FW * FW;
constexpr int64_t FM_SIZE = FM_W3 + FW * FW;
// Fragment-major fitting weights of the BF16 paths (split and plain). A fragment is the A operand
// of one v_mfma_f32_16x16x32_bf16 for one 16-row tile and one 32-wide K-chunk: the BF16 hi parts
// of the 64 lanes (8 values, 16 B each), then the lo parts. Lane 16g + i holds row 16t + i and
// the K values kidx32(c, g, j), j = 0..7, so that the output tile pair (2c, 2c+1) of one layer
// is the K-chunk c of the next. K of the 240-wide layers is zero-padded to 256 (8 chunks).
// Offsets in fragments per type; fragment (c, t) of a matrix sits at base + c * ntiles + t.
constexpr int XF_ELEMS = 1024;                 // BF16 values per fragment (hi 512 + lo 512)
constexpr int XF_NCH1 = DD / 32;               // 50 K-chunks of layer 1
constexpr int XF_NCH2 = 8;                     // K-chunks of the 240-wide layers
constexpr int XF_W1F = 0;                      // layer 1 forward: rows = 240 outputs, K = 1600
constexpr int XF_W2F = XF_W1F + XF_NCH1 * 15;  // layer 2 forward: rows = outputs, K = inputs
constexpr int XF_W3F = XF_W2F + XF_NCH2 * 15;
constexpr int XF_W3B = XF_W3F + XF_NCH2 * 15;  // layer 3 backward: rows = inputs, K = outputs
constexpr int XF_W2B = XF_W3B + XF_NCH2 * 15;
constexpr int XF_W1B = XF_W2B + XF_NCH2 * 15;  // layer 1 backward: rows = 1600 D entries, K = outputs
constexpr int XF_NFRAG = XF_W1B + XF_NCH2 * 100;
constexpr int XF_ACT = 3 * 16 * 256;           // fitting scratch floats per 16-atom tile

// Skip-aligned feature order of the embedding net (network path; the table path keeps features in
// order). The layer widths double (25 -> 50 -> 100), so each layer adds its input to its output
// with feature o taking input o mod n_in (Sec. II.A.6, eq. NN). Every layer is evaluated with one
// neighbour per lane column and a lane group g holding a fixed set of rows in registers u; the
// features are placed so that the input of every skip sits in the same lane, at register u / 2:
//   layer 1, register u1 of group g: feature kb(g) + u1 for u1 < ns(g) (ns = 7, 6, 6, 6), else none;
//   layer 2, register u2: feature f1(u2 / 2) + 25 (u2 % 2);
//   layer 3, register u3: feature f2(u3 / 2) + 50 (u3 % 2).
// That fills 7 + 6 + 6 + 6 = 25, 50 and 100 features with 7, 4 and 7 padding rows, whose weights
// are zero (their outputs are exactly zero). Registers map to row positions through the
// instruction's layout: layer-1 register u = c VPL + v is K position kidx(c, g, v); register u of
// layers 2 and 3 is row 16 (u / 4) + orow(g, u % 4).
__host__ __device__ constexpr int emb_ns(int g) { return g == 0 ? 7 : 6; }
__host__ __device__ constexpr int emb_kb(int g) { return g == 0 ? 0 : 6 * g + 1; }
// feature held by register u of lane group g in layer l (1, 2, 3), or -1 for a padding row
__host__ __device__ constexpr int emb_feat(int l, int g, int u)
{
    const int u1 = u >> (l - 1);
    if (u1 >= emb_ns(g)) return -1;
    const int k = emb_kb(g) + u1;
    return l == 1 ? k : (l == 2 ? k + E0 * (u & 1) : k + E0 * ((u >> 1) & 1) + E1 * (u & 1));
}
// lane group and register of layer-3 feature f (inverse of emb_feat(3, ., .))
__host__ __device__ constexpr void emb_reg3(int f, int& g, int& u)
{
    const int h3 = f >= E1 ? 1 : 0, n = f - E1 * h3;
    const int h2 = n >= E0 ? 1 : 0, k = n - E0 * h2;
    g = k < 7 ? 0 : (k - 1) / 6;
    u = 4 * (k - emb_kb(g)) + 2 * h2 + h3;
}

// The quintic table of the compressed embedding (Sec. II.A.6, eq. compress) is uploaded in three
// layouts, one after the other in one buffer of the accumulation type:
//   [nets][nint][100][6]        per interval and feature its six coefficients (three-body table);
//   [nets][tab_kp][N3P]         row K = 6 l + j, column m: coefficient j of feature m on interval l;
//   [nets][N3P][tab_kp]         the same transposed.
// Coefficient j multiplies t^(5 - j), t = x - l dx. Rows past 6 nint and columns past 100 are zero;
// tab_kp leaves at least 64 zero rows past the last interval (the product kernels read whole
// groups of 16-row tiles there).
__host__ __device__ constexpr int tab_kp(int nint) { return (6 * nint + 15) / 16 * 16 + 64; }

constexpr int64_t EM_W2T = 0;                          // [64][32]
constexpr int64_t EM_W3T = N2P * K2P;                  // [112][64]
constexpr int64_t EM_SIZE = EM_W3T + N3P * N2P;

// Split BF16 of two FP32 values: hi = bf16(x) (round to nearest even), lo = bf16(x - hi), so
// hi + lo is within 2^-17 of x. Written on two-element vectors so that each conversion is one
// packed v_cvt_pk_bf16_f32 (two values per instruction) instead of one per value.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16x2(float x0, float x1, bf16x2_t& hi, bf16x2_t& lo)
{
    const f32x2_t x = {x0, x1};
    hi = __builtin_convertvector(x, bf16x2_t);
    lo = __builtin_convertvector(x - __builtin_convertvector(hi, f32x2_t), bf16x2_t);
}

// Geometry of the frame for neighbour search.
struct GeomParams {
    int periodic;
    int nb[3];          // bins per axis
    int K[3];           // stencil half-width per axis (bins)
    double h[9];        // cell rows (periodic)
    double hinv[9];
    double origin[3];   // open boundary: lower corner of the bin grid
    double binw[3];     // open boundary: bin widths
    double rc2;
    int ntypes, nc;
    int sel[MAXT], off[MAXT];
    int cap;            // candidate buffer entries per atom (256, 512 or NL_CAP)
};

// Device-side error / statistics block of one frame.
struct DevStats {
    unsigned long long nbr_dropped;
    unsigned long long table_oor;
    int max_cand;
    int err_type;       // atom type out of range
    int err_overflow;   // candidate buffer overflow
    int order_local;    // consecutive internal atoms that share a bin (tabulated backward's order)
};

// Neighbours dropped by sel are counted per atom into NL_DROP_SLOTS counters that follow the
// statistics block in memory (atom a adds to counter a mod NL_DROP_SLOTS: one shared counter
// serialised every atom's atomic), cleared with the block at the start of a frame and added into
// nbr_dropped by the frame's final reduction.
constexpr int NL_DROP_SLOTS = 256;
constexpr int STATS_WORDS = (int)((sizeof(DevStats) + sizeof(unsigned long long) * NL_DROP_SLOTS) / 4);
__host__ __device__ inline unsigned long long* drop_slots(DevStats* st)
{
    return reinterpret_cast<unsigned long long*>(st + 1);
}

// One frame of a batch evaluated in shared launches (serving).
constexpr int BATCH_MAX_FRAMES = 64;
struct FrameDesc {
    int atom_off;          // first atom (caller order over the batch) and first candidate record
    int natoms;
    int cell_off;          // first of the frame's ncell + 1 entries in the concatenated cell_start
    int ncell;
    int out_off;           // first double of the frame's outputs: E, virial[9], F[3n], E_i[n]
    int want_ei;           // write E_i
    int type_base[MAXT];   // device: per-frame type counts, then internal position of the frame's first atom of each type
    int bad;               // device: an atom type was out of range
    int pad;
};

// Kept neighbours per atom of the three-body descriptor (sum of sel): the backward pass holds
// dE/dR of every slot of a wave's atom in LDS.
constexpr int E3_MAXN = 128;

// Arguments of the embedding kernels.
struct EmbArgs {
    int natoms, ntypes, nc, type_one_side;
    int ncu;                 // compute units of the device (sizes the launch)
    int apw;                 // atoms per wave (set by the launcher)
    int off[MAXT];
    const int* itype;        // [N] type of internal atom
    const int* nnei;         // [N][ntypes] kept neighbours per type block
    const int* nl_j;         // [N][nc] caller index of each kept neighbour, -1 past the kept ones
    const double* nl_r;      // [N][nc][3]
    double rs, rc, inv_nc;
    // network (packed per policy) or table
    const void* evec;        // [nets][EVEC] of acc type
    const void* emat;        // [planes][nets][EM_SIZE] of weight type
    const void* table;       // the table's three layouts (tab_kp) of acc type
    double tab_dx; int tab_nint;
    void* T;                 // [N][100][4] of acc type (forward output)
    const void* dT;          // [N][100][4] (backward input)
    const int* perm;         // [N] caller index of each internal atom
    double* F;               // [N][3] caller order (backward output, atomics; zero on entry)
    void* env;               // three-body descriptor: [N][nc][4] environment rows R_j (acc type)
    double* vir_part;        // [gridDim][10]: E of the block's atoms (single frame), virial
    double* vir_atom;        // [N][9] virial per centre atom (batched frames), or nullptr
    DevStats* stats;
    // single frame (nullptr for a batch): E_i of the fitting net, summed per block into vir_part
    // and copied to atom_energy (caller order) if that is not nullptr
    const double* Ei;        // [N] internal order
    double* atom_energy;     // [N] caller order, or nullptr
    // tabulated backward: the centres in bin order (internal index of the k-th) and the number of
    // consecutive internal atoms that share a bin; where fewer than a quarter do (the caller's order
    // is not spatial) the backward takes its groups in bin order. nullptr: internal order
    const int* order;
    const int* order_cnt;
    // Model ensemble (model deviation, one launch for all models): blockIdx.y selects model k,
    // whose parameters and per-model buffers start k times these byte strides past the pointers
    // above; the geometry (types, neighbour list, perm) and the statistics block are shared.
    // nmodels 0 or 1: a single model.
    int nmodels = 0;
    int64_t ms_evec = 0, ms_emat = 0, ms_table = 0, ms_T = 0, ms_F = 0, ms_Ei = 0, ms_vir = 0, ms_ae = 0;
};

// The arguments of the model that blockIdx.y selects.
template <class T> __host__ __device__ inline T* byte_offset(T* p, int64_t bytes)
{
    return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + bytes) : p;
}
__device__ inline EmbArgs model_args(const EmbArgs& A0)
{
    EmbArgs A = A0;
    const int64_t k = blockIdx.y;
    if (k) {
        A.evec = byte_offset(A0.evec, k * A0.ms_evec);
        A.emat = byte_offset(A0.emat, k * A0.ms_emat);
        A.table = byte_offset(A0.table, k * A0.ms_table);
        A.T = byte_offset(A0.T, k * A0.ms_T);
        A.dT = byte_offset(A0.dT, k * A0.ms_T);
        A.F = byte_offset(A0.F, k * A0.ms_F);
        A.Ei = byte_offset(A0.Ei, k * A0.ms_Ei);
        A.vir_part = byte_offset(A0.vir_part, k * A0.ms_vir);
        A.atom_energy = byte_offset(A0.atom_energy, k * A0.ms_ae);
    }
    return A;
}

struct FitArgs {
    int natoms, ntypes;
    int ncu;                // compute units of the device (sizes the BF16 fitting grid)
    const int* itype;
    const int* toff;        // [ntypes+1] internal type offsets (device)
    const void* fvec;       // [ntypes][FVEC] acc type
    const void* fmat;       // FP64: [ntypes][FM_SIZE]; BF16 paths: [ntypes][XF_NFRAG][XF_ELEMS]
    const void* T;          // [N][100][4]
    void* dT;               // [N][100][4]
    void* act;              // forward activations and gradients (scratch)
    double* Ei;             // [N]
    int radial;             // descriptor of M values D_m = T[m][0] (se_e2_r, se_e3) instead of M x M_<
    // model ensemble: as in EmbArgs (blockIdx.y = model, byte strides of the per-model pointers)
    int nmodels = 0;
    int64_t ms_fvec = 0, ms_fmat = 0, ms_T = 0, ms_act = 0, ms_Ei = 0;
};

__device__ inline FitArgs model_args(const FitArgs& A0)
{
    FitArgs A = A0;
    const int64_t k = blockIdx.y;
    if (k) {
        A.fvec = byte_offset(A0.fvec, k * A0.ms_fvec);
        A.fmat = byte_offset(A0.fmat, k * A0.ms_fmat);
        A.T = byte_offset(A0.T, k * A0.ms_T);
        A.dT = byte_offset(A0.dT, k * A0.ms_T);
        A.act = byte_offset(A0.act, k * A0.ms_act);
        A.Ei = byte_offset(A0.Ei, k * A0.ms_Ei);
    }
    return A;
}

}  // namespace dpk
