// kernels_nn.hip -- embedding net with the descriptor contraction, fitting net, and the
// hand-written adjoint (prod_force / prod_virial) of the se_e2_a Deep Potential.
//
// Paper: Sec. II.A.1 (environment rows, switching function eq. switch, embedding eq. G2,
// D = N_c^-2 G^T R R^T G_<), Sec. II.A.2 (E_i = F_0(D), F = -dE/dr, virial), Sec. II.A.6 (layers
// eq. NN; tabulated embedding eq. compress; operator merging: G never leaves registers; precise
// neighbour indexing: only kept neighbours are evaluated).
//
// Matrix-core mapping (16x16 output tiles, one 64-lane wave):
//   * An MFMA computes D[i][j] += sum_k A[i][k] B[k][j] over a 16-wide K-chunk. Lane l supplies row
//     i = l%16 of A and column j = l%16 of B, with the lane group g = l/16 holding the K values
//     kidx(c, g, v), v = 0..3; the output holds D[orow(g, r)][l%16] in register r. The two maps
//     depend on the instruction (see the policies); with them, the output of one tile is the
//     B operand of the next K-chunk without any data movement.
//   * Embedding, per chunk of 16 neighbours of one centre atom: layer 1 (1 -> 25) on the VALU
//     straight into B-operand layout; layer 2 (25 -> 50) transposed (W^T as A, activations as B);
//     forward pass: layer 3 (50 -> 100) untransposed (activations as A), which puts 4 neighbours
//     in each lane's registers for the contraction T += G^T R; backward pass: layer 3 transposed,
//     which keeps one neighbour per lane column so the reductions over the 100 channels (dE/dR_j
//     and dE/ds_j) are lane-local plus two cross-group shuffles. Both contractions run as rank-1
//     updates on the matrix cores (outer4) in the FP32-accumulating paths.
//   * The features of the embedding net are stored in a skip-aligned order (emb_feat): the input
//     of every skip connection is a register of the same lane, so no layer output goes through
//     LDS except the forward pass's layer 2 (the untransposed layer 3 reads it transposed).
//   * The backward pass re-evaluates the net with its forward-mode derivative d/ds (the input is
//     a scalar), rather than storing G: G would cost 400 B per neighbour in HBM.
//   * Fitting: 16 atoms per wave, all 240 features per wave; every layer transposed (W^T as A)
//     so each layer's output tiles are the next layer's B operand; the descriptor D = T T_<^T
//     is formed on the fly in B-operand layout; the input gradient uses W as A.
#include <hip/hip_runtime.h>
#include "dpk_device.h"
#include "dpk_internal.h"
#include "dpk_launch.h"

namespace dpk {

typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------------
// Precision policies
// ---------------------------------------------------------------------------------------------

// FP64 hyperbolic tangent, tanh x = m / (m + 2) with m = e^{2x} - 1, written for the FP64 paths
// (the device library's general routine costs about three times the instructions; the
// embedding's FP64 passes are bound by these evaluations). Range reduction: 2x = n ln 2 + g with
// n = rint(2x log2 e), |g| <= ln 2 / 2; e^g - 1 = g (1 + g/2! + ... + g^12/13!) (Taylor remainder
// below 1e-17 relative on that interval); m = 2^n (e^g - 1) + (2^n - 1), free of cancellation for
// small |x|. The quotient uses the hardware reciprocal refined by two Newton steps. |x| is clamped
// to 20, past which tanh is +-1 in double; NaN propagates. Measured against the C library over
// [-25, 25] and down to |x| = 1e-15: relative error within 3 ulp, absolute within 1.5 ulp(1).
__device__ __forceinline__ double tanh_f64(double x)
{
    const double xc = x > 20.0 ? 20.0 : (x < -20.0 ? -20.0 : x);
    const double n = __builtin_rint(xc * 2.8853900817779268);       // 2 log2 e
    const double g = __builtin_fma(-n, 0.69314718055994531, 2.0 * xc);
    double p = 1.0 / 6227020800.0;                                   // 1/13!
    p = __builtin_fma(p, g, 1.0 / 479001600.0);
    p = __builtin_fma(p, g, 1.0 / 39916800.0);
    p = __builtin_fma(p, g, 1.0 / 3628800.0);
    p = __builtin_fma(p, g, 1.0 / 362880.0);
    p = __builtin_fma(p, g, 1.0 / 40320.0);
    p = __builtin_fma(p, g, 1.0 / 5040.0);
    p = __builtin_fma(p, g, 1.0 / 720.0);
    p = __builtin_fma(p, g, 1.0 / 120.0);
    p = __builtin_fma(p, g, 1.0 / 24.0);
    p = __builtin_fma(p, g, 1.0 / 6.0);
    p = __builtin_fma(p, g, 0.5);
    p = __builtin_fma(p, g, 1.0);
    const double s = __builtin_amdgcn_ldexp(1.0, (int)n);
    const double m = __builtin_fma(s, g * p, s - 1.0), d = m + 2.0;
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    return m * r;
}

// FP64: v_mfma_f64_16x16x4f64, four instructions per 16-wide K-chunk. Output register r of lane
// group g holds row g + 4r. Weight matrices are stored with each 16-wide K-chunk permuted so that
// the four K values a lane needs (g, g+4, g+8, g+12) are contiguous.
struct PF64 {
    typedef double acc;
    typedef double wt;
    typedef d4 accv;
    static constexpr int NPL = 1;
    static constexpr int KC = 16;    // K per fragment (four instructions)
    static constexpr int VPL = 4;    // K values per lane per fragment
    static constexpr int GB = 32;    // bytes of one lane's fragment in LDS
    struct frag { d4 v; };
    __device__ static int orow(int g, int r) { return g + 4 * r; }
    __device__ static int ogrp(int row) { return row & 3; }    // inverse of orow
    __device__ static int oreg(int row) { return row >> 2; }
    __device__ static int kidx(int c, int g, int v) { return 16 * c + g + 4 * v; }
    __device__ static frag make(acc x0, acc x1, acc x2, acc x3) { frag f; f.v = d4{x0, x1, x2, x3}; return f; }
    __device__ static frag make(const acc* x) { return make(x[0], x[1], x[2], x[3]); }
    __device__ static frag lds(const char* p) { return *reinterpret_cast<const frag*>(p); }
    __device__ static frag load(const wt* p, int64_t) {
        frag f;
        f.v = *reinterpret_cast<const d4*>(p);
        return f;
    }
    __device__ static void mma(accv& d, const frag& a, const frag& b) {
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[0], b.v[0], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[1], b.v[1], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[2], b.v[2], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[3], b.v[3], d, 0, 0, 0);
    }
    __device__ static acc act(acc x) { return tanh_f64(x); }
    // tanh(x + b) from the bias as staged (unscaled)
    __device__ static acc act_b(acc x, acc b) { return tanh_f64(x + b); }
    static constexpr double BIAS_SCALE = 1.0;
};

// FP32 hyperbolic tangent: 1 - 2 / (exp(2x) + 1), with exp(2x) = 2^(K x), K = 2 log2 e, on the
// hardware exp2 and the hardware reciprocal. Saturates to +-1 without overflow trouble (2^inf =
// inf, 1/inf = 0). Absolute error about 1e-7. tanh_scaled takes y = K x, so that a bias staged as
// K b folds into one FMA: tanh(x + b) = tanh_scaled(K x + K b).
constexpr float TANH_K = 2.885390081777927f;
__device__ __forceinline__ float tanh_scaled(float y)
{
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f);
}
__device__ __forceinline__ float tanh_fast(float x) { return tanh_scaled(x * TANH_K); }

// Split BF16 on v_mfma_f32_16x16x32_bf16: each FP32 operand is hi + lo with both parts BF16; the
// product is formed as lo*hi + hi*lo + hi*hi with FP32 accumulation, about 16 significant bits per
// operand. Lane group g supplies K values 8g..8g+7 of a 32-wide chunk; they are the logical
// indices kidx(c, g, v): rows 4g..4g+3 of output tile 2c (v < 4) and of tile 2c + 1 (v >= 4), so
// that a layer's output tiles feed the next layer's K-chunk in place (weights are stored with
// their K order permuted to match). Output register r of lane group g holds row 4g + r.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ int kidx32(int c, int g, int v) { return 32 * c + (v < 4 ? 4 * g + v : 16 + 4 * g + (v - 4)); }

struct PMIX {
    typedef float acc;
    typedef __bf16 wt;
    typedef f4 accv;
    static constexpr int NPL = 2;
    static constexpr int KC = 32, VPL = 8, GB = 32;
    struct frag { bf8 h, l; };
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static int ogrp(int row) { return row >> 2; }   // inverse of orow
    __device__ static int oreg(int row) { return row & 3; }
    __device__ static int kidx(int c, int g, int v) { return kidx32(c, g, v); }
    __device__ static frag make(const acc* x) {
        frag f;
#pragma unroll
        for (int v = 0; v < 8; v += 2) {
            bf16x2_t h, l;
            split_bf16x2(x[v], x[v + 1], h, l);
            f.h[v] = h[0]; f.h[v + 1] = h[1];
            f.l[v] = l[0]; f.l[v + 1] = l[1];
        }
        return f;
    }
    __device__ static frag load(const wt* p, int64_t plane) {
        frag f;
        f.h = *reinterpret_cast<const bf8*>(p);
        f.l = *reinterpret_cast<const bf8*>(p + plane);
        return f;
    }
    __device__ static frag lds(const char* p) {
        frag f;
        f.h = *reinterpret_cast<const bf8*>(p);
        f.l = *reinterpret_cast<const bf8*>(p + 16);
        return f;
    }
    __device__ static void mma(accv& d, const frag& a, const frag& b) {
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, d, 0, 0, 0);
    }
    __device__ static acc act(acc x) { return tanh_fast(x); }
    // tanh(x + b) from the bias as staged (K b)
    __device__ static acc act_b(acc x, acc kb) { return tanh_scaled(__builtin_fmaf(x, TANH_K, kb)); }
    static constexpr float BIAS_SCALE = TANH_K;
};

// Plain BF16 operands on the same instruction, one product (fast, about 1e-2 relative force error).
struct PBF16 {
    typedef float acc;
    typedef __bf16 wt;
    typedef f4 accv;
    static constexpr int NPL = 1;
    static constexpr int KC = 32, VPL = 8, GB = 16;
    struct frag { bf8 h; };
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static int ogrp(int row) { return row >> 2; }   // inverse of orow
    __device__ static int oreg(int row) { return row & 3; }
    __device__ static int kidx(int c, int g, int v) { return kidx32(c, g, v); }
    __device__ static frag make(const acc* x) {
        frag f;
#pragma unroll
        for (int v = 0; v < 8; v += 2) {
            const bf16x2_t h = __builtin_convertvector((f32x2_t){x[v], x[v + 1]}, bf16x2_t);
            f.h[v] = h[0];
            f.h[v + 1] = h[1];
        }
        return f;
    }
    __device__ static frag load(const wt* p, int64_t) {
        frag f;
        f.h = *reinterpret_cast<const bf8*>(p);
        return f;
    }
    __device__ static frag lds(const char* p) {
        frag f;
        f.h = *reinterpret_cast<const bf8*>(p);
        return f;
    }
    __device__ static void mma(accv& d, const frag& a, const frag& b) {
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, d, 0, 0, 0);
    }
    __device__ static acc act(acc x) { return tanh_fast(x); }
    // tanh(x + b) from the bias as staged (K b)
    __device__ static acc act_b(acc x, acc kb) { return tanh_scaled(__builtin_fmaf(x, TANH_K, kb)); }
    static constexpr float BIAS_SCALE = TANH_K;
};

// FP32 on v_mfma_f32_16x16x4f32, four instructions per 16-wide K-chunk (the FP32 precision of
// the paper's reduced-precision inference, Sec. IV). In instruction v lane group g supplies one K
// value, register v of its fragment; with kidx(c, g, v) = 16c + 4g + v that is row 4g + v of the
// previous layer's output tile c, which is exactly what output register v of lane group g holds
// (orow(g, r) = 4g + r, probed on gfx950), so a layer's output is the next layer's B operand in
// place and the weights are stored in plain K order.
struct PF32 {
    typedef float acc;
    typedef float wt;
    typedef f4 accv;
    static constexpr int NPL = 1;
    static constexpr int KC = 16, VPL = 4, GB = 16;
    struct frag { f4 v; };
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static int ogrp(int row) { return row >> 2; }   // inverse of orow
    __device__ static int oreg(int row) { return row & 3; }
    __device__ static int kidx(int c, int g, int v) { return 16 * c + 4 * g + v; }
    __device__ static frag make(acc x0, acc x1, acc x2, acc x3) { frag f; f.v = f4{x0, x1, x2, x3}; return f; }
    __device__ static frag make(const acc* x) { return make(x[0], x[1], x[2], x[3]); }
    __device__ static frag lds(const char* p) { frag f; f.v = *reinterpret_cast<const f4*>(p); return f; }
    __device__ static frag load(const wt* p, int64_t) { frag f; f.v = *reinterpret_cast<const f4*>(p); return f; }
    __device__ static void mma(accv& d, const frag& a, const frag& b) {
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[0], b.v[0], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[1], b.v[1], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[2], b.v[2], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[3], b.v[3], d, 0, 0, 0);
    }
    __device__ static acc act(acc x) { return tanh_fast(x); }
    // tanh(x + b) from the bias as staged (K b)
    __device__ static acc act_b(acc x, acc kb) { return tanh_scaled(__builtin_fmaf(x, TANH_K, kb)); }
    static constexpr float BIAS_SCALE = TANH_K;
};

template <class V> __device__ __forceinline__ void zero4(V& v) { v[0] = 0; v[1] = 0; v[2] = 0; v[3] = 0; }

// Rank-1 updates on the matrix cores. v_mfma_f32_4x4x1f32 runs 16 independent 4 x 4 x 1 products,
// one per block of four lanes b: register i of lane 4b + j gains A(lane 4b + i) * B(lane 4b + j).
// With a = X[lane % 4] (an entry of a 4-vector X that is the same for the lane's quad) and b the
// lane's own scalar y, register k of every lane gains X[k] * y: 16 products per instruction, none
// wasted. The forward embedding kernel contracts T += G^T R this way (its layer-3 output puts one
// feature per lane and the neighbours in registers), the backward kernel dE/dR_j = G dT and
// dE/ds_j = (dG/ds) dT (one row m per lane quad, one neighbour per lane): the FMAs leave the vector
// ALUs and the accumulators the general registers.
__device__ __forceinline__ void outer4(f4& d, float a, float b)
{
    d = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, d, 0, 0, 0);
}


// Cross-lane sums over the four 16-lane groups of a wave on v_permlane32_swap (exchanges the
// upper half of one register with the lower half of another: pairs groups g, g + 2) and
// v_permlane16_swap (odd rows of one with even rows of the other: pairs g, g + 1).
__device__ __forceinline__ void swap_halves(float& a, float& b, bool rows16)
{
    const auto r = rows16 ? __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false)
                          : __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap_halves(double& a, double& b, bool rows16)
{
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
    const auto rl = rows16 ? __builtin_amdgcn_permlane16_swap(alo, blo, false, false)
                           : __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto rh = rows16 ? __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false)
                           : __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    a = __longlong_as_double((long long)(((unsigned long long)rh[0] << 32) | rl[0]));
    b = __longlong_as_double((long long)(((unsigned long long)rh[1] << 32) | rl[1]));
}
// Every lane receives the sum of v over the four lanes of its column (lane & 15).
template <class T> __device__ __forceinline__ T sum_groups(T v)
{
    T a = v, b = v;
    swap_halves(a, b, false);
    v = a + b;
    a = v;
    b = v;
    swap_halves(a, b, true);
    return a + b;
}
// Lane group G receives the column sum of p[ksel(G)], ksel = {0, 2, 1, 3}.
__device__ __forceinline__ int ksel(int g) { return ((g & 1) << 1) | (g >> 1); }
template <class T> __device__ __forceinline__ T sum_groups4(const T* p)
{
    T a = p[0], b = p[1], c = p[2], d = p[3];
    swap_halves(a, b, false);
    swap_halves(c, d, false);
    T q0 = a + b, q1 = c + d;
    swap_halves(q0, q1, true);
    return q0 + q1;
}


// Row stride of the forward pass's neighbour-major layer-2 buffer (64 rows used): a multiple of 4
// but not of 8, so the reads at (neighbour orow(g, r), row n) of the four lane groups fall in
// different banks, and rows stay 16-B aligned, so a lane's four consecutive rows go out as one
// 128-bit store (odd strides split them into 32-bit pairs: the bank-conflict counter rose 60 %).
constexpr int Z2S = 68;

// Launch shape of the embedding kernels: NW waves per block share one staged net; each wave takes
// A.apw atoms, chosen per launch (embed_apw) between 1 and APW_MAX so that a large frame gets about
// one block per CU (fewer net stagings per atom) and a small one still spreads over the CUs. Every
// path stages W3^T in LDS. FP64 runs 8 waves (network; two per SIMD, in at most 256 registers) or
// 4 (table; three blocks per CU). The FP32-accumulating policies run:
//   * forward (network): 16 waves, four per SIMD, in at most 128 VGPRs (the contraction's
//     accumulators live in the matrix cores' operands, see outer4): the extra waves per SIMD hide
//     more of the exp/rcp, MFMA and LDS latency;
//   * forward (table): 8 waves (the polynomial path needs more registers);
//   * backward: 12 waves, three per SIMD, in at most 168 VGPRs (skips in registers, the
//     contraction on the matrix cores, the pair sums of force and virial in LDS).
template <class P, bool FWD = false, bool TAB = false> struct EmbCfg {
    typedef typename P::wt wt;
    static constexpr bool F64 = sizeof(typename P::acc) == 8;
    static constexpr int NW = F64 ? (TAB ? 4 : 8) : (FWD ? (TAB ? 8 : 16) : 12);
    static constexpr int APW_MAX = F64 ? 3 : (FWD ? (TAB ? 3 : 4) : 6);
    static constexpr bool W3LDS = true;
    // LDS rows of staged weights: one lane's fragment per group (VPL K values; [hi lo] for split
    // BF16), rows padded by 16 B so 16 consecutive rows fall in distinct banks.
    static constexpr int ROW2 = (K2P / P::VPL) * P::GB + 16;
    static constexpr int ROW3 = (N2P / P::VPL) * P::GB + 16;
    static constexpr int NC1 = K2P / P::KC;     // K-chunks of layer 2 (input 25, padded)
    static constexpr int NC2 = N2P / P::KC;     // K-chunks of layer 3 (input 50, padded)
};

// Fragment of row `row`, K-group `grp` (= 4 * chunk + lane group) from a staged block with `rowb`
// bytes per row.
template <class P>
__device__ __forceinline__ typename P::frag lds_frag(const char* base, int rowb, int row, int grp)
{
    return P::lds(base + row * rowb + grp * P::GB);
}

// Stage rows x K of a per-plane row-major matrix into LDS rows of fragment groups.
template <class P>
__device__ void stage_rows(char* dst, int rowb, const typename P::wt* src, int64_t plane, int rows, int K)
{
    typedef typename P::wt wt;
    const int G = K / P::VPL;
    for (int i = threadIdx.x; i < rows * G; i += blockDim.x) {
        const int row = i / G, grp = i - row * G;
        const wt* sp = src + (int64_t)row * K + P::VPL * grp;
        char* d = dst + row * rowb + grp * P::GB;
        if constexpr (sizeof(wt) == 8) {
            *reinterpret_cast<d4*>(d) = *reinterpret_cast<const d4*>(sp);
        } else {
            *reinterpret_cast<u32x4*>(d) = *reinterpret_cast<const u32x4*>(sp);
            if constexpr (P::NPL == 2) *reinterpret_cast<u32x4*>(d + 16) = *reinterpret_cast<const u32x4*>(sp + plane);
        }
    }
}

// Stage one embedding net: vector block, W2^T and (split BF16) W3^T.
template <class P>
__device__ void stage_net(const EmbArgs& A, int net, typename P::acc* s_vec, char* s_w2, char* s_w3)
{
    typedef typename P::acc acc;
    typedef typename P::wt wt;
    typedef EmbCfg<P> Cfg;
    const acc* ev = reinterpret_cast<const acc*>(A.evec) + (size_t)net * EVEC;
    // biases of layers 2 and 3 staged pre-scaled for P::act_b
    for (int i = threadIdx.x; i < EVEC; i += blockDim.x) {
        const bool bias = (i >= EV_B2 && i < EV_B2 + N2P) || (i >= EV_B3 && i < EV_B3 + N3P);
        s_vec[i] = bias ? ev[i] * (acc)P::BIAS_SCALE : ev[i];
    }
    const int nets = A.type_one_side ? A.ntypes : A.ntypes * A.ntypes;
    const wt* src = reinterpret_cast<const wt*>(A.emat) + (size_t)net * EM_SIZE;
    const int64_t plane = (int64_t)nets * EM_SIZE;
    stage_rows<P>(s_w2, Cfg::ROW2, src + EM_W2T, plane, N2P, K2P);
    if (Cfg::W3LDS) stage_rows<P>(s_w3, Cfg::ROW3, src + EM_W3T, plane, N3P, N2P);
}

// Per-wave walk over (atom, 16-neighbour chunk) work items of one (type_i, type_j) pass, with the
// next item's neighbour vector and index loaded one item ahead. With LDSW the wave's atoms' type,
// neighbour count and caller index are loaded once per pass into a small LDS table (wl) and read
// from there when the walk reaches an atom: a global load there has to wait for every vector
// memory operation in flight (force atomics, prefetches), since that counter is in order. (The
// table backward pass uses it; in the network passes it cost more registers than it saved.)
constexpr int WL_MAX = 8;   // atoms per wave at most (APW_MAX)
template <bool LDSW = false>
struct ChunkWalk {
    int i, a, np, c0;
    int ac;   // caller index of atom a (backward pass)
    bool have;
    double px, py, pz;
    int pj;
    // wl: this wave's [2][WL_MAX] LDS table (type << 16 | neighbour count of atom k; its caller index)
    template <bool J = false>
    __device__ __forceinline__ void load_atoms(int* wl, const EmbArgs& A, int a0, int a1, int wave, int nw, int apw,
                                               int tj, int lane) {
        if (!LDSW) return;
        const int a = a0 + wave + nw * lane;
        if (lane < apw) {
            wl[lane] = a < a1 ? (A.itype[a] << 16) | A.nnei[(size_t)a * A.ntypes + tj] : -1;
            if (J) wl[WL_MAX + lane] = a < a1 ? A.perm[a] : 0;
        }
        wave_sync();
    }
    template <bool J = false>
    __device__ __forceinline__ bool find_atom(const EmbArgs& A, const int* wl, int a0, int a1, int wave, int nw,
                                              int apw, int ti, int tj, bool skip_empty) {
        for (; i < apw; ++i) {
            a = a0 + wave + nw * i;
            if (a >= a1) return false;
            if constexpr (LDSW) {
                const int tn = __builtin_amdgcn_readfirstlane(wl[i]);
                if ((tn >> 16) != ti) continue;
                np = tn & 0xffff;
                if (skip_empty && np == 0) continue;
                if (J) ac = __builtin_amdgcn_readfirstlane(wl[WL_MAX + i]);
            } else {
                if (A.itype[a] != ti) continue;
                np = A.nnei[(size_t)a * A.ntypes + tj];
                if (skip_empty && np == 0) continue;
                if (J) ac = A.perm[a];
            }
            return true;
        }
        return false;
    }
    // Prefetch of the chunk's r_ij; J: also the neighbour's caller index (the backward pass adds
    // forces in caller order). The reads are unconditional and their values used as read: a lane
    // past its atom's kept neighbours reads another slot of the atom's row (clamped to the row;
    // slot 0 once the walk has ended). Every slot of every row holds finite values (padding is
    // written as zero), and the kernels use r of such a lane only under `valid` or multiplied by
    // its zero s. A read under a branch, or a select of its value, makes the compiler wait for
    // this prefetch early (reads retire in order).
    template <bool J = false>
    __device__ __forceinline__ void fetch(const EmbArgs& A, int tj, int c16) {
        const int e = min(A.off[tj] + c0 + c16, A.nc - 1);
        const size_t slot = have ? (size_t)a * A.nc + e : 0;
        const double* v = A.nl_r + 3 * slot;
        px = v[0];
        py = v[1];
        pz = v[2];
        if (J) pj = A.nl_j[slot];
    }
};

// Three-body descriptor (Sec. II.A.1, eq. descrpt-e3, eq. nn-descrpt-e3): the rows of the
// embedding net are the ordered pairs (j, k) of an atom's kept neighbours, with input
// theta_jk = R_j . R_k. A pass takes one net (a_j, a_k) and walks the pairs of the neighbour-type
// blocks a_j x a_k of each atom: pair p is (slot off[a_j] + p / n_k, slot off[a_k] + p % n_k), n_k
// the atom's kept count of type a_k. Within one type block (a_j = a_k) the pairs (j, k) and (k, j)
// have the same theta and the same net, so that pass walks k <= j only (p = j (j + 1) / 2 + k) and
// weighs j != k twice. The two environment rows are loaded one item ahead (they come from the
// per-frame env buffer, k_e3_env). The pass index q encodes (a_j, a_k) = (q / nt, q % nt).
template <class P>
struct PairWalk {
    typedef typename P::acc acc;
    typedef typename P::accv accv;
    int i, a, np, nb, c0, ac;
    bool have;
    accv ra, rb;   // environment rows of the item's pair (prefetched)
    int sa, sb;    // their slots
    acc wgt;       // 1, or 2 for an off-diagonal pair of one type block
    template <bool J = false>
    __device__ __forceinline__ bool find_atom(const EmbArgs& A, const int*, int a0, int a1, int wave, int nw, int apw,
                                              int ti, int q, bool skip_empty) {
        const int nt = A.ntypes, ta = q / nt, tb = q - ta * nt;
        for (; i < apw; ++i) {
            a = a0 + wave + nw * i;
            if (a >= a1) return false;
            if (A.itype[a] != ti) continue;
            nb = A.nnei[(size_t)a * nt + tb];
            np = ta == tb ? nb * (nb + 1) / 2 : A.nnei[(size_t)a * nt + ta] * nb;
            if (skip_empty && np == 0) continue;
            if (J) ac = A.perm[a];
            return true;
        }
        return false;
    }
    // Lanes past the atom's last pair (and every lane once the walk has ended) read the pair of the
    // first slots, whose rows are finite (padding rows are zero); their values are used only under
    // `valid`.
    template <bool J = false>
    __device__ __forceinline__ void fetch(const EmbArgs& A, int q, int c16) {
        const int nt = A.ntypes, ta = q / nt, tb = q - ta * nt;
        int ia = 0, ib = 0;
        wgt = 1;
        if (have && np > 0) {
            const int p = min(c0 + c16, np - 1);
            if (ta == tb) {
                // p = j (j + 1) / 2 + k with k <= j
                int j = (int)((sqrtf(8.0f * p + 1.0f) - 1.0f) * 0.5f);
                j -= j * (j + 1) / 2 > p;
                j += (j + 1) * (j + 2) / 2 <= p;
                ia = j;
                ib = p - j * (j + 1) / 2;
                wgt = ia == ib ? (acc)1 : (acc)2;
            } else {
                ia = p / nb;
                ib = p - ia * nb;
            }
        }
        sa = min(A.off[ta] + ia, A.nc - 1);   // (a type with sel 0 starts at nc)
        sb = min(A.off[tb] + ib, A.nc - 1);
        const acc* e = reinterpret_cast<const acc*>(A.env) + (have ? (size_t)a * A.nc * 4 : 0);
        ra = *reinterpret_cast<const accv*>(e + 4 * sa);
        rb = *reinterpret_cast<const accv*>(e + 4 * sb);
    }
    // keep the prefetched rows in place (see the pair walk's use in the backward pass)
    __device__ __forceinline__ void pin() const { asm volatile("" ::"v"(ra), "v"(rb), "v"(sa), "v"(sb)); }
};

// Environment rows of the three-body descriptor, R_j = s(r_j) (1, x_j / r_j, y_j / r_j, z_j / r_j)
// (Sec. II.A.1, eq. rij, eq. switch), for every slot of every atom: zero past an atom's kept
// neighbours of each type block. One thread per (atom, slot).
template <class acc>
__global__ void __launch_bounds__(256) k_e3_env(EmbArgs A)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)A.natoms * A.nc) return;
    const int a = (int)(e / A.nc), sl = (int)(e - (int64_t)a * A.nc);
    int t = 0;
    while (t + 1 < A.ntypes && sl >= A.off[t + 1]) ++t;
    acc out[4] = {0, 0, 0, 0};
    if (sl - A.off[t] < A.nnei[(size_t)a * A.ntypes + t]) {
        const double* v = A.nl_r + 3 * e;
        const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]), ir = 1.0 / r;
        double s, ds;
        switch_fn(r, ir, A.rs, A.rc, 1.0 / (A.rc - A.rs), s, ds);
        const double sr = s * ir;
        out[0] = (acc)s;
        out[1] = (acc)(sr * v[0]);
        out[2] = (acc)(sr * v[1]);
        out[3] = (acc)(sr * v[2]);
    }
    acc* o = reinterpret_cast<acc*>(A.env) + 4 * e;
    o[0] = out[0];
    o[1] = out[1];
    o[2] = out[2];
    o[3] = out[3];
}

// ---------------------------------------------------------------------------------------------
// Forward: T_a = N_c^-1 sum_j G_j^T R_j for every atom a (G evaluated and contracted in
// registers, never stored). The neighbour-type blocks of atom a are separate passes (one staged
// net each) that add into T[a]; the same lane owns T[a][m][k] in every pass.
// E3 (three-body descriptor): the rows are neighbour pairs (PairWalk) with net input theta and
// row (theta, 0, 0, 0), so that T[a][m][0] = D_m with A.inv_nc = N_c^-2 and T[a][m][1..3] = 0.
// ---------------------------------------------------------------------------------------------
template <class P, bool TAB, bool ENS, bool E3>
__global__ void __launch_bounds__((EmbCfg<P, true, TAB>::NW * 64)) k_embed_fwd(EmbArgs A_)
{
    // ENS: a model ensemble, blockIdx.y selects the model (a separate instantiation, so that the
    // single-model kernels carry no per-model pointer arithmetic in their registers)
    const EmbArgs A = ENS ? model_args(A_) : A_;
    typedef typename P::acc acc;
    typedef typename P::wt wt;
    typedef typename P::accv accv;
    typedef typename P::frag frag;
    typedef EmbCfg<P, true, TAB> Cfg;
    constexpr int NW = Cfg::NW;
    const int APW = A.apw, APB = NW * APW;
    constexpr bool W3LDS = Cfg::W3LDS;
    __shared__ acc s_vec[EVEC];
    __shared__ __attribute__((aligned(16))) char s_w2[TAB ? 16 : N2P * Cfg::ROW2];
    __shared__ __attribute__((aligned(16))) char s_w3[(TAB || !W3LDS) ? 16 : N3P * Cfg::ROW3];
    // layer-2 outputs for the skip into layer 3, neighbour-major: the untransposed layer 3 reads
    // them as (neighbour orow(g, r), row of the lane's column); the layer-1 skip stays in registers
    __shared__ acc s_z2[TAB ? 1 : NW][16][Z2S];
    __shared__ acc s_R[NW][16][4];
    __shared__ double s_x[NW][16];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar registers)
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const double inv_w = 1.0 / (A.rc - A.rs);
    const int a0 = blockIdx.x * APB;
    const int a1 = min(a0 + APB, A.natoms);
    if (a0 >= a1) return;
    const int t_lo = A.itype[a0], t_hi = A.itype[a1 - 1];
    const int nets = A.type_one_side ? A.ntypes : A.ntypes * A.ntypes;
    const int npass = E3 ? A.ntypes * A.ntypes : A.ntypes;

    for (int ti = t_lo; ti <= t_hi; ++ti) {
        for (int tj = 0; tj < npass; ++tj) {
            const int net = (E3 || A.type_one_side) ? tj : ti * A.ntypes + tj;
            __syncthreads();
            if (!TAB) stage_net<P>(A, net, s_vec, s_w2, s_w3);
            __syncthreads();
            const wt* gw3 = reinterpret_cast<const wt*>(A.emat) + (size_t)net * EM_SIZE + EM_W3T;
            const int64_t gpl = (int64_t)nets * EM_SIZE;
            const acc* tab = reinterpret_cast<const acc*>(A.table) + (size_t)net * A.tab_nint * E2 * 6;
            acc* Tout = reinterpret_cast<acc*>(A.T);

            std::conditional_t<E3, PairWalk<P>, ChunkWalk<>> w;
            w.i = 0;
            w.c0 = 0;
            w.ac = 0;
            w.have = w.find_atom(A, nullptr, a0, a1, wave, NW, APW, ti, tj, false);
            w.fetch(A, tj, c16);
            accv Tacc[7];
            while (w.have) {
                double x = 0.0, y = 0.0, z = 0.0;
                acc th = 0, wt = 1;
                if constexpr (E3) {
                    th = w.ra[0] * w.rb[0] + w.ra[1] * w.rb[1] + w.ra[2] * w.rb[2] + w.ra[3] * w.rb[3];
                    wt = w.wgt;
                } else {
                    x = w.px; y = w.py; z = w.pz;
                }
                const int ca = w.a, cc0 = w.c0, cnp = w.np;
                bool last = false;
                w.c0 += 16;
                if (w.c0 >= w.np) {
                    ++w.i;
                    w.c0 = 0;
                    w.have = w.find_atom(A, nullptr, a0, a1, wave, NW, APW, ti, tj, false);
                    last = true;
                }
                w.fetch(A, tj, c16);
                if (cc0 == 0)
                    for (int t = 0; t < 7; ++t) zero4(Tacc[t]);

                const int p = c16;
                const bool valid = cc0 + p < cnp;
                double s = 0.0, R[4] = {0.0, 0.0, 0.0, 0.0};
                if (valid) {
                    if constexpr (E3) {
                        s = (double)th;
                        R[0] = (double)(wt * th);   // the pair and its mirror image
                    } else {
                        const double r = sqrt(x * x + y * y + z * z);
                        const double ir = 1.0 / r;
                        double ds;
                        switch_fn(r, ir, A.rs, A.rc, inv_w, s, ds);
                        const double sr = s * ir;
                        R[0] = s; R[1] = sr * x; R[2] = sr * y; R[3] = sr * z;
                    }
                }
                wave_sync();
                if (g == 0) {
                    for (int k = 0; k < 4; ++k) s_R[wave][p][k] = (acc)R[k];
                    s_x[wave][p] = s;
                }
                // T[m][k] += G_qm R_qk for feature m = 16 tm + c16 and neighbour q = orow(g, r) of this
                // lane: FP64 on the VALU; FP32 as outer4 with A = R_q[lane % 4] (register k gets
                // R_qk G_qm: all of T's row m over lane group g's neighbours)
                float Rq[4];
                auto add_G = [&](int tm, int r, int q, acc G) {
                    if constexpr (Cfg::F64) {
                        for (int k = 0; k < 4; ++k) Tacc[tm][k] += G * s_R[wave][q][k];
                    } else {
                        outer4(Tacc[tm], Rq[r], G);
                    }
                };
                if (TAB) {
                    wave_sync();
                    if constexpr (!Cfg::F64)
                        for (int r = 0; r < 4; ++r) Rq[r] = s_R[wave][P::orow(g, r)][c16 & 3];
                    for (int tm = 0; tm < 7; ++tm) {
                        const int m = 16 * tm + c16;
                        if (Cfg::F64 && m >= E2) continue;
                        for (int r = 0; r < 4; ++r) {
                            const int q = P::orow(g, r);
                            const double xs = s_x[wave][q];
                            int li = (int)floor(xs / A.tab_dx);
                            li = li < 0 ? 0 : (li >= A.tab_nint ? A.tab_nint - 1 : li);
                            const acc t = (acc)(xs - li * A.tab_dx);
                            const acc* cf = tab + ((size_t)li * E2 + (m < E2 ? m : 0)) * 6;
                            acc G = ((((cf[0] * t + cf[1]) * t + cf[2]) * t + cf[3]) * t + cf[4]) * t + cf[5];
                            if (m >= E2) G = 0;   // rows past 100 are not stored
                            add_G(tm, r, q, G);
                        }
                    }
                    if (blockIdx.y == 0 && g == 0 && valid && (s < 0.0 || s > A.tab_nint * A.tab_dx))
                        atomicAdd(&A.stats->table_oor, 1ull);
                } else {
                    // layer 1 (1 -> 25) straight into the B operand of layer 2 (register u = c VPL + v;
                    // padding rows have zero weights and give exact zeros)
                    frag B1[Cfg::NC1];
                    acc z1[Cfg::NC1 * P::VPL];
#pragma unroll
                    for (int c = 0; c < Cfg::NC1; ++c) {
#pragma unroll
                        for (int v = 0; v < P::VPL; ++v) {
                            const int k = P::kidx(c, g, v);
                            z1[c * P::VPL + v] = s_vec[EV_WH1 + k] * P::act((acc)s * s_vec[EV_W1 + k] + s_vec[EV_B1 + k]);
                        }
                        B1[c] = P::make(&z1[c * P::VPL]);
                    }
                    // layer 2 (25 -> 50), transposed: pre2^T = W2^T z1^T
                    accv acc2[4];
                    for (int t = 0; t < 4; ++t) {
                        zero4(acc2[t]);
                        for (int c = 0; c < Cfg::NC1; ++c)
                            P::mma(acc2[t], lds_frag<P>(s_w2, Cfg::ROW2, 16 * t + c16, 4 * c + g), B1[c]);
                    }
                    wave_sync();
                    // skip: register u = 4t + r of layer 2 adds register u / 2 of layer 1 (same lane)
                    acc zt[4][4];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int n = 16 * t + P::orow(g, r);
                            zt[t][r] = s_vec[EV_WH2 + n] * P::act_b(acc2[t][r], s_vec[EV_B2 + n]) + z1[(4 * t + r) >> 1];
                            s_z2[wave][p][n] = zt[t][r];
                        }
                    // output tiles -> K-chunks of layer 3: chunk c, value v is tile c*KC/16 + v/4, row r = v%4
                    frag A3[Cfg::NC2];
                    for (int c = 0; c < Cfg::NC2; ++c) {
                        acc x[P::VPL];
                        for (int v = 0; v < P::VPL; ++v) x[v] = zt[c * (P::KC / 16) + v / 4][v % 4];
                        A3[c] = P::make(x);
                    }
                    // layer 3 (50 -> 100), untransposed: pre3 = z2 W3
                    accv acc3[7];
                    for (int tm = 0; tm < 7; ++tm) {
                        zero4(acc3[tm]);
                        for (int c = 0; c < Cfg::NC2; ++c) {
                            const frag Bw = W3LDS ? lds_frag<P>(s_w3, Cfg::ROW3, 16 * tm + c16, 4 * c + g)
                                                  : P::load(gw3 + (16 * tm + c16) * N2P + P::KC * c + P::VPL * g, gpl);
                            P::mma(acc3[tm], A3[c], Bw);
                        }
                    }
                    wave_sync();
                    if constexpr (!Cfg::F64)
                        for (int r = 0; r < 4; ++r) Rq[r] = s_R[wave][P::orow(g, r)][c16 & 3];
                    // G = w_hat tanh(pre3 + b) + z2 at the skip source of row m = 16 tm + c16 (its
                    // register u in lane group ogrp(c16) takes layer-2 register u / 2 of that group);
                    // contraction T += G^T R (padding rows have zero weights, G = 0, and are not stored)
                    const int gc = P::ogrp(c16), rc = P::oreg(c16);
                    for (int tm = 0; tm < 7; ++tm) {
                        const int m = 16 * tm + c16;
                        if (Cfg::F64 && emb_feat(3, gc, 4 * tm + rc) < 0) continue;
                        const int u2 = (4 * tm + rc) >> 1;
                        const int n2 = 16 * (u2 >> 2) + P::orow(gc, u2 & 3);
                        const acc wh = s_vec[EV_WH3 + m], bb = s_vec[EV_B3 + m];
                        for (int r = 0; r < 4; ++r) {
                            const int q = P::orow(g, r);
                            const acc G = wh * P::act_b(acc3[tm][r], bb) + s_z2[wave][q][n2];
                            add_G(tm, r, q, G);
                        }
                    }
                }
                if (last) {
                    // T accumulates over the neighbour-type passes (lane group g owns component
                    // ksel(g) of row 16 tm + c16); the earlier passes' sum is read only here, so
                    // that it holds no registers during the network
                    // (row 16 tm + c16 is feature f: the same row for the table, the skip-aligned
                    // order for the network; f < 0 is a padding row)
                    const int gc = P::ogrp(c16), rc = P::oreg(c16);
                    auto feat = [&](int tm) { return TAB ? (16 * tm + c16 < E2 ? 16 * tm + c16 : -1) : emb_feat(3, gc, 4 * tm + rc); };
                    acc Tprev[7];
                    for (int tm = 0; tm < 7; ++tm) {
                        const int f = feat(tm);
                        Tprev[tm] = (tj > 0 && f >= 0) ? Tout[((size_t)ca * E2 + f) * 4 + ksel(g)] : (acc)0;
                    }
                    // sum the four lane groups (they hold different neighbours) and store T
                    for (int tm = 0; tm < 7; ++tm) {
                        const acc tv[4] = {Tacc[tm][0], Tacc[tm][1], Tacc[tm][2], Tacc[tm][3]};
                        const acc v = sum_groups4(tv);
                        const int f = feat(tm);
                        if (f >= 0)
                            Tout[((size_t)ca * E2 + f) * 4 + ksel(g)] = v * (acc)A.inv_nc + Tprev[tm];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Backward (input gradient only): re-evaluate G_j and dG_j/ds, then
//   dE/dR_j = N_c^-1 G_j dT,  dE/ds_j|_G = N_c^-1 sum_m dG_jm/ds (dT R_j)_m,
//   g_ij = dE/dr_ij = [(dR_0 + dE/ds) s' + q (s' - s/r)] r^ + (s/r) dR_{1:3},  q = dR_{1:3} . r^,
//   F_i += g_ij, F_j -= g_ij (FP64 atomics into caller order), Xi_ab -= g_ij,a r_ij,b (FP64,
//   per-block partials, with E over the block's atoms for a single frame).
// E3 (three-body descriptor, one atom per wave): a pair row gives
//   dE/dtheta_jk = N_c^-2 sum_m dD_m (G_m + theta dG_m/dtheta)   (dT[m][0] = dE/dD_m),
// and theta_jk = R_j . R_k adds dE/dtheta R_k to dE/dR_j and dE/dtheta R_j to dE/dR_k (LDS
// atomics into the wave's slot rows); after the last pass each slot's dE/dR_j goes through the
// same g_ij formula (with dE/ds folded into dR_0).
// ---------------------------------------------------------------------------------------------
template <class P, bool TAB, bool ENS, bool E3>
__global__ void __launch_bounds__((EmbCfg<P, false, TAB>::NW * 64)) k_embed_bwd(EmbArgs A_)
{
    const EmbArgs A = ENS ? model_args(A_) : A_;
    typedef typename P::acc acc;
    typedef typename P::wt wt;
    typedef typename P::accv accv;
    typedef typename P::frag frag;
    typedef EmbCfg<P, false, TAB> Cfg;
    constexpr int NW = Cfg::NW;
    const int APW = A.apw, APB = NW * APW;
    constexpr bool W3LDS = Cfg::W3LDS;
    constexpr int DTL = (E2 * 4 + 63) / 64;     // dT values per lane
    __shared__ acc s_vec[EVEC];
    __shared__ __attribute__((aligned(16))) char s_w2[TAB ? 16 : N2P * Cfg::ROW2];
    __shared__ __attribute__((aligned(16))) char s_w3[(TAB || !W3LDS) ? 16 : N3P * Cfg::ROW3];
    // dT of the wave's current atom by layer-3 row (the feature's row position; padding rows zero)
    __shared__ __attribute__((aligned(16))) acc s_dT[NW][N3P][4];
    // per neighbour column of a wave: [0, 3) the centre atom's force over its pairs, [3, 12) the
    // virial sum -g r^T over the wave's pairs (kept here rather than in every lane's registers);
    // 13 doubles per column (the 16 columns' read-modify-writes conflict less in the banks than
    // with 12: the backward's bank-conflict counter reads 8 % lower)
    __shared__ __attribute__((aligned(16))) double s_pair[NW][16][13];
    // the LDS atom table of the walk (its reads do not wait on the in-order vector memory counter,
    // which also holds the force atomics)
    __shared__ int s_wl[NW][2 * WL_MAX];
    // three-body: dE/dR_j of every slot of the wave's atom
    __shared__ __attribute__((aligned(16))) acc s_dRs[E3 ? NW : 1][E3 ? E3_MAXN : 1][4];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar registers)
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    for (int e = lane; e < N3P * 4; e += 64) s_dT[wave][e >> 2][e & 3] = 0;
    for (int e = lane; e < 16 * 12; e += 64) s_pair[wave][e / 12][e % 12] = 0.0;
    if constexpr (E3)
        for (int e = lane; e < E3_MAXN * 4; e += 64) s_dRs[wave][e >> 2][e & 3] = 0;
    const double inv_w = 1.0 / (A.rc - A.rs);
    const int a0 = blockIdx.x * APB;
    const int a1 = min(a0 + APB, A.natoms);
    const int nets = A.type_one_side ? A.ntypes : A.ntypes * A.ntypes;
    const acc* dTin = reinterpret_cast<const acc*>(A.dT);
    const int t_lo = a0 < a1 ? A.itype[a0] : 0, t_hi = a0 < a1 ? A.itype[a1 - 1] : -1;
    const int npass = E3 ? A.ntypes * A.ntypes : A.ntypes;

    for (int ti = t_lo; ti <= t_hi; ++ti) {
        for (int tj = 0; tj < npass; ++tj) {
            const int net = (E3 || A.type_one_side) ? tj : ti * A.ntypes + tj;
            __syncthreads();
            if (!TAB) stage_net<P>(A, net, s_vec, s_w2, s_w3);
            __syncthreads();
            const wt* gw3 = reinterpret_cast<const wt*>(A.emat) + (size_t)net * EM_SIZE + EM_W3T;
            const int64_t gpl = (int64_t)nets * EM_SIZE;
            const acc* tab = reinterpret_cast<const acc*>(A.table) + (size_t)net * A.tab_nint * E2 * 6;

            std::conditional_t<E3, PairWalk<P>, ChunkWalk<true>> w;
            w.i = 0;
            w.c0 = 0;
            w.ac = 0;
            if constexpr (!E3) w.template load_atoms<true>(s_wl[wave], A, a0, a1, wave, NW, APW, tj, lane);
            w.have = w.template find_atom<true>(A, s_wl[wave], a0, a1, wave, NW, APW, ti, tj, true);
            w.template fetch<true>(A, tj, c16);
            acc pdT[DTL];
            for (int q = 0; q < DTL; ++q) {
                const int e = lane + 64 * q;
                pdT[q] = (w.have && e < E2 * 4) ? dTin[(size_t)w.a * E2 * 4 + e] : (acc)0;
            }
            // the first chunk's r and j are in place before the loop, as every later chunk's are
            // at the end of the previous one, so the loop itself never waits for them
            if constexpr (E3) w.pin();
            else asm volatile("" ::"v"(w.px), "v"(w.py), "v"(w.pz), "v"(w.pj));
            while (w.have) {
                double x = 0.0, y = 0.0, z = 0.0;
                int jn = 0;
                accv ra, rb;   // three-body: the pair's rows, slots and weight
                int sa = 0, sb = 0;
                acc wt = 1;
                if constexpr (E3) {
                    ra = w.ra; rb = w.rb; sa = w.sa; sb = w.sb; wt = w.wgt;
                } else {
                    x = w.px; y = w.py; z = w.pz;
                    jn = w.pj;
                }
                const int ca = w.a, cac = w.ac, cc0 = w.c0, cnp = w.np;
                bool last = false;
                w.c0 += 16;
                if (w.c0 >= w.np) {
                    ++w.i;
                    w.c0 = 0;
                    w.have = w.template find_atom<true>(A, s_wl[wave], a0, a1, wave, NW, APW, ti, tj, true);
                    last = true;
                }
                w.template fetch<true>(A, tj, c16);
                if (cc0 == 0) {
                    // the prefetched dT of this atom goes to LDS, feature f to its layer-3 row; the
                    // next atom's is requested
                    wave_sync();
                    for (int q = 0; q < DTL; ++q) {
                        const int e = lane + 64 * q, f = e >> 2;
                        if (e < E2 * 4) {
                            int gf = 0, uf = 0;
                            emb_reg3(f, gf, uf);
                            const int row = TAB ? f : 16 * (uf >> 2) + P::orow(gf, uf & 3);
                            s_dT[wave][row][e & 3] = pdT[q];
                        }
                    }
                    wave_sync();
                }
                if (last) {
                    for (int q = 0; q < DTL; ++q) {
                        const int e = lane + 64 * q;
                        pdT[q] = (w.have && e < E2 * 4) ? dTin[(size_t)w.a * E2 * 4 + e] : (acc)0;
                    }
                }

                const int p = c16;
                const bool valid = cc0 + p < cnp;
                double ir = 1.0, s = 0.0, ds = 0.0;
                if (valid) {
                    if constexpr (E3) {
                        s = (double)(ra[0] * rb[0] + ra[1] * rb[1] + ra[2] * rb[2] + ra[3] * rb[3]);
                    } else {
                        const double r = sqrt(x * x + y * y + z * z);
                        ir = 1.0 / r;
                        switch_fn(r, ir, A.rs, A.rc, inv_w, s, ds);
                    }
                }
                acc dR[4] = {0, 0, 0, 0}, H[4] = {0, 0, 0, 0};
                if (TAB) {
                    int li = (int)floor(s / A.tab_dx);
                    li = li < 0 ? 0 : (li >= A.tab_nint ? A.tab_nint - 1 : li);
                    const acc t = (acc)(s - li * A.tab_dx);
                    for (int tm = 0; tm < 7; ++tm)
                        for (int rr = 0; rr < 4; ++rr) {
                            const int m = 16 * tm + P::orow(g, rr);
                            if (m >= E2) continue;
                            const acc* cf = tab + ((size_t)li * E2 + m) * 6;
                            const acc G = ((((cf[0] * t + cf[1]) * t + cf[2]) * t + cf[3]) * t + cf[4]) * t + cf[5];
                            const acc Gd = (((5 * cf[0] * t + 4 * cf[1]) * t + 3 * cf[2]) * t + 2 * cf[3]) * t + cf[4];
                            for (int k = 0; k < 4; ++k) {
                                const acc dt = s_dT[wave][m][k];
                                dR[k] += G * dt;
                                H[k] += Gd * dt;
                            }
                        }
                } else {
                    // layer 1 and its derivative d/ds (register u = c VPL + v; padding rows have zero
                    // weights and give exact zeros)
                    frag B1[Cfg::NC1], B1d[Cfg::NC1];
                    acc z1[Cfg::NC1 * P::VPL], z1d[Cfg::NC1 * P::VPL];
#pragma unroll
                    for (int c = 0; c < Cfg::NC1; ++c) {
#pragma unroll
                        for (int v = 0; v < P::VPL; ++v) {
                            const int k = P::kidx(c, g, v);
                            const acc w1 = s_vec[EV_W1 + k], wh = s_vec[EV_WH1 + k];
                            const acc t1 = P::act((acc)s * w1 + s_vec[EV_B1 + k]);
                            z1[c * P::VPL + v] = wh * t1;
                            z1d[c * P::VPL + v] = wh * (1 - t1 * t1) * w1;
                        }
                        B1[c] = P::make(&z1[c * P::VPL]);
                        B1d[c] = P::make(&z1d[c * P::VPL]);
                    }
                    accv acc2[4], acc2d[4];
                    for (int t = 0; t < 4; ++t) {
                        zero4(acc2[t]);
                        zero4(acc2d[t]);
                        for (int c = 0; c < Cfg::NC1; ++c) {
                            const frag W = lds_frag<P>(s_w2, Cfg::ROW2, 16 * t + c16, 4 * c + g);
                            P::mma(acc2[t], W, B1[c]);
                            P::mma(acc2d[t], W, B1d[c]);
                        }
                    }
                    // skip: register u = 4t + rr of layer 2 adds register u / 2 of layer 1 (same lane)
                    acc zt[4][4], ztd[4][4];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) {
                            const int n = 16 * t + P::orow(g, rr), u1 = (4 * t + rr) >> 1;
                            const acc t2 = P::act_b(acc2[t][rr], s_vec[EV_B2 + n]);
                            const acc wh = s_vec[EV_WH2 + n];
                            zt[t][rr] = wh * t2 + z1[u1];
                            ztd[t][rr] = wh * (1 - t2 * t2) * acc2d[t][rr] + z1d[u1];
                        }
                    // output tiles -> K-chunks of layer 3 (chunk c, value v: tile c*KC/16 + v/4, row v%4)
                    frag B3[Cfg::NC2], B3d[Cfg::NC2];
                    for (int c = 0; c < Cfg::NC2; ++c) {
                        acc x[P::VPL], xd[P::VPL];
                        for (int v = 0; v < P::VPL; ++v) {
                            x[v] = zt[c * (P::KC / 16) + v / 4][v % 4];
                            xd[v] = ztd[c * (P::KC / 16) + v / 4][v % 4];
                        }
                        B3[c] = P::make(x);
                        B3d[c] = P::make(xd);
                    }
                    // layer 3 transposed (one neighbour per lane column), one output tile at a time:
                    // the products of tile tm + 1 are issued before the epilogue of tile tm, so only
                    // two tiles of accumulators are live
                    auto mm3 = [&](int tm, accv& o, accv& od) {
                        zero4(o);
                        zero4(od);
#pragma unroll
                        for (int c = 0; c < Cfg::NC2; ++c) {
                            const frag W = W3LDS ? lds_frag<P>(s_w3, Cfg::ROW3, 16 * tm + c16, 4 * c + g)
                                                 : P::load(gw3 + (16 * tm + c16) * N2P + P::KC * c + P::VPL * g, gpl);
                            P::mma(o, W, B3[c]);
                            P::mma(od, W, B3d[c]);
                        }
                    };
                    f4 dRq, Hq;   // FP32 paths: the contraction's accumulators (see outer4)
                    // skip: register u = 4 tm + rr of layer 3 adds register u / 2 of layer 2 (same
                    // lane); padding rows give G = Gd = 0 against zero rows of dT
                    auto epi3 = [&](int tm, const accv& o, const accv& od) {
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) {
                            const int m = 16 * tm + P::orow(g, rr), u2 = (4 * tm + rr) >> 1;
                            const acc t3 = P::act_b(o[rr], s_vec[EV_B3 + m]);
                            const acc wh = s_vec[EV_WH3 + m];
                            const acc G = wh * t3 + zt[u2 >> 2][u2 & 3];
                            const acc Gd = wh * (1 - t3 * t3) * od[rr] + ztd[u2 >> 2][u2 & 3];
                            if constexpr (Cfg::F64) {
                                const acc* dt = s_dT[wave][m];
                                dR[0] += G * dt[0]; dR[1] += G * dt[1]; dR[2] += G * dt[2]; dR[3] += G * dt[3];
                                H[0] += Gd * dt[0]; H[1] += Gd * dt[1]; H[2] += Gd * dt[2]; H[3] += Gd * dt[3];
                            } else {
                                // rank-1 updates on the matrix cores: every lane of a quad has the
                                // same row m, so register k gains dT[m][k] G (and dT[m][k] Gd)
                                const acc dtq = s_dT[wave][m][lane & 3];
                                outer4(dRq, dtq, G);
                                outer4(Hq, dtq, Gd);
                            }
                        }
                    };
                    zero4(dRq);
                    zero4(Hq);
                    accv a3[2], a3d[2];
                    mm3(0, a3[0], a3d[0]);
#pragma unroll
                    for (int tm = 0; tm < 7; ++tm) {
                        if (tm + 1 < 7) mm3(tm + 1, a3[(tm + 1) & 1], a3d[(tm + 1) & 1]);
                        epi3(tm, a3[tm & 1], a3d[tm & 1]);
                    }
                    if constexpr (!Cfg::F64)
                        for (int k = 0; k < 4; ++k) { dR[k] = dRq[k]; H[k] = Hq[k]; }
                }
                // column sums over the lane groups (they hold different rows m): dR component ksel(g)
                // in lane group g, gathered into group 0; sum_k H_k R_k as one value
                const double ux = x * ir, uy = y * ir, uz = z * ir, sr = s * ir;
                const acc Ra[4] = {E3 ? (acc)(wt * (acc)s) : (acc)s, (acc)(sr * x), (acc)(sr * y), (acc)(sr * z)};
                const acc dRg = sum_groups4(dR);
                const acc hR = sum_groups(H[0] * Ra[0] + H[1] * Ra[1] + H[2] * Ra[2] + H[3] * Ra[3]);
                if constexpr (E3) {
                    // dE/dtheta of the row (weight w: the pair and its mirror image; lane group 0
                    // holds component 0 of dR), to every group; group g adds component g of both
                    // rows' gradients
                    const acc de = __shfl((acc)A.inv_nc * (wt * dRg + hR), c16);
                    w.pin();
                    if (valid) {
                        const acc rag = g == 0 ? ra[0] : g == 1 ? ra[1] : g == 2 ? ra[2] : ra[3];
                        const acc rbg = g == 0 ? rb[0] : g == 1 ? rb[1] : g == 2 ? rb[2] : rb[3];
                        atomicAdd(&s_dRs[wave][sa][g], de * rbg);
                        atomicAdd(&s_dRs[wave][sb][g], de * rag);
                    }
                    continue;
                }
                const acc dR2 = __shfl(dRg, c16 + 16), dR1 = __shfl(dRg, c16 + 32), dR3 = __shfl(dRg, c16 + 48);
                // The next chunk's prefetched r and j are put in place here, after this chunk's work
                // and before its force atomics: reads and atomics retire in order, so waiting for the
                // prefetch after the atomics (where the compiler otherwise sinks it) waits for them too.
                if constexpr (!E3) asm volatile("" ::"v"(w.px), "v"(w.py), "v"(w.pz), "v"(w.pj));
                if (valid && g == 0) {
                    const double inc = A.inv_nc;
                    const double d0 = inc * (double)dRg, d1 = inc * (double)dR1;
                    const double d2 = inc * (double)dR2, d3 = inc * (double)dR3;
                    const double dEds = inc * (double)hR;
                    const double q = d1 * ux + d2 * uy + d3 * uz;
                    const double rad = (d0 + dEds) * ds + q * (ds - sr);
                    const double gx = rad * ux + sr * d1, gy = rad * uy + sr * d2, gz = rad * uz + sr * d3;
                    unsafeAtomicAdd(&A.F[3 * (size_t)jn], -gx);
                    unsafeAtomicAdd(&A.F[3 * (size_t)jn + 1], -gy);
                    unsafeAtomicAdd(&A.F[3 * (size_t)jn + 2], -gz);
                    double* pa = s_pair[wave][p];
                    pa[0] += gx; pa[1] += gy; pa[2] += gz;
                    pa[3] -= gx * x; pa[4] -= gx * y; pa[5] -= gx * z;
                    pa[6] -= gy * x; pa[7] -= gy * y; pa[8] -= gy * z;
                    pa[9] -= gz * x; pa[10] -= gz * y; pa[11] -= gz * z;
                }
                if (last) {
                    // the centre atom's force (and, for batched frames, its share of the virial:
                    // one wave owns the atom in every pass) summed over the 16 columns
                    wave_sync();
                    const int nk = A.vir_atom ? 12 : 3;
                    for (int k = 0; k < nk; ++k) {
                        double v = s_pair[wave][c16][k];
                        v += __shfl_xor(v, 1);
                        v += __shfl_xor(v, 2);
                        v += __shfl_xor(v, 4);
                        v += __shfl_xor(v, 8);
                        if (lane == 0) {
                            if (k < 3) {
                                unsafeAtomicAdd(&A.F[3 * (size_t)cac + k], v);
                            } else {
                                A.vir_atom[9 * (size_t)ca + k - 3] += v;
                            }
                        }
                    }
                    wave_sync();
                    if (g == 0)
                        for (int k = 0; k < nk; ++k) s_pair[wave][c16][k] = 0.0;
                }
            }
        }
    }
    if constexpr (E3) {
        // slot gradients -> forces and virial (Sec. II.A.2) for the wave's atom (apw = 1)
        wave_sync();
        const int a = a0 + wave;
        if (a < a1) {
            const int nt = A.ntypes;
            double f[3] = {0.0, 0.0, 0.0}, vir[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int sl = lane; sl < A.nc; sl += 64) {
                int t = 0;
                while (t + 1 < nt && sl >= A.off[t + 1]) ++t;
                if (sl - A.off[t] >= A.nnei[(size_t)a * nt + t]) continue;
                const size_t slot = (size_t)a * A.nc + sl;
                const double x = A.nl_r[3 * slot], y = A.nl_r[3 * slot + 1], z = A.nl_r[3 * slot + 2];
                const int j = A.nl_j[slot];
                const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
                double s, ds;
                switch_fn(r, ir, A.rs, A.rc, inv_w, s, ds);
                const double ux = x * ir, uy = y * ir, uz = z * ir, sr = s * ir;
                const double d0 = s_dRs[wave][sl][0], d1 = s_dRs[wave][sl][1], d2 = s_dRs[wave][sl][2],
                             d3 = s_dRs[wave][sl][3];
                const double q = d1 * ux + d2 * uy + d3 * uz;
                const double rad = d0 * ds + q * (ds - sr);
                const double gx = rad * ux + sr * d1, gy = rad * uy + sr * d2, gz = rad * uz + sr * d3;
                unsafeAtomicAdd(&A.F[3 * (size_t)j], -gx);
                unsafeAtomicAdd(&A.F[3 * (size_t)j + 1], -gy);
                unsafeAtomicAdd(&A.F[3 * (size_t)j + 2], -gz);
                f[0] += gx; f[1] += gy; f[2] += gz;
                vir[0] -= gx * x; vir[1] -= gx * y; vir[2] -= gx * z;
                vir[3] -= gy * x; vir[4] -= gy * y; vir[5] -= gy * z;
                vir[6] -= gz * x; vir[7] -= gz * y; vir[8] -= gz * z;
            }
            auto wsum = [](double v) {
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
                return v;
            };
            for (int k = 0; k < 3; ++k) f[k] = wsum(f[k]);
            for (int k = 0; k < 9; ++k) vir[k] = wsum(vir[k]);
            if (lane == 0) {
                const int ac = A.perm[a];
                for (int k = 0; k < 3; ++k) unsafeAtomicAdd(&A.F[3 * (size_t)ac + k], f[k]);
                for (int k = 0; k < 9; ++k) {
                    if (A.vir_atom) A.vir_atom[9 * (size_t)a + k] += vir[k];
                    else s_pair[wave][0][3 + k] += vir[k];
                }
            }
        }
    }
    __syncthreads();
    // block partial [E, virial]: the virial over the waves' columns, E over this block's atoms (a
    // shuffle tree, a fixed order; single frame), and E_i in caller order if asked for
    double* part = A.vir_part + 10 * (size_t)blockIdx.x;
    if (threadIdx.x < 9) {
        double v = 0.0;
        for (int q = 0; q < NW; ++q)
            for (int c = 0; c < 16; ++c) v += s_pair[q][c][3 + threadIdx.x];
        part[1 + threadIdx.x] = v;
    }
    if (A.Ei) {
        if (threadIdx.x < 64) {
            double e = 0.0;
            for (int a = a0 + lane; a < a1; a += 64) e += A.Ei[a];
            for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
            if (lane == 0) part[0] = e;
        }
        if (A.atom_energy)
            for (int a = a0 + (int)threadIdx.x; a < a1; a += NW * 64) A.atom_energy[A.perm[a]] = A.Ei[a];
    }
}

// ---------------------------------------------------------------------------------------------
// Fitting net F_0 of the FP64 path (Sec. II.A.2, eq. fitting_energy): forward E_i and the input
// gradient dE_i/dT through D = T T_<^T. Each wave owns 16 atoms and computes all 240 features of
// every layer; the four waves of a block share the weight K-chunks, staged through LDS with
// register double buffering. (The BF16 paths use k_fitx in kernels_fit.hip.)
// ---------------------------------------------------------------------------------------------

// Weight staging for the FP64 fitting kernel. A stage is ROWS rows x KC columns (K) of a row-major
// matrix in global memory, stored per plane (BF16 hi, BF16 lo) or once (FP64). In LDS each row
// holds KC/4 groups of four K values; a group is [hi0..3 lo0..3] (16 B) or [four doubles] (32 B),
// exactly one lane's A fragment, and rows are padded by 16 B so the 16 rows a wave reads at once
// fall in distinct banks. Global reads are 16-B pieces, issued into registers by load() one stage
// ahead and written to LDS by store() after the MFMAs of the current stage.
template <class P, int ROWS, int KC, int NT = 256>
struct FitStage {
    typedef typename P::wt wt;
    static constexpr int GB = 4 * sizeof(wt) * P::NPL;       // bytes per group in LDS
    static constexpr int ROWB = (KC / 4) * GB + 16;           // bytes per LDS row
    static constexpr int BYTES = ROWS * ROWB;
    static constexpr int EPP = 16 / sizeof(wt);               // elements per 16-B piece
    static constexpr int PPR = KC / EPP;                      // pieces per row and plane
    static constexpr int TOTAL = ROWS * PPR * P::NPL;
    static constexpr int NP = (TOTAL + NT - 1) / NT;          // pieces per thread (NT threads)
    u32x4 r[NP];

    // Only the first nrows <= ROWS source rows are read; staged rows past them repeat the last one.
    __device__ __forceinline__ void load(const wt* src, int64_t ld, int64_t plane, int k0, int nrows = ROWS) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int q = threadIdx.x + NT * p;
            if (TOTAL % NT == 0 || q < TOTAL) {
                const int pl = q / (ROWS * PPR), rem = q - pl * ROWS * PPR;
                const int row = rem / PPR, pc = rem - row * PPR;
                const int rs = row < nrows ? row : nrows - 1;
                r[p] = *reinterpret_cast<const u32x4*>(src + pl * plane + (int64_t)rs * ld + k0 + pc * EPP);
            }
        }
    }
    // Two row ranges in one stage: rows [0, ROWS/2) from the first n0 rows of src0 and rows
    // [ROWS/2, ROWS) from the first n1 rows of src1 (n0, n1 >= 1; past them the last row repeats).
    __device__ __forceinline__ void load2(const wt* src0, int n0, const wt* src1, int n1, int64_t ld, int k0) {
        static_assert(P::NPL == 1, "one plane");
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int q = threadIdx.x + NT * p;
            if (TOTAL % NT == 0 || q < TOTAL) {
                const int row = q / PPR, pc = q - row * PPR;
                const bool hi = row >= ROWS / 2;
                const int lr = hi ? row - ROWS / 2 : row, n = hi ? n1 : n0;
                const int rs = lr < n ? lr : n - 1;
                r[p] = *reinterpret_cast<const u32x4*>((hi ? src1 : src0) + (int64_t)rs * ld + k0 + pc * EPP);
            }
        }
    }
    __device__ __forceinline__ void store(char* dst) const {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int q = threadIdx.x + NT * p;
            if (TOTAL % NT == 0 || q < TOTAL) {
                const int pl = q / (ROWS * PPR), rem = q - pl * ROWS * PPR;
                const int row = rem / PPR, pc = rem - row * PPR;
                char* rowp = dst + row * ROWB;
                if (sizeof(wt) == 8) {
                    // two doubles: half of group pc/2
                    *reinterpret_cast<u32x4*>(rowp + (pc >> 1) * GB + (pc & 1) * 16) = r[p];
                } else if (sizeof(wt) == 4) {
                    // four floats: group pc
                    *reinterpret_cast<u32x4*>(rowp + pc * GB) = r[p];
                } else {
                    // eight BF16 of one plane: the plane's half of groups 2pc and 2pc+1
                    *reinterpret_cast<uint2*>(rowp + (2 * pc) * GB + pl * 8) = make_uint2(r[p].x, r[p].y);
                    *reinterpret_cast<uint2*>(rowp + (2 * pc + 1) * GB + pl * 8) = make_uint2(r[p].z, r[p].w);
                }
            }
        }
    }
};

// A fragment of row `row`, group `grp` of a staged block.
template <class P, int ROWB>
__device__ __forceinline__ typename P::frag fit_afrag(const char* base, int row, int grp)
{
    typename P::frag f;
    const char* p = base + row * ROWB + grp * (4 * sizeof(typename P::wt) * P::NPL);
    if constexpr (P::NPL == 2) {
        f.h = *reinterpret_cast<const bf4*>(p);
        f.l = *reinterpret_cast<const bf4*>(p + 8);
    } else {
        f = *reinterpret_cast<const typename P::frag*>(p);
    }
    return f;
}

// ---------------------------------------------------------------------------------------------
// Fitting net on the 16x16x4 MFMA of one element type: FP64 (PF64) or FP32 (PF32). FP64
// accumulators take twice the registers, so every product runs in passes of eight 16-row output
// tiles and the layer outputs go to a per-atom scratch row instead of registers. Values are stored
// in the K order the MFMA lanes read (position 16c + 4g + v holds logical index kidx(c, g, v):
// 16c + g + 4v in FP64, 16c + 4g + v in FP32): the four outputs a lane produces and the four
// B-operand values it later reads are the same 32 (FP64) or 16 (FP32) bytes, written and read by
// the same lane, so the scratch row needs no synchronisation.
// Scratch row per atom: a1, a2, a3 (tanh outputs), ga (two ping-pong buffers), gh; during the
// forward pass the slots of the second ga buffer and of gh hold the inputs of layers 2 and 3.
// RAD: a descriptor of M values D_m = T[m][0] (se_e2_r, se_e3): layer 1 has K = 100 (padded to
// 112, zero weights past 100; W1^T is [240][112] and W1 [112][240] in the same slots), and the
// input gradient is dT[m] = (dE/dD_m, 0, 0, 0).
// ---------------------------------------------------------------------------------------------
constexpr int F64_TP = 8;
constexpr int FS_A1 = 0, FS_A2 = FW, FS_A3 = 2 * FW, FS_GA = 3 * FW, FS_GB = 4 * FW, FS_GH = 5 * FW, FS_ROW = 6 * FW;
constexpr int RAD_K = N3P;   // padded width of a descriptor of M values

// HALVES = 2: eight waves per block, two per atom tile; each layer's output tiles are split
// between the two (the first ceil(n/2) tiles and the rest), and one LDS stage holds both halves'
// weight rows. Every layer's input is read by both halves, so the scratch row is then shared between
// two waves of the block (ordered by the barriers at the start of every product).
template <class P, bool ENS, bool RAD, int HALVES>
__global__ void __launch_bounds__(256 * HALVES) k_fit_dense(FitArgs A_)
{
    const FitArgs A = ENS ? model_args(A_) : A_;
    typedef typename P::acc acc;
    typedef typename P::accv accv;
    typedef typename P::wt wt;
    typedef typename P::frag frag;
    typedef accv d4;   // four values of the element type (the lane's 4-row output or K group)
    // output tiles per pass: eight, or four in the two-half shape (two waves per SIMD: half the
    // registers per wave)
    constexpr int TP = HALVES == 2 ? 4 : F64_TP;
    typedef FitStage<P, 16 * TP * HALVES, 16, 256 * HALVES> SW;
    __shared__ __attribute__((aligned(32))) char s_w[2][SW::BYTES];
    __shared__ acc s_p1[4][16][16][4];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar registers)
    const int aw = wave & 3, h = HALVES == 2 ? wave >> 2 : 0;           // atom tile, half
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const int a0 = blockIdx.x * FIT_AF;
    const int a1 = min(a0 + FIT_AF, A.natoms);
    if (a0 >= a1) return;
    const int t_lo = A.itype[a0], t_hi = A.itype[a1 - 1];
    const acc* Tin = reinterpret_cast<const acc*>(A.T);
    acc* dTout = reinterpret_cast<acc*>(A.dT);
    const int atom = a0 + 16 * aw + c16;
    const bool real = atom < A.natoms;
    const int arow = real ? atom : a0;
    const acc* Ta = Tin + (size_t)arow * E2 * 4;
    acc* row = reinterpret_cast<acc*>(A.act) + (size_t)atom * FS_ROW;   // a row for every lane of the grid
    auto rd4 = [&](int off) { return *reinterpret_cast<const d4*>(row + off); };
    auto wr4 = [&](int off, const acc* x) { *reinterpret_cast<d4*>(row + off) = d4{x[0], x[1], x[2], x[3]}; };

#pragma unroll 1
    for (int ti = t_lo; ti <= t_hi; ++ti) {
        const bool mine = real && A.itype[atom] == ti;
        const acc* fv = reinterpret_cast<const acc*>(A.fvec) + (size_t)ti * FVEC;
        const wt* fm = reinterpret_cast<const wt*>(A.fmat) + (size_t)ti * FM_SIZE;
        acc Tn[4][4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int k = 0; k < 4; ++k) Tn[v][k] = RAD ? (acc)0 : Ta[P::kidx(0, g, v) * 4 + k];

        // y = W x for ntiles 16-row output tiles of the row-major matrix at fm + mo (K columns,
        // stored in the MFMA K order); x for K-chunk c is make(fetch(c)), where fetch(c) is the one
        // memory read (32 B per lane) and make works on registers only; epi(t, out) receives
        // output tile t (rows 16t + orow(g, r)). Reads retire in issue order, so each chunk's
        // fetch is issued one chunk ahead and before the weight loads it would otherwise wait on.
        // tiles of this wave: [tb, te) of ntiles (all of them, or its half)
        auto tiles_of = [&](int ntiles, int& tb, int& te) {
            const int hs = HALVES == 2 ? (ntiles + 1) / 2 : ntiles;
            tb = h * hs;
            te = min(ntiles, tb + hs);
        };
        auto gemm = [&](int64_t mo, int K, int ntiles, auto&& fetch, auto&& make, auto&& epi) {
            const int nchunk = K / 16;
            const int hs = HALVES == 2 ? (ntiles + 1) / 2 : ntiles;   // tiles of the first half
            int tb, te;
            tiles_of(ntiles, tb, te);
#pragma unroll 1
            for (int t0 = 0; t0 < hs; t0 += TP) {
                const int nt = min(TP, te - tb - t0);   // this wave's tiles in the pass (may be <= 0)
                const int n0 = min(TP, hs - t0), n1 = max(1, min(TP, ntiles - hs - t0));
                accv accs[TP];
#pragma unroll
                for (int t = 0; t < TP; ++t) zero4(accs[t]);
                // Weight chunks are fetched two ahead (two register stages in flight, alternated by
                // unrolling the chunk loop twice) and staged through two LDS buffers: chunk c + 1
                // goes to LDS after chunk c's products, into the buffer the previous barrier freed.
                // Every read is unconditional (past the last chunk it repeats the last one), so that
                // the compiler's in-order wait counts stay exact instead of draining all reads.
                SW st0, st1;
                const wt* src = fm + mo + (int64_t)16 * t0 * K;
                const wt* src1 = fm + mo + (int64_t)16 * (hs + t0) * K;
                auto ld = [&](SW& st, int k0) {
                    if constexpr (HALVES == 2) st.load2(src, 16 * n0, src1, 16 * n1, K, k0);
                    else st.load(src, K, 0, k0, 16 * n0);
                };
                const int clast = nchunk - 1;
                __syncthreads();
                d4 x0 = fetch(0), x1 = {0, 0, 0, 0};
                ld(st0, 0);
                st0.store(s_w[0]);
                ld(st1, 16 * min(1, clast));
                __syncthreads();
                // chunk c from LDS; `nxt` holds chunk c + 1 in flight, `fut` receives chunk c + 2;
                // xc holds chunk c's fetch, xn receives chunk c + 1's
                const int rb = 16 * TP * h;   // this half's first staged row
                auto step = [&](int c, SW& nxt, SW& fut, const d4& xc, d4& xn) {
                    xn = fetch(min(c + 1, clast));
                    ld(fut, 16 * min(c + 2, clast));
                    const frag B = make(xc);
                    const char* buf = s_w[c & 1];
#pragma unroll
                    for (int t = 0; t < TP; ++t)
                        if (t < nt) P::mma(accs[t], fit_afrag<P, SW::ROWB>(buf, rb + 16 * t + c16, g), B);
                    nxt.store(s_w[(c + 1) & 1]);
                    __syncthreads();
                };
#pragma unroll 1
                for (int c = 0; c + 1 < nchunk; c += 2) {
                    step(c, st1, st0, x0, x1);
                    step(c + 1, st0, st1, x1, x0);
                }
                if (nchunk & 1) step(clast, st1, st0, x0, x1);
#pragma unroll
                for (int t = 0; t < TP; ++t)
                    if (t < nt) {
                        const acc o[4] = {accs[t][0], accs[t][1], accs[t][2], accs[t][3]};
                        epi(tb + t0 + t, o);
                    }
            }
        };
        auto vec = [&](int off, int t, int r) { return fv[off + 16 * t + P::orow(g, r)]; };
        auto rdrow = [&](int off) { return [&, off](int c) { return rd4(off + 16 * c + 4 * g); }; };
        auto asis = [](const d4& x) { return P::make(x[0], x[1], x[2], x[3]); };

        // a = tanh(y + b) in place over the 15 tiles of a layer output (a loop, so that the
        // activation is inlined once rather than once per tile); side(t, a) forms the next
        // layer's input from it
        int ab, ae;   // this wave's tiles of a 240-wide layer
        tiles_of(15, ab, ae);
        auto activate = [&](int off, int boff, auto&& side) {
#pragma unroll 1
            for (int t = ab; t < ae; ++t) {
                const d4 y = rd4(off + 16 * t + 4 * g);
                acc a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = P::act(y[r] + vec(boff, t, r));
                wr4(off + 16 * t + 4 * g, a);
                side(t, a);
            }
        };

        // ---------------------------------------------------------- forward
        // layer 1: a1 = tanh(W1 D + b1), D formed on the fly from T (Eq. 7); RAD: D_m = T[m][0]
        if constexpr (RAD) {
            gemm(FM_W1T, RAD_K, 15,
                 [&](int c) {
                     d4 x;
#pragma unroll
                     for (int v = 0; v < 4; ++v) {
                         const int m = P::kidx(c, g, v);
                         x[v] = Ta[(m < E2 ? m : 0) * 4];
                         if (m >= E2) x[v] = 0;
                     }
                     return x;
                 },
                 asis, [&](int t, const acc* o) { wr4(FS_A1 + 16 * t + 4 * g, o); });
        } else {
            gemm(FM_W1T, DD, 15, [&](int c) { return *reinterpret_cast<const d4*>(Ta + c * 4); },
                 [&](const d4& T) {
                     acc d[4];
#pragma unroll
                     for (int v = 0; v < 4; ++v) d[v] = T[0] * Tn[v][0] + T[1] * Tn[v][1] + T[2] * Tn[v][2] + T[3] * Tn[v][3];
                     return P::make(d[0], d[1], d[2], d[3]);
                 },
                 [&](int t, const acc* o) { wr4(FS_A1 + 16 * t + 4 * g, o); });
        }
        // layer 2 input h1 = wh1 a1 and layer 3 input h2 = wh2 a2 + h1, formed as the activations
        // are, in the slots GB and GH (the backward pass's, free until then)
        activate(FS_A1, FV_B1, [&](int t, const acc* a) {
            acc h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) h[r] = vec(FV_WH1, t, r) * a[r];
            wr4(FS_GB + 16 * t + 4 * g, h);
        });
        gemm(FM_W2T, FW, 15, rdrow(FS_GB), asis, [&](int t, const acc* o) { wr4(FS_A2 + 16 * t + 4 * g, o); });
        activate(FS_A2, FV_B2, [&](int t, const acc* a) {
            const d4 h1 = rd4(FS_GB + 16 * t + 4 * g);
            acc h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) h[r] = vec(FV_WH2, t, r) * a[r] + h1[r];
            wr4(FS_GH + 16 * t + 4 * g, h);
        });
        gemm(FM_W3T, FW, 15, rdrow(FS_GH), asis, [&](int t, const acc* o) { wr4(FS_A3 + 16 * t + 4 * g, o); });
        activate(FS_A3, FV_B3, [](int, const acc*) {});
        // ---------------------------------------------------------- energy (Eq. 9) and ga3
        if (HALVES == 2) __syncthreads();   // both halves' a3 in place
        if (h == 0) {
            acc e = 0;
#pragma unroll 1
            for (int t = 0; t < 15; ++t) {
                const d4 x1 = rd4(FS_A1 + 16 * t + 4 * g), x2 = rd4(FS_A2 + 16 * t + 4 * g),
                         x3 = rd4(FS_A3 + 16 * t + 4 * g);
                acc ga[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const acc h3 = vec(FV_WH3, t, r) * x3[r] + vec(FV_WH2, t, r) * x2[r] + vec(FV_WH1, t, r) * x1[r];
                    e += h3 * vec(FV_W4, t, r);
                    ga[r] = fv[FV_WH4] * vec(FV_W4, t, r) * vec(FV_WH3, t, r) * (1 - x3[r] * x3[r]);
                }
                wr4(FS_GA + 16 * t + 4 * g, ga);
            }
            e += __shfl_xor(e, 16);
            e += __shfl_xor(e, 32);
            if (g == 0 && mine) A.Ei[atom] = fv[FV_WH4] * (e + fv[FV_B4]);
        }
        // ---------------------------------------------------------- backward through layers 3, 2
        // gh2 = W3^T ga3 + gh3 with gh3 = wh4 w4; ga2 = gh2 wh2 (1 - a2^2)
        gemm(FM_W3, FW, 15, rdrow(FS_GA), asis,
             [&](int t, const acc* o) {
                 const d4 x2 = rd4(FS_A2 + 16 * t + 4 * g);
                 acc gh[4], ga[4];
#pragma unroll
                 for (int r = 0; r < 4; ++r) {
                     gh[r] = o[r] + fv[FV_WH4] * vec(FV_W4, t, r);
                     ga[r] = gh[r] * vec(FV_WH2, t, r) * (1 - x2[r] * x2[r]);
                 }
                 wr4(FS_GH + 16 * t + 4 * g, gh);
                 wr4(FS_GB + 16 * t + 4 * g, ga);
             });
        // gh1 = W2^T ga2 + gh2; ga1 = gh1 wh1 (1 - a1^2)
        gemm(FM_W2, FW, 15, rdrow(FS_GB), asis,
             [&](int t, const acc* o) {
                 const d4 x1 = rd4(FS_A1 + 16 * t + 4 * g), gh2 = rd4(FS_GH + 16 * t + 4 * g);
                 acc ga[4];
#pragma unroll
                 for (int r = 0; r < 4; ++r) ga[r] = (o[r] + gh2[r]) * vec(FV_WH1, t, r) * (1 - x1[r] * x1[r]);
                 wr4(FS_GA + 16 * t + 4 * g, ga);
             });
        // ---------------------------------------------------------- dD = W1^T ga1 and dT (Eq. 7)
        if constexpr (RAD) {
            // rows 16t + orow(g, r) of the 7 tiles are dE/dD_m (m < 100 stored)
            gemm(FM_W1, FW, RAD_K / 16, rdrow(FS_GA), asis,
                 [&](int t, const acc* dd) {
#pragma unroll
                     for (int r = 0; r < 4; ++r) {
                         const int m = 16 * t + P::orow(g, r);
                         if (mine && m < E2) *reinterpret_cast<d4*>(dTout + ((size_t)atom * E2 + m) * 4) = d4{dd[r], 0, 0, 0};
                     }
                 });
            continue;
        }
        // Tile m of dD holds dD[m][n], n < 16: dT[m] += sum_n dD[m][n] T[n] (reduced over the lane
        // groups, tiles m < 16 parked in LDS) and dT[n] += sum_m dD[m][n] T[m] (kept per lane).
        acc q2[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k) q2[r][k] = 0;
        gemm(FM_W1, FW, E2, rdrow(FS_GA), asis,
             [&](int m, const acc* dd) {
                 const acc T0 = Ta[m * 4 + 0], T1 = Ta[m * 4 + 1], T2 = Ta[m * 4 + 2], T3 = Ta[m * 4 + 3];
                 acc part[4] = {0, 0, 0, 0};
#pragma unroll
                 for (int r = 0; r < 4; ++r) {
#pragma unroll
                     for (int k = 0; k < 4; ++k) part[k] += dd[r] * Tn[r][k];
                     q2[r][0] += dd[r] * T0;
                     q2[r][1] += dd[r] * T1;
                     q2[r][2] += dd[r] * T2;
                     q2[r][3] += dd[r] * T3;
                 }
#pragma unroll
                 for (int k = 0; k < 4; ++k) {
                     part[k] += __shfl_xor(part[k], 16);
                     part[k] += __shfl_xor(part[k], 32);
                 }
                 if (g == 0) {
                     if (m < 16) {
#pragma unroll
                         for (int k = 0; k < 4; ++k) s_p1[aw][c16][m][k] = part[k];
                     } else if (mine) {
                         *reinterpret_cast<d4*>(dTout + ((size_t)atom * E2 + m) * 4) = d4{part[0], part[1], part[2], part[3]};
                     }
                 }
             });
        __syncthreads();
        // two halves: the second one's share of dT[n], n < 16, goes through LDS (the weight stages
        // are free until the next product's first barrier)
        acc* xq = reinterpret_cast<acc*>(&s_w[0][0]) + ((size_t)aw * 64 + lane) * 16;
        if (HALVES == 2) {
            if (h == 1)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int k = 0; k < 4; ++k) xq[4 * r + k] = q2[r][k];
            __syncthreads();
        }
        if (h == 0 && mine) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = P::orow(g, r);
                d4 o;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    o[k] = s_p1[aw][c16][n][k] + q2[r][k] + (HALVES == 2 ? xq[4 * r + k] : (acc)0);
                *reinterpret_cast<d4*>(dTout + ((size_t)atom * E2 + n) * 4) = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
// Atoms per wave of one launch (see EmbCfg).
static int embed_apw(int nw, int apw_max, int64_t natoms, int ncu)
{
    const int64_t a = natoms / ((int64_t)nw * (ncu > 0 ? ncu : 1));
    return (int)std::max<int64_t>(1, std::min<int64_t>(apw_max, a));
}

// Atoms per wave of the backward launch: one for the three-body descriptor (a wave keeps its
// atom's slot gradients in LDS over all passes).
template <class P, bool TAB>
static int embed_bwd_apw(int64_t natoms, int ncu, bool e3)
{
    typedef EmbCfg<P, false, TAB> Cfg;
    return e3 ? 1 : embed_apw(Cfg::NW, Cfg::APW_MAX, natoms, ncu);
}

template <class P, bool TAB>
static int embed_bwd_blocks_p(int64_t natoms, int ncu, bool e3)
{
    typedef EmbCfg<P, false, TAB> Cfg;
    const int64_t apb = (int64_t)Cfg::NW * embed_bwd_apw<P, TAB>(natoms, ncu, e3);
    return (int)((natoms + apb - 1) / apb);
}

int embed_bwd_blocks(int precision, bool table, int64_t natoms, int ncu, bool e3)
{
    if (table && !e3) return tab_blocks(natoms, ncu);
    if (precision == 0) return table ? embed_bwd_blocks_p<PF64, true>(natoms, ncu, e3) : embed_bwd_blocks_p<PF64, false>(natoms, ncu, e3);
    if (precision == 1) return table ? embed_bwd_blocks_p<PMIX, true>(natoms, ncu, e3) : embed_bwd_blocks_p<PMIX, false>(natoms, ncu, e3);
    if (precision == 3) return table ? embed_bwd_blocks_p<PF32, true>(natoms, ncu, e3) : embed_bwd_blocks_p<PF32, false>(natoms, ncu, e3);
    return table ? embed_bwd_blocks_p<PBF16, true>(natoms, ncu, e3) : embed_bwd_blocks_p<PBF16, false>(natoms, ncu, e3);
}

// at least one atom per wave: the smallest block (in atoms) over both paths bounds the count
int64_t embed_bwd_max_blocks(int precision, int64_t natoms)
{
    const int nw = std::min(tab_atoms_per_block_min(),
                            precision == 0 ? std::min(EmbCfg<PF64, false, false>::NW, EmbCfg<PF64, false, true>::NW)
                                           : std::min(EmbCfg<PMIX, false, false>::NW, EmbCfg<PMIX, false, true>::NW));
    static_assert(EmbCfg<PBF16, false, false>::NW == EmbCfg<PMIX, false, false>::NW &&
                  EmbCfg<PBF16, false, true>::NW == EmbCfg<PMIX, false, true>::NW &&
                  EmbCfg<PF32, false, false>::NW == EmbCfg<PMIX, false, false>::NW &&
                  EmbCfg<PF32, false, true>::NW == EmbCfg<PMIX, false, true>::NW, "backward shapes");
    return (natoms + nw - 1) / nw;
}
int fit_atoms_per_block(int) { return FIT_AF; }

// The three-body backward kernels are instantiated explicitly: the host pass emitted no launch stub
// for the FP64 network variant from its implicit instantiation alone.
template __global__ void k_embed_bwd<PF64, false, false, true>(EmbArgs);
template __global__ void k_embed_bwd<PF64, true, false, true>(EmbArgs);
template __global__ void k_embed_bwd<PF64, false, true, true>(EmbArgs);
template __global__ void k_embed_bwd<PF64, true, true, true>(EmbArgs);

// e3: the three-body descriptor's pair passes (also for a model ensemble, blockIdx.y = model). The table runs here only for the three-body descriptor (the two-body
// descriptors' table has the product kernels of kernels_tab.hip).
template <class P, bool FWD, bool TAB>
static void launch_embed_shape(const EmbArgs& a0, bool e3, hipStream_t s)
{
    typedef EmbCfg<P, FWD, TAB> Cfg;
    EmbArgs a = a0;
    a.apw = FWD ? embed_apw(Cfg::NW, Cfg::APW_MAX, a.natoms, a.ncu) : embed_bwd_apw<P, TAB>(a.natoms, a.ncu, e3);
    const int apb = Cfg::NW * a.apw;
    const bool ens = a.nmodels > 1;
    const dim3 grid((a.natoms + apb - 1) / apb, ens ? a.nmodels : 1), block(Cfg::NW * 64);
    if constexpr (FWD) {
        if (e3 && ens) hipLaunchKernelGGL((k_embed_fwd<P, TAB, true, true>), grid, block, 0, s, a);
        else if (e3) hipLaunchKernelGGL((k_embed_fwd<P, TAB, false, true>), grid, block, 0, s, a);
        else if constexpr (!TAB) {
            if (ens) hipLaunchKernelGGL((k_embed_fwd<P, TAB, true, false>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_embed_fwd<P, TAB, false, false>), grid, block, 0, s, a);
        }
    } else {
        if (e3 && ens) hipLaunchKernelGGL((k_embed_bwd<P, TAB, true, true>), grid, block, 0, s, a);
        else if (e3) hipLaunchKernelGGL((k_embed_bwd<P, TAB, false, true>), grid, block, 0, s, a);
        else if constexpr (!TAB) {
            if (ens) hipLaunchKernelGGL((k_embed_bwd<P, TAB, true, false>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_embed_bwd<P, TAB, false, false>), grid, block, 0, s, a);
        }
    }
}

template <class P>
static void launch_embed(bool fwd, bool table, const EmbArgs& a, bool e3, hipStream_t s)
{
    if (fwd) {
        if (table) launch_embed_shape<P, true, true>(a, e3, s);
        else launch_embed_shape<P, true, false>(a, e3, s);
    } else {
        if (table) launch_embed_shape<P, false, true>(a, e3, s);
        else launch_embed_shape<P, false, false>(a, e3, s);
    }
}

// The two-body descriptors' table runs on the matrix-product kernels of kernels_tab.hip; the
// three-body table on the pair walk here.
void launch_embed_fwd(int precision, bool table, const EmbArgs& a, hipStream_t s, bool e3)
{
    if (table && !e3) return launch_tab(true, precision, a, s);
    if (precision == 0) launch_embed<PF64>(true, table, a, e3, s);
    else if (precision == 1) launch_embed<PMIX>(true, table, a, e3, s);
    else if (precision == 3) launch_embed<PF32>(true, table, a, e3, s);
    else launch_embed<PBF16>(true, table, a, e3, s);
}

void launch_embed_bwd(int precision, bool table, const EmbArgs& a, hipStream_t s, bool e3)
{
    if (table && !e3) return launch_tab(false, precision, a, s);
    if (precision == 0) launch_embed<PF64>(false, table, a, e3, s);
    else if (precision == 1) launch_embed<PMIX>(false, table, a, e3, s);
    else if (precision == 3) launch_embed<PF32>(false, table, a, e3, s);
    else launch_embed<PBF16>(false, table, a, e3, s);
}

void launch_e3_env(int precision, const EmbArgs& a, hipStream_t s)
{
    const int64_t n = (int64_t)a.natoms * a.nc;
    if (n == 0) return;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (precision == 0) hipLaunchKernelGGL((k_e3_env<double>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_e3_env<float>), grid, block, 0, s, a);
}

// The fitting net: FP64 and FP32 on the dense kernel, the BF16 paths on k_fitx; a descriptor of M
// values (a.radial) always on the dense kernel (FP64, else FP32), whose first layer is then small.
// Shape of the dense kernel: FP64 always in two halves (four 4-wave blocks run one wave per SIMD);
// FP32 in two halves when the 64-atom blocks do not outnumber the CUs, else in the 4-wave shape,
// whose blocks then share the CUs two at a time (measured: the 12,288-atom water box 0.424 -> 0.387
// ms with halves, the 32,000-atom fcc box 0.730 -> 0.857 ms).
template <class P, bool RAD, int HALVES>
static void launch_dense_shape(const FitArgs& a, hipStream_t s)
{
    const bool ens = a.nmodels > 1;
    const dim3 grid((a.natoms + FIT_AF - 1) / FIT_AF, ens ? a.nmodels : 1), block(256 * HALVES);
    if (ens) hipLaunchKernelGGL((k_fit_dense<P, true, RAD, HALVES>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_fit_dense<P, false, RAD, HALVES>), grid, block, 0, s, a);
}

template <class P, bool RAD>
static void launch_dense(const FitArgs& a, hipStream_t s)
{
    const int64_t blocks = (int64_t)((a.natoms + FIT_AF - 1) / FIT_AF) * (a.nmodels > 1 ? a.nmodels : 1);
    if (sizeof(typename P::acc) == 8 || blocks <= (a.ncu > 0 ? a.ncu : 256)) launch_dense_shape<P, RAD, 2>(a, s);
    else launch_dense_shape<P, RAD, 1>(a, s);
}

void launch_fit(int precision, const FitArgs& a, hipStream_t s)
{
    if (a.radial) {
        if (precision == 0) launch_dense<PF64, true>(a, s);
        else launch_dense<PF32, true>(a, s);
    } else if (precision == 0) {
        launch_dense<PF64, false>(a, s);
    } else if (precision == 3) {
        launch_dense<PF32, false>(a, s);
    } else {
        launch_fitx(precision == 1, a, s);
    }
}

}  // namespace dpk
