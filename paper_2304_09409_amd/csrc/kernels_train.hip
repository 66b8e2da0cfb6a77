// kernels_train.hip -- training-mode backward of the se_e2_a model (Sec. II.B), FP64.
//
// The gradient of the loss of eq. loss with respect to every parameter, force and virial terms
// included. With g_ij = dE/dr_ij, the force and virial terms are linear in the g_ij, so
//   dL/dtheta = d/dtheta [ cE E + sum_ij g_ij . rdot_ij ],
//   cE = 2 p_E (E - E*) / N,  rdot_ij = vdir_j - vdir_i + CV r_ij,
//   vdir_k = -2 p_F q_k (F_k - F*_k) / (3N),  CV = -2 p_Xi (Xi - Xi*) / (9N),
// and sum_ij g_ij . rdot_ij is the derivative of E along the pair displacements rdot_ij: a
// forward-mode tangent through the model (s, R, G = N(s), T, D, F_0), then reverse mode through
// the model and its tangent. Every layer y = w_hat tanh(x W + b) + skip(x) carries (y, ydot); its
// adjoint pair (ybar, ydotbar) gives
//   zbar = w_hat (1 - a^2) ybar - 2 w_hat a (1 - a^2) zdot ydotbar,  zdotbar = w_hat (1 - a^2) ydotbar,
//   Wbar += x zbar^T + xdot zdotbar^T,  bbar += zbar,  w_hatbar += a ybar + (1 - a^2) zdot ydotbar,
//   xbar = W zbar + skip^T ybar,  xdotbar = W zdotbar + skip^T ydotbar.
// The embedding net has a scalar input s, so its tangent along any direction is sdot times its
// unit tangent d/ds: the forward pass (which the forces need anyway) stores the unit tangents and
// the reverse pass scales them per pair.
//
// Layout: the activations of every layer are materialised per row (rows = neighbour pairs grouped
// by embedding net, or atoms grouped by type), and every layer is a row GEMM (tr_gemm) with a fused
// epilogue; the weight gradients are GEMMs over the rows (tr_wgrad, split over rows with FP64
// atomics). 64 x 64 output tiles, 16-deep K chunks staged in LDS, four waves of 2 x 2 tiles of the
// 16 x 16 x 4 FP64 matrix instruction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dpk_train.h"

namespace dpk {

constexpr int TB = 64, TK = 16;

// ---------------------------------------------------------------------------------------------
// Row GEMM with layer epilogues, on v_mfma_f64_16x16x4f64. A block computes a 64 x 64 tile of C
// with four waves of 32 x 32 (2 x 2 MFMA tiles); K runs in chunks of 16 staged in LDS. For one
// instruction, lane l (group g = l / 16, column c = l % 16) supplies A[c][g] and B[g][c] of the
// 16 x 16 x 4 step and receives D[g + 4r][c] in register r.
// ---------------------------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));
constexpr int TAP = TK + 1;   // LDS row pitch of the A tiles (doubles): rows c = 0..15 fall in distinct banks

__device__ __forceinline__ void tr_epilogue(const TrGemm& g, int m, int n, double c, double c2, bool dual)
{
    const int64_t o = (int64_t)m * g.N + n;
    if (g.mode == TR_FWD) {
        // skip source: the input row at n (N == K) or n mod K (N == 2K)
        const int ks = g.N == g.K ? n : (g.N == 2 * g.K ? (n < g.K ? n : n - g.K) : -1);
        const double a = tanh(c + g.bias[n]);
        g.C[o] = a;
        g.Y[o] = g.wh[n] * a + (ks >= 0 ? g.A[(int64_t)m * g.K + ks] : 0.0);
        if (dual) {
            g.Zd[o] = c2;
            g.Yd[o] = g.wh[n] * (1.0 - a * a) * c2 + (ks >= 0 ? g.A2[(int64_t)m * g.K + ks] : 0.0);
        }
    } else if (g.mode == TR_BWD) {
        double sk = 0.0, sk2 = 0.0;
        if (g.NS == g.N) {
            sk = g.S[(int64_t)m * g.NS + n];
            if (dual) sk2 = g.S2[(int64_t)m * g.NS + n];
        } else if (g.NS == 2 * g.N) {
            sk = g.S[(int64_t)m * g.NS + n] + g.S[(int64_t)m * g.NS + n + g.N];
            if (dual) sk2 = g.S2[(int64_t)m * g.NS + n] + g.S2[(int64_t)m * g.NS + n + g.N];
        }
        g.C[o] = c + sk;
        if (dual) g.C2[o] = c2 + sk2;
    } else {
        g.C[o] = c;
        if (dual) g.C2[o] = c2;
    }
}

template <bool DUAL>
__global__ void __launch_bounds__(256) k_tr_gemm(TrGemm g)
{
    __shared__ double sA[TB][TAP];
    __shared__ double sA2[DUAL ? TB : 1][TAP];
    __shared__ double sB[TK][TB + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lg = lane >> 4, lc = lane & 15;
    const int wr = wave >> 1, wc = wave & 1;
    const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
    d4v acc[2][2], acc2[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = acc2[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < g.K; k0 += TK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            // A tile: 64 rows x 16 k, read along k
            const int r = idx >> 4, kk = idx & 15;
            const int m = m0 + r, k = k0 + kk;
            const bool in = m < g.M && k < g.K;
            sA[r][kk] = in ? g.A[(int64_t)m * g.K + k] : 0.0;
            if (DUAL) sA2[r][kk] = in ? g.A2[(int64_t)m * g.K + k] : 0.0;
            // B tile: 16 k x 64 n
            if (g.transB) {
                const int c = idx >> 4, kb = idx & 15;
                const int n = n0 + c, k2 = k0 + kb;
                sB[kb][c] = (n < g.N && k2 < g.K) ? g.W[(int64_t)n * g.K + k2] : 0.0;
            } else {
                const int kb = idx >> 6, c = idx & 63;
                const int n = n0 + c, k2 = k0 + kb;
                sB[kb][c] = (n < g.N && k2 < g.K) ? g.W[(int64_t)k2 * g.N + n] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            double a[2], a2[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = sA[wr * 32 + i * 16 + lc][ks + lg];
                if (DUAL) a2[i] = sA2[wr * 32 + i * 16 + lc][ks + lg];
                b[i] = sB[ks + lg][wc * 32 + i * 16 + lc];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                    if (DUAL) acc2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i], b[j], acc2[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr * 32 + i * 16 + lg + 4 * r, n = n0 + wc * 32 + j * 16 + lc;
                if (m < g.M && n < g.N) tr_epilogue(g, m, n, acc[i][j][r], DUAL ? acc2[i][j][r] : 0.0, DUAL);
            }
}

void tr_gemm(const TrGemm& g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return;
    const dim3 grid((g.N + TB - 1) / TB, (g.M + TB - 1) / TB), block(256);
    if (g.A2) hipLaunchKernelGGL((k_tr_gemm<true>), grid, block, 0, s, g);
    else hipLaunchKernelGGL((k_tr_gemm<false>), grid, block, 0, s, g);
}

// ---------------------------------------------------------------------------------------------
// Weight gradient: Wbar[K][N] += A1^T B1 + A2^T (scale2 B2) over the rows, on the FP64 MFMA with
// the rows as the reduction index; blockIdx.z takes a row range (FP64 atomics into Wbar).
// ---------------------------------------------------------------------------------------------
template <bool DUAL>
__global__ void __launch_bounds__(256) k_tr_wgrad(int M, int N, int K, int rows_per, const double* A1,
                                                  const double* B1, const double* A2, const double* B2,
                                                  const double* scale2, double* Wbar)
{
    __shared__ double sA[TK][TB + 1], sB[TK][TB + 1];
    __shared__ double sA2[DUAL ? TK : 1][TB + 1], sB2[DUAL ? TK : 1][TB + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lg = lane >> 4, lc = lane & 15;
    const int wr = wave >> 1, wc = wave & 1;
    const int k0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
    const int r0 = blockIdx.z * rows_per, r1 = min(M, r0 + rows_per);
    d4v acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int m0 = r0; m0 < r1; m0 += TK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            const int mm = idx >> 6, c = idx & 63;
            const int m = m0 + mm;
            const bool row = m < r1;
            const int k = k0 + c, n = n0 + c;
            sA[mm][c] = (row && k < K) ? A1[(int64_t)m * K + k] : 0.0;
            sB[mm][c] = (row && n < N) ? B1[(int64_t)m * N + n] : 0.0;
            if (DUAL) {
                sA2[mm][c] = (row && k < K) ? A2[(int64_t)m * K + k] : 0.0;
                sB2[mm][c] = (row && n < N) ? B2[(int64_t)m * N + n] * (scale2 ? scale2[m] : 1.0) : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            double a[2], b[2], a2[2], b2[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = sA[ks + lg][wr * 32 + i * 16 + lc];
                b[i] = sB[ks + lg][wc * 32 + i * 16 + lc];
                if (DUAL) {
                    a2[i] = sA2[ks + lg][wr * 32 + i * 16 + lc];
                    b2[i] = sB2[ks + lg][wc * 32 + i * 16 + lc];
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                    if (DUAL) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i], b2[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = k0 + wr * 32 + i * 16 + lg + 4 * r, n = n0 + wc * 32 + j * 16 + lc;
                if (k < K && n < N) atomicAdd(&Wbar[(int64_t)k * N + n], acc[i][j][r]);
            }
}

void tr_wgrad(int M, int N, int K, const double* A1, const double* B1, const double* A2, const double* B2,
              const double* scale2, double* Wbar, hipStream_t s)
{
    if (M <= 0) return;
    const int tiles = ((N + TB - 1) / TB) * ((K + TB - 1) / TB);
    // about 2,048 blocks, at least 256 rows each
    int splits = std::max(1, std::min((M + 255) / 256, 2048 / tiles));
    const int rows_per = ((M + splits - 1) / splits + TK - 1) / TK * TK;
    splits = (M + rows_per - 1) / rows_per;
    const dim3 grid((N + TB - 1) / TB, (K + TB - 1) / TB, splits), block(256);
    if (A2) hipLaunchKernelGGL((k_tr_wgrad<true>), grid, block, 0, s, M, N, K, rows_per, A1, B1, A2, B2, scale2, Wbar);
    else hipLaunchKernelGGL((k_tr_wgrad<false>), grid, block, 0, s, M, N, K, rows_per, A1, B1, A2, B2, scale2, Wbar);
}

// ---------------------------------------------------------------------------------------------
// Column sums (bias and w_hat gradients)
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_colsum(int M, int N, int rows_per, const double* X1, double* o1,
                                                   const double* X2, double* o2)
{
    __shared__ double s1[4][64], s2[4][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int m0 = blockIdx.y * rows_per, m1 = min(M, m0 + rows_per);
    double a = 0.0, b = 0.0;
    if (n < N)
        for (int m = m0 + r; m < m1; m += 4) {
            a += X1[(int64_t)m * N + n];
            if (X2) b += X2[(int64_t)m * N + n];
        }
    s1[r][c] = a;
    s2[r][c] = b;
    __syncthreads();
    if (r == 0 && n < N) {
        atomicAdd(&o1[n], s1[0][c] + s1[1][c] + s1[2][c] + s1[3][c]);
        if (X2) atomicAdd(&o2[n], s2[0][c] + s2[1][c] + s2[2][c] + s2[3][c]);
    }
}

void tr_colsum(int M, int N, const double* X1, double* o1, const double* X2, double* o2, hipStream_t s)
{
    if (M <= 0) return;
    const int rows_per = 1024;
    const dim3 grid((N + 63) / 64, (M + rows_per - 1) / rows_per), block(256);
    hipLaunchKernelGGL(k_tr_colsum, grid, block, 0, s, M, N, rows_per, X1, o1, X2, o2);
}

// ---------------------------------------------------------------------------------------------
// Element-wise adjoint of a tanh layer
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_adj_elem(int64_t total, int N, const double* A, const double* Zd,
                                                     const double* sigma, const double* Yb, const double* Ydb,
                                                     const double* wh, double* Zb, double* Zdb, double* H)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t m = e / N;
        const int n = (int)(e - m * N);
        const double a = A[e], gd = 1.0 - a * a, w = wh[n], yb = Yb[e];
        const double sg = sigma ? sigma[m] : 1.0;
        const double zd = Zd ? sg * Zd[e] : 0.0, ydb = Ydb ? Ydb[e] : 0.0;
        Zb[e] = w * gd * yb - 2.0 * w * a * gd * zd * ydb;
        H[e] = a * yb + gd * zd * ydb;
        if (Zdb) Zdb[e] = w * gd * ydb;
    }
}

// The same with the column sums of zbar and h added into bsum and hsum (the bias and w_hat
// gradients): 64 columns x a range of rows per block, the four row groups reduced in LDS.
__global__ void __launch_bounds__(256) k_tr_adj_sum(int M, int N, int rows_per, const double* A, const double* Zd,
                                                    const double* sigma, const double* Yb, const double* Ydb,
                                                    const double* wh, double* Zb, double* Zdb, double* bsum,
                                                    double* hsum)
{
    __shared__ double s1[4][64], s2[4][64];
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int m0 = blockIdx.y * rows_per, m1 = min(M, m0 + rows_per);
    double sb = 0.0, sh = 0.0;
    if (n < N) {
        const double w = wh[n];
        for (int m = m0 + rg; m < m1; m += 4) {
            const int64_t e = (int64_t)m * N + n;
            const double a = A[e], gd = 1.0 - a * a, yb = Yb[e];
            const double sg = sigma ? sigma[m] : 1.0;
            const double zd = Zd ? sg * Zd[e] : 0.0, ydb = Ydb ? Ydb[e] : 0.0;
            const double zb = w * gd * yb - 2.0 * w * a * gd * zd * ydb;
            Zb[e] = zb;
            if (Zdb) Zdb[e] = w * gd * ydb;
            sb += zb;
            sh += a * yb + gd * zd * ydb;
        }
    }
    s1[rg][c] = sb;
    s2[rg][c] = sh;
    __syncthreads();
    if (rg == 0 && n < N) {
        atomicAdd(&bsum[n], s1[0][c] + s1[1][c] + s1[2][c] + s1[3][c]);
        atomicAdd(&hsum[n], s2[0][c] + s2[1][c] + s2[2][c] + s2[3][c]);
    }
}

void tr_adj_sum(int M, int N, const double* A, const double* Zd, const double* sigma, const double* Yb,
                const double* Ydb, const double* wh, double* Zb, double* Zdb, double* bsum, double* hsum, hipStream_t s)
{
    if (M <= 0) return;
    const int rows_per = 256;
    const dim3 grid((N + 63) / 64, (M + rows_per - 1) / rows_per), block(256);
    hipLaunchKernelGGL(k_tr_adj_sum, grid, block, 0, s, M, N, rows_per, A, Zd, sigma, Yb, Ydb, wh, Zb, Zdb, bsum, hsum);
}

void tr_adj_elem(int M, int N, const double* A, const double* Zd, const double* sigma, const double* Yb,
                 const double* Ydb, const double* wh, double* Zb, double* Zdb, double* H, hipStream_t s)
{
    const int64_t total = (int64_t)M * N;
    if (total <= 0) return;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_tr_adj_elem, dim3(blocks), dim3(256), 0, s, total, N, A, Zd, sigma, Yb, Ydb, wh, Zb, Zdb, H);
}

// ---------------------------------------------------------------------------------------------
// Pair environment and its tangent
// ---------------------------------------------------------------------------------------------
// Switching function of eq. switch and ds/dr (the quintic in factored form, as the inference path).
__device__ __forceinline__ void tr_switch(double r, double rs, double rc, double& s, double& ds)
{
    if (r < rs) {
        s = 1.0 / r;
        ds = -s * s;
    } else if (r < rc) {
        const double w = rc - rs, x = (r - rs) / w, y = 1.0 - x;
        const double u = y * y * y * (1.0 + x * (3.0 + 6.0 * x)), du = -30.0 * x * x * y * y;
        s = u / r;
        ds = du / (w * r) - u / (r * r);
    } else {
        s = 0.0;
        ds = 0.0;
    }
}

__global__ void __launch_bounds__(256) k_tr_env(TrEnv E)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= E.P) return;
    const int64_t slot = (int64_t)E.pa[p] * E.nc + E.ps[p];
    const double x = E.nl_r[3 * slot], y = E.nl_r[3 * slot + 1], z = E.nl_r[3 * slot + 2];
    const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
    double s, ds;
    tr_switch(r, E.rs, E.rc, s, ds);
    const double sr = s * ir, ux = x * ir, uy = y * ir, uz = z * ir;
    double* R = E.R + 4 * (int64_t)p;
    R[0] = s;
    R[1] = sr * x;
    R[2] = sr * y;
    R[3] = sr * z;
    E.X0[p] = s;
    E.ones[p] = 1.0;
    if (E.vdir) {
        const int j = E.nl_j[slot], i = E.perm[E.pa[p]];
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = E.vdir[3 * (int64_t)j + k] - E.vdir[3 * (int64_t)i + k] + E.CV[3 * k] * x + E.CV[3 * k + 1] * y +
                   E.CV[3 * k + 2] * z;
        const double q = ux * d[0] + uy * d[1] + uz * d[2];   // rate of change of r
        const double sd = ds * q, c = (ds - sr) * q;
        E.sigma[p] = sd;
        double* Rd = E.Rd + 4 * (int64_t)p;
        Rd[0] = sd;
        Rd[1] = c * ux + sr * d[0];
        Rd[2] = c * uy + sr * d[1];
        Rd[3] = c * uz + sr * d[2];
    }
}

void tr_env(const TrEnv& e, hipStream_t s)
{
    if (e.P <= 0) return;
    hipLaunchKernelGGL(k_tr_env, dim3((e.P + 255) / 256), dim3(256), 0, s, e);
}

// ---------------------------------------------------------------------------------------------
// Contraction T = N_c^-1 sum G (x) R, its tangent, and D = T T_<^T (one block per atom)
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_contract(TrContract C)
{
    // two atoms per block, 128 threads each: thread m < 100 accumulates T[m][0..3] (and Td) over the
    // atom's pairs, reading row p of G at column m (consecutive threads, consecutive columns)
    __shared__ double sT[2][E2][4], sTd[2][E2][4];
    const int half = threadIdx.x >> 7, m = threadIdx.x & 127;
    const int a = blockIdx.x * 2 + half;
    const bool tan = C.Td != nullptr;
    if (a < C.n && m < E2) {
        double t[4] = {0, 0, 0, 0}, td[4] = {0, 0, 0, 0};
        for (int tj = 0; tj < C.nt; ++tj) {
            const int p0 = C.apo[(int64_t)a * C.nt + tj], cnt = C.nnei[(int64_t)a * C.nt + tj];
            for (int p = p0; p < p0 + cnt; ++p) {
                const double g = C.G[(int64_t)p * E2 + m];
                const double* r = C.R + 4 * (int64_t)p;
                const double r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
                t[0] += g * r0; t[1] += g * r1; t[2] += g * r2; t[3] += g * r3;
                if (tan) {
                    const double gd = C.sigma[p] * C.Gd[(int64_t)p * E2 + m];
                    const double* rd = C.Rd + 4 * (int64_t)p;
                    td[0] += gd * r0 + g * rd[0];
                    td[1] += gd * r1 + g * rd[1];
                    td[2] += gd * r2 + g * rd[2];
                    td[3] += gd * r3 + g * rd[3];
                }
            }
        }
        for (int k = 0; k < 4; ++k) {
            t[k] *= C.inv_nc;
            sT[half][m][k] = t[k];
            C.T[((int64_t)a * E2 + m) * 4 + k] = t[k];
            if (tan) {
                td[k] *= C.inv_nc;
                sTd[half][m][k] = td[k];
                C.Td[((int64_t)a * E2 + m) * 4 + k] = td[k];
            }
        }
    }
    __syncthreads();
    if (a >= C.n) return;
    for (int e = m; e < DD; e += 128) {
        const int mm = e / AX, nn = e - mm * AX;
        double d = 0.0, dd = 0.0;
        for (int k = 0; k < 4; ++k) {
            d += sT[half][mm][k] * sT[half][nn][k];
            if (tan) dd += sTd[half][mm][k] * sT[half][nn][k] + sT[half][mm][k] * sTd[half][nn][k];
        }
        C.D[(int64_t)a * DD + e] = d;
        if (tan) C.Dd[(int64_t)a * DD + e] = dd;
    }
}

void tr_contract(const TrContract& c, hipStream_t s)
{
    if (c.n <= 0) return;
    hipLaunchKernelGGL(k_tr_contract, dim3((c.n + 1) / 2), dim3(256), 0, s, c);
}

// ---------------------------------------------------------------------------------------------
// Adjoint of D = T T_<^T
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_dT(const double* T, const double* Td, const double* Db, const double* Ddb,
                                               double* Tb, double* Tdb)
{
    __shared__ double sT[E2][4], sTd[E2][4], sDb[DD], sDdb[DD];
    const int a = blockIdx.x;
    const bool tan = Ddb != nullptr;
    for (int e = threadIdx.x; e < E2 * 4; e += 256) {
        sT[e >> 2][e & 3] = T[(int64_t)a * E2 * 4 + e];
        if (tan) sTd[e >> 2][e & 3] = Td[(int64_t)a * E2 * 4 + e];
    }
    for (int e = threadIdx.x; e < DD; e += 256) {
        sDb[e] = Db[(int64_t)a * DD + e];
        if (tan) sDdb[e] = Ddb[(int64_t)a * DD + e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < E2 * 4; e += 256) {
        const int p = e >> 2, k = e & 3;
        double tb = 0.0, tdb = 0.0;
        for (int n = 0; n < AX; ++n) {
            tb += sDb[p * AX + n] * sT[n][k];
            if (tan) {
                tb += sDdb[p * AX + n] * sTd[n][k];
                tdb += sDdb[p * AX + n] * sT[n][k];
            }
        }
        if (p < AX)
            for (int m = 0; m < E2; ++m) {
                tb += sDb[m * AX + p] * sT[m][k];
                if (tan) {
                    tb += sDdb[m * AX + p] * sTd[m][k];
                    tdb += sDdb[m * AX + p] * sT[m][k];
                }
            }
        Tb[(int64_t)a * E2 * 4 + e] = tb;
        if (tan) Tdb[(int64_t)a * E2 * 4 + e] = tdb;
    }
}

void tr_dT(int n, const double* T, const double* Td, const double* Db, const double* Ddb, double* Tb, double* Tdb,
           hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tr_dT, dim3(n), dim3(256), 0, s, T, Td, Db, Ddb, Tb, Tdb);
}

// ---------------------------------------------------------------------------------------------
// Fitting output layer (one wave per row)
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_fit_out(int M, const double* Y, const double* Yd, const double* W4,
                                                    const double* b4, const double* wh4, double cE, double* Ei,
                                                    double* sums, double* Yb, double* Ydb)
{
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (m >= M) return;
    double o = 0.0, od = 0.0;
    for (int n = lane; n < FW; n += 64) {
        const double w = W4[n];
        o += Y[(int64_t)m * FW + n] * w;
        if (Yd) od += Yd[(int64_t)m * FW + n] * w;
        Yb[(int64_t)m * FW + n] = cE * wh4[0] * w;
        if (Ydb) Ydb[(int64_t)m * FW + n] = wh4[0] * w;
    }
    for (int s = 32; s > 0; s >>= 1) {
        o += __shfl_xor(o, s);
        od += __shfl_xor(od, s);
    }
    if (lane == 0) {
        o += b4[0];
        Ei[m] = wh4[0] * o;
        atomicAdd(&sums[0], o);
        atomicAdd(&sums[1], od);
    }
}

void tr_fit_out(int M, const double* Y, const double* Yd, const double* W4, const double* b4, const double* wh4,
                double cE, double* Ei, double* sums, double* Yb, double* Ydb, hipStream_t s)
{
    if (M <= 0) return;
    hipLaunchKernelGGL(k_tr_fit_out, dim3((M + 3) / 4), dim3(256), 0, s, M, Y, Yd, W4, b4, wh4, cE, Ei, sums, Yb, Ydb);
}

__global__ void k_tr_out_grad(int M, const double* S1, const double* S2, const double* sums, const double* wh4,
                              double cE, double* W4b, double* b4b, double* wh4b)
{
    for (int n = threadIdx.x; n < FW; n += blockDim.x) W4b[n] += wh4[0] * (cE * S1[n] + (S2 ? S2[n] : 0.0));
    if (threadIdx.x == 0) {
        b4b[0] += cE * wh4[0] * M;
        wh4b[0] += cE * sums[0] + sums[1];
    }
}

void tr_out_grad(int M, const double* S1, const double* S2, const double* sums, const double* wh4, double cE,
                 double* W4b, double* b4b, double* wh4b, hipStream_t s)
{
    hipLaunchKernelGGL(k_tr_out_grad, dim3(1), dim3(256), 0, s, M, S1, S2, sums, wh4, cE, W4b, b4b, wh4b);
}

// ---------------------------------------------------------------------------------------------
// Pair adjoints
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_pair_force(TrPairForce f)
{
    __shared__ double sv[9][256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (p < f.P) {
        const int a = f.pa[p];
        const int64_t slot = (int64_t)a * f.nc + f.ps[p];
        const double x = f.nl_r[3 * slot], y = f.nl_r[3 * slot + 1], z = f.nl_r[3 * slot + 2];
        const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
        double s, ds;
        tr_switch(r, f.rs, f.rc, s, ds);
        const double* R = f.R + 4 * (int64_t)p;
        const double* G = f.G + (int64_t)p * E2;
        const double* Gd = f.Gd + (int64_t)p * E2;
        const double* dT = f.dT + (int64_t)a * E2 * 4;
        double dR[4] = {0, 0, 0, 0}, h = 0.0;
        for (int m = 0; m < E2; ++m) {
            const double g = G[m], gd = Gd[m];
            const double t0 = dT[4 * m], t1 = dT[4 * m + 1], t2 = dT[4 * m + 2], t3 = dT[4 * m + 3];
            dR[0] += g * t0;
            dR[1] += g * t1;
            dR[2] += g * t2;
            dR[3] += g * t3;
            h += gd * (t0 * R[0] + t1 * R[1] + t2 * R[2] + t3 * R[3]);
        }
        for (int k = 0; k < 4; ++k) dR[k] *= f.inv_nc;
        h *= f.inv_nc;
        const double ux = x * ir, uy = y * ir, uz = z * ir, sr = s * ir;
        const double q = dR[1] * ux + dR[2] * uy + dR[3] * uz;
        const double rad = (dR[0] + h) * ds + q * (ds - sr);
        const double gx = rad * ux + sr * dR[1], gy = rad * uy + sr * dR[2], gz = rad * uz + sr * dR[3];
        const int j = f.nl_j[slot], i = f.perm[a];
        atomicAdd(&f.F[3 * (int64_t)i], gx);
        atomicAdd(&f.F[3 * (int64_t)i + 1], gy);
        atomicAdd(&f.F[3 * (int64_t)i + 2], gz);
        atomicAdd(&f.F[3 * (int64_t)j], -gx);
        atomicAdd(&f.F[3 * (int64_t)j + 1], -gy);
        atomicAdd(&f.F[3 * (int64_t)j + 2], -gz);
        v[0] = -gx * x; v[1] = -gx * y; v[2] = -gx * z;
        v[3] = -gy * x; v[4] = -gy * y; v[5] = -gy * z;
        v[6] = -gz * x; v[7] = -gz * y; v[8] = -gz * z;
    }
    for (int k = 0; k < 9; ++k) sv[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 9; ++k) sv[k][threadIdx.x] += sv[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 9) atomicAdd(&f.vir[threadIdx.x], sv[threadIdx.x][0]);
}

void tr_pair_force(const TrPairForce& f, hipStream_t s)
{
    if (f.P <= 0) return;
    hipLaunchKernelGGL(k_tr_pair_force, dim3((f.P + 255) / 256), dim3(256), 0, s, f);
}

__global__ void __launch_bounds__(256) k_tr_pair_adj(int64_t total, double inv_nc, const int* pa, const double* Tb,
                                                     const double* Tdb, const double* R, const double* Rd, double* Yb,
                                                     double* Ydb)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t p = e / E2;
        const int m = (int)(e - p * E2);
        const int a = pa[p];
        const double* tb = Tb + ((int64_t)a * E2 + m) * 4;
        const double* tdb = Tdb + ((int64_t)a * E2 + m) * 4;
        const double* r = R + 4 * p;
        const double* rd = Rd + 4 * p;
        double yb = 0.0, ydb = 0.0;
        for (int k = 0; k < 4; ++k) {
            yb += tb[k] * r[k] + tdb[k] * rd[k];
            ydb += tdb[k] * r[k];
        }
        Yb[e] = inv_nc * yb;
        Ydb[e] = inv_nc * ydb;
    }
}

void tr_pair_adj(int P, double inv_nc, const int* pa, const double* Tb, const double* Tdb, const double* R,
                 const double* Rd, double* Yb, double* Ydb, hipStream_t s)
{
    const int64_t total = (int64_t)P * E2;
    if (total <= 0) return;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_tr_pair_adj, dim3(blocks), dim3(256), 0, s, total, inv_nc, pa, Tb, Tdb, R, Rd, Yb, Ydb);
}

// ---------------------------------------------------------------------------------------------
// Adam and zero fill
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tr_adam(int64_t n, double* th, double* g, double* m, double* v, double lr,
                                                 double b1, double b2, double eps, double c1, double c2)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double gi = g[i];
        const double mi = b1 * m[i] + (1.0 - b1) * gi, vi = b2 * v[i] + (1.0 - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
        g[i] = 0.0;
    }
}

void tr_adam(int64_t n, double* theta, double* g, double* m, double* v, double lr, double b1, double b2, double eps,
             double c1, double c2, hipStream_t s)
{
    if (n <= 0) return;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_tr_adam, dim3(blocks), dim3(256), 0, s, n, theta, g, m, v, lr, b1, b2, eps, c1, c2);
}

__global__ void __launch_bounds__(256) k_tr_zero(double* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0;
}

void tr_zero(double* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_tr_zero, dim3(blocks), dim3(256), 0, s, p, n);
}

}  // namespace dpk
