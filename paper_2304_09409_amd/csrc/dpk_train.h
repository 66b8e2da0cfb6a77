// dpk_train.h -- internal declarations of the training-mode backward (Sec. II.B): FP64 kernels over
// materialised per-pair and per-atom layer activations, and the frame-geometry hook they use.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpk_internal.h"

struct dpk_ctx;

namespace dpk {

// The neighbour list of a frame as the geometry launches left it (internal atom order).
struct FrameGeom {
    int n, nc, nt;
    int off[MAXT];
    const int* itype;      // [n]
    const int* nnei;       // [n][nt]
    const int* nl_j;       // [n][nc] caller index of each kept neighbour
    const double* nl_r;    // [n][nc][3]
    const int* perm;       // [n] caller index of each internal atom
    hipStream_t stream;
};
// Partition, bin and search one host frame on the context's device and stream (no network); the
// context keeps the buffers until its next frame.
int frame_geometry(dpk_ctx* c, int64_t natoms, const double* coord, const int32_t* atype, const double* box,
                   FrameGeom* g);

// Row GEMM C[M][N] = A[M][K] B with B[k][n] = W[k N + n] (transB = 0) or W[n K + k] (transB = 1),
// a second product C2 = A2 B on the same B when A2 is set, and one of three epilogues:
//   TR_PLAIN: C (and C2) stored;
//   TR_FWD:   a hidden layer of eq. NN: z = C + b, a = tanh z, y = w_hat a + skip(x) with x the
//             row of A (skip: x when N == K, (x, x) when N == 2K); tangent: zd = C2,
//             yd = w_hat (1 - a^2) zd + skip(A2 row); stores a, y and (dual) zd, yd;
//   TR_BWD:   input adjoint of such a layer, C = zbar W^T + skip^T(ybar) with ybar the rows of S
//             (width NS = the layer's output width: adds ybar[n] when NS == N, ybar[n] + ybar[n + N]
//             when NS == 2N), and the same for the tangent from A2 and S2.
enum { TR_PLAIN = 0, TR_FWD = 1, TR_BWD = 2 };
struct TrGemm {
    int M, N, K, transB, mode, NS;
    const double *A, *A2, *W, *bias, *wh, *S, *S2;
    double *C, *C2, *Y, *Zd, *Yd;   // FWD: C receives a
};
void tr_gemm(const TrGemm& g, hipStream_t s);

// Weight gradient Wbar[K][N] += sum_m A1[m][k] B1[m][n] + A2[m][k] scale2[m] B2[m][n] (A2 optional;
// scale2 optional, 1 if absent).
void tr_wgrad(int M, int N, int K, const double* A1, const double* B1, const double* A2, const double* B2,
              const double* scale2, double* Wbar, hipStream_t s);
// Column sums: o1[n] += sum_m X1[m][n]; o2[n] += sum_m X2[m][n] (X2 optional).
void tr_colsum(int M, int N, const double* X1, double* o1, const double* X2, double* o2, hipStream_t s);
// Adjoint of a tanh layer's pre-activation, element-wise over [M][N]:
//   zbar = w_hat (1 - a^2) ybar - 2 w_hat a (1 - a^2) zd ydbar,  zdbar = w_hat (1 - a^2) ydbar,
//   h = a ybar + (1 - a^2) zd ydbar (summed into w_hat's gradient),
// with zd = sigma_m Zd (sigma optional, 1 if absent; Zd, Ydb optional: no tangent).
void tr_adj_elem(int M, int N, const double* A, const double* Zd, const double* sigma, const double* Yb,
                 const double* Ydb, const double* wh, double* Zb, double* Zdb, double* H, hipStream_t s);
// The same, with the column sums of zbar added into bsum and of h into hsum (h not stored).
void tr_adj_sum(int M, int N, const double* A, const double* Zd, const double* sigma, const double* Yb,
                const double* Ydb, const double* wh, double* Zb, double* Zdb, double* bsum, double* hsum, hipStream_t s);

// Per-pair environment (pair p = (atom pa[p], slot ps[p])): R[p] = s (1, r/r), X0[p] = s, ones[p] = 1;
// with vdir (training): the pair tangent rdot = vdir[j] - vdir[i] + CV r_ij, sigma[p] = ds/dt,
// Rd[p] = dR/dt.
struct TrEnv {
    int P, nc;
    const int *pa, *ps, *nl_j, *perm;
    const double* nl_r;
    double rs, rc;
    const double* vdir;   // [caller atoms][3] or nullptr
    double CV[9];
    double *R, *X0, *ones, *sigma, *Rd;
};
void tr_env(const TrEnv& e, hipStream_t s);

// Per-atom contraction T = N_c^-1 sum_p G_p (x) R_p over the atom's pairs (nt segments from apo and
// nnei), its tangent Td = N_c^-1 sum_p (sigma_p Gd_p (x) R_p + G_p (x) Rd_p) when Td is set, and
// D = T T_<^T ([m 16 + n]) with Dd.
struct TrContract {
    int n, nt;
    double inv_nc;
    const int *apo, *nnei;
    const double *G, *Gd, *R, *Rd, *sigma;
    double *T, *Td, *D, *Dd;
};
void tr_contract(const TrContract& c, hipStream_t s);

// Adjoint of D = T T_<^T per atom: Tb from Db (and from Ddb through Td when training), Tdb from Ddb.
void tr_dT(int n, const double* T, const double* Td, const double* Db, const double* Ddb, double* Tb, double* Tdb,
           hipStream_t s);

// Fitting output layer over rows [0, M): o = y W4 + b4, E_i = w_hat4 o, od = yd W4; sums[0] += sum o,
// sums[1] += sum od; and the adjoints of its input: Yb[m][n] = cE w_hat4 W4[n], Ydb[m][n] = w_hat4 W4[n].
void tr_fit_out(int M, const double* Y, const double* Yd, const double* W4, const double* b4, const double* wh4,
                double cE, double* Ei, double* sums, double* Yb, double* Ydb, hipStream_t s);
// Output-layer gradients from the column sums of y3 (S1) and yd3 (S2): W4bar += w_hat4 (cE S1 + S2),
// b4bar += cE w_hat4 M, wh4bar += cE sums[0] + sums[1].
void tr_out_grad(int M, const double* S1, const double* S2, const double* sums, const double* wh4, double cE,
                 double* W4b, double* b4b, double* wh4b, hipStream_t s);

// Inference adjoint per pair: forces (caller order, atomics) and the virial (9 atomics per block).
struct TrPairForce {
    int P, nc;
    double inv_nc, rs, rc;
    const int *pa, *ps, *nl_j, *perm;
    const double *nl_r, *R, *G, *Gd, *dT;
    double *F, *vir;
};
void tr_pair_force(const TrPairForce& f, hipStream_t s);

// Training adjoint per pair: Yb[p][m] = N_c^-1 (Tb[a] R_p + Tdb[a] Rd_p)_m, Ydb[p][m] = N_c^-1 (Tdb[a] R_p)_m.
void tr_pair_adj(int P, double inv_nc, const int* pa, const double* Tb, const double* Tdb, const double* R,
                 const double* Rd, double* Yb, double* Ydb, hipStream_t s);

// Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); then g = 0.
void tr_adam(int64_t n, double* theta, double* g, double* m, double* v, double lr, double b1, double b2, double eps,
             double c1, double c2, hipStream_t s);
void tr_zero(double* p, int64_t n, hipStream_t s);

}  // namespace dpk
