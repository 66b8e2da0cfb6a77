// kernels_tab.hip -- the compressed embedding of the two-body descriptors (se_e2_a, se_e2_r): the
// quintic table (Sec. II.A.6, eq. compress) contracted with the environment matrix as matrix
// products, forward (T of Sec. II.A.1) and backward (forces and virial of Sec. II.A.2).
//
// On interval l of the table every feature is a quintic in the local variable t = s - l dx,
//   G_m(s) = sum_j C[l][j][m] t^(5 - j),
// linear in the coefficients. For one centre atom with environment rows R_q (eq. G2) the
// contraction T = N_c^-1 G^T R is therefore
//   T[m][k] = N_c^-1 sum_{l,j} C[l][j][m] P[l][j][k],   P[l][j][k] = sum_{q on l} t_q^(5-j) R_qk,
// and the backward pass needs, with dT = dE/dT from the fitting net,
//   sum_m G_qm dT[m][k] = sum_j W[l][j][k] t_q^(5-j),   W[l][j][k] = sum_m C[l][j][m] dT[m][k],
//   sum_m (dG_qm/ds) dT[m][k] = the derivative in t of the same quintic.
// The moments P and the adjoint coefficients W are 6 x 4 numbers per interval and atom. Their
// products with the table run on v_mfma_f32_16x16x4f32 (FP32 table) or v_mfma_f64_16x16x4f64
// (FP64), four centre atoms at a time (16 columns: atom x component), so each table row is read
// once per four atoms and streams through the vector caches. A neighbour costs its geometry and
// 24 moment terms (forward; summed per interval by a segmented scan over the wave) or two quintics
// in four components (backward): nothing per feature.
//
// Within a type block the neighbours are sorted by distance, so their intervals fall along the
// list. A group's intervals are processed in windows of WIN intervals whose P or W sits in LDS; a
// window takes each atom's neighbours from a cursor on for as long as their interval is inside it.
// At the rounding level the interval of s is not strictly monotone in r: a neighbour found above
// the window is evaluated on the window's top interval (and in the last window one below it on the
// lowest), i.e. on the adjacent piece extrapolated by a rounding error; the pieces agree in value,
// slope and curvature at the nodes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dpk_device.h"
#include "dpk_internal.h"
#include "dpk_launch.h"

namespace dpk {

template <class T> struct TabPol;
// FP32 table: output register r of lane group g holds row 4g + r of the 16 x 16 tile.
template <> struct TabPol<float> {
    typedef f4 accv;
    static constexpr int WIN = 32;
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static void mma(f4& d, float a, float b) { d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0); }
};
// FP64 table: output register r of lane group g holds row g + 4r.
template <> struct TabPol<double> {
    typedef d4 accv;
    static constexpr int WIN = 16;
    __device__ static int orow(int g, int r) { return g + 4 * r; }
    __device__ static void mma(d4& d, double a, double b) { d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0); }
};

constexpr int TGA = 4;            // centre atoms per group (16 product columns)
constexpr int TNW = 4;            // waves per block
// groups per wave at most: one (blocks of 16 atoms) balanced the fcc box's 2,000 blocks best, in
// both passes, also with the backward's force hash
#ifndef TAB_GPW_MAX
#define TAB_GPW_MAX 1
#endif
constexpr int TGPW_MAX = TAB_GPW_MAX;
constexpr int TPS = 6 * 16 + 4;   // LDS stride of one interval's six moment rows (16-B aligned;
                                  // consecutive intervals start 36 banks apart)

// Neighbour forces of a backward block are summed in LDS before they reach the force array: an
// open-addressing hash on the neighbour's caller index (2^TAB_HLOG slots, linear probing over at
// most TAB_PROBE slots; a neighbour that finds no slot adds to the force array directly). A block's
// atoms are neighbours in space (consecutive internal atoms where the caller's order is spatial,
// as an MD code keeps it; else consecutive in bin order, k_spatial_order), so their neighbour lists
// overlap and the block flushes each distinct neighbour once.
#ifndef TAB_HLOG
#define TAB_HLOG 10
#endif
#ifndef TAB_PROBE
#define TAB_PROBE 4
#endif
constexpr int TH = TAB_HLOG > 0 ? 1 << TAB_HLOG : 1;

__device__ __forceinline__ bool tab_hash_add(int* hk, double (*hf)[TH], int j, double fx, double fy, double fz)
{
    if (TAB_HLOG == 0) return false;
    unsigned h = ((unsigned)j * 2654435761u) >> (32 - (TAB_HLOG > 0 ? TAB_HLOG : 1));
#pragma unroll
    for (int p = 0; p < TAB_PROBE; ++p) {
        // a key once stored stays, so a plain read settles most lookups; an empty slot is claimed
        // by compare-and-swap (which returns the key that won if another lane came first)
        int old = __hip_atomic_load(&hk[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == -1) old = atomicCAS(&hk[h], -1, j);
        if (old == -1 || old == j) {
            unsafeAtomicAdd(&hf[0][h], fx);
            unsafeAtomicAdd(&hf[1][h], fy);
            unsafeAtomicAdd(&hf[2][h], fz);
            return true;
        }
        h = (h + 1) & (TH - 1);
    }
    return false;
}

// Geometry of one kept neighbour: r_ij, 1/r, s(r) and ds/dr (eq. switch), and the table interval
// of s (clamped to the table; inputs past it use the end pieces extrapolated).
struct TabGeo {
    double x, y, z, ir, s, ds;
    int li;
};
__device__ __forceinline__ TabGeo tab_geo_of(const EmbArgs& A, double x, double y, double z, double inv_w)
{
    TabGeo o;
    o.x = x;
    o.y = y;
    o.z = z;
    const double r = sqrt(o.x * o.x + o.y * o.y + o.z * o.z);
    o.ir = 1.0 / r;
    switch_fn(r, o.ir, A.rs, A.rc, inv_w, o.s, o.ds);
    const int li = (int)floor(o.s / A.tab_dx);
    o.li = li < 0 ? 0 : (li >= A.tab_nint ? A.tab_nint - 1 : li);
    return o;
}
__device__ __forceinline__ TabGeo tab_geo(const EmbArgs& A, size_t slot, double inv_w)
{
    return tab_geo_of(A, A.nl_r[3 * slot], A.nl_r[3 * slot + 1], A.nl_r[3 * slot + 2], inv_w);
}

// One neighbour-type block tj of a group for centre type ti: the atoms' kept counts (0 for an atom
// of another type or past the end) and the interval range [lo, top] (the intervals of the atoms'
// nearest and farthest neighbours).
struct TabPass {
    int cnt[TGA];
    int top, lo;
    bool any;
    // windows of equal size (at most win intervals) over [lo, top]
    __device__ int wsz(int win) const {
        const int span = max(top - lo + 1, 1), nw = (span + win - 1) / win;
        return (span + nw - 1) / nw;
    }
};
// The group's atom a: position a0 + a of the centres' order (bin order, or internal order).
__device__ __forceinline__ int group_atom(const int* order, int a0, int a) { return order ? order[a0 + a] : a0 + a; }

__device__ __forceinline__ TabPass tab_pass(const EmbArgs& A, const int* order, int a0, int na, int ti, int tj,
                                            bool all_types, int lane, double inv_w)
{
    int cnt = 0, li = 0;
    if (lane < 2 * TGA) {
        const int a = lane & (TGA - 1);
        const int at = a < na ? group_atom(order, a0, a) : 0;
        if (a < na && (all_types || A.itype[at] == ti)) cnt = A.nnei[(size_t)at * A.ntypes + tj];
        if (cnt > 0) li = tab_geo(A, (size_t)at * A.nc + A.off[tj] + (lane < TGA ? 0 : cnt - 1), inv_w).li;
    }
    TabPass p;
    p.top = -1;
    p.lo = 1 << 30;
    p.any = false;
#pragma unroll
    for (int a = 0; a < TGA; ++a) {
        p.cnt[a] = __builtin_amdgcn_readlane(cnt, a);
        if (p.cnt[a] > 0) {
            p.any = true;
            p.top = max(p.top, __builtin_amdgcn_readlane(li, a));
            p.lo = min(p.lo, __builtin_amdgcn_readlane(li, a + TGA));
        }
    }
    return p;
}

// Lane shifts on DPP (GFX9 controls): row_shr:n = 0x110 + n within rows of 16 lanes; row_bcast:15
// (0x142) gives rows 1 and 3 the last lane of the row before; row_bcast:31 (0x143) gives rows 2 and
// 3 lane 31. Lanes left out (row mask, or no source lane) read `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v, int old)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_t(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_t(double v)
{
    const int lo = dpp_i<CTRL, ROWS>(__double2loint(v), 0), hi = dpp_i<CTRL, ROWS>(__double2hiint(v), 0);
    return __hiloint2double(hi, lo);
}

// Segmented inclusive sums over the 64 lanes, segments being runs of lanes with equal keys (keys
// must be non-increasing along the lanes, so that equal keys are adjacent): after the call the last
// lane of each run holds the run's sum. Six Hillis-Steele steps (shifts 1, 2, 4, 8 in the rows,
// then across rows); a step adds the shifted partial sum where the source lane lies in the same run.
template <class T, int NV>
struct SegScan {
    T m[6];   // per step: 1 where the step's source lane has this lane's key, else 0
    __device__ __forceinline__ explicit SegScan(int key) {
        m[0] = dpp_i<0x111, 0xf>(key, -2) == key ? (T)1 : (T)0;
        m[1] = dpp_i<0x112, 0xf>(key, -2) == key ? (T)1 : (T)0;
        m[2] = dpp_i<0x114, 0xf>(key, -2) == key ? (T)1 : (T)0;
        m[3] = dpp_i<0x118, 0xf>(key, -2) == key ? (T)1 : (T)0;
        m[4] = dpp_i<0x142, 0xa>(key, -2) == key ? (T)1 : (T)0;
        m[5] = dpp_i<0x143, 0xc>(key, -2) == key ? (T)1 : (T)0;
    }
    __device__ __forceinline__ void run(T* v) const {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += dpp_t<0x111, 0xf>(v[i]) * m[0];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += dpp_t<0x112, 0xf>(v[i]) * m[1];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += dpp_t<0x114, 0xf>(v[i]) * m[2];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += dpp_t<0x118, 0xf>(v[i]) * m[3];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += dpp_t<0x142, 0xa>(v[i]) * m[4];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += dpp_t<0x143, 0xc>(v[i]) * m[5];
    }
};

// Leading lanes of a wave whose predicate holds (the neighbours a window takes from its cursor).
__device__ __forceinline__ int leading(bool pred)
{
    const uint64_t m = __ballot(pred);
    return ~m ? __builtin_ctzll(~m) : 64;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Centre types of a group: of consecutive internal atoms, one type except at a type boundary or
// where the atoms of a batch change frames; of atoms in bin order, any of them.
__device__ __forceinline__ void group_types(const EmbArgs& A, const int* order, int a0, int na, int& tmin, int& tmax)
{
    tmin = A.itype[group_atom(order, a0, 0)];
    tmax = tmin;
    for (int a = 1; a < na; ++a) {
        const int t = A.itype[group_atom(order, a0, a)];
        tmin = min(tmin, t);
        tmax = max(tmax, t);
    }
}

// ---------------------------------------------------------------------------------------------
// Forward: T of every atom. Each wave takes A.apw groups of TGA consecutive atoms; per (centre
// type, neighbour type) pass and window, the moments P go to LDS (atomics: neighbours on one
// interval share a row), then T^T += P^T C over the window's rows (K-steps of four rows, seven
// 16-feature tiles). T accumulates over every pass in registers and is stored once.
// ---------------------------------------------------------------------------------------------
template <class T, bool ENS>
__global__ void __launch_bounds__(TNW * 64) k_tab_fwd(EmbArgs A_)
{
    const EmbArgs A = ENS ? model_args(A_) : A_;
    typedef TabPol<T> Pol;
    typedef typename Pol::accv accv;
    constexpr int WIN = Pol::WIN;
    __shared__ T s_P[TNW][WIN * TPS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    T* sP = s_P[wave];
    const double inv_w = 1.0 / (A.rc - A.rs);
    const int nt = A.ntypes, kp = tab_kp(A.tab_nint);
    const bool tos = A.type_one_side;
    const int nets = tos ? nt : nt * nt;
    const T* tabk = reinterpret_cast<const T*>(A.table) + (size_t)nets * A.tab_nint * E2 * 6;
    T* Tout = reinterpret_cast<T*>(A.T);
    const int64_t grp0 = ((int64_t)blockIdx.x * TNW + wave) * A.apw;

    for (int gi = 0; gi < A.apw; ++gi) {
        const int64_t a0l = (grp0 + gi) * TGA;
        if (a0l >= A.natoms) break;
        const int a0 = (int)a0l, na = min(TGA, A.natoms - a0);
        accv acc[7];
#pragma unroll
        for (int tm = 0; tm < 7; ++tm) acc[tm] = accv{0, 0, 0, 0};
        int tmin, tmax;
        group_types(A, nullptr, a0, na, tmin, tmax);
        if (tos) tmax = tmin;   // the nets depend on the neighbour type only: one pass covers all
        for (int ti = tmin; ti <= tmax; ++ti)
            for (int tj = 0; tj < nt; ++tj) {
                const TabPass ps = tab_pass(A, nullptr, a0, na, ti, tj, tos, lane, inv_w);
                if (!ps.any) continue;
                const int net = tos ? tj : ti * nt + tj;
                const T* tk = tabk + (size_t)net * kp * N3P;
                int cur[TGA] = {0, 0, 0, 0};
                const int wsz = ps.wsz(WIN);
                for (int wtop = ps.top;; wtop -= wsz) {
                    const int L = max(wtop - wsz + 1, 0);
                    const bool lastw = L <= ps.lo;
                    for (int e = lane; e < WIN * TPS; e += 64) sP[e] = (T)0;
                    wave_sync();
#pragma unroll
                    for (int a = 0; a < TGA; ++a) {
                        const int n = ps.cnt[a];
                        const size_t row0 = (size_t)(a0 + a) * A.nc + A.off[tj];
                        while (cur[a] < n) {
                            const int q = cur[a] + lane;
                            const bool valid = q < n;
                            const TabGeo o = tab_geo(A, row0 + (valid ? q : n - 1), inv_w);
                            const int take = leading(valid && (lastw || o.li >= L));
                            // interval of each taken lane, made non-increasing along the lanes (a
                            // prefix minimum, needed only where rounding broke the order); -1 past them
                            // (every shuffle runs on all 64 lanes: a lane reading an inactive one
                            // would not see its key)
                            int le = lane < take ? min(max(o.li, L), wtop) : -1;
                            const int prv = __shfl_up(le, 1);
                            if (__ballot(lane > 0 && le > prv)) {
                                for (int d = 1; d < 64; d <<= 1) {
                                    const int u = __shfl_up(le, d);
                                    if (lane >= d) le = min(le, u);
                                }
                            }
                            // the lane's moment terms t^(5-j) R_k, summed over each interval's run
                            T v[24];
                            {
                                const T t = (T)(o.s - max(le, 0) * A.tab_dx);
                                const double sr = o.s * o.ir;
                                const T R[4] = {(T)o.s, (T)(sr * o.x), (T)(sr * o.y), (T)(sr * o.z)};
                                T tp = lane < take ? (T)1 : (T)0;
#pragma unroll
                                for (int j = 5; j >= 0; --j) {
#pragma unroll
                                    for (int k = 0; k < 4; ++k) v[4 * j + k] = tp * R[k];
                                    tp *= t;
                                }
                            }
                            SegScan<T, 24>(le).run(v);
                            // the last lane of each run adds it to the interval's rows (one lane per
                            // interval, so plain read-modify-writes)
                            const int nxt = __shfl_down(le, 1);
                            if (le >= 0 && (lane == 63 || nxt != le)) {
                                T* pp = sP + (le - L) * TPS + 4 * a;
#pragma unroll
                                for (int j = 0; j < 6; ++j)
#pragma unroll
                                    for (int k = 0; k < 4; ++k) pp[16 * j + k] += v[4 * j + k];
                            }
                            if (blockIdx.y == 0 && lane < take && (o.s < 0.0 || o.s > A.tab_nint * A.tab_dx))
                                atomicAdd(&A.stats->table_oor, 1ull);
                            cur[a] += take;
                            if (take < 64) break;
                        }
                    }
                    wave_sync();
                    // T^T += P^T C over the window's rows: lane (g, c) gives P[row 4 ks + g][column c]
                    // and C[row][feature 16 tm + c]. The table rows of the next K-steps are read
                    // while these multiply (FP32 two steps ahead, FP64 one; rows past the window
                    // lie in the table's zero padding, P past its last K-step counts as zero).
                    const int nks = (6 * (wtop - L + 1) + 3) >> 2;
                    const T* tb = tk + (size_t)(6 * L + g) * N3P + c;
                    constexpr int AHEAD = sizeof(T) == 4 ? 2 : 1;
                    T bq[AHEAD][7];
#pragma unroll
                    for (int d = 0; d < AHEAD; ++d)
#pragma unroll
                        for (int tm = 0; tm < 7; ++tm) bq[d][tm] = tb[(size_t)(4 * d) * N3P + 16 * tm];
                    for (int ks = 0; ks < nks; ks += AHEAD) {
#pragma unroll
                        for (int d = 0; d < AHEAD; ++d) {
                            const int row = 4 * (ks + d) + g;
                            const T av = (d == 0 || ks + d < nks) ? sP[(row / 6) * TPS + (row % 6) * 16 + c] : (T)0;
#pragma unroll
                            for (int tm = 0; tm < 7; ++tm) Pol::mma(acc[tm], av, bq[d][tm]);
                            const T* bn = tb + (size_t)(4 * (ks + d + AHEAD)) * N3P;
#pragma unroll
                            for (int tm = 0; tm < 7; ++tm) bq[d][tm] = bn[16 * tm];
                        }
                    }
                    wave_sync();
                    if (lastw) break;
                }
            }
        // T[atom][m][k] with row i = 4 atom + k of the product, m = 16 tm + c
#pragma unroll
        for (int tm = 0; tm < 7; ++tm) {
            const int m = 16 * tm + c;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = Pol::orow(g, r), a = i >> 2, k = i & 3;
                if (a < na && m < E2) Tout[((size_t)(a0 + a) * E2 + m) * 4 + k] = acc[tm][r] * (T)A.inv_nc;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Backward: per window W^T = dT^T C^T (16 rows at a time, K over the 100 features in steps of
// four) into LDS; then per neighbour
//   dE/dR_q = N_c^-1 (quintic in t of W[l][.][k]),  dE/ds_q|_G = N_c^-1 sum_k R_qk (its t-derivative)_k,
//   g_ij = dE/dr_ij = [(dR_0 + dE/ds) s' + p (s' - s/r)] r^ + (s/r) dR_{1:3},  p = dR_{1:3} . r^,
// F_j -= g_ij (FP64 atomics into caller order), F_i += g_ij (per lane over the group, then one
// atomic per atom and component), Xi -= g_ij r_ij^T (per lane over the block, or per atom for a
// batch of frames), and the block's [E, virial] partial as the network path writes it.
// ---------------------------------------------------------------------------------------------
template <class T, bool ENS>
__global__ void __launch_bounds__(TNW * 64) k_tab_bwd(EmbArgs A_)
{
    const EmbArgs A = ENS ? model_args(A_) : A_;
    typedef TabPol<T> Pol;
    typedef typename Pol::accv accv;
    constexpr int WIN = Pol::WIN, ROWS = 6 * WIN, KC = 3;
    // groups of atoms neighbouring in space (see the force hash): the internal order where it is
    // spatial, else the bin order
    const int* ord = (A.order && 4 * (int64_t)*A.order_cnt < (int64_t)A.natoms) ? A.order : nullptr;
    static_assert(ROWS % 16 == 0, "whole 16-row tiles of W per window");
    __shared__ __attribute__((aligned(16))) T s_W[TNW][TGA][ROWS][4];
    __shared__ double s_vir[TNW][9];
    __shared__ int s_hk[TH];
    __shared__ double s_hf[3][TH];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const double inv_w = 1.0 / (A.rc - A.rs), inc = A.inv_nc;
    if (TAB_HLOG > 0) {
        for (int i = threadIdx.x; i < TH; i += TNW * 64) {
            s_hk[i] = -1;
            s_hf[0][i] = s_hf[1][i] = s_hf[2][i] = 0.0;
        }
        __syncthreads();
    }
    const int nt = A.ntypes, kp = tab_kp(A.tab_nint);
    const bool tos = A.type_one_side;
    const int nets = tos ? nt : nt * nt;
    const T* tabm = reinterpret_cast<const T*>(A.table) + (size_t)nets * A.tab_nint * E2 * 6 + (size_t)nets * kp * N3P;
    const T* dTin = reinterpret_cast<const T*>(A.dT);
    const bool batched = A.vir_atom != nullptr;
    const int64_t grp0 = ((int64_t)blockIdx.x * TNW + wave) * A.apw;
    double vir[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

    for (int gi = 0; gi < A.apw; ++gi) {
        const int64_t a0l = (grp0 + gi) * TGA;
        if (a0l >= A.natoms) break;
        const int a0 = (int)a0l, na = min(TGA, A.natoms - a0);
        double fc[TGA][3];
#pragma unroll
        for (int a = 0; a < TGA; ++a) fc[a][0] = fc[a][1] = fc[a][2] = 0.0;
        int tmin, tmax;
        group_types(A, ord, a0, na, tmin, tmax);
        if (tos) tmax = tmin;
        for (int ti = tmin; ti <= tmax; ++ti) {
            // dT^T as the A operand: lane (g, c) holds dT[atom c/4][feature 4 ms + g][component c%4]
            // (zero for atoms outside the pass)
            T adt[E2 / 4];
            {
                const int ai = c >> 2;
                const int at = group_atom(ord, a0, ai < na ? ai : 0);
                const bool ok = ai < na && (tos || A.itype[at] == ti);
                const T* src = dTin + ((size_t)at * E2 + g) * 4 + (c & 3);
#pragma unroll
                for (int ms = 0; ms < E2 / 4; ++ms) adt[ms] = ok ? src[16 * ms] : (T)0;
            }
            for (int tj = 0; tj < nt; ++tj) {
                const TabPass ps = tab_pass(A, ord, a0, na, ti, tj, tos, lane, inv_w);
                if (!ps.any) continue;
                const int net = tos ? tj : ti * nt + tj;
                const T* tmat = tabm + (size_t)net * N3P * kp;
                int cur[TGA] = {0, 0, 0, 0};
                const int wsz = ps.wsz(WIN);
                for (int wtop = ps.top;; wtop -= wsz) {
                    const int L = max(wtop - wsz + 1, 0);
                    const bool lastw = L <= ps.lo;
                    // W^T[atom, k][row] for the window's rows 6 L + [0, 16 nkt), KC K-tiles at a time
                    // (independent accumulators; the sum over the features runs inside them and the
                    // next feature step's table rows are read while this one multiplies; tiles past
                    // nkt read the table's zero padding and are not stored)
                    const int nkt = (6 * (wtop - L + 1) + 15) >> 4;
                    const T* bc = tmat + (size_t)g * kp + 6 * L + c;
                    for (int k0 = 0; k0 < nkt; k0 += KC) {
                        accv w[KC];
                        T bq[KC];
                        const T* bk = bc + 16 * k0;
#pragma unroll
                        for (int j = 0; j < KC; ++j) {
                            w[j] = accv{0, 0, 0, 0};
                            bq[j] = bk[16 * j];
                        }
#pragma unroll
                        for (int ms = 0; ms < E2 / 4; ++ms) {
                            T bn[KC];
                            if (ms + 1 < E2 / 4) {
#pragma unroll
                                for (int j = 0; j < KC; ++j) bn[j] = bk[(size_t)(4 * ms + 4) * kp + 16 * j];
                            }
#pragma unroll
                            for (int j = 0; j < KC; ++j) Pol::mma(w[j], adt[ms], bq[j]);
                            if (ms + 1 < E2 / 4) {
#pragma unroll
                                for (int j = 0; j < KC; ++j) bq[j] = bn[j];
                            }
                        }
#pragma unroll
                        for (int j = 0; j < KC; ++j) {
                            if (k0 + j >= nkt) break;
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int i = Pol::orow(g, r);
                                s_W[wave][i >> 2][16 * (k0 + j) + c][i & 3] = w[j][r];
                            }
                        }
                    }
                    wave_sync();
#pragma unroll
                    for (int a = 0; a < TGA; ++a) {
                        const int n = ps.cnt[a];
                        if (n == 0) continue;
                        const size_t row0 = (size_t)group_atom(ord, a0, a) * A.nc + A.off[tj];
                        // r_ij and j of the chunk at the cursor; each chunk reads the next one's
                        // before its force atomics (reads and atomics retire in order, so a read
                        // issued after them would wait for them)
                        size_t slot = row0 + min(cur[a] + lane, n - 1);
                        double px = A.nl_r[3 * slot], py = A.nl_r[3 * slot + 1], pz = A.nl_r[3 * slot + 2];
                        int pj = A.nl_j[slot];
                        while (cur[a] < n) {
                            const int q = cur[a] + lane;
                            const bool valid = q < n;
                            const TabGeo o = tab_geo_of(A, px, py, pz, inv_w);
                            const int jn = pj;
                            const int take = leading(valid && (lastw || o.li >= L));
                            if (take == 64 && cur[a] + 64 < n) {
                                slot = row0 + min(cur[a] + 64 + lane, n - 1);
                                px = A.nl_r[3 * slot];
                                py = A.nl_r[3 * slot + 1];
                                pz = A.nl_r[3 * slot + 2];
                                pj = A.nl_j[slot];
                            }
                            if (lane < take) {
                                const int le = min(max(o.li, L), wtop);
                                const T t = (T)(o.s - le * A.tab_dx);
                                const T* wr = &s_W[wave][a][(le - L) * 6][0];
                                const double sr = o.s * o.ir;
                                const double ux = o.x * o.ir, uy = o.y * o.ir, uz = o.z * o.ir;
                                const T R[4] = {(T)o.s, (T)(sr * o.x), (T)(sr * o.y), (T)(sr * o.z)};
                                T dR[4], hR = (T)0;
#pragma unroll
                                for (int k = 0; k < 4; ++k) {
                                    T v = wr[k], h = 5 * wr[k];
                                    v = v * t + wr[4 + k];
                                    h = h * t + 4 * wr[4 + k];
                                    v = v * t + wr[8 + k];
                                    h = h * t + 3 * wr[8 + k];
                                    v = v * t + wr[12 + k];
                                    h = h * t + 2 * wr[12 + k];
                                    v = v * t + wr[16 + k];
                                    h = h * t + wr[16 + k];
                                    dR[k] = v * t + wr[20 + k];
                                    hR += h * R[k];
                                }
                                const double d0 = inc * (double)dR[0], d1 = inc * (double)dR[1];
                                const double d2 = inc * (double)dR[2], d3 = inc * (double)dR[3];
                                const double dEds = inc * (double)hR;
                                const double p = d1 * ux + d2 * uy + d3 * uz;
                                const double rad = (d0 + dEds) * o.ds + p * (o.ds - sr);
                                const double gx = rad * ux + sr * d1, gy = rad * uy + sr * d2, gz = rad * uz + sr * d3;
                                asm volatile("" ::"v"(px), "v"(py), "v"(pz), "v"(pj));
                                if (!tab_hash_add(s_hk, s_hf, jn, -gx, -gy, -gz)) {
                                    unsafeAtomicAdd(&A.F[3 * (size_t)jn], -gx);
                                    unsafeAtomicAdd(&A.F[3 * (size_t)jn + 1], -gy);
                                    unsafeAtomicAdd(&A.F[3 * (size_t)jn + 2], -gz);
                                }
                                fc[a][0] += gx;
                                fc[a][1] += gy;
                                fc[a][2] += gz;
                                vir[0] -= gx * o.x; vir[1] -= gx * o.y; vir[2] -= gx * o.z;
                                vir[3] -= gy * o.x; vir[4] -= gy * o.y; vir[5] -= gy * o.z;
                                vir[6] -= gz * o.x; vir[7] -= gz * o.y; vir[8] -= gz * o.z;
                            }
                            cur[a] += take;
                            if (take < 64) break;
                        }
                        if (batched) {
                            // a batch of frames keeps the virial per centre atom (one wave owns it)
#pragma unroll
                            for (int k = 0; k < 9; ++k) {
                                const double v = wave_sum(vir[k]);
                                if (lane == 0) A.vir_atom[9 * (size_t)group_atom(ord, a0, a) + k] += v;
                                vir[k] = 0.0;
                            }
                        }
                    }
                    wave_sync();
                    if (lastw) break;
                }
            }
        }
        // the centre atoms' forces, caller order
#pragma unroll
        for (int a = 0; a < TGA; ++a) {
            if (a >= na) break;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double v = wave_sum(fc[a][k]);
                if (lane == 0) unsafeAtomicAdd(&A.F[3 * (size_t)A.perm[group_atom(ord, a0, a)] + k], v);
            }
        }
    }
    // block partial [E, virial]: the virial over the waves' lanes, E over this block's atoms (a
    // shuffle tree, a fixed order; single frame), and E_i in caller order if asked for
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double v = batched ? 0.0 : wave_sum(vir[k]);
        if (lane == 0) s_vir[wave][k] = v;
    }
    __syncthreads();
    // the block's summed neighbour forces, once per distinct neighbour
    if (TAB_HLOG > 0) {
        for (int i = threadIdx.x; i < TH; i += TNW * 64) {
            const int j = s_hk[i];
            if (j >= 0) {
                unsafeAtomicAdd(&A.F[3 * (size_t)j], s_hf[0][i]);
                unsafeAtomicAdd(&A.F[3 * (size_t)j + 1], s_hf[1][i]);
                unsafeAtomicAdd(&A.F[3 * (size_t)j + 2], s_hf[2][i]);
            }
        }
    }
    double* part = A.vir_part + 10 * (size_t)blockIdx.x;
    if (threadIdx.x < 9) {
        double v = 0.0;
        for (int q = 0; q < TNW; ++q) v += s_vir[q][threadIdx.x];
        part[1 + threadIdx.x] = v;
    }
    if (A.Ei) {
        const int64_t apb = (int64_t)TNW * A.apw * TGA;
        const int b0 = (int)std::min<int64_t>((int64_t)blockIdx.x * apb, A.natoms);
        const int b1 = (int)std::min<int64_t>((int64_t)b0 + apb, A.natoms);
        if (threadIdx.x < 64) {
            double e = 0.0;
            for (int a = b0 + lane; a < b1; a += 64) e += A.Ei[a];
            e = wave_sum(e);
            if (lane == 0) part[0] = e;
        }
        if (A.atom_energy)
            for (int a = b0 + (int)threadIdx.x; a < b1; a += TNW * 64) A.atom_energy[A.perm[a]] = A.Ei[a];
    }
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
// Groups per wave: about two resident blocks' worth of groups per CU before a wave takes more.
static int tab_gpw(int64_t natoms, int ncu)
{
    const int64_t groups = (natoms + TGA - 1) / TGA;
    const int64_t per = groups / ((int64_t)TNW * 2 * (ncu > 0 ? ncu : 256));
    return (int)std::max<int64_t>(1, std::min<int64_t>(TGPW_MAX, per));
}

int tab_blocks(int64_t natoms, int ncu)
{
    const int64_t apb = (int64_t)TNW * tab_gpw(natoms, ncu) * TGA;
    return (int)((natoms + apb - 1) / apb);
}

int tab_atoms_per_block_min() { return TNW * TGA; }

// The centres in bin order, from the candidate records (bin order, one per atom; the tag's low 30
// bits are the internal index): groups of consecutive positions in this order are atoms in one or
// two bins, whose neighbour lists overlap in the force hash. The caller's own order (kept within
// each type by the internal order) is usually more compact still where it is spatial (a lattice, or
// an MD code's periodic sort), so the backward keeps it unless fewer than a quarter of consecutive
// internal atoms share a bin, the count this kernel makes (one atomic per wave into *cnt, which
// starts the frame at zero).
__global__ void __launch_bounds__(256) k_spatial_order(int n, const double4* cand, const int* cell_of, int* order,
                                                       int* cnt)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) order[k] = (int)(__double_as_longlong(cand[k].w) & ((1LL << 30) - 1));
    const bool same = k + 1 < n && cell_of[k] == cell_of[k + 1];
    const int w = __popcll(__ballot(same));
    if ((threadIdx.x & 63) == 0 && w) atomicAdd(cnt, w);
}

void launch_spatial_order(int n, const double4* cand, const int* cell_of, int* order, int* cnt, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_spatial_order, dim3((n + 255) / 256), dim3(256), 0, s, n, cand, cell_of, order, cnt);
}

template <class T>
static void launch_tab_p(bool fwd, const EmbArgs& a0, hipStream_t s)
{
    EmbArgs a = a0;
    a.apw = tab_gpw(a.natoms, a.ncu);
    const int blocks = tab_blocks(a.natoms, a.ncu);
    if (blocks <= 0) return;
    const bool ens = a.nmodels > 1;
    const dim3 grid(blocks, ens ? a.nmodels : 1), block(TNW * 64);
    if (fwd) {
        if (ens) hipLaunchKernelGGL((k_tab_fwd<T, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_tab_fwd<T, false>), grid, block, 0, s, a);
    } else {
        if (ens) hipLaunchKernelGGL((k_tab_bwd<T, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_tab_bwd<T, false>), grid, block, 0, s, a);
    }
}

void launch_tab(bool fwd, int precision, const EmbArgs& a, hipStream_t s)
{
    if (precision == 0) launch_tab_p<double>(fwd, a, s);
    else launch_tab_p<float>(fwd, a, s);
}

}  // namespace dpk
