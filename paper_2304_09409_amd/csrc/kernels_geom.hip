// kernels_geom.hip -- ingest, cell list and neighbour list of one frame (FP64 geometry).
//
// Compiled with FP contraction off: every coordinate difference, image shift and squared
// distance is evaluated with separately rounded multiplies and adds in a fixed order, so the
// neighbour selection (Sec. II.A: n(i), capacities padded to N_c; Sec. III.B.1: order by type,
// distance, index) is a deterministic function of the input bits.
#include <hip/hip_runtime.h>
#include "dpk_internal.h"
#include "dpk_launch.h"

namespace dpk {

__global__ void k_fill_zero(unsigned int* p, size_t nwords)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < nwords; i += stride) p[i] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t s)
{
    size_t words = (bytes + 3) / 4;
    if (!words) return;
    int blocks = (int)((words + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (unsigned int*)p, words);
}

// ---- atom types: validation, counts, stable partition by type (atoms are kept sorted by
// species so that each fitting GEMM and each embedding net runs over contiguous atoms) ----

__global__ void k_type_count(int n, const int* atype, int ntypes, int* tcount, DevStats* st)
{
    __shared__ int h[MAXT];
    if (threadIdx.x < MAXT) h[threadIdx.x] = 0;
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        // Out-of-range types raise the error flag and are counted as the nearest valid type,
        // the same clamp the partition below applies, so the permutation stays complete.
        int t = atype[i];
        if (t < 0 || t >= ntypes) atomicExch(&st->err_type, 1);
        t = t < 0 ? 0 : (t >= ntypes ? ntypes - 1 : t);
        atomicAdd(&h[t], 1);
    }
    __syncthreads();
    if (threadIdx.x < ntypes && h[threadIdx.x]) atomicAdd(&tcount[threadIdx.x], h[threadIdx.x]);
}

// One block of 1024 threads: stable counting-sort scatter. perm[a] = caller index of internal
// atom a; inv_perm is its inverse; itype[a] the type.
__global__ void __launch_bounds__(1024) k_type_perm(int n, const int* atype, int ntypes, const int* tcount,
                                                     int* toff, int* perm, int* inv_perm, int* itype)
{
    __shared__ int cursor[MAXT];
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        int acc = 0;
        for (int t = 0; t < ntypes; ++t) { cursor[t] = acc; toff[t] = acc; acc += tcount[t]; }
        toff[ntypes] = acc;
    }
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int base = 0; base < n; base += 1024) {
        int i = base + tid;
        int t = -1;
        if (i < n) {
            t = atype[i];
            if (t < 0) t = 0;
            if (t >= ntypes) t = ntypes - 1;
        }
        for (int k = 0; k < ntypes; ++k) {
            bool f = (t == k);
            unsigned long long m = __ballot(f);
            if (lane == 0) wsum[wid] = __popcll(m);
            __syncthreads();
            int before = 0, total = 0;
            for (int w = 0; w < 16; ++w) { if (w < wid) before += wsum[w]; total += wsum[w]; }
            if (f) {
                int pos = cursor[k] + before + __popcll(m & lt);
                perm[pos] = i;
                inv_perm[i] = pos;
                itype[pos] = k;
            }
            __syncthreads();
            if (tid == 0) cursor[k] += total;
            __syncthreads();
        }
    }
}

// Bounding box of an open cluster: out = {min xyz, max xyz}.
__global__ void __launch_bounds__(1024) k_bbox(int n, const double* coord, double* out)
{
    __shared__ double red[6][1024];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = threadIdx.x; i < n; i += 1024)
        for (int c = 0; c < 3; ++c) {
            double x = coord[3 * (size_t)i + c];
            lo[c] = fmin(lo[c], x);
            hi[c] = fmax(hi[c], x);
        }
    for (int c = 0; c < 3; ++c) { red[c][threadIdx.x] = lo[c]; red[3 + c][threadIdx.x] = hi[c]; }
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + s]);
                red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// Wrap into the cell (periodic) and assign bins. Fractional s = r h^-1 (row vector), wrapped to
// [0,1), and the wrapped position s h, each component summed in the fixed order 0, 1, 2.
__global__ void k_wrap_bin(int n, const double* coord, const int* perm, GeomParams gp, double* pos,
                           int* cell_of, int* cell_count)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    int i = perm[a];
    double x[3] = {coord[3 * (size_t)i], coord[3 * (size_t)i + 1], coord[3 * (size_t)i + 2]};
    int b[3];
    double p[3];
    if (gp.periodic) {
        double s[3];
        for (int c = 0; c < 3; ++c) {
            s[c] = (x[0] * gp.hinv[c] + x[1] * gp.hinv[3 + c]) + x[2] * gp.hinv[6 + c];
            s[c] -= floor(s[c]);
            if (s[c] >= 1.0) s[c] = 0.0;
        }
        for (int c = 0; c < 3; ++c) p[c] = (s[0] * gp.h[c] + s[1] * gp.h[3 + c]) + s[2] * gp.h[6 + c];
        for (int c = 0; c < 3; ++c) {
            int bb = (int)floor(s[c] * gp.nb[c]);
            b[c] = bb < 0 ? 0 : (bb >= gp.nb[c] ? gp.nb[c] - 1 : bb);
        }
    } else {
        for (int c = 0; c < 3; ++c) {
            p[c] = x[c];
            int bb = (int)floor((x[c] - gp.origin[c]) / gp.binw[c]);
            b[c] = bb < 0 ? 0 : (bb >= gp.nb[c] ? gp.nb[c] - 1 : bb);
        }
    }
    for (int c = 0; c < 3; ++c) pos[3 * (size_t)a + c] = p[c];
    int cell = (b[2] * gp.nb[1] + b[1]) * gp.nb[0] + b[0];
    cell_of[a] = cell;
    atomicAdd(&cell_count[cell], 1);
}

// Exclusive scan of the bin counts (one block).
__global__ void __launch_bounds__(1024) k_cell_scan(int ncell, const int* count, int* start, int* cursor)
{
    __shared__ int part[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ncell; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < ncell ? count[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < 1024; s <<= 1) {
            int add = (int)threadIdx.x >= s ? part[threadIdx.x - s] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ncell) { start[i] = carry + part[threadIdx.x] - v; cursor[i] = start[i]; }
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) start[ncell] = carry;
}

__global__ void k_cell_fill(int n, const int* cell_of, int* cursor, int* cell_atoms)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    int slot = atomicAdd(&cursor[cell_of[a]], 1);
    cell_atoms[slot] = a;
}

// ---- neighbour list: one wave per centre atom --------------------------------------------
// Candidates (every atom image within r_c found through the bin stencil) are compacted into
// LDS as 128-bit keys that compare like (type, r^2, caller index j, image n0, n1, n2):
//   hi = type << 59 | bits(r^2) >> 5
//   lo = (bits(r^2) & 31) << 59 | j << 21 | code(n)
// (r^2 is a non-negative double, whose bit pattern orders like its value). A bitonic sort in LDS
// orders them; the first sel[t] of each type fill that type's block of slots, the rest are
// counted as dropped; unfilled slots get index -1.

__device__ __forceinline__ bool key_less(unsigned long long ah, unsigned long long al,
                                         unsigned long long bh, unsigned long long bl)
{
    return ah < bh || (ah == bh && al < bl);
}

__device__ __forceinline__ void image_shift(const GeomParams& gp, int n0, int n1, int n2, double sh[3])
{
    if (gp.periodic) {
        for (int c = 0; c < 3; ++c)
            sh[c] = ((double)n0 * gp.h[c] + (double)n1 * gp.h[3 + c]) + (double)n2 * gp.h[6 + c];
    } else {
        sh[0] = sh[1] = sh[2] = 0.0;
    }
}

__global__ void __launch_bounds__(64) k_nlist(int n, const double* pos, const int* itype, const int* perm,
                                              const int* inv_perm, const int* cell_of, const int* cell_start,
                                              const int* cell_atoms, GeomParams gp, int* nl_j, double* nl_r,
                                              int* nnei, DevStats* st)
{
    __shared__ unsigned long long khi[NL_CAP], klo[NL_CAP];
    __shared__ int tcnt[MAXT];
    const int a = blockIdx.x, lane = threadIdx.x;
    if (lane < MAXT) tcnt[lane] = 0;
    const double pi[3] = {pos[3 * (size_t)a], pos[3 * (size_t)a + 1], pos[3 * (size_t)a + 2]};
    const int ci = cell_of[a];
    const int bi[3] = {ci % gp.nb[0], (ci / gp.nb[0]) % gp.nb[1], ci / (gp.nb[0] * gp.nb[1])};
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();
    int count = 0;   // wave-uniform
    for (int o0 = -gp.K[0]; o0 <= gp.K[0]; ++o0)
        for (int o1 = -gp.K[1]; o1 <= gp.K[1]; ++o1)
            for (int o2 = -gp.K[2]; o2 <= gp.K[2]; ++o2) {
                int tg[3] = {bi[0] + o0, bi[1] + o1, bi[2] + o2}, nn[3], bb[3];
                bool skip = false;
                for (int c = 0; c < 3; ++c) {
                    if (gp.periodic) {
                        int q = tg[c] / gp.nb[c];
                        if ((tg[c] % gp.nb[c] != 0) && (tg[c] < 0)) --q;
                        nn[c] = q;
                        bb[c] = tg[c] - q * gp.nb[c];
                    } else {
                        nn[c] = 0;
                        bb[c] = tg[c];
                        if (tg[c] < 0 || tg[c] >= gp.nb[c]) skip = true;
                    }
                }
                if (skip) continue;
                double sh[3];
                image_shift(gp, nn[0], nn[1], nn[2], sh);
                const bool self_image = (nn[0] == 0 && nn[1] == 0 && nn[2] == 0);
                const unsigned long long code =
                    ((unsigned long long)(nn[0] + 64) << 14) | ((unsigned long long)(nn[1] + 64) << 7) |
                    (unsigned long long)(nn[2] + 64);
                const int cell = (bb[2] * gp.nb[1] + bb[1]) * gp.nb[0] + bb[0];
                const int qs = cell_start[cell], qe = cell_start[cell + 1];
                for (int q0 = qs; q0 < qe; q0 += 64) {
                    int q = q0 + lane;
                    bool pass = false;
                    int j = 0;
                    double r2 = 0.0;
                    if (q < qe) {
                        j = cell_atoms[q];
                        if (!(j == a && self_image)) {
                            double d0 = (pos[3 * (size_t)j] + sh[0]) - pi[0];
                            double d1 = (pos[3 * (size_t)j + 1] + sh[1]) - pi[1];
                            double d2 = (pos[3 * (size_t)j + 2] + sh[2]) - pi[2];
                            r2 = d0 * d0 + d1 * d1 + d2 * d2;
                            pass = r2 < gp.rc2;
                        }
                    }
                    unsigned long long m = __ballot(pass);
                    if (pass) {
                        int idx = count + __popcll(m & lt);
                        if (idx < NL_CAP) {
                            int tj = itype[j];
                            unsigned long long rb = (unsigned long long)__double_as_longlong(r2);
                            khi[idx] = ((unsigned long long)tj << 59) | (rb >> 5);
                            klo[idx] = ((rb & 31ull) << 59) | ((unsigned long long)perm[j] << 21) | code;
                            atomicAdd(&tcnt[tj], 1);
                        }
                    }
                    count += __popcll(m);
                }
            }
    if (lane == 0) {
        atomicMax(&st->max_cand, count);
        if (count > NL_CAP) atomicExch(&st->err_overflow, 1);
    }
    if (count > NL_CAP) count = NL_CAP;
    int S = 64;
    while (S < count) S <<= 1;
    for (int q = count + lane; q < S; q += 64) { khi[q] = ~0ull; klo[q] = ~0ull; }
    __syncthreads();
    for (int k = 2; k <= S; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < S; i += 64) {
                int ixj = i ^ j;
                if (ixj > i) {
                    unsigned long long ah = khi[i], al = klo[i], bh = khi[ixj], bl = klo[ixj];
                    bool up = (i & k) == 0;
                    if (key_less(bh, bl, ah, al) == up) {
                        khi[i] = bh; klo[i] = bl; khi[ixj] = ah; klo[ixj] = al;
                    }
                }
            }
            __syncthreads();
        }
    }
    int tstart[MAXT], kept[MAXT];
    int acc = 0, drops = 0;
    for (int t = 0; t < gp.ntypes; ++t) {
        tstart[t] = acc;
        acc += tcnt[t];
        kept[t] = tcnt[t] < gp.sel[t] ? tcnt[t] : gp.sel[t];
        drops += tcnt[t] - kept[t];
    }
    const size_t rowj = (size_t)a * gp.nc;
    for (int q = lane; q < count; q += 64) {
        int t = (int)(khi[q] >> 59);
        int rank = q - tstart[t];
        if (rank < gp.sel[t]) {
            unsigned long long lo = klo[q];
            int jo = (int)((lo >> 21) & ((1ull << 38) - 1));
            int code = (int)(lo & ((1ull << 21) - 1));
            int n0 = (code >> 14) - 64, n1 = ((code >> 7) & 127) - 64, n2 = (code & 127) - 64;
            int j = inv_perm[jo];
            double sh[3];
            image_shift(gp, n0, n1, n2, sh);
            size_t slot = rowj + gp.off[t] + rank;
            nl_j[slot] = j;
            for (int c = 0; c < 3; ++c) nl_r[3 * slot + c] = (pos[3 * (size_t)j + c] + sh[c]) - pi[c];
        }
    }
    for (int s = lane; s < gp.nc; s += 64) {
        int t = 0;
        while (t + 1 < gp.ntypes && s >= gp.off[t + 1]) ++t;
        if (s - gp.off[t] >= kept[t]) {
            nl_j[rowj + s] = -1;
            for (int c = 0; c < 3; ++c) nl_r[3 * (rowj + s) + c] = 0.0;
        }
    }
    if (lane < gp.ntypes) nnei[(size_t)a * gp.ntypes + lane] = kept[lane];
    if (lane == 0 && drops) atomicAdd(&st->nbr_dropped, (unsigned long long)drops);
}

// ---- reductions and output ----------------------------------------------------------------

// E = sum_i E_i and Xi = sum of per-block partials, in a fixed order (one block).
__global__ void __launch_bounds__(1024) k_finalize(int n, const double* ei, int nvp, const double* vir_part,
                                                    double* energy, double* virial)
{
    __shared__ double red[1024];
    for (int c = -1; c < 9; ++c) {
        double s = 0.0;
        if (c < 0) {
            for (int i = threadIdx.x; i < n; i += 1024) s += ei[i];
        } else {
            for (int i = threadIdx.x; i < nvp; i += 1024) s += vir_part[9 * (size_t)i + c];
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (c < 0) *energy = red[0];
            else virial[c] = red[0];
        }
        __syncthreads();
    }
}

__global__ void k_output(int n, const int* perm, const double* f_int, const double* ei, double* force,
                         double* atom_energy)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    int i = perm[a];
    for (int c = 0; c < 3; ++c) force[3 * (size_t)i + c] = f_int[3 * (size_t)a + c];
    if (atom_energy) atom_energy[i] = ei[a];
}

// Debug: neighbour list in caller numbering, rows in caller order.
__global__ void k_debug_nlist(int n, int nc, const int* perm, const int* nl_j, int* out)
{
    int a = blockIdx.x;
    int i = perm[a];
    for (int s = threadIdx.x; s < nc; s += blockDim.x) {
        int j = nl_j[(size_t)a * nc + s];
        out[(size_t)i * nc + s] = j < 0 ? -1 : perm[j];
    }
}

// ---- launchers --------------------------------------------------------------------------

void launch_types(int n, const int* atype, int ntypes, int* tcount, int* toff, int* perm, int* inv_perm,
                  int* itype, DevStats* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_type_count, dim3((n + 255) / 256), dim3(256), 0, s, n, atype, ntypes, tcount, st);
    hipLaunchKernelGGL(k_type_perm, dim3(1), dim3(1024), 0, s, n, atype, ntypes, tcount, toff, perm, inv_perm,
                       itype);
}

void launch_bbox(int n, const double* coord, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, s, n, coord, out);
}

void launch_cells(int n, const double* coord, const int* perm, const GeomParams& gp, double* pos, int* cell_of,
                  int* cell_count, int* cell_start, int* cursor, int* cell_atoms, hipStream_t s)
{
    int ncell = gp.nb[0] * gp.nb[1] * gp.nb[2];
    hipLaunchKernelGGL(k_wrap_bin, dim3((n + 255) / 256), dim3(256), 0, s, n, coord, perm, gp, pos, cell_of,
                       cell_count);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, s, ncell, cell_count, cell_start, cursor);
    hipLaunchKernelGGL(k_cell_fill, dim3((n + 255) / 256), dim3(256), 0, s, n, cell_of, cursor, cell_atoms);
}

void launch_nlist(int n, const double* pos, const int* itype, const int* perm, const int* inv_perm,
                  const int* cell_of, const int* cell_start, const int* cell_atoms, const GeomParams& gp, int* nl_j,
                  double* nl_r, int* nnei, DevStats* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_nlist, dim3(n), dim3(64), 0, s, n, pos, itype, perm, inv_perm, cell_of, cell_start,
                       cell_atoms, gp, nl_j, nl_r, nnei, st);
}

void launch_finalize(int n, const double* ei, int nvp, const double* vir_part, double* energy, double* virial,
                     const int* perm, const double* f_int, double* force, double* atom_energy, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, n, ei, nvp, vir_part, energy, virial);
    hipLaunchKernelGGL(k_output, dim3((n + 255) / 256), dim3(256), 0, s, n, perm, f_int, ei, force, atom_energy);
}

void launch_debug_nlist(int n, int nc, const int* perm, const int* nl_j, int* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_nlist, dim3(n), dim3(64), 0, s, n, nc, perm, nl_j, out);
}

}  // namespace dpk
