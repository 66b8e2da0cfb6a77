// kernels_geom.hip -- ingest, cell list and neighbour list of one frame (FP64 geometry).
//
// Compiled with FP contraction off: every coordinate difference, image shift and squared
// distance is evaluated with separately rounded multiplies and adds in a fixed order, so the
// neighbour selection (Sec. II.A: n(i), capacities padded to N_c; Sec. III.B.1: order by type,
// distance, index) is a deterministic function of the input bits.
#include <hip/hip_runtime.h>

#include <mutex>

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

// Workspace of the allocation-free entry point: one array per device, held from the library's
// load until the process ends, shared by every call on that device. In host code `scratch` names
// a host-side stand-in; kernels get the device address that scratch_region looks up.
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int scratch_region(int device, void** ptr)
{
    if (device < 0 || device >= MAX_DEVICES) return -1;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        // the caller has made `device` current: this is that device's copy of the array
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return -1;
        }
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return 0;
}

// ---- atom types: validation, counts, stable partition by type (atoms are kept sorted by
// species so that each fitting GEMM and each embedding net runs over contiguous atoms; the order
// within a type is the caller order) ----
constexpr int TP_BLOCK = PREP_BLOCK;   // atoms per block of the multi-block preparation

__device__ __forceinline__ int clamp_type(int t, int ntypes) { return t < 0 ? 0 : (t >= ntypes ? ntypes - 1 : t); }

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

// ---- fused preparation for frames of up to PS_MAX_ATOMS atoms and PS_MAX_CELLS bins --------
// One workgroup runs every preparation phase with barriers in between instead of seven dependent
// launches: type counts (ballots), the stable type partition (chunks of 1024 atoms in caller
// order, ballot ranks), wrap and bin (bin counts as LDS atomics), the bin scan, and the bin fill,
// which writes the candidate records directly. Results equal those of the multi-kernel path,
// except the order of atoms within a bin, which nothing downstream depends on (the neighbour
// list sorts its hits by a key that is unique per candidate).
constexpr int PS_THREADS = 1024;
constexpr int PS_APT = 8;                           // atoms per thread, held in registers
constexpr int PS_MAX_ATOMS = PS_THREADS * PS_APT;   // 8192
constexpr int PS_MAX_CELLS = 8192;

__device__ __forceinline__ void wrap_bin_one(const GeomParams& gp, const double* x, double* p, int* b)
{
    if (gp.periodic) {
        double s[3];
        for (int c = 0; c < 3; ++c) {
            s[c] = (x[0] * gp.hinv[c] + x[1] * gp.hinv[3 + c]) + x[2] * gp.hinv[6 + c];
            s[c] -= floor(s[c]);
            if (s[c] >= 1.0) s[c] = 0.0;
        }
        for (int c = 0; c < 3; ++c) p[c] = (s[0] * gp.h[c] + s[1] * gp.h[3 + c]) + s[2] * gp.h[6 + c];
        for (int c = 0; c < 3; ++c) {
            const int bb = (int)floor(s[c] * gp.nb[c]);
            b[c] = bb < 0 ? 0 : (bb >= gp.nb[c] ? gp.nb[c] - 1 : bb);
        }
    } else {
        for (int c = 0; c < 3; ++c) {
            p[c] = x[c];
            const int bb = (int)floor((x[c] - gp.origin[c]) / gp.binw[c]);
            b[c] = bb < 0 ? 0 : (bb >= gp.nb[c] ? gp.nb[c] - 1 : bb);
        }
    }
}

// One frame's preparation in one workgroup. Single frame (BATCH = false): counts the types itself
// and zeroes the statistics block. Frame f of a batch (BATCH = true): the per-type internal bases
// come from k_batch_scan; atoms, candidate records and bins sit at the frame's offsets.
// Ghost atoms (single frame, caller indices nlocal.. n - 1; nlocal = n without ghosts) form one
// more partition class after the types, so the owned atoms take internal positions 0.. nlocal - 1
// sorted by type; itype and the candidate records keep every atom's real type.
template <bool BATCH>
__device__ __forceinline__ void prep_frame(int f, int n, int nlocal, int atom_off, const double* coord, const int* atype,
                                           int ntypes, const GeomParams& gp, int ncell, int cell_off,
                                           const int* type_base, int* tcount, int* toff, int* perm, int* inv_perm,
                                           int* itype, int* frame_of, DevStats* st, double* pos, int* cell_of,
                                           int* cell_start, double4* cand, double* f_int, double* vir_atom)
{
    __shared__ int s_cnt[PS_MAX_CELLS];        // bin counts, then bin cursors
    __shared__ int s_w[PS_THREADS / 64][MAXT]; // per-wave type counts
    __shared__ int s_base[MAXT];               // next internal position per type
    __shared__ int s_part[PS_THREADS];         // scan partials
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (!BATCH)
        for (int w = tid; w < STATS_WORDS; w += PS_THREADS) reinterpret_cast<int*>(st)[w] = 0;
    for (int c = tid; c < ncell; c += PS_THREADS) s_cnt[c] = 0;
    if (BATCH && tid < ntypes) s_base[tid] = type_base[tid];
    __syncthreads();   // the statistics block is zero before anything raises a flag in it
    // types of this thread's atoms tid + PS_THREADS j, read once; tv is the partition class (the
    // type, or ntypes for a ghost), rv the type
    const int ncls = ntypes + (nlocal < n ? 1 : 0);
    int tv[PS_APT], rv[PS_APT];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < PS_APT; ++j) {
        const int a = tid + PS_THREADS * j;
        const int t0 = a < n ? atype[atom_off + a] : 0;
        bad |= t0 < 0 || t0 >= ntypes;
        rv[j] = clamp_type(t0, ntypes);
        tv[j] = a < n ? (a < nlocal ? rv[j] : ntypes) : -1;
    }
    if (!BATCH) {
        if (__ballot(bad) != 0 && lane == 0) atomicExch(&st->err_type, 1);
        for (int k = 0; k < ncls; ++k) {
            int v = 0;
#pragma unroll
            for (int j = 0; j < PS_APT; ++j) v += tv[j] == k;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) s_w[wid][k] = v;
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int k = 0; k < ncls; ++k) {
                int c = 0;
                for (int w = 0; w < PS_THREADS / 64; ++w) c += s_w[w][k];
                toff[k] = acc;
                tcount[k] = c;
                s_base[k] = acc;
                acc += c;
            }
            toff[ncls] = acc;
        }
        __syncthreads();
    }
    // stable partition by type: chunk j = atoms PS_THREADS j .. in caller order; this thread's
    // internal positions are kept for the next phase
    int qv[PS_APT];
#pragma unroll
    for (int j = 0; j < PS_APT; ++j) {
        qv[j] = -1;
        if (PS_THREADS * j >= n) continue;   // uniform
        const int a = tid + PS_THREADS * j;
        const int t = tv[j];
        unsigned long long mine = 0;
        for (int k = 0; k < (BATCH ? ntypes : ncls); ++k) {
            const unsigned long long m = __ballot(t == k);
            if (t == k) mine = m;
            if (lane == 0) s_w[wid][k] = __popcll(m);
        }
        __syncthreads();
        if (t >= 0) {
            int before = s_base[t];
            for (int w = 0; w < wid; ++w) before += s_w[w][t];
            const int q = before + __popcll(mine & lt);
            qv[j] = q;
            perm[q] = atom_off + a;
            inv_perm[atom_off + a] = q;
            itype[q] = rv[j];
            if (BATCH) frame_of[q] = f;
        }
        __syncthreads();
        if (tid < (BATCH ? ntypes : ncls)) {
            int c = 0;
            for (int w = 0; w < PS_THREADS / 64; ++w) c += s_w[w][tid];
            s_base[tid] += c;
        }
        __syncthreads();
    }
    // wrap and bin this thread's atoms (caller index atom_off + a, internal index qv[j]); zero the
    // frame's force (and, batched, virial) accumulators
    double xv[PS_APT][3];
#pragma unroll
    for (int j = 0; j < PS_APT; ++j) {
        const int a = atom_off + tid + PS_THREADS * j;
        for (int c = 0; c < 3; ++c) xv[j][c] = qv[j] >= 0 ? coord[3 * (size_t)a + c] : 0.0;
    }
    int cv[PS_APT];
#pragma unroll
    for (int j = 0; j < PS_APT; ++j) {
        cv[j] = -1;
        const int q = qv[j];
        if (q < 0) continue;
        double p[3];
        int b[3];
        wrap_bin_one(gp, xv[j], p, b);
        for (int c = 0; c < 3; ++c) {
            pos[3 * (size_t)q + c] = p[c];
            xv[j][c] = p[c];
            f_int[3 * (size_t)q + c] = 0.0;
        }
        if (BATCH)
            for (int k = 0; k < 9; ++k) vir_atom[9 * (size_t)q + k] = 0.0;
        const int cell = (b[2] * gp.nb[1] + b[1]) * gp.nb[0] + b[0];
        cell_of[q] = cell;
        cv[j] = cell;
        atomicAdd(&s_cnt[cell], 1);
    }
    __syncthreads();
    // exclusive scan of the bin counts: contiguous segments per thread, then a scan of the partials
    const int seg = (ncell + PS_THREADS - 1) / PS_THREADS;
    const int c0 = tid * seg, c1 = min(c0 + seg, ncell);
    int sum = 0;
    for (int c = c0; c < c1; ++c) sum += s_cnt[c];
    s_part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < PS_THREADS; o <<= 1) {
        const int v = tid >= o ? s_part[tid - o] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    int run = s_part[tid] - sum;
    for (int c = c0; c < c1; ++c) {
        const int v = s_cnt[c];
        cell_start[cell_off + c] = atom_off + run;
        s_cnt[c] = run;   // cursor
        run += v;
    }
    if (tid == 0) cell_start[cell_off + ncell] = atom_off + n;
    __syncthreads();
    // bin fill: candidate records in bin order (tag: internal index, caller index, type)
#pragma unroll
    for (int j = 0; j < PS_APT; ++j) {
        const int q = qv[j];
        if (q < 0) continue;
        const int slot = atomicAdd(&s_cnt[cv[j]], 1);
        const long long tag = (long long)q | ((long long)(atom_off + tid + PS_THREADS * j) << 30) |
                              ((long long)rv[j] << 60);
        cand[atom_off + slot] = make_double4(xv[j][0], xv[j][1], xv[j][2], __longlong_as_double(tag));
    }
}

// ---- preparation of larger frames in three launches ---------------------------------------
// Blocks of TP_BLOCK atoms in caller order.
//   k_prep_count: per-block type counts (types clamped; the scatter raises the error flag) and
//                 the bin of every atom, counted into cell_count with atomics. cell_count is zero
//                 on entry: k_prep_scan clears what it read, and the host clears the array after
//                 allocating it.
//   k_prep_scan (one block): clears the statistics block, scans the block type counts over blocks
//                 and the bin counts (bin starts and fill cursors), and clears the bin counts.
//   k_prep_scatter: the stable partition by type (ballot ranks within the block plus the block's
//                 base), the wrapped position and bin in internal order (wrap_bin_one again, the
//                 same bits as in k_prep_count), zeroed force accumulators, and the candidate
//                 record of every atom at the next free slot of its bin (the order within a bin
//                 is not fixed: the neighbour list sorts its hits by a key unique per candidate).
__global__ void __launch_bounds__(TP_BLOCK) k_prep_count(int n, int nlocal, const double* coord, const int* atype,
                                                         int ntypes, GeomParams gp, int* bcount, int* cell_tmp,
                                                         int* cell_count)
{
    __shared__ int h[MAXT];
    if (threadIdx.x < MAXT) h[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * TP_BLOCK + threadIdx.x;
    if (i < n) {
        atomicAdd(&h[i < nlocal ? clamp_type(atype[i], ntypes) : ntypes], 1);   // ghosts: one class after the types
        const double x[3] = {coord[3 * (size_t)i], coord[3 * (size_t)i + 1], coord[3 * (size_t)i + 2]};
        double p[3];
        int b[3];
        wrap_bin_one(gp, x, p, b);
        const int cell = (b[2] * gp.nb[1] + b[1]) * gp.nb[0] + b[0];
        cell_tmp[i] = cell;
        atomicAdd(&cell_count[cell], 1);
    }
    __syncthreads();
    if (threadIdx.x < MAXT) bcount[blockIdx.x * MAXT + threadIdx.x] = h[threadIdx.x];
}

// Exclusive scan of v[0..m) by one block of 1024 threads (passes of 1024 with a carry): out[i] =
// base + sum of v[0..i); returns the total to every thread. part holds 1024 ints of LDS.
__device__ int block_scan_1024(int m, const int* v, int vstride, int* out, int ostride, int base, int* part,
                               int* carry)
{
    const int tid = threadIdx.x;
    if (tid == 0) *carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < m; b0 += 1024) {
        const int i = b0 + tid;
        const int x = i < m ? v[(size_t)i * vstride] : 0;
        part[tid] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int add = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        if (i < m) out[(size_t)i * ostride] = base + *carry + part[tid] - x;
        __syncthreads();
        if (tid == 1023) *carry += part[1023];
        __syncthreads();
    }
    const int total = *carry;
    __syncthreads();   // every thread has read the total before the next scan resets it
    return total;
}

__global__ void __launch_bounds__(1024) k_prep_scan(int nblocks, int ntypes, const int* bcount, int* boff, int* toff,
                                                    int* tcount, int ncell, int* cell_count, int* cell_start,
                                                    int* cursor, DevStats* st)
{
    __shared__ int part[1024];
    __shared__ int carry;
    const int tid = threadIdx.x;
    for (int w = tid; w < STATS_WORDS; w += (int)blockDim.x) reinterpret_cast<int*>(st)[w] = 0;
    // types: block offsets within each type (type t's atoms follow those of types < t)
    int acc = 0;
    for (int t = 0; t < ntypes; ++t) {
        const int c = block_scan_1024(nblocks, bcount + t, MAXT, boff + t, MAXT, acc, part, &carry);
        if (tid == 0) {
            toff[t] = acc;
            tcount[t] = c;
        }
        acc += c;
    }
    if (tid == 0) toff[ntypes] = acc;
    // bins: starts and fill cursors; the counts are cleared for the next frame
    const int total = block_scan_1024(ncell, cell_count, 1, cell_start, 1, 0, part, &carry);
    for (int i = tid; i < ncell; i += 1024) {
        cursor[i] = cell_start[i];
        cell_count[i] = 0;
    }
    if (tid == 0) cell_start[ncell] = total;
}

__global__ void __launch_bounds__(TP_BLOCK) k_prep_scatter(int n, int nlocal, const double* coord, const int* atype,
                                                           int ntypes, GeomParams gp, const int* boff,
                                                           const int* cell_tmp, int* perm, int* inv_perm, int* itype,
                                                           double* pos, int* cell_of, int* cursor, double4* cand,
                                                           double* f_int, DevStats* st)
{
    __shared__ int wsum[TP_BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int i = blockIdx.x * TP_BLOCK + tid;
    const int ncls = ntypes + (nlocal < n ? 1 : 0);
    int t = -1, cls = -1;
    if (i < n) {
        const int t0 = atype[i];
        if (t0 < 0 || t0 >= ntypes) atomicExch(&st->err_type, 1);
        t = clamp_type(t0, ntypes);
        cls = i < nlocal ? t : ntypes;   // ghosts: one class after the types
    }
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int q = -1;
    for (int k = 0; k < ncls; ++k) {
        const bool f = (cls == k);
        const unsigned long long m = __ballot(f);
        if (lane == 0) wsum[wid] = __popcll(m);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wid; ++w) before += wsum[w];
        if (f) q = boff[blockIdx.x * MAXT + k] + before + __popcll(m & lt);
        __syncthreads();
    }
    if (q < 0) return;
    perm[q] = i;
    inv_perm[i] = q;
    itype[q] = t;
    const double x[3] = {coord[3 * (size_t)i], coord[3 * (size_t)i + 1], coord[3 * (size_t)i + 2]};
    double p[3];
    int b[3];
    wrap_bin_one(gp, x, p, b);
    const int cell = cell_tmp[i];
    for (int c = 0; c < 3; ++c) {
        pos[3 * (size_t)q + c] = p[c];
        f_int[3 * (size_t)q + c] = 0.0;
    }
    cell_of[q] = cell;
    const int slot = atomicAdd(&cursor[cell], 1);
    const long long tag = (long long)q | ((long long)i << 30) | ((long long)t << 60);
    cand[slot] = make_double4(p[0], p[1], p[2], __longlong_as_double(tag));
}

__global__ void __launch_bounds__(PS_THREADS) k_prep_small(int n, int nlocal, const double* coord, const int* atype,
                                                            int ntypes, GeomParams gp, int ncell, int* tcount,
                                                            int* toff, int* perm, int* inv_perm, int* itype,
                                                            DevStats* st, double* pos, int* cell_of, int* cell_start,
                                                            double4* cand, double* f_int)
{
    prep_frame<false>(0, n, nlocal, 0, coord, atype, ntypes, gp, ncell, 0, nullptr, tcount, toff, perm, inv_perm,
                      itype, nullptr, st, pos, cell_of, cell_start, cand, f_int, nullptr);
}

// ---- batched frames (serving): per-frame type counts, cross-frame type bases, per-frame prep --

__global__ void __launch_bounds__(256) k_batch_count(const int* atype, int ntypes, FrameDesc* fd)
{
    __shared__ int s_c[4][MAXT];
    __shared__ int s_bad[4];
    FrameDesc& d = fd[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int cnt[MAXT];
    for (int k = 0; k < MAXT; ++k) cnt[k] = 0;
    bool bad = false;
    for (int a = tid; a < d.natoms; a += 256) {
        const int t0 = atype[d.atom_off + a];
        bad |= t0 < 0 || t0 >= ntypes;
        const int t = clamp_type(t0, ntypes);
        for (int k = 0; k < MAXT; ++k) cnt[k] += t == k;
    }
    for (int k = 0; k < MAXT; ++k) {
        int v = cnt[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) s_c[wid][k] = v;
    }
    if (lane == 0) s_bad[wid] = __ballot(bad) != 0;
    __syncthreads();
    if (tid < MAXT) d.type_base[tid] = s_c[0][tid] + s_c[1][tid] + s_c[2][tid] + s_c[3][tid];
    if (tid == 0) d.bad = s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3];
}

// Per-type totals and each frame's internal base per type (atoms sorted by type over the whole
// batch, frames in order within a type); zeroes the statistics block of the batch.
__global__ void k_batch_scan(int nframes, int ntypes, FrameDesc* fd, int* tcount, int* toff, DevStats* st)
{
    for (int w = threadIdx.x; w < STATS_WORDS; w += (int)blockDim.x) reinterpret_cast<int*>(st)[w] = 0;
    __syncthreads();
    if (threadIdx.x != 0) return;
    int acc = 0, bad = 0;
    for (int t = 0; t < ntypes; ++t) {
        toff[t] = acc;
        int c = 0;
        for (int f = 0; f < nframes; ++f) {
            const int v = fd[f].type_base[t];
            fd[f].type_base[t] = acc + c;
            c += v;
        }
        tcount[t] = c;
        acc += c;
    }
    toff[ntypes] = acc;
    for (int f = 0; f < nframes; ++f) bad |= fd[f].bad;
    if (bad) st->err_type = 1;
}

__global__ void __launch_bounds__(PS_THREADS) k_prep_batch(const double* coord, const int* atype, int ntypes,
                                                            const GeomParams* gps, const FrameDesc* fd, int* perm,
                                                            int* inv_perm, int* itype, int* frame_of, double* pos,
                                                            int* cell_of, int* cell_start, double4* cand, double* f_int,
                                                            double* vir_atom)
{
    const int f = blockIdx.x;
    const FrameDesc& d = fd[f];
    prep_frame<true>(f, d.natoms, d.natoms, d.atom_off, coord, atype, ntypes, gps[f], d.ncell, d.cell_off, d.type_base,
                     nullptr, nullptr, perm, inv_perm, itype, frame_of, nullptr, pos, cell_of, cell_start, cand, f_int,
                     vir_atom);
}

// ---- neighbour list: one wave per centre atom --------------------------------------------
// Candidate records are stored in bin order (by the preparation): position and a tag holding the
// internal index, the caller index and the type (30 + 30 + 4 bits), so one 32-B load gives
// everything the candidate test and the output need.
// The wave first loads the ranges of all stencil bins at once (one lane per bin) and scans their
// sizes; it then sweeps the flat candidate range, several candidates per lane in flight (each
// lane finds its candidate's bin by binary search in the scanned offsets).
// Candidates within r_c are compacted into LDS as 128-bit keys that compare like
// (type, r^2, caller index j, image n0, n1, n2):
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

constexpr int NL_UNROLL = 4;
constexpr int RANK_MAX = 256;   // hits per atom up to which the neighbour list ranks instead of sorting

// Ordering of LDS traffic between the lanes of the (single-wave) workgroup.
__device__ __forceinline__ void wave_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Rank sort of count <= RANK_MAX keys in LDS, EA = ceil(count / 64) of them per lane (key lane +
// 64 e): a key's position is the number of smaller keys, counted against every stored key read once
// from LDS (one broadcast per key, no exchange chain). The high words decide unless two are equal
// (equal type and r^2 to 2^-47, i.e. in practice equal distances): equal ranks then collide in a
// slot check and the ranks are recounted on the full 128-bit keys, which are unique. The keys end
// sorted in LDS.
template <int EA>
__device__ __forceinline__ void rank_keys(int count, int lane, unsigned long long* khi, unsigned long long* klo,
                                          int* kq)
{
    unsigned long long kh[EA], kl[EA];
    int kx[EA], rk[EA];
#pragma unroll
    for (int e = 0; e < EA; ++e) {
        const int i = lane + 64 * e;
        const bool have = i < count;
        kh[e] = have ? khi[i] : ~0ull;
        kl[e] = have ? klo[i] : ~0ull;
        kx[e] = have ? kq[i] : 0;
        rk[e] = 0;
    }
    for (int q = 0; q < count; ++q) {
        const unsigned long long h = khi[q];
#pragma unroll
        for (int e = 0; e < EA; ++e) rk[e] += h < kh[e] ? 1 : 0;
    }
    wave_barrier();
#pragma unroll
    for (int e = 0; e < EA; ++e)
        if (lane + 64 * e < count) kq[rk[e]] = lane + 64 * e;
    wave_barrier();
    bool clash = false;
#pragma unroll
    for (int e = 0; e < EA; ++e)
        if (lane + 64 * e < count) clash |= kq[rk[e]] != lane + 64 * e;
    if (__ballot(clash) != 0) {
#pragma unroll
        for (int e = 0; e < EA; ++e) rk[e] = 0;
        for (int q = 0; q < count; ++q) {
            const unsigned long long h = khi[q], l = klo[q];
#pragma unroll
            for (int e = 0; e < EA; ++e) rk[e] += key_less(h, l, kh[e], kl[e]) ? 1 : 0;
        }
    }
    wave_barrier();
#pragma unroll
    for (int e = 0; e < EA; ++e)
        if (lane + 64 * e < count) {
            khi[rk[e]] = kh[e];
            klo[rk[e]] = kl[e];
            kq[rk[e]] = kx[e];
        }
    wave_barrier();
}

// Bitonic sort in LDS of count keys (padded to a power of two with keys that order last): the path
// for more than RANK_MAX atoms within r_c, rare, kept out of registers so that the buffer size does
// not set the kernel's register count.
__device__ void bitonic_keys_lds(int count, int lane, unsigned long long* khi, unsigned long long* klo, int* kq)
{
    int n2 = 64;
    while (n2 < count) n2 <<= 1;
    for (int i = count + lane; i < n2; i += 64) {
        khi[i] = ~0ull;
        klo[i] = ~0ull;
        kq[i] = 0;
    }
    wave_barrier();
    for (int k = 2; k <= n2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = lane; p < (n2 >> 1); p += 64) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));   // p with a zero bit inserted at j
                const int l = i | j;
                const bool up = (i & k) == 0;
                const unsigned long long ih = khi[i], il = klo[i], lh = khi[l], ll = klo[l];
                if (key_less(lh, ll, ih, il) == up) {
                    const int ix = kq[i];
                    khi[i] = lh; klo[i] = ll; kq[i] = kq[l];
                    khi[l] = ih; klo[l] = il; kq[l] = ix;
                }
            }
            wave_barrier();
        }
}

// The selection of one atom's list from its count hits (keys in LDS: type, r^2, caller index,
// image code; kq the candidate each key came from; tcount the hits per type, which may exceed the
// CAP stored keys): keys sorted in LDS, the first sel[t] of each type block written to row a of
// the list (fetch(kq, code, r, j) gives the candidate's r_ij and caller index), padding -1, the
// kept counts, and the neighbours dropped by sel.
template <int CAP, class Fetch>
__device__ __forceinline__ void nlist_select(int a, int lane, int count, int* tcount, const GeomParams& gp,
                                             unsigned long long* khi, unsigned long long* klo, int* kq, int* nl_j,
                                             double* nl_r, int* nnei, DevStats* st, Fetch&& fetch)
{
    // one word shared by every atom: only the few atoms that raise the maximum touch it atomically
    if (lane == 0 && count > __atomic_load_n(&st->max_cand, __ATOMIC_RELAXED)) {
        atomicMax(&st->max_cand, count);
        if (count > CAP) atomicExch(&st->err_overflow, 1);
    }
    const bool overflow = count > CAP;   // wave-uniform; the frame is flagged and its list incomplete
    if (overflow) count = CAP;
    __syncthreads();
    // the keys are put in order in LDS
    static_assert(RANK_MAX <= 256, "rank sort dispatch covers at most four keys per lane");
    if (count <= RANK_MAX) {
        const int ER = (count + 63) >> 6;
        if (ER <= 1) rank_keys<1>(count, lane, khi, klo, kq);
        else if (ER == 2) rank_keys<2>(count, lane, khi, klo, kq);
        else if (ER == 3) rank_keys<3>(count, lane, khi, klo, kq);
        else rank_keys<4>(count, lane, khi, klo, kq);
    } else {
        bitonic_keys_lds(count, lane, khi, klo, kq);
    }
    // per-type counts of the sorted keys: every hit, unless the buffer overflowed; then only the
    // stored hits count, so that each type block starts where its keys do and every slot the
    // list claims is written (the overflowed frame is reported and not used)
    int tsorted[MAXT];
    for (int t = 0; t < gp.ntypes; ++t) tsorted[t] = tcount[t];
    if (overflow) {
        for (int t = 0; t < gp.ntypes; ++t) {
            int c = 0;
            for (int q0 = 0; q0 < count; q0 += 64) {
                const int q = q0 + lane;
                c += __popcll(__ballot(q < count && (int)(khi[q] >> 59) == t));
            }
            tsorted[t] = c;
        }
    }
    int tstart[MAXT], kept[MAXT];
    int acc = 0, drops = 0;
    for (int t = 0; t < gp.ntypes; ++t) {
        tstart[t] = acc;
        acc += tsorted[t];
        kept[t] = tsorted[t] < gp.sel[t] ? tsorted[t] : gp.sel[t];
        drops += tcount[t] - kept[t];
    }
    const size_t rowj = (size_t)a * gp.nc;
    for (int q = lane; q < count; q += 64) {
        const unsigned long long kh = khi[q], kl = klo[q];
        const int t = (int)(kh >> 59);
        const int rank = q - tstart[t];
        if (rank < gp.sel[t]) {
            double r[3];
            int j;
            fetch(kq[q], (int)(kl & ((1ull << 21) - 1)), r, j);
            const size_t slot = rowj + gp.off[t] + rank;
            nl_j[slot] = j;
            nl_r[3 * slot + 0] = r[0];
            nl_r[3 * slot + 1] = r[1];
            nl_r[3 * slot + 2] = r[2];
        }
    }
    for (int s2 = lane; s2 < gp.nc; s2 += 64) {
        int t = 0;
        while (t + 1 < gp.ntypes && s2 >= gp.off[t + 1]) ++t;
        if (s2 - gp.off[t] >= kept[t]) {
            nl_j[rowj + s2] = -1;
            for (int c = 0; c < 3; ++c) nl_r[3 * (rowj + s2) + c] = 0.0;
        }
    }
    if (lane < gp.ntypes) nnei[(size_t)a * gp.ntypes + lane] = kept[lane];
    if (lane == 0 && drops) atomicAdd(drop_slots(st) + (a & (NL_DROP_SLOTS - 1)), (unsigned long long)drops);
}

// BATCH: atom a belongs to frame frame_of[a]; its geometry is gps[frame] and its bins start at
// fd[frame].cell_off of the concatenated cell_start (candidate records hold batch-wide indices).
template <int CAP, bool BATCH>
__global__ void __launch_bounds__(64) k_nlist(int n, const double* pos, const int* perm, const int* inv_perm,
                                              const int* cell_of, const int* cell_start0, const double4* cand,
                                              GeomParams gp0, const GeomParams* gps, const FrameDesc* fd,
                                              const int* frame_of, int* nl_j, double* nl_r, int* nnei, DevStats* st)
{
    const int fr = BATCH ? frame_of[blockIdx.x] : 0;
    const GeomParams& gp = BATCH ? gps[fr] : gp0;
    const int* cell_start = BATCH ? cell_start0 + fd[fr].cell_off : cell_start0;
    // LDS sized per launch (nlist_lds_bytes): keys of CAP candidates, then the stencil tables
    extern __shared__ __attribute__((aligned(16))) unsigned long long nl_lds[];
    unsigned long long* khi = nl_lds;
    unsigned long long* klo = khi + CAP;
    const int S = (2 * gp.K[0] + 1) * (2 * gp.K[1] + 1) * (2 * gp.K[2] + 1);
    double* s_sh = reinterpret_cast<double*>(klo + CAP);   // [S][3] image shift of each stencil bin
    int* kq = reinterpret_cast<int*>(s_sh + 3 * S);       // flat candidate index, moved with its key
    int* s_base = kq + CAP;                        // [S + 1]
    int* s_start = s_base + S + 1;                 // [S]
    int* s_code = s_start + S;                     // [S]
    const int a = blockIdx.x, lane = threadIdx.x;
    const double pi[3] = {pos[3 * (size_t)a], pos[3 * (size_t)a + 1], pos[3 * (size_t)a + 2]};
    const long long self_tag = (long long)a;
    const int ci = cell_of[a];
    const int bi[3] = {ci % gp.nb[0], (ci / gp.nb[0]) % gp.nb[1], ci / (gp.nb[0] * gp.nb[1])};
    const int w1 = 2 * gp.K[1] + 1, w2 = 2 * gp.K[2] + 1;
    const int self_code = (64 << 14) | (64 << 7) | 64;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // ranges of every stencil bin, scanned across the wave
    int total = 0;   // wave-uniform
    // stencil index -> offsets: divisions by w2 and w1 w2 (at most 49) of an index below 343 as a
    // multiply by ceil(2^16 / d) and a shift, exact in that range
    const unsigned m2 = (65536u + w2 - 1) / w2, m12 = (65536u + w1 * w2 - 1) / (w1 * w2);
    for (int sb = 0; sb < S; sb += 64) {
        const int sidx = sb + lane;
        int cnt = 0, start = 0, code = 0;
        if (sidx < S) {
            const int d12 = (int)(((unsigned)sidx * m12) >> 16), d2 = (int)(((unsigned)sidx * m2) >> 16);
            const int o0 = d12 - gp.K[0];
            const int o1 = d2 - d12 * w1 - gp.K[1];
            const int o2 = sidx - d2 * w2 - gp.K[2];
            const int tg[3] = {bi[0] + o0, bi[1] + o1, bi[2] + o2};
            int nn[3], bb[3];
            bool skip = false;
            for (int c = 0; c < 3; ++c) {
                if (gp.periodic) {
                    // image (floor division by the bins per axis); at least K bins per axis leave
                    // tg within one box length of the cell, so the image is -1, 0 or 1
                    int q;
                    if (gp.nb[c] >= gp.K[c]) {
                        q = tg[c] < 0 ? -1 : (tg[c] >= gp.nb[c] ? 1 : 0);
                    } else {
                        q = tg[c] / gp.nb[c];
                        if ((tg[c] % gp.nb[c] != 0) && (tg[c] < 0)) --q;
                    }
                    nn[c] = q;
                    bb[c] = tg[c] - q * gp.nb[c];
                } else {
                    nn[c] = 0;
                    bb[c] = tg[c];
                    if (tg[c] < 0 || tg[c] >= gp.nb[c]) skip = true;
                }
            }
            code = ((nn[0] + 64) << 14) | ((nn[1] + 64) << 7) | (nn[2] + 64);
            if (!skip) {
                const int cell = (bb[2] * gp.nb[1] + bb[1]) * gp.nb[0] + bb[0];
                start = cell_start[cell];
                cnt = cell_start[cell + 1] - start;
            }
        }
        int incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (sidx < S) {
            s_base[sidx] = total + incl - cnt;
            s_start[sidx] = start;
            s_code[sidx] = code;
            // the bin's image shift, once (the same expression the output uses, so the same bits)
            double sh[3];
            image_shift(gp, (code >> 14) - 64, ((code >> 7) & 127) - 64, (code & 127) - 64, sh);
            for (int c = 0; c < 3; ++c) s_sh[3 * sidx + c] = sh[c];
        }
        total += __shfl(incl, 63);
    }
    if (lane == 0) s_base[S] = total;
    __syncthreads();

    int count = 0;   // wave-uniform
    int tcount[MAXT];   // wave-uniform, per type (may exceed CAP)
    for (int t = 0; t < MAXT; ++t) tcount[t] = 0;
    int b = 0;       // this lane's current stencil bin
    for (int q0 = 0; q0 < total; q0 += 64 * NL_UNROLL) {
        double4 c4[NL_UNROLL];
        int bin[NL_UNROLL], cq[NL_UNROLL];
#pragma unroll
        for (int u = 0; u < NL_UNROLL; ++u) {
            const int q = q0 + 64 * u + lane;
            bin[u] = -1;
            if (q < total) {
                // bin of flat candidate q: the last b with s_base[b] <= q (s_base is non-decreasing
                // with s_base[S] = total > q); q only grows, so the search starts at the last bin
                int hi = S;
                while (hi - b > 1) {
                    const int mid = (b + hi) >> 1;
                    if (s_base[mid] <= q) b = mid;
                    else hi = mid;
                }
                bin[u] = b;
                cq[u] = s_start[b] + (q - s_base[b]);
                c4[u] = cand[cq[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < NL_UNROLL; ++u) {
            bool pass = false;
            double r2 = 0.0;
            long long tag = 0;
            int code = 0;
            if (bin[u] >= 0) {
                code = s_code[bin[u]];
                tag = __double_as_longlong(c4[u].w);
                const double* sh = s_sh + 3 * bin[u];
                if (!((tag & 0x3fffffffll) == self_tag && code == self_code)) {
                    const double d0 = (c4[u].x + sh[0]) - pi[0];
                    const double d1 = (c4[u].y + sh[1]) - pi[1];
                    const double d2 = (c4[u].z + sh[2]) - pi[2];
                    r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    pass = r2 < gp.rc2;
                }
            }
            const unsigned long long m = __ballot(pass);
            const int tj = (int)((unsigned long long)tag >> 60);
            if (pass) {
                const int idx = count + __popcll(m & lt);
                if (idx < CAP) {
                    const unsigned long long jo = ((unsigned long long)tag >> 30) & 0x3fffffffull;
                    const unsigned long long rb = (unsigned long long)__double_as_longlong(r2);
                    khi[idx] = ((unsigned long long)tj << 59) | (rb >> 5);
                    klo[idx] = ((rb & 31ull) << 59) | (jo << 21) | (unsigned long long)code;
                    kq[idx] = cq[u];
                }
            }
            // per-type counts from ballots (no shared-word atomics)
            for (int t = 0; t < gp.ntypes; ++t) tcount[t] += __popcll(__ballot(pass && tj == t));
            count += __popcll(m);
        }
    }
    nlist_select<CAP>(a, lane, count, tcount, gp, khi, klo, kq, nl_j, nl_r, nnei, st,
                      [&](int q, int code, double* r, int& j) {
                          const int n0 = (code >> 14) - 64, n1 = ((code >> 7) & 127) - 64, n2 = (code & 127) - 64;
                          const double4 c4 = cand[q];
                          j = (int)((__double_as_longlong(c4.w) >> 30) & 0x3fffffffll);   // caller index
                          double sh[3];
                          image_shift(gp, n0, n1, n2, sh);
                          r[0] = (c4.x + sh[0]) - pi[0];
                          r[1] = (c4.y + sh[1]) - pi[1];
                          r[2] = (c4.z + sh[2]) - pi[2];
                      });
}

// External neighbour candidates (an MD code's own list, with or without a skin; Sec. III.B.2):
// owned atom a (internal index, caller index i = perm[a]) takes the candidates
// ext[ext_start[i] .. ext_start[i + 1]), caller indices of owned or ghost atoms in any order,
// without duplicates. Positions are used as given (open geometry: a ghost carries the image
// position its owner's domain sent), so r_ij = r_j - r_i; those within r_c are ordered by (type,
// distance, index) and selected exactly as k_nlist does. Indices outside [0, ntot) and the atom
// itself are skipped (the host entry point rejects such lists before the launch).
template <int CAP>
__global__ void __launch_bounds__(64) k_nlist_ext(int ntot, const double* pos, const int* perm, const int* inv_perm,
                                                  const int* itype, const int* ext_start, const int* ext,
                                                  GeomParams gp, int* nl_j, double* nl_r, int* nnei, DevStats* st)
{
    extern __shared__ __attribute__((aligned(16))) unsigned long long nl_lds[];
    unsigned long long* khi = nl_lds;
    unsigned long long* klo = khi + CAP;
    int* kq = reinterpret_cast<int*>(klo + CAP);   // internal index of the candidate, moved with its key
    const int a = blockIdx.x, lane = threadIdx.x;
    const int ci = perm[a];
    const double pi[3] = {pos[3 * (size_t)a], pos[3 * (size_t)a + 1], pos[3 * (size_t)a + 2]};
    const int b0 = ext_start[ci], b1 = ext_start[ci + 1];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int count = 0;   // wave-uniform
    int tcount[MAXT];
    for (int t = 0; t < MAXT; ++t) tcount[t] = 0;
    for (int q0 = b0; q0 < b1; q0 += 64) {
        const int q = q0 + lane;
        bool pass = false;
        double r2 = 0.0;
        int tj = 0, j = -1, jq = 0;
        if (q < b1) {
            j = ext[q];
            if (j >= 0 && j < ntot && j != ci) {
                jq = inv_perm[j];
                tj = itype[jq];
                const double d0 = pos[3 * (size_t)jq] - pi[0];
                const double d1 = pos[3 * (size_t)jq + 1] - pi[1];
                const double d2 = pos[3 * (size_t)jq + 2] - pi[2];
                r2 = d0 * d0 + d1 * d1 + d2 * d2;
                pass = r2 < gp.rc2;
            }
        }
        const unsigned long long m = __ballot(pass);
        if (pass) {
            const int idx = count + __popcll(m & lt);
            if (idx < CAP) {
                const unsigned long long rb = (unsigned long long)__double_as_longlong(r2);
                khi[idx] = ((unsigned long long)tj << 59) | (rb >> 5);
                klo[idx] = ((rb & 31ull) << 59) | ((unsigned long long)j << 21);   // no image: code 0
                kq[idx] = jq;
            }
        }
        for (int t = 0; t < gp.ntypes; ++t) tcount[t] += __popcll(__ballot(pass && tj == t));
        count += __popcll(m);
    }
    nlist_select<CAP>(a, lane, count, tcount, gp, khi, klo, kq, nl_j, nl_r, nnei, st,
                      [&](int q, int, double* r, int& jj) {
                          jj = perm[q];
                          for (int c = 0; c < 3; ++c) r[c] = pos[3 * (size_t)q + c] - pi[c];
                      });
}

// ---- reductions and output ----------------------------------------------------------------

// Compensated (Neumaier) running sum: the error of a long sum stays about one rounding of the
// result instead of growing with the number of terms (this file is built without FMA contraction,
// which the compensation relies on).
struct NeumaierSum {
    double s = 0.0, c = 0.0;
    __device__ void add(double x) {
        const double t = s + x;
        c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ double value() const { return s + c; }
};

// Single frame: E and the virial from the embedding backward's block partials [E, virial[9]], in a
// fixed order with compensated sums: thread t < 250 sums component t % 10 of the partials t / 10,
// t / 10 + 25, ..., then ten threads add their component's 25 sums. Also the frame's count of
// neighbours dropped by sel from its per-atom counters (one wave, lane = its lane index).
__device__ void sum_drop_slots(DevStats* st, int lane)
{
    const unsigned long long* ds = drop_slots(st);
    unsigned long long v = 0;
    for (int i = lane; i < NL_DROP_SLOTS; i += 64) v += ds[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) st->nbr_dropped = v;
}

__global__ void __launch_bounds__(256) k_finalize(int nb, const double* part, double* energy, double* virial,
                                                  DevStats* st)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    NeumaierSum v;
    if (t < 250)
        for (int i = t; i < 10 * nb; i += 250) v.add(part[i]);
    red[t] = v.value();
    __syncthreads();
    if (t < 10) {
        NeumaierSum x;
        for (int k = t; k < 250; k += 10) x.add(red[k]);
        if (t == 0) *energy = x.value();
        else virial[t - 1] = x.value();
    }
    if (t >= 192) sum_drop_slots(st, t - 192);   // the fourth wave, beside the ten sums above
}

// Batched frames: per frame (one block each) E = sum E_i and the virial = sum over the frame's
// atoms of their per-atom virial, both in a fixed order, and the frame's forces (and E_i) in its
// caller order. Output of frame f at out + out_off: E, virial[9], F[3n], E_i[n].
__global__ void __launch_bounds__(256) k_finalize_batch(const FrameDesc* fd, const int* inv_perm, const double* ei,
                                                        const double* vir_atom, const double* f_int, double* out,
                                                        DevStats* st)
{
    __shared__ double red[10][256];
    const FrameDesc& d = fd[blockIdx.x];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < 64) sum_drop_slots(st, tid);   // one count for the batch
    double* o = out + d.out_off;
    double acc[10];
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    for (int a = tid; a < d.natoms; a += 256) {
        const int q = inv_perm[d.atom_off + a];
        acc[0] += ei[q];
        for (int k = 0; k < 9; ++k) acc[1 + k] += vir_atom[9 * (size_t)q + k];
        for (int c = 0; c < 3; ++c) o[10 + 3 * (size_t)a + c] = f_int[3 * ((size_t)d.atom_off + a) + c];
        if (d.want_ei) o[10 + 3 * (size_t)d.natoms + a] = ei[q];
    }
    for (int k = 0; k < 10; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < 10; ++k) red[k][tid] += red[k][tid + w];
        __syncthreads();
    }
    if (tid < 10) o[tid] = red[tid][0];
}

// Debug: neighbour list (caller numbering already), rows in caller order.
__global__ void k_debug_nlist(int n, int ncentre, int nc, const int* perm, const int* nl_j, int* out)
{
    int a = blockIdx.x;
    int i = perm[a];
    // atoms past the centres (ghost atoms) have no list
    for (int s = threadIdx.x; s < nc; s += blockDim.x) out[(size_t)i * nc + s] = a < ncentre ? nl_j[(size_t)a * nc + s] : -1;
}

// ---- launchers --------------------------------------------------------------------------

void launch_prep_large(int n, const double* coord, const int* atype, int ntypes, const GeomParams& gp, int* tcount,
                       int* toff, int* bcount, int* boff, int* perm, int* inv_perm, int* itype, DevStats* st,
                       double* pos, int* cell_of, int* cell_count, int* cell_start, int* cursor, int* cell_tmp,
                       double4* cand, double* f_int, hipStream_t s, int nlocal)
{
    if (nlocal < 0) nlocal = n;
    const int nb = (n + TP_BLOCK - 1) / TP_BLOCK;
    const int ncell = gp.nb[0] * gp.nb[1] * gp.nb[2];
    const int ncls = ntypes + (nlocal < n ? 1 : 0);
    hipLaunchKernelGGL(k_prep_count, dim3(nb), dim3(TP_BLOCK), 0, s, n, nlocal, coord, atype, ntypes, gp, bcount,
                       cell_tmp, cell_count);
    hipLaunchKernelGGL(k_prep_scan, dim3(1), dim3(1024), 0, s, nb, ncls, bcount, boff, toff, tcount, ncell,
                       cell_count, cell_start, cursor, st);
    hipLaunchKernelGGL(k_prep_scatter, dim3(nb), dim3(TP_BLOCK), 0, s, n, nlocal, coord, atype, ntypes, gp, boff,
                       cell_tmp, perm, inv_perm, itype, pos, cell_of, cursor, cand, f_int, st);
}

bool launch_prep_small(int n, const double* coord, const int* atype, int ntypes, const GeomParams& gp, int* tcount,
                       int* toff, int* perm, int* inv_perm, int* itype, DevStats* st, double* pos, int* cell_of,
                       int* cell_start, double4* cand, double* f_int, hipStream_t s, int nlocal)
{
    if (nlocal < 0) nlocal = n;
    const int ncell = gp.nb[0] * gp.nb[1] * gp.nb[2];
    if (n > PS_MAX_ATOMS || ncell > PS_MAX_CELLS) return false;
    hipLaunchKernelGGL(k_prep_small, dim3(1), dim3(PS_THREADS), 0, s, n, nlocal, coord, atype, ntypes, gp, ncell,
                       tcount, toff, perm, inv_perm, itype, st, pos, cell_of, cell_start, cand, f_int);
    return true;
}

void launch_batch_prep(int nframes, int ntypes, const double* coord, const int* atype, const GeomParams* gps,
                       FrameDesc* fd, int* tcount, int* toff, int* perm, int* inv_perm, int* itype, int* frame_of,
                       DevStats* st, double* pos, int* cell_of, int* cell_start, double4* cand, double* f_int,
                       double* vir_atom, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_count, dim3(nframes), dim3(256), 0, s, atype, ntypes, fd);
    hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(64), 0, s, nframes, ntypes, fd, tcount, toff, st);
    hipLaunchKernelGGL(k_prep_batch, dim3(nframes), dim3(PS_THREADS), 0, s, coord, atype, ntypes, gps, fd, perm,
                       inv_perm, itype, frame_of, pos, cell_of, cell_start, cand, f_int, vir_atom);
}

void launch_finalize(int nb, const double* part, double* energy, double* virial, DevStats* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, nb, part, energy, virial, st);
}

void launch_finalize_batch(int nframes, const FrameDesc* fd, const int* inv_perm, const double* ei,
                           const double* vir_atom, const double* f_int, double* out, DevStats* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_batch, dim3(nframes), dim3(256), 0, s, fd, inv_perm, ei, vir_atom, f_int, out, st);
}

int prep_small_max_atoms() { return PS_MAX_ATOMS; }
int prep_small_max_cells() { return PS_MAX_CELLS; }

void launch_bbox(int n, const double* coord, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, s, n, coord, out);
}

void launch_nlist(int n, const double* pos, const int* perm, const int* inv_perm, const int* cell_of,
                  const int* cell_start, const double4* cand, const GeomParams& gp, int* nl_j, double* nl_r,
                  int* nnei, DevStats* st, hipStream_t s, const GeomParams* gps, const FrameDesc* fd,
                  const int* frame_of, int max_stencil, int max_cap)
{
    // candidate buffer sized from the expected count within r_c (the synchronous entry point reruns
    // a frame that overflowed with the largest buffer); LDS = 20 B per candidate slot + 36 B per
    // stencil bin, so small stencils leave room for more resident waves. A batch passes the
    // largest stencil and buffer of its frames.
    const bool batch = gps != nullptr;
    const int S = batch ? max_stencil : (2 * gp.K[0] + 1) * (2 * gp.K[1] + 1) * (2 * gp.K[2] + 1);
    const int want = batch ? max_cap : gp.cap;
    const int cap = want <= 256 ? 256 : (want <= 512 ? 512 : NL_CAP);
    const size_t lds = (size_t)cap * 20 + (size_t)S * 24 + (size_t)(3 * S + 1) * 4;
#define DPK_NL(C, B)                                                                                              \
    hipLaunchKernelGGL((k_nlist<C, B>), dim3(n), dim3(64), lds, s, n, pos, perm, inv_perm, cell_of, cell_start,   \
                       cand, gp, gps, fd, frame_of, nl_j, nl_r, nnei, st)
    if (batch) {
        if (cap == 256) DPK_NL(256, true);
        else if (cap == 512) DPK_NL(512, true);
        else DPK_NL(NL_CAP, true);
    } else {
        if (cap == 256) DPK_NL(256, false);
        else if (cap == 512) DPK_NL(512, false);
        else DPK_NL(NL_CAP, false);
    }
#undef DPK_NL
}

// Model deviation of the forces (Sec. II.C): over the nm models of an ensemble (ensemble averages
// with weight 1/nm), eps_i = sqrt(< |F_i - <F_i>|^2 >); with nu >= 0 the relative form
// eps_i / (|<F_i>| + nu). F holds model k's forces (caller order) at F + k * stride doubles.
__global__ void k_force_devi(int n, int nm, const double* F, int64_t stride, double nu, double* eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int k = 0; k < nm; ++k) {
        const double* f = F + k * stride + 3 * (size_t)i;
        m0 += f[0];
        m1 += f[1];
        m2 += f[2];
    }
    const double inv = 1.0 / nm;
    m0 *= inv;
    m1 *= inv;
    m2 *= inv;
    double v = 0.0;
    for (int k = 0; k < nm; ++k) {
        const double* f = F + k * stride + 3 * (size_t)i;
        const double d0 = f[0] - m0, d1 = f[1] - m1, d2 = f[2] - m2;
        v += d0 * d0 + d1 * d1 + d2 * d2;
    }
    double e = sqrt(v * inv);
    if (nu >= 0.0) e /= sqrt(m0 * m0 + m1 * m1 + m2 * m2) + nu;
    eps[i] = e;
}

void launch_force_devi(int n, int nm, const double* F, int64_t stride, double nu, double* eps, hipStream_t s)
{
    hipLaunchKernelGGL(k_force_devi, dim3((n + 255) / 256), dim3(256), 0, s, n, nm, F, stride, nu, eps);
}

void launch_nlist_ext(int nlocal, int ntot, const double* pos, const int* perm, const int* inv_perm, const int* itype,
                      const int* ext_start, const int* ext, const GeomParams& gp, int* nl_j, double* nl_r, int* nnei,
                      DevStats* st, hipStream_t s)
{
    const size_t lds = (size_t)NL_CAP * 20;
    hipLaunchKernelGGL((k_nlist_ext<NL_CAP>), dim3(nlocal), dim3(64), lds, s, ntot, pos, perm, inv_perm, itype,
                       ext_start, ext, gp, nl_j, nl_r, nnei, st);
}

void launch_debug_nlist(int n, int ncentre, int nc, const int* perm, const int* nl_j, int* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_nlist, dim3(n), dim3(64), 0, s, n, ncentre, nc, perm, nl_j, out);
}

}  // namespace dpk
