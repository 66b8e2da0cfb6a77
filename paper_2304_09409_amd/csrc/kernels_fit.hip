// kernels_fit.hip -- fitting net of the BF16 paths (split BF16 and plain BF16).
//
// Fitting net F_0 (Sec. II.A.2, eq. fitting_energy) for every atom, forward E_i and the input
// gradient dE_i/dT through D = T T_<^T (Sec. II.A.1). The products run on
// v_mfma_f32_16x16x32_bf16, which issues twice the K of the 16x16x16 form in the same cycles.
//
// Work split: a block holds NAT tiles of 16 atoms and four waves; wave w owns the 16-row feature
// tiles w, w+4, w+8, w+12 (< 15) of every layer for all atoms of the block, and in the backward
// dD product the D-row tiles w, w+4, ... Weights are read by exactly one wave each, straight from
// global memory (fragment-major, one coalesced 1 KB load per plane), one K-chunk ahead. The B
// operands (D for layer 1, then h_l or ga_l) are shared through LDS as split BF16 fragments; a
// layer's output tiles 2c and 2c+1 fill the two halves of K-chunk c of the next layer (the
// weights' K order matches, see XF_* in dpk_internal.h). D is formed from T by the wave that owns
// the atom tile, a group of K-chunks ahead, so layer 1 has one barrier per group.
// Blocks are placed so that each XCD (block b runs on XCD b % 8) works on a contiguous range of
// atoms: with atoms sorted by species, an XCD's L2 mostly holds one species' weights.
#include <hip/hip_runtime.h>
#include "dpk_internal.h"
#include "dpk_launch.h"

namespace dpk {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct F8 {
    bf8 h, l;
};

constexpr int FX_G = 4;    // layer-1 K-chunks per D group
#ifndef FITX_PD
#define FITX_PD 4          // weight lookahead (K-chunks) of the 32-atom block shape
#endif

// FP32 hyperbolic tangent on the hardware exp2 and reciprocal: 1 - 2 / (2^(2x log2 e) + 1).
__device__ __forceinline__ float fx_tanh(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.885390081777927f);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// acc += a b with a, b split as hi + lo: lo*hi + hi*lo + hi*hi (SPLIT), or hi*hi only.
template <bool SPLIT>
__device__ __forceinline__ void mma32(f4& c, const F8& a, const F8& b)
{
    if constexpr (SPLIT) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    }
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}

// One lane's part of a fragment: hi at lane*8, lo at 512 + lane*8 (global memory or LDS).
template <bool SPLIT>
__device__ __forceinline__ F8 ld_frag(const __bf16* f, int lane)
{
    F8 r;
    r.h = *reinterpret_cast<const bf8*>(f + lane * 8);
    if constexpr (SPLIT) r.l = *reinterpret_cast<const bf8*>(f + 512 + lane * 8);
    else r.l = bf8{};
    return r;
}

// Buffer-resource loads of the (read-only) weights: the per-lane part of an address is one VGPR
// offset (lane * 16 B) shared by all loads, the fragment offset a scalar. Keeps 64-bit per-lane
// addresses out of the register file; loads past num_records read 0.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
// Weight fragment f of the buffer r (fragment-major, XF_ELEMS BF16 values = 2 KB each).
template <bool SPLIT>
__device__ __forceinline__ F8 ld_wfrag(rsrc_t r, int lane16, int f)
{
    F8 x;
    x.h = __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(r, lane16, f * 2048, 0));
    if constexpr (SPLIT) x.l = __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(r, lane16, f * 2048 + 1024, 0));
    else x.l = bf8{};
    return x;
}

// Write four values (half `half` of a lane's eight) of a fragment in LDS, split into hi and lo.
template <bool SPLIT>
__device__ __forceinline__ void st_half(__bf16* f, int lane, int half, const float* x)
{
    bf4 hi, lo;
#pragma unroll
    for (int r = 0; r < 4; r += 2) {
        bf16x2_t h, l;
        split_bf16x2(x[r], x[r + 1], h, l);
        hi[r] = h[0]; hi[r + 1] = h[1];
        lo[r] = l[0]; lo[r + 1] = l[1];
    }
    *reinterpret_cast<bf4*>(f + lane * 8 + half * 4) = hi;
    if constexpr (SPLIT) *reinterpret_cast<bf4*>(f + 512 + lane * 8 + half * 4) = lo;
}

// Sum of p[0..3] over the four 16-lane groups of the wave: v_permlane32_swap pairs groups g and
// g+2, v_permlane16_swap pairs g and g+1. Lane group G receives the total of p[ksel(G)],
// ksel = {0, 2, 1, 3}.
__device__ __forceinline__ float sum_groups4(const float* p)
{
    const auto s01 = __builtin_amdgcn_permlane32_swap(__float_as_uint(p[0]), __float_as_uint(p[1]), false, false);
    const auto s23 = __builtin_amdgcn_permlane32_swap(__float_as_uint(p[2]), __float_as_uint(p[3]), false, false);
    const float q0 = __uint_as_float(s01[0]) + __uint_as_float(s01[1]);
    const float q1 = __uint_as_float(s23[0]) + __uint_as_float(s23[1]);
    const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(q0), __float_as_uint(q1), false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}
__device__ __forceinline__ int ksel(int g) { return ((g & 1) << 1) | (g >> 1); }

template <int NAT, bool SPLIT, int NW, bool ENS, int PD>
__global__ void __launch_bounds__(64 * NW) k_fitx(FitArgs A_)
{
    const FitArgs A = ENS ? model_args(A_) : A_;
    constexpr int NA = 16 * NAT;                       // atoms per block
    constexpr int FR = XF_ELEMS;
    constexpr int TPW = (15 + NW - 1) / NW;            // feature tiles per wave (at most)
    constexpr int NWA = NW / NAT;                      // waves sharing one atom tile's D fragments
    // the dD phase splits the waves into NW / 4 atom groups of NAT / (NW / 4) atom tiles each
    static_assert(NW % NAT == 0 && NW % 4 == 0 && NAT % (NW / 4) == 0, "wave layout");
    static_assert(FX_G % PD == 0 && XF_NCH2 % PD == 0, "prefetch ring slots are compile-time");
    // B operands [K-chunk][atom tile] (layer 1: two groups of FX_G chunks); at the end the
    // per-wave dT partials (floats) of the D rows n < 16.
    __shared__ __attribute__((aligned(16))) __bf16 s_b[XF_NCH2 * NAT * FR];
    __shared__ float s_e[NW][NA];
    // rows padded to 17 entries so that the 16 atoms a wave touches at once fall in distinct banks
    __shared__ __attribute__((aligned(16))) float s_p1[NA][17][4];
    __shared__ __attribute__((aligned(16))) float s_tq[NA][17][4];     // T rows n < 16 of the block's atoms

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar registers)
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const int nblk = gridDim.x, xcd = blockIdx.x & 7, per = nblk >> 3, rem = nblk & 7;
    const int blk = xcd * per + min(xcd, rem) + (blockIdx.x >> 3);
    // tile blk of the species-aligned tiling: species t has ceil(count_t / NA) tiles of its own,
    // so that no block runs the net twice for a boundary between species (the grid holds
    // ceil(N / NA) + ntypes blocks, an upper bound; the surplus ones leave here)
    int a0 = -1, ty = 0;
    {
        int tb = blk;
        for (int t = 0; t < A.ntypes; ++t) {
            const int lo = A.toff[t], nb = (A.toff[t + 1] - lo + NA - 1) / NA;
            if (tb < nb) {
                a0 = lo + tb * NA;
                ty = t;
                break;
            }
            tb -= nb;
        }
    }
    if (a0 < 0) return;
    const int t_lo = ty, t_hi = ty;
    const float* Tg = reinterpret_cast<const float*>(A.T);
    float* dTg = reinterpret_cast<float*>(A.dT);
    float* scr = reinterpret_cast<float*>(A.act) + (size_t)blk * NAT * XF_ACT;
    const int nown = (15 - wave + NW - 1) / NW;       // feature tiles wave + NW i < 15

    // activation scratch of (layer l, feature tile t, atom tile a): this lane's four values
    const int lane16 = lane * 16;
    // this lane's four values of (layer l, feature tile t, atom tile a) in the scratch: a
    // wave-uniform base plus the lane's 16-byte offset (read back by the same lane)
    const unsigned ulane16 = (unsigned)lane16;
    auto sptr = [&](int l, int t, int a) {
        char* base = reinterpret_cast<char*>(scr) + (unsigned)(((l * 16 + t) * NAT + a) * 1024);
        return reinterpret_cast<f4*>(base + ulane16);
    };
    auto sb = [&](int c, int a) { return s_b + (c * NAT + a) * FR; };

#pragma unroll 1
    for (int ti = t_lo; ti <= t_hi; ++ti) {
        const float* fv = reinterpret_cast<const float*>(A.fvec) + (size_t)ti * FVEC;
        const __bf16* W = reinterpret_cast<const __bf16*>(A.fmat) + (size_t)ti * XF_NFRAG * FR;
        const rsrc_t wrs = make_rsrc(W, XF_NFRAG * FR * 2);

        f4 acc[TPW][NAT];
        float h[TPW][NAT][4];
        auto zero_acc = [&]() {
#pragma unroll
            for (int i = 0; i < TPW; ++i)
#pragma unroll
                for (int a = 0; a < NAT; ++a) acc[i][a] = f4{0.f, 0.f, 0.f, 0.f};
        };
        // Weight fragment of K-chunk c of the product at wb for the wave's tile i (a wave without a
        // tile i reads its last valid tile again: every read is unconditional, since a read skipped
        // by a branch makes the compiler wait for every read in flight).
        auto wtile = [&](int i) { return min(wave + NW * i, 14); };
        // The first PD K-chunks of the next 240-wide product, requested before the preceding
        // epilogue and barrier so that their latency is hidden; each product step then requests
        // the chunk PD ahead (a ring of PD register slots).
        F8 Apf[PD][TPW];
        auto prefetch8 = [&](int wb) {
#pragma unroll
            for (int d = 0; d < PD; ++d)
#pragma unroll
                for (int i = 0; i < TPW; ++i) Apf[d][i] = ld_wfrag<SPLIT>(wrs, lane16, wb + d * 15 + wtile(i));
        };
        // acc[i][a] = sum over the 8 K-chunks of W(own tile i, c) B(c, a), B from s_b; Apf must
        // hold the first chunk of product wb (prefetch8)
        auto gemm8 = [&](int wb) {
            zero_acc();
            F8 Rg[PD][TPW];
#pragma unroll
            for (int d = 0; d < PD; ++d)
#pragma unroll
                for (int i = 0; i < TPW; ++i) Rg[d][i] = Apf[d][i];
#pragma unroll
            for (int c = 0; c < XF_NCH2; ++c) {
                F8 Ac[TPW];
#pragma unroll
                for (int i = 0; i < TPW; ++i) Ac[i] = Rg[c % PD][i];
                if (c + PD < XF_NCH2) {
#pragma unroll
                    for (int i = 0; i < TPW; ++i) Rg[c % PD][i] = ld_wfrag<SPLIT>(wrs, lane16, wb + (c + PD) * 15 + wtile(i));
                }
                F8 B[NAT];
#pragma unroll
                for (int a = 0; a < NAT; ++a) B[a] = ld_frag<SPLIT>(sb(c, a), lane);
#pragma unroll
                for (int i = 0; i < TPW; ++i)
                    if (i < nown) {
#pragma unroll
                        for (int a = 0; a < NAT; ++a) mma32<SPLIT>(acc[i][a], Ac[i], B[a]);
                    }
            }
        };
        auto vec4 = [&](int off, int t) { return *reinterpret_cast<const f4*>(fv + off + 16 * t + 4 * g); };

        __syncthreads();   // s_b, s_e, s_p1 of the previous species are no longer read
        for (int idx = threadIdx.x; idx < NA * 16; idx += 64 * NW) {
            const int al = idx >> 4, n = idx & 15;
            const int at = a0 + al < A.natoms ? a0 + al : a0;
            *reinterpret_cast<f4*>(&s_tq[al][n][0]) = *reinterpret_cast<const f4*>(Tg + ((size_t)at * E2 + n) * 4);
        }
        // ------------------------------------------------------------ layer 1: D (1600) -> 240
        // D fragment of K-chunk c for atom tile `wave`: lane group g holds D[2c][4g+r] and
        // D[2c+1][4g+r], D[m][n] = sum_k T[m][k] T[n][k] (Sec. II.A.1, D = T T_<^T).
        // wave w forms the D fragments of atom tile wa = w % NAT for the K-chunks cc = ph (mod NWA)
        const int wa = wave % NAT, ph = wave / NAT;
        const float* Tw = Tg + (size_t)(a0 + 16 * wa + c16 < A.natoms ? a0 + 16 * wa + c16 : a0) * (E2 * 4);
        float Tn[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const f4 v = *reinterpret_cast<const f4*>(Tw + (4 * g + r) * 4);
#pragma unroll
            for (int k = 0; k < 4; ++k) Tn[r][k] = v[k];
        }
        // T rows 2c and 2c + 1 of this lane's atom, and the D fragment of K-chunk c formed from them
        auto trows = [&](int c, f4& ta, f4& tb) {
            ta = *reinterpret_cast<const f4*>(Tw + (2 * c) * 4);
            tb = *reinterpret_cast<const f4*>(Tw + (2 * c + 1) * 4);
        };
        auto dform = [&](const f4& ta, const f4& tb, __bf16* f) {
            float d0[4], d1[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                d0[r] = ta[0] * Tn[r][0] + ta[1] * Tn[r][1] + ta[2] * Tn[r][2] + ta[3] * Tn[r][3];
                d1[r] = tb[0] * Tn[r][0] + tb[1] * Tn[r][1] + tb[2] * Tn[r][2] + tb[3] * Tn[r][3];
            }
            st_half<SPLIT>(f, lane, 0, d0);
            st_half<SPLIT>(f, lane, 1, d1);
        };
#pragma unroll
        for (int cc = 0; cc < FX_G; ++cc)
            if (cc % NWA == ph) {
                f4 ta, tb;
                trows(cc, ta, tb);
                dform(ta, tb, sb(cc, wa));
            }
        __syncthreads();
        {
            zero_acc();
            const int wb = XF_W1F;
            F8 R1[PD][TPW];
#pragma unroll
            for (int d = 0; d < PD; ++d)
#pragma unroll
                for (int i = 0; i < TPW; ++i) R1[d][i] = ld_wfrag<SPLIT>(wrs, lane16, wb + d * 15 + wtile(i));
            constexpr int NGRP = (XF_NCH1 + FX_G - 1) / FX_G;
            // One group of FX_G K-chunks. Reads retire in issue order, so the T rows of the D
            // fragment formed after a chunk's products are read before that chunk's weight
            // prefetch, and every read is unconditional (clamped to valid rows and fragments; a
            // wave with fewer tiles reads one it does not use): a read skipped by a branch would
            // make the compiler drain all reads in flight. The last, partial group is peeled so
            // that its chunk bounds are constants.
            auto group = [&](int grp) {
                const int p = grp & 1;
#pragma unroll
                for (int cc = 0; cc < FX_G; ++cc) {
                    const int c = grp * FX_G + cc;
                    if (c < XF_NCH1) {
                        F8 Ac[TPW];
#pragma unroll
                        for (int i = 0; i < TPW; ++i) Ac[i] = R1[cc % PD][i];
                        const int cn = c + FX_G;
                        f4 ta, tb;
                        trows(min(cn, XF_NCH1 - 1), ta, tb);
                        const int c1 = min(c + PD, XF_NCH1 - 1);
#pragma unroll
                        for (int i = 0; i < TPW; ++i) R1[cc % PD][i] = ld_wfrag<SPLIT>(wrs, lane16, wb + c1 * 15 + wtile(i));
                        F8 B[NAT];
#pragma unroll
                        for (int a = 0; a < NAT; ++a) B[a] = ld_frag<SPLIT>(sb(p * FX_G + cc, a), lane);
#pragma unroll
                        for (int i = 0; i < TPW; ++i)
                            if (i < nown) {
#pragma unroll
                                for (int a = 0; a < NAT; ++a) mma32<SPLIT>(acc[i][a], Ac[i], B[a]);
                            }
                        if (cn < XF_NCH1 && cc % NWA == ph) dform(ta, tb, sb((p ^ 1) * FX_G + cc, wa));
                    }
                }
                __syncthreads();
            };
#pragma unroll 1
            for (int grp = 0; grp < NGRP - 1; ++grp) group(grp);
            group(NGRP - 1);
        }
        prefetch8(XF_W2F);
        // a1 = tanh(W1 D + b1), h1 = wh1 a1
#pragma unroll
        for (int i = 0; i < TPW; ++i)
            if (i < nown) {
                const int t = wave + NW * i;
                const f4 b = vec4(FV_B1, t), wh = vec4(FV_WH1, t);
#pragma unroll
                for (int a = 0; a < NAT; ++a) {
                    f4 av;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        av[r] = fx_tanh(acc[i][a][r] + b[r]);
                        h[i][a][r] = wh[r] * av[r];
                    }
                    *sptr(0, t, a) = av;
                    st_half<SPLIT>(sb(t >> 1, a), lane, t & 1, h[i][a]);
                }
            }
        if (wave == NW - 1) {   // feature tile 15 does not exist: the second half of K-chunk 7 is zero
            const float z[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < NAT; ++a) st_half<SPLIT>(sb(7, a), lane, 1, z);
        }
        __syncthreads();
        // ------------------------------------------------------------ layers 2, 3: h += wh tanh(W h + b)
#pragma unroll 1
        for (int layer = 2; layer <= 3; ++layer) {
            gemm8(layer == 2 ? XF_W2F : XF_W3F);
            prefetch8(layer == 2 ? XF_W3F : XF_W3B);
            __syncthreads();
            const int ob = layer == 2 ? FV_B2 : FV_B3, ow = layer == 2 ? FV_WH2 : FV_WH3;
#pragma unroll
            for (int i = 0; i < TPW; ++i)
                if (i < nown) {
                    const int t = wave + NW * i;
                    const f4 b = vec4(ob, t), wh = vec4(ow, t);
#pragma unroll
                    for (int a = 0; a < NAT; ++a) {
                        f4 av;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            av[r] = fx_tanh(acc[i][a][r] + b[r]);
                            h[i][a][r] += wh[r] * av[r];
                        }
                        *sptr(layer - 1, t, a) = av;
                        if (layer == 2) st_half<SPLIT>(sb(t >> 1, a), lane, t & 1, h[i][a]);
                    }
                }
            if (layer == 2) __syncthreads();
        }
        // ------------------------------------------------------------ energy E_i = wh4 (w4 . h3 + b4)
        {
            float e[NAT];
#pragma unroll
            for (int a = 0; a < NAT; ++a) e[a] = 0.f;
#pragma unroll
            for (int i = 0; i < TPW; ++i)
                if (i < nown) {
                    const f4 w4 = vec4(FV_W4, wave + NW * i);
#pragma unroll
                    for (int a = 0; a < NAT; ++a)
#pragma unroll
                        for (int r = 0; r < 4; ++r) e[a] += w4[r] * h[i][a][r];
                }
            static_assert(NAT <= 4, "one energy sum per lane group");
            float ep[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < NAT; ++a) ep[a] = e[a];
            const float es = sum_groups4(ep);
            if (ksel(g) < NAT) s_e[wave][16 * ksel(g) + c16] = es;
        }
        // ------------------------------------------------------------ backward through layers 3, 2
        // gh3 = wh4 w4, ga3 = gh3 wh3 (1 - a3^2); gh_{l-1} = W_l^T ga_l + gh_l, ga_l = gh_l wh_l (1 - a_l^2)
        const float wh4 = fv[FV_WH4];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
            if (i < nown) {
                const int t = wave + NW * i;
                const f4 w4 = vec4(FV_W4, t), wh = vec4(FV_WH3, t);
#pragma unroll
                for (int a = 0; a < NAT; ++a) {
                    const f4 av = *sptr(2, t, a);
                    float ga[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        h[i][a][r] = wh4 * w4[r];
                        ga[r] = h[i][a][r] * wh[r] * (1.f - av[r] * av[r]);
                    }
                    st_half<SPLIT>(sb(t >> 1, a), lane, t & 1, ga);
                }
            }
        __syncthreads();
        if (threadIdx.x < NA) {
            const int at = a0 + threadIdx.x;
            if (at < A.natoms && A.itype[at] == ti)
            {
                double es = 0.0;
                for (int w = 0; w < NW; ++w) es += (double)s_e[w][threadIdx.x];
                A.Ei[at] = (double)wh4 * (es + (double)fv[FV_B4]);
            }
        }
#pragma unroll 1
        for (int layer = 3; layer >= 2; --layer) {
            gemm8(layer == 3 ? XF_W3B : XF_W2B);
            if (layer == 3) prefetch8(XF_W2B);
            __syncthreads();
            const int ow = layer == 3 ? FV_WH2 : FV_WH1;
#pragma unroll
            for (int i = 0; i < TPW; ++i)
                if (i < nown) {
                    const int t = wave + NW * i;
                    const f4 wh = vec4(ow, t);
#pragma unroll
                    for (int a = 0; a < NAT; ++a) {
                        const f4 av = *sptr(layer - 2, t, a);
                        float ga[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            h[i][a][r] += acc[i][a][r];
                            ga[r] = h[i][a][r] * wh[r] * (1.f - av[r] * av[r]);
                        }
                        st_half<SPLIT>(sb(t >> 1, a), lane, t & 1, ga);
                    }
                }
            __syncthreads();
        }
        // ------------------------------------------------------------ dD = W1 ga1 and dT
        // D-row tile m of dD holds dD[m][n = 4g + r] for 16 atoms. dT[m][k] collects
        // sum_n dD[m][n] T[n][k] (part 1, reduced over lane groups) and, for rows n < 16,
        // sum_m dD[m][n] T[m][k] (part 2, q2, per wave; reduced over waves at the end).
        // Waves form AG atom groups x 4 row groups: wave w takes atom tiles ag*NATD.. of its
        // group ag = w % AG and the D-row tiles mw + 4j, mw = w / AG (each W1 fragment is read
        // by AG waves, each ga1 fragment by 4 waves per atom group).
        {
            constexpr int AG = NW / 4, NATD = NAT / AG, MGD = NW == 4 ? 4 : 2;
            const int ag = wave % AG, mw = wave / AG;
            const float* Td[NATD];
            int atd[NATD];
            bool mined[NATD];
#pragma unroll
            for (int a2 = 0; a2 < NATD; ++a2) {
                const int at = a0 + 16 * (ag * NATD + a2) + c16;
                atd[a2] = at;
                Td[a2] = Tg + (size_t)(at < A.natoms ? at : a0) * (E2 * 4);
                mined[a2] = at < A.natoms && A.itype[at] == ti;
            }
            float q2[NATD][4][4];
#pragma unroll
            for (int a2 = 0; a2 < NATD; ++a2)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int k = 0; k < 4; ++k) q2[a2][r][k] = 0.f;
            const int wb = XF_W1B;
            constexpr int NMT = E2 / 4;                   // D-row tiles per row group: mw + 4 j
            constexpr int NPASS = (NMT + MGD - 1) / MGD;
            // one flat loop over (pass, K-chunk): the weight fragments of the next step, also
            // across a pass boundary, are requested one step ahead
            auto wfrag = [&](int pass, int c, int j) {
                return ld_wfrag<SPLIT>(wrs, lane16, wb + c * E2 + mw + 4 * (pass * MGD + j));
            };
            // a ring of PD steps of weight fragments (a row tile past the last pass reads tile
            // 0 of the pass again: unconditional reads)
            constexpr int NSTEP = NPASS * XF_NCH2;
            static_assert(NSTEP % PD == 0, "whole ring turns");
            auto wstep = [&](int st, int j) {
                const int pn = st / XF_NCH2, cn = st - pn * XF_NCH2;
                return wfrag(pn, cn, j < min(MGD, NMT - pn * MGD) ? j : 0);
            };
            F8 RD[PD][MGD];
#pragma unroll
            for (int d = 0; d < PD; ++d)
#pragma unroll
                for (int j = 0; j < MGD; ++j) RD[d][j] = wstep(d, j);
            f4 dd[MGD][NATD];
            f4 tmv[MGD][NATD];
#pragma unroll 1
            for (int s0 = 0; s0 < NSTEP; s0 += PD)
#pragma unroll
            for (int dstep = 0; dstep < PD; ++dstep) {
                const int step = s0 + dstep;
                const int pass = step / XF_NCH2, c = step - pass * XF_NCH2;
                const int nm = min(MGD, NMT - pass * MGD);
                if (c == 0) {
#pragma unroll
                    for (int j = 0; j < MGD; ++j)
#pragma unroll
                        for (int a2 = 0; a2 < NATD; ++a2) {
                            dd[j][a2] = f4{0.f, 0.f, 0.f, 0.f};
                            // rows T[m] of this pass, used by the epilogue
                            const int m = mw + 4 * (pass * MGD + (j < nm ? j : 0));
                            tmv[j][a2] = *reinterpret_cast<const f4*>(Td[a2] + m * 4);
                        }
                }
                F8 Ac[MGD];
#pragma unroll
                for (int j = 0; j < MGD; ++j) Ac[j] = RD[dstep][j];
                if (step + PD < NSTEP) {
#pragma unroll
                    for (int j = 0; j < MGD; ++j) RD[dstep][j] = wstep(step + PD, j);
                }
                F8 B[NATD];
#pragma unroll
                for (int a2 = 0; a2 < NATD; ++a2) B[a2] = ld_frag<SPLIT>(sb(c, ag * NATD + a2), lane);
#pragma unroll
                for (int j = 0; j < MGD; ++j)
                    if (j < nm) {
#pragma unroll
                        for (int a2 = 0; a2 < NATD; ++a2) mma32<SPLIT>(dd[j][a2], Ac[j], B[a2]);
                    }
                if (c == XF_NCH2 - 1) {
#pragma unroll
                    for (int a2 = 0; a2 < NATD; ++a2) {
                        const int al = 16 * (ag * NATD + a2) + c16;   // atom within the block
                        f4 tn[4];                                     // T rows 4g..4g+3 of the atom
#pragma unroll
                        for (int r = 0; r < 4; ++r) tn[r] = *reinterpret_cast<const f4*>(&s_tq[al][4 * g + r][0]);
#pragma unroll
                        for (int j = 0; j < MGD; ++j)
                            if (j < nm) {
                                const int m = mw + 4 * (pass * MGD + j);
                                const f4 tm = tmv[j][a2];
                                float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                                for (int r = 0; r < 4; ++r)
#pragma unroll
                                    for (int k = 0; k < 4; ++k) {
                                        part[k] += dd[j][a2][r] * tn[r][k];
                                        q2[a2][r][k] += dd[j][a2][r] * tm[k];
                                    }
                                const float pk = sum_groups4(part);   // lane group g: component ksel(g)
                                if (m < 16) s_p1[al][m][ksel(g)] = pk;
                                else if (mined[a2]) dTg[((size_t)atd[a2] * E2 + m) * 4 + ksel(g)] = pk;
                            }
                    }
                }
            }
            __syncthreads();   // every wave is done with ga1 in s_b
            // part 2 partials: slot (row group, atom tile) [lane][16], each written by one wave
            float* qs = reinterpret_cast<float*>(s_b);
#pragma unroll
            for (int a2 = 0; a2 < NATD; ++a2)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    *reinterpret_cast<f4*>(qs + ((mw * NAT + ag * NATD + a2) * 64 + lane) * 16 + 4 * r) =
                        f4{q2[a2][r][0], q2[a2][r][1], q2[a2][r][2], q2[a2][r][3]};
            __syncthreads();
            // rows n < 16 of dT: part 1 + the four row groups' part 2
            for (int idx = threadIdx.x; idx < NA * 16; idx += 64 * NW) {
                const int al = idx >> 4, n = idx & 15;
                const int at = a0 + al;
                if (at < A.natoms && A.itype[at] == ti) {
                    const int a = al >> 4, lp = (n >> 2) * 16 + (al & 15), r = n & 3;
                    f4 v = *reinterpret_cast<const f4*>(&s_p1[al][n][0]);
#pragma unroll
                    for (int w = 0; w < 4; ++w) v += *reinterpret_cast<const f4*>(qs + ((w * NAT + a) * 64 + lp) * 16 + 4 * r);
                    *reinterpret_cast<f4*>(dTg + ((size_t)at * E2 + n) * 4) = v;
                }
            }
        }
    }
}

}  // namespace

int fitx_tiles_per_block(int, int)
{
    // Four 16-atom tiles per block: the weights a block streams are amortised over 64 atoms. (On
    // the 12,288-atom box, 192 blocks of 64 atoms ran the kernel in 0.17 ms, 256 blocks of 48 atoms
    // in 0.27 ms.)
    return 4;
}

// Block shape: 64 atoms with a one-chunk weight lookahead when the frame fills the CUs; otherwise
// 32 atoms per block (twice the blocks, so twice the CUs stream a frame's weights) and a ring of
// FITX_PD chunks per wave, which the smaller accumulator set leaves registers for.
template <int NAT, int PD>
static void launch_fitx_shape(bool split, const FitArgs& a, hipStream_t s)
{
    constexpr int NW = 8;
    const bool ens = a.nmodels > 1;
    dim3 grid((a.natoms + 16 * NAT - 1) / (16 * NAT) + a.ntypes, ens ? a.nmodels : 1), block(64 * NW);
    // ens: one launch for a model ensemble, blockIdx.y = model (a separate instantiation)
    if (split) {
        if (ens) hipLaunchKernelGGL((k_fitx<NAT, true, NW, true, PD>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_fitx<NAT, true, NW, false, PD>), grid, block, 0, s, a);
    } else {
        if (ens) hipLaunchKernelGGL((k_fitx<NAT, false, NW, true, PD>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_fitx<NAT, false, NW, false, PD>), grid, block, 0, s, a);
    }
}

void launch_fitx(bool split, const FitArgs& a, hipStream_t s)
{
    if (a.natoms <= 0) return;
    const int64_t blocks64 = ((int64_t)a.natoms + 63) / 64 * (a.nmodels > 1 ? a.nmodels : 1);
    if (blocks64 * 2 <= (a.ncu > 0 ? a.ncu : 256)) launch_fitx_shape<2, FITX_PD>(split, a, s);
    else launch_fitx_shape<4, 1>(split, a, s);
}

}  // namespace dpk
