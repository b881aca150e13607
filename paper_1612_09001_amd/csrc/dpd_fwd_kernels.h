// Forward kernels of the APH predistorter (Eq. 1 / Algorithm 1) for gfx950.
//
// One pass per sample does all three steps of Algorithm 1 -- basis
// (polynomial), filtering and accumulation + c -- in registers.  The paper's
// own fused single kernel (section 3.2.2) keeps intermediates out of global
// memory too; it fetches the L-1 preceding basis values with warp shuffles and
// spends (L-1)/32 of the lanes on redundant samples (section 3.3.2).  Here
// a block instead stages its tile plus an (L-1)-sample halo once (LDS or
// direct cached loads), and each thread produces S consecutive outputs from a
// register window of S+L-1 samples, so no lane is redundant.
//
// Arithmetic per output.  With s = |x|^2 and v = (Re x, Im x), the main and
// conjugate taps of order 2j+1 combine into one real 2x2 matrix M_{j,k}
// (h w + hbar conj(w) is real-linear in w), so
//     z_n = c + sum_k W_k(s_{n-k}) v_{n-k},   W_k(s) = sum_j M_{j,k} s^j,
// and W_k is evaluated by Horner in s: 4*NI fused multiply-adds per tap and
// output, the minimum for 4*NI*L independent real coefficients.  No sqrt or
// transcendental is needed for odd orders.
#pragma once

#include "dpd_internal.h"

namespace dpd {

typedef float v4f __attribute__((ext_vector_type(4)));

// Coefficient tables are read through the constant address space: uniform,
// read-only loads from it become scalar loads (SGPR operands of the FMAs).
typedef const float __attribute__((address_space(4))) cfloat;
__device__ __forceinline__ const cfloat *as_const(const float *p)
{
    return (const cfloat *)p;
}

// Consecutive tiles share a halo; keep neighbours on one XCD (one L2) by
// mapping dispatch order (round-robin over the 8 XCDs) to contiguous ranges.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G)
{
    const uint32_t q = G >> 3, r = G & 7u;
    const uint32_t x = b & 7u, l = b >> 3;
    return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Sample m of a row; zero before the start unless a history is given
// (hist[L-1+m] for -(L-1) <= m < 0).
template <int L>
__device__ __forceinline__ float2 sample_or_hist(const float2 *__restrict__ x, int64_t m, int64_t n,
                                                 const float2 *__restrict__ hist)
{
    if (m >= 0) return m < n ? x[m] : make_float2(0.f, 0.f);
    if (hist != nullptr && m >= -(int64_t)(L - 1)) return hist[(L - 1) + m];
    return make_float2(0.f, 0.f);
}

// S outputs from a window of S+L-1 samples; window index w = i + (L-1) - k
// holds x_{n_i - k}.  `top` holds M_{NI-1,k} (4 floats per tap) in VGPRs; the
// remaining levels are read through the uniform pointer M (scalar loads).
template <int NI, int L, int S>
__device__ __forceinline__ void fir_outputs(const float (&a)[S + L - 1], const float (&b)[S + L - 1],
                                            const float (&s)[S + L - 1], const float (&top)[4 * L],
                                            const cfloat *M, float (&zr)[S], float (&zi)[S])
{
    const float cr = M[4 * L * NI], ci = M[4 * L * NI + 1];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        zr[i] = cr;
        zi[i] = ci;
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const cfloat *Mk = M + 4 * NI * k;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int w = i + (L - 1) - k;
            float w00 = top[4 * k + 0], w01 = top[4 * k + 1];
            float w10 = top[4 * k + 2], w11 = top[4 * k + 3];
#pragma unroll
            for (int j = NI - 2; j >= 0; --j) {
                w00 = __builtin_fmaf(w00, s[w], Mk[4 * j + 0]);
                w01 = __builtin_fmaf(w01, s[w], Mk[4 * j + 1]);
                w10 = __builtin_fmaf(w10, s[w], Mk[4 * j + 2]);
                w11 = __builtin_fmaf(w11, s[w], Mk[4 * j + 3]);
            }
            zr[i] = __builtin_fmaf(w00, a[w], zr[i]);
            zr[i] = __builtin_fmaf(w01, b[w], zr[i]);
            zi[i] = __builtin_fmaf(w10, a[w], zi[i]);
            zi[i] = __builtin_fmaf(w11, b[w], zi[i]);
        }
    }
}

template <int W>
__device__ __forceinline__ void split_window(const float2 (&win)[W], float (&a)[W], float (&b)[W],
                                             float (&s)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) {
        a[w] = win[w].x;
        b[w] = win[w].y;
        s[w] = __builtin_fmaf(a[w], a[w], b[w] * b[w]);
    }
}

// Store S consecutive outputs starting at sample m0 (< n) of a row.
template <int S>
__device__ __forceinline__ void store_outputs(float2 *__restrict__ z, int64_t m0, int64_t n,
                                              bool full, const float (&zr)[S], const float (&zi)[S])
{
    if (full) {
        v4f *z4 = reinterpret_cast<v4f *>(z + m0);
#pragma unroll
        for (int i = 0; i < S / 2; ++i) {
            v4f v = {zr[2 * i], zi[2 * i], zr[2 * i + 1], zi[2 * i + 1]};
            __builtin_nontemporal_store(v, z4 + i);
        }
    } else {
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (m0 + i < n) z[m0 + i] = make_float2(zr[i], zi[i]);
    }
}

// Tile = kBlock*S samples.  STAGE_LDS: the block loads its tile with coalesced
// 16-byte loads into LDS (plus an even-padded halo of L-1 samples), then every
// thread reads its S+L-1 window from LDS.  Otherwise each thread loads its own
// window with 16-byte loads; the halo part re-reads its neighbour's samples,
// which the vector L1 / L2 serve.
template <int NI, int L, int S, bool STAGE_LDS>
__global__ void __launch_bounds__(kBlock) fwd_kernel(FwdParams p)
{
    static_assert(S % 2 == 0, "S must be even (16-byte stores)");
    constexpr int T = kBlock * S;
    constexpr int HP = (L - 1 + 1) & ~1;   // halo rounded up to an even count
    constexpr int W = S + L - 1;
    __shared__ float ctop[4 * L];
    __shared__ __align__(16) float2 xs[STAGE_LDS ? HP + T : 2];

    const int tid = threadIdx.x;
    if (tid < 4 * L) ctop[tid] = p.M[(tid >> 2) * 4 * NI + 4 * (NI - 1) + (tid & 3)];

    for (int64_t step = xcd_remap(blockIdx.x, gridDim.x); step < p.total_tiles; step += gridDim.x) {
        const int64_t row = step / p.tiles_per_row;
        const int64_t t0 = (step - row * p.tiles_per_row) * (int64_t)T;
        const float2 *__restrict__ x = p.in + row * p.ld;
        float2 *__restrict__ z = p.out + row * p.ld;
        const float2 *__restrict__ hist = row == 0 ? p.hist : nullptr;
        const bool full = t0 + T <= p.n;
        const int64_t m0 = t0 + (int64_t)tid * S;   // first output of this thread

        float2 win[W];
        if constexpr (STAGE_LDS) {
            if (full) {
                const float4 *x4 = reinterpret_cast<const float4 *>(x + t0);
                float4 v[S / 2];
#pragma unroll
                for (int i = 0; i < S / 2; ++i) v[i] = x4[tid + i * kBlock];
#pragma unroll
                for (int i = 0; i < S / 2; ++i)
                    reinterpret_cast<float4 *>(xs + HP)[tid + i * kBlock] = v[i];
            } else {
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    const int q = tid + i * kBlock;
                    xs[HP + q] = (t0 + q < p.n) ? x[t0 + q] : make_float2(0.f, 0.f);
                }
            }
            if (tid < HP) xs[tid] = sample_or_hist<L>(x, t0 - HP + tid, p.n, hist);
            __syncthreads();
            const int base = HP + tid * S - (L - 1);
#pragma unroll
            for (int w = 0; w < W; ++w) win[w] = xs[base + w];
        } else {
            __syncthreads();   // ctop
            constexpr int WL = HP + S;                  // loaded samples (even)
            float2 raw[WL];
            const int64_t lo = m0 - HP;
            if (full && lo >= 0) {
                const float4 *x4 = reinterpret_cast<const float4 *>(x + lo);
#pragma unroll
                for (int i = 0; i < WL / 2; ++i) {
                    float4 v = x4[i];
                    raw[2 * i] = make_float2(v.x, v.y);
                    raw[2 * i + 1] = make_float2(v.z, v.w);
                }
            } else {
#pragma unroll
                for (int i = 0; i < WL; ++i) raw[i] = sample_or_hist<L>(x, lo + i, p.n, hist);
            }
#pragma unroll
            for (int w = 0; w < W; ++w) win[w] = raw[HP - (L - 1) + w];
        }

        float top[4 * L];
#pragma unroll
        for (int e = 0; e < 4 * L; ++e) top[e] = ctop[e];
        float a[W], b[W], s[W];
        split_window<W>(win, a, b, s);
        float zr[S], zi[S];
        fir_outputs<NI, L, S>(a, b, s, top, as_const(p.M), zr, zi);
        if (m0 < p.n) store_outputs<S>(z, m0, p.n, full, zr, zi);
        if constexpr (STAGE_LDS) __syncthreads();   // xs is reused by the next tile
    }
}

template <int NI, int L, int S, bool STAGE_LDS>
hipError_t launch_fwd(const FwdParams &p, hipStream_t stream)
{
    // Enough blocks to fill the chip several times over; larger inputs loop.
    const int64_t cap = 1 << 20;
    const int64_t grid = p.total_tiles < cap ? p.total_tiles : cap;
    hipLaunchKernelGGL((fwd_kernel<NI, L, S, STAGE_LDS>), dim3((uint32_t)grid), dim3(kBlock), 0,
                       stream, p);
    return hipGetLastError();
}

template <int NI, int L>
void register_fwd_one(FwdTable &t)
{
    t.fn[NI - 1][L - 1][0] = &launch_fwd<NI, L, 2, false>;
    t.fn[NI - 1][L - 1][1] = &launch_fwd<NI, L, 2, true>;
    t.fn[NI - 1][L - 1][2] = &launch_fwd<NI, L, 4, false>;
    t.fn[NI - 1][L - 1][3] = &launch_fwd<NI, L, 4, true>;
    t.fn[NI - 1][L - 1][4] = &launch_fwd<NI, L, 8, false>;
    t.fn[NI - 1][L - 1][5] = &launch_fwd<NI, L, 8, true>;
}

}  // namespace dpd
