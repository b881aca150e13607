// Batched multi-stream apply: many streams of uneven length, each with its own
// orders, L and coefficients, in one persistent launch.
//
// Work item = one block tile of 4 waves x R chunks x 64*S samples of one
// stream (R = 16 / S, 4096 samples).  The host orders the items most
// expensive first (cost ~ NI * L * samples) and the persistent blocks claim
// them from a device counter, so long-running classes start first and the
// tail is short.  The counter resets itself: the last block to leave sets it
// back to zero, so the launch needs no memset and can be replayed from a
// hipGraph.  Each item dispatches on its stream's (NI, L) class to a fully
// unrolled tile function; every stream starts from zero history.
#pragma once

#include "dpd_fwd_kernels.h"

namespace dpd {

constexpr int kBatchMaxNI = 5;   // orders up to 9 in the persistent kernel
constexpr int kBatchMaxL = 8;
constexpr int kBatchItem = 4096; // samples per work item

struct BatchStream {
    const float2 *in;
    float2 *out;
    int64_t n;
    int32_t cls;      // (NI-1)*kBatchMaxL + (L-1), or -1 (handled by separate launches)
    int32_t tab;      // float offset of the stream's precombined table
};

struct BatchItem {
    int32_t stream;
    int32_t pad_;
    int64_t t0;
};

struct BatchPrep {
    const float2 *raw;
    CoefMap map;
    int32_t tab;
    int32_t pad_;
};

struct BatchParams {
    const BatchStream *streams;
    const BatchItem *items;
    int64_t n_items;
    const float *tables;
    unsigned int *counter;   // [0] next item, [1] blocks done
};

// Largest padded wave buffer over the classes of the persistent kernel.
template <int S>
struct BatchSlots {
    static constexpr int value = PadLayout<kBatchMaxL, S>::SLOTS;
};

// One chunk of C = 64*S samples starting at t (< n) of a stream.
template <int NI, int L, int S>
__device__ __forceinline__ void batch_chunk(const float2 *__restrict__ x, float2 *__restrict__ z,
                                            int64_t n, int64_t t, const float (&top)[4 * L],
                                            const cfloat *M, float2 *X, float *SX, int lane)
{
    constexpr int C = 64 * S;
    constexpr int W = S + L - 1;
    constexpr int NV = S / 2;
    constexpr int HS = L - 1;
    using PL = PadLayout<L, S>;
    const bool full = t + C <= n;
    float4 v[NV];
    if (full) {
        const float4 *x4 = reinterpret_cast<const float4 *>(x + t);
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = x4[lane + 64 * i];
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int64_t m = t + 2 * (lane + 64 * i);
            const float2 u = m < n ? x[m] : make_float2(0.f, 0.f);
            const float2 w = m + 1 < n ? x[m + 1] : make_float2(0.f, 0.f);
            v[i] = make_float4(u.x, u.y, w.x, w.y);
        }
    }
    float2 h = make_float2(0.f, 0.f);
    if (HS > 0) {
        const int hl = lane < HS ? lane : HS - 1;
        const int64_t m = t - HS + hl;
        const float2 r = x[m >= 0 ? m : 0];
        h = m >= 0 ? r : make_float2(0.f, 0.f);
    }
    wave_lds_order();
    if (HS > 0 && lane < HS) {
        const int q = PL::slot(lane - HS);
        X[q] = h;
        SX[q] = __builtin_fmaf(h.x, h.x, h.y * h.y);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int j = 2 * (lane + 64 * i);
        const int q = PL::OFF + j + j / S;
        X[q] = make_float2(v[i].x, v[i].y);
        X[q + 1] = make_float2(v[i].z, v[i].w);
        SX[q] = __builtin_fmaf(v[i].x, v[i].x, v[i].y * v[i].y);
        SX[q + 1] = __builtin_fmaf(v[i].z, v[i].z, v[i].w * v[i].w);
    }
    wave_lds_order();
    float a[W], b[W], s[W];
    const int lb = lane * (S + 1);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int q = lb + PL::slot(w - (L - 1));
        const float2 u = X[q];
        a[w] = u.x;
        b[w] = u.y;
        s[w] = SX[q];
    }
    float zr[S], zi[S];
    fir_outputs<NI, L, S>(a, b, s, top, M, zr, zi);
    if (full) {
        if constexpr (S == 2) {
            store_outputs<S>(z, t + lane * S, n, true, zr, zi);
        } else {
            wave_lds_order();
            const int ob = lb + PL::OFF;
#pragma unroll
            for (int i = 0; i < S; ++i) X[ob + i] = make_float2(zr[i], zi[i]);
            wave_lds_order();
            v4f *z4 = reinterpret_cast<v4f *>(z + t);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int j = 2 * (lane + 64 * i);
                const int q = PL::OFF + j + j / S;
                const float2 u = X[q], w = X[q + 1];
                const v4f o = {u.x, u.y, w.x, w.y};
                __builtin_nontemporal_store(o, z4 + lane + 64 * i);
            }
        }
    } else {
        const int64_t m0 = t + (int64_t)lane * S;
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (m0 + i < n) z[m0 + i] = make_float2(zr[i], zi[i]);
    }
}

// The wave's chunks of one work item: chunk wv + 4 r, r < R.
template <int NI, int L, int S>
__device__ __forceinline__ void batch_item(const BatchStream &st, int64_t t0, const float *table,
                                        float2 *X, float *SX, int lane, int wv)
{
    constexpr int C = 64 * S;
    constexpr int R = kBatchItem / (4 * C);
    const cfloat *M = as_const(table);
    float top[4 * L];
#pragma unroll
    for (int e = 0; e < 4 * L; ++e) top[e] = M[(e >> 2) * 4 * NI + 4 * (NI - 1) + (e & 3)];
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
        const int64_t t = t0 + (int64_t)(wv + 4 * r) * C;
        if (t >= st.n) break;
        batch_chunk<NI, L, S>(st.in, st.out, st.n, t, top, M, X, SX, lane);
    }
}

template <int S>
__global__ void __launch_bounds__(kBlock) batch_kernel(BatchParams bp)
{
    constexpr int WAVES = kBlock / 64;
    constexpr int SLOTS = BatchSlots<S>::value;
    __shared__ __align__(16) float2 xs[WAVES][SLOTS];
    __shared__ __align__(16) float ss[WAVES][SLOTS];
    __shared__ unsigned int item_sh;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (;;) {
        if (tid == 0)
            item_sh = __hip_atomic_fetch_add(&bp.counter[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(item_sh);
        __syncthreads();
        if (item >= bp.n_items) break;
        const BatchItem it = bp.items[item];
        const BatchStream st = bp.streams[it.stream];
        const float *tab = bp.tables + st.tab;
        switch (st.cls) {
#define DPD_BATCH_CASE(NI, L)                                                          \
    case (NI - 1) * kBatchMaxL + (L - 1):                                              \
        batch_item<NI, L, S>(st, it.t0, tab, xs[wv], ss[wv], lane, wv);                \
        break;
#define DPD_BATCH_ROW(NI)                                                              \
    DPD_BATCH_CASE(NI, 1) DPD_BATCH_CASE(NI, 2) DPD_BATCH_CASE(NI, 3) DPD_BATCH_CASE(NI, 4) \
    DPD_BATCH_CASE(NI, 5) DPD_BATCH_CASE(NI, 6) DPD_BATCH_CASE(NI, 7) DPD_BATCH_CASE(NI, 8)
            DPD_BATCH_ROW(1)
            DPD_BATCH_ROW(2)
            DPD_BATCH_ROW(3)
            DPD_BATCH_ROW(4)
            DPD_BATCH_ROW(5)
#undef DPD_BATCH_ROW
#undef DPD_BATCH_CASE
        default:
            break;
        }
    }
    // the last block out resets the counters for the next launch
    if (tid == 0) {
        const unsigned int done =
            __hip_atomic_fetch_add(&bp.counter[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(&bp.counter[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bp.counter[1], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace dpd

namespace dpd {

typedef hipError_t (*BatchLaunch)(const BatchParams &, hipStream_t, int grid);
struct BatchTable {
    BatchLaunch fn[kNumSIdx];
    const void *kern[kNumSIdx];
};
void register_batch_s2(BatchTable &);
void register_batch_s4(BatchTable &);
void register_batch_s8(BatchTable &);

template <int S>
hipError_t launch_batch(const BatchParams &bp, hipStream_t stream, int grid)
{
    hipLaunchKernelGGL((batch_kernel<S>), dim3((uint32_t)grid), dim3(kBlock), 0, stream, bp);
    return hipGetLastError();
}

}  // namespace dpd
