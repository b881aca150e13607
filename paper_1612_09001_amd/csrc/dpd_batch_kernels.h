// Batched multi-stream apply: many streams of uneven length, each with its own
// orders, L and coefficients, in one persistent launch.
//
// The host cuts every stream into chunks of C = 64*S samples and lists them
// in one array of 32-byte chunk descriptors: all full chunks first, streams
// ordered most expensive class first (per-sample cost ~ NI * L), then the
// ragged last chunk of each stream (a second, small launch filters those),
// then one idle entry.  The persistent grid walks the full chunks the way the
// single-stream kernel walks one stream: wave g
// takes entries g, g + nw, g + 2 nw, ... (nw = waves in the grid), so
// neighbouring waves filter neighbouring chunks, every wave's sequence has the
// same cost profile (balanced without atomics), and the waves that run
// together mostly run the same class (code stays in the instruction cache).
//
// Per chunk everything is fetched one chunk ahead with vector loads, which the
// hardware completes in order, so the compiler's counter waits never stall on
// the prefetch: the descriptor (two chunks ahead), then the samples
// (nontemporal, 1 KiB contiguous per instruction), the 7 samples before the
// chunk and the stream's precombined coefficient table.  The table goes
// through a wave-private LDS area and is read back as broadcast 16-byte LDS
// reads, one tap at a time.  Each chunk dispatches on its stream's (NI, L)
// class to a fully unrolled filter.  Every stream starts from zero history.
// There is no device counter and no memset: the launch replays from a hipGraph
// as it is.
#pragma once

#include "dpd_fwd_kernels.h"

namespace dpd {

constexpr int kBatchMaxNI = 5;   // orders up to 9 in the persistent kernel
constexpr int kBatchMaxL = 8;
constexpr int kBatchHalo = kBatchMaxL - 1;   // samples before a chunk fetched for every class
constexpr int kBatchTabFloats = 256;         // per-wave LDS coefficient area (64 lanes x 16 B)
static_assert(4 * kBatchMaxL * kBatchMaxNI + 2 <= kBatchTabFloats, "table does not fit the LDS area");

// One chunk of one stream.
struct BatchChunk {
    const float2 *in;   // first input sample of the chunk
    float2 *out;        // first output sample of the chunk
    int32_t tab;        // float offset of the stream's table (16-byte aligned)
    uint32_t meta;      // class | hist << 8 | nc4 << 16 (see BatchDesc)
    int32_t valid;      // samples in the chunk (C except for a stream's ragged end)
    int32_t pad_;
};
static_assert(sizeof(BatchChunk) == 32, "descriptor is read as 8 dwords");

__host__ __device__ constexpr uint32_t batch_meta(int cls, int hist, int nc4)
{
    return (uint32_t)cls | ((uint32_t)hist << 8) | ((uint32_t)nc4 << 16);
}

// One entry of a stream's precombined table, rebuilt from the stream's
// coefficients at every apply: the 2x2 matrix of (order 2j+1, tap k) from the
// main and conjugate coefficients (either may be absent), or the DC term.
struct BatchPrepJob {
    const float2 *h;   // main-branch coefficient, or the DC term; nullptr: absent
    const float2 *g;   // conjugate-branch coefficient; nullptr: absent
    int32_t out;       // float offset in the tables (4 floats, 16-byte aligned; 2 for the DC term)
    int32_t dc;        // 1: DC term
    int64_t pad_;
};
static_assert(sizeof(BatchPrepJob) == 32, "job layout");

struct BatchParams {
    const BatchChunk *chunks;   // [0, n_full) full, [n_full, n_chunks) ragged, [n_chunks] idle
    int64_t n_full;
    int64_t n_chunks;
    const float *tables;
    // Full chunks [0, n_heavy) go to the waves of the blocks in the dispatch
    // slots not in light_mask, [n_heavy, n_full) to those in it (slot of a
    // block: blockIdx / ncu).  light_mask 0: every wave walks the whole list.
    int64_t n_heavy;
    int32_t ncu;
    int32_t light_mask;
};

// Wave-uniform view of a descriptor (scalar registers).
struct BatchDesc {
    const gcv2f *in;
    gv2f *out;
    int tab;
    int cls;     // (NI-1) * kBatchMaxL + (L-1)
    int hist;    // samples of the stream before the chunk, capped at kBatchHalo
    int nc4;     // 16-byte groups of the coefficient table
    int valid;
};

// Lane l (mod 8) fetches dword l of descriptor c.
__device__ __forceinline__ uint32_t batch_desc_load(const BatchChunk *chunks, int64_t c, int lane)
{
    return reinterpret_cast<const uint32_t *>(chunks + c)[lane & 7];
}

__device__ __forceinline__ BatchDesc batch_desc_read(uint32_t d)
{
    const auto rl = [&](int k) { return (uint32_t)__builtin_amdgcn_readlane((int)d, k); };
    BatchDesc D;
    D.in = (const gcv2f *)((uint64_t)rl(0) | ((uint64_t)rl(1) << 32));
    D.out = (gv2f *)((uint64_t)rl(2) | ((uint64_t)rl(3) << 32));
    D.tab = (int)rl(4);
    const uint32_t meta = rl(5);
    D.cls = (int)(meta & 0xffu);
    D.hist = (int)((meta >> 8) & 0xffu);
    D.nc4 = (int)(meta >> 16);
    D.valid = (int)rl(6);
    return D;
}

// Registers of one chunk in flight.
template <int S>
struct BatchRegs {
    float4 v[S / 2];   // lane l, part i: samples 2 (l + 64 i) and 2 (l + 64 i) + 1
    float2 h;          // lane l < kBatchHalo: sample l - kBatchHalo (clamped into the stream)
    float4 m;          // coefficient table floats 4 l .. 4 l + 3 (clamped to the table)
};

template <int S, bool FULL>
__device__ __forceinline__ void batch_load(BatchRegs<S> &R, const BatchDesc &D, const float *tables,
                                           int lane)
{
    constexpr int NV = S / 2;
    if constexpr (FULL) {
        const gcv4f *x4 = (const gcv4f *)D.in;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f u = __builtin_nontemporal_load(x4 + lane + 64 * i);
            R.v[i] = make_float4(u.x, u.y, u.z, u.w);
        }
    } else {
        const v2f zero = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int m = 2 * (lane + 64 * i);
            const v2f u = m < D.valid ? D.in[m] : zero;
            const v2f w = m + 1 < D.valid ? D.in[m + 1] : zero;
            R.v[i] = make_float4(u.x, u.y, w.x, w.y);
        }
    }
    // Fixed issue order (samples, halo, table): the prologue and the loop
    // then leave the same loads in flight, and the compiler's counter waits
    // at the loop head stay exact for both.
    __builtin_amdgcn_sched_barrier(0);
    const int d = (lane < kBatchHalo ? lane : kBatchHalo - 1) - kBatchHalo;   // -7 .. -1
    const v2f h = D.in[d >= -D.hist ? d : 0];
    __builtin_amdgcn_sched_barrier(0);
    R.h = make_float2(h.x, h.y);
    const int q = lane < D.nc4 ? lane : D.nc4 - 1;
    const v4f m = ((const gcv4f *)(tables + D.tab))[q];
    R.m = make_float4(m.x, m.y, m.z, m.w);
}

// fir_outputs with the table in LDS (CS): each tap's 4*NI floats are read as
// broadcast 16-byte LDS loads one tap ahead of their use.  Scheduling
// barriers between taps keep the compiler from hoisting every tap's reads to
// the top (which would hold the whole table in registers).
template <int NI>
__device__ __forceinline__ void batch_tap_load(const float *CS, int k, float (&Mk)[4 * NI])
{
    const float4 *ck = reinterpret_cast<const float4 *>(CS + 4 * NI * k);
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const float4 u = ck[j];
        Mk[4 * j + 0] = u.x;
        Mk[4 * j + 1] = u.y;
        Mk[4 * j + 2] = u.z;
        Mk[4 * j + 3] = u.w;
    }
}

template <int NI, int L, int S>
__device__ __forceinline__ void fir_outputs_lds(const float (&a)[S + L - 1], const float (&b)[S + L - 1],
                                                const float (&s)[S + L - 1], const float *CS,
                                                float (&zr)[S], float (&zi)[S])
{
    const float2 c = *reinterpret_cast<const float2 *>(CS + 4 * L * NI);
#pragma unroll
    for (int i = 0; i < S; ++i) {
        zr[i] = c.x;
        zi[i] = c.y;
    }
    float Mk[4 * NI];
    batch_tap_load<NI>(CS, 0, Mk);
#pragma unroll
    for (int k = 0; k < L; ++k) {
        float Mn[4 * NI];
        if (k + 1 < L) batch_tap_load<NI>(CS, k + 1, Mn);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int w = i + (L - 1) - k;
            float w00 = Mk[4 * (NI - 1) + 0], w01 = Mk[4 * (NI - 1) + 1];
            float w10 = Mk[4 * (NI - 1) + 2], w11 = Mk[4 * (NI - 1) + 3];
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
        __builtin_amdgcn_sched_barrier(0);
        if (k + 1 < L) {
#pragma unroll
            for (int e = 0; e < 4 * NI; ++e) Mk[e] = Mn[e];
        }
    }
}

// LDS layout shared by all classes: the padded layout of the longest filter,
// so a chunk is staged the same way whatever its class.
template <int S>
using BatchPad = PadLayout<kBatchMaxL, S>;

// Stage a chunk whose registers have arrived into the wave's LDS: samples and
// |x|^2 (X, SX, padded layout), the kBatchHalo samples before it (zero before
// the stream start) and the coefficient table (CS).  The registers are free
// afterwards.
template <int S>
__device__ __forceinline__ void batch_stage(const BatchRegs<S> &R, const BatchDesc &D, float2 *X, float *SX,
                                            float *CS, int lane)
{
    constexpr int NV = S / 2;
    using PL = BatchPad<S>;
    wave_lds_order();   // the previous chunk's LDS reads are done
    reinterpret_cast<float4 *>(CS)[lane] = R.m;
    if (lane < kBatchHalo) {
        const int d = lane - kBatchHalo;
        const float2 h = d >= -D.hist ? R.h : make_float2(0.f, 0.f);
        const int q = PL::slot(d);
        X[q] = h;
        SX[q] = __builtin_fmaf(h.x, h.x, h.y * h.y);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int j = 2 * (lane + 64 * i);
        const int q = PL::OFF + j + j / S;
        X[q] = make_float2(R.v[i].x, R.v[i].y);
        X[q + 1] = make_float2(R.v[i].z, R.v[i].w);
        SX[q] = __builtin_fmaf(R.v[i].x, R.v[i].x, R.v[i].y * R.v[i].y);
        SX[q + 1] = __builtin_fmaf(R.v[i].z, R.v[i].z, R.v[i].w * R.v[i].w);
    }
    wave_lds_order();
}

// Filter a staged chunk of class (NI, L) and store its outputs.
template <int NI, int L, int S, bool FULL>
__device__ __forceinline__ void batch_step(const BatchDesc &D, float2 *X0, float *SX0, float *CS0, int lane0)
{
    constexpr int W = S + L - 1;
    constexpr int NV = S / 2;
    using PL = BatchPad<S>;
    // An opaque zero keeps this class's LDS address arithmetic inside its own
    // code: hoisted out of the chunk loop, the constant-offset addresses of
    // all classes would each hold a register for the whole loop instead of
    // folding into the LDS instructions' offset fields.
    int z = 0;
    asm volatile("" : "+v"(z));
    const int lane = lane0 + z;
    float2 *X = X0 + z;
    float *SX = SX0 + z;
    const float *CS = CS0 + z;
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
    fir_outputs_lds<NI, L, S>(a, b, s, CS, zr, zi);
    if constexpr (!FULL) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const v2f o = {zr[i], zi[i]};
            if (lane * S + i < D.valid) D.out[lane * S + i] = o;
        }
    } else if constexpr (S == 2) {
        const v4f o = {zr[0], zi[0], zr[1], zi[1]};
        __builtin_nontemporal_store(o, (gv4f *)D.out + lane);
    } else {
        // outputs back through LDS so every store writes 1 KiB contiguously
        wave_lds_order();
        const int ob = lb + PL::OFF;
#pragma unroll
        for (int i = 0; i < S; ++i) X[ob + i] = make_float2(zr[i], zi[i]);
        wave_lds_order();
        gv4f *z4 = (gv4f *)D.out;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = 2 * (lane + 64 * i);
            const int q = PL::OFF + j + j / S;
            const float2 u = X[q], w = X[q + 1];
            const v4f o = {u.x, u.y, w.x, w.y};
            __builtin_nontemporal_store(o, z4 + lane + 64 * i);
        }
    }
}

template <int S, bool FULL>
__device__ __forceinline__ void batch_dispatch(const BatchDesc &D, float2 *X, float *SX, float *CS, int lane)
{
    switch (D.cls) {
#define DPD_BATCH_CASE(NI, L)                                                          \
    case (NI - 1) * kBatchMaxL + (L - 1):                                              \
        batch_step<NI, L, S, FULL>(D, X, SX, CS, lane);                                \
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
        __builtin_unreachable();   // the host lists only these classes
    }
}

template <int S>
__global__ void __launch_bounds__(kBlock) batch_kernel(BatchParams bp)
{
    static_assert(S % 2 == 0, "S must be even (16-byte loads and stores)");
    constexpr int WAVES = kBlock / 64;
    constexpr int SLOTS = BatchPad<S>::SLOTS;
    __shared__ __align__(16) float2 xs[WAVES][SLOTS];
    __shared__ __align__(16) float ss[WAVES][SLOTS];
    __shared__ __align__(16) float cs[WAVES][kBatchTabFloats];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *X = xs[wv];
    float *SX = ss[wv];
    float *CS = cs[wv];
    int64_t nw = (int64_t)gridDim.x * WAVES;
    int64_t gw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * WAVES + wv;
    int64_t nf = bp.n_full, base = 0;
    // Heavy and light chunks side by side: the dispatcher fills one block slot
    // of every CU before the next, so the blocks of one slot share no SIMD
    // with each other and the waves of a light-slot block run beside waves of
    // heavy-slot blocks -- VALU-bound and memory-bound chunks on one SIMD at
    // once.  Each group walks its own part of the cost-sorted list, wave-
    // strided in its own rank order (XCD-contiguous, as xcd_remap).  Any
    // placement of the blocks still covers every chunk exactly once.
    if (bp.light_mask != 0) {
        const int slot = blockIdx.x / bp.ncu, cu = blockIdx.x - slot * bp.ncu;
        const int nslots = gridDim.x / bp.ncu;
        const bool light = (bp.light_mask >> slot) & 1;
        int r = 0, cnt = 0;
        for (int s2 = 0; s2 < nslots; ++s2) {
            const bool l2 = (bp.light_mask >> s2) & 1;
            if (l2 == light) {
                if (s2 < slot) ++r;
                ++cnt;
            }
        }
        gw = ((int64_t)r * bp.ncu + xcd_remap(cu, bp.ncu)) * WAVES + wv;
        nw = (int64_t)cnt * bp.ncu * WAVES;
        base = light ? bp.n_heavy : 0;
        nf = (light ? bp.n_full : bp.n_heavy) - base;
    }

    // full chunks gw, gw + nw, ...: while one staged chunk is filtered, the
    // next chunk's loads are in flight (its descriptor was fetched one chunk
    // earlier); it is staged into LDS right after the stores, so its
    // registers are free again before the following loads.  Past the wave's
    // last chunk the loads read the idle entry, whose samples stay in the L2.
    if (gw < nf) {
        const int64_t left = (nf - 1 - gw) / nw + 1;
        const auto idx = [&](int64_t i) { return i < left ? base + gw + i * nw : bp.n_chunks; };
        BatchRegs<S> R;
        BatchDesc Dc = batch_desc_read(batch_desc_load(bp.chunks, idx(0), lane));
        uint32_t dn = batch_desc_load(bp.chunks, idx(1), lane);
        __builtin_amdgcn_sched_barrier(0);   // descriptor before samples, as in the loop
        batch_load<S, true>(R, Dc, bp.tables, lane);
        batch_stage<S>(R, Dc, X, SX, CS, lane);
        for (int64_t i = 0; i < left; ++i) {
            const BatchDesc Dn = batch_desc_read(dn);
            dn = batch_desc_load(bp.chunks, idx(i + 2), lane);
            __builtin_amdgcn_sched_barrier(0);
            batch_load<S, true>(R, Dn, bp.tables, lane);
            batch_dispatch<S, true>(Dc, X, SX, CS, lane);
            batch_stage<S>(R, Dn, X, SX, CS, lane);
            Dc = Dn;
        }
    }
}

// The ragged last chunks of the streams (entries [n_full, n_chunks)), one per
// wave: a second, small launch, so that the guarded code of a ragged chunk
// does not raise the register count of the streaming kernel.
template <int S>
__global__ void __launch_bounds__(kBlock) batch_tail_kernel(BatchParams bp)
{
    constexpr int WAVES = kBlock / 64;
    constexpr int SLOTS = BatchPad<S>::SLOTS;
    __shared__ __align__(16) float2 xs[WAVES][SLOTS];
    __shared__ __align__(16) float ss[WAVES][SLOTS];
    __shared__ __align__(16) float cs[WAVES][kBatchTabFloats];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    for (int64_t c = bp.n_full + (int64_t)blockIdx.x * WAVES + wv; c < bp.n_chunks; c += nw) {
        const BatchDesc D = batch_desc_read(batch_desc_load(bp.chunks, c, lane));
        BatchRegs<S> R;
        batch_load<S, false>(R, D, bp.tables, lane);
        batch_stage<S>(R, D, xs[wv], ss[wv], cs[wv], lane);
        batch_dispatch<S, false>(D, xs[wv], ss[wv], cs[wv], lane);
    }
}

// grid: blocks of the streaming kernel (0: no full chunk); tail_grid: blocks
// of the ragged-chunk kernel (0: none).
typedef hipError_t (*BatchLaunch)(const BatchParams &, hipStream_t, int grid, int tail_grid);
struct BatchTable {
    BatchLaunch fn[kNumSIdx];
    const void *kern[kNumSIdx];
};
void register_batch_s2(BatchTable &);
void register_batch_s4(BatchTable &);
void register_batch_s8(BatchTable &);

template <int S>
hipError_t launch_batch(const BatchParams &bp, hipStream_t stream, int grid, int tail_grid)
{
    if (grid > 0) {
        hipLaunchKernelGGL((batch_kernel<S>), dim3((uint32_t)grid), dim3(kBlock), 0, stream, bp);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tail_grid > 0) {
        hipLaunchKernelGGL((batch_tail_kernel<S>), dim3((uint32_t)tail_grid), dim3(kBlock), 0, stream, bp);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace dpd
