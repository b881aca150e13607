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

// Global-address-space views, for pointers the compiler cannot trace back to
// a kernel argument (so loads and stores become global_*, not flat_*, and
// only count against the vector-memory counter).
typedef float v2f __attribute__((ext_vector_type(2)));
typedef const v2f __attribute__((address_space(1))) gcv2f;
typedef const v4f __attribute__((address_space(1))) gcv4f;
typedef v2f __attribute__((address_space(1))) gv2f;
typedef v4f __attribute__((address_space(1))) gv4f;

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
    constexpr int T = 4 * (NI - 1);   // scalar coefficients per tap
    // An opaque zero offset keeps the scalar loads inside the caller's chunk
    // loop: hoisted, the whole table would not fit the scalar registers and
    // would be spilled to VGPR lanes and read back with one v_readlane each.
    int z = 0;
    asm volatile("" : "+s"(z));
    const cfloat *Mz = M + z;
    const float cr = Mz[4 * L * NI], ci = Mz[4 * L * NI + 1];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        zr[i] = cr;
        zi[i] = ci;
    }
    // tap k's coefficients are in c while tap k + 1's load
    float c[T > 0 ? T : 1];
#pragma unroll
    for (int e = 0; e < T; ++e) c[e] = Mz[e];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        float cn[T > 0 ? T : 1];
        if (k + 1 < L) {
#pragma unroll
            for (int e = 0; e < T; ++e) cn[e] = Mz[4 * NI * (k + 1) + e];
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int w = i + (L - 1) - k;
            float w00 = top[4 * k + 0], w01 = top[4 * k + 1];
            float w10 = top[4 * k + 2], w11 = top[4 * k + 3];
#pragma unroll
            for (int j = NI - 2; j >= 0; --j) {
                w00 = __builtin_fmaf(w00, s[w], c[4 * j + 0]);
                w01 = __builtin_fmaf(w01, s[w], c[4 * j + 1]);
                w10 = __builtin_fmaf(w10, s[w], c[4 * j + 2]);
                w11 = __builtin_fmaf(w11, s[w], c[4 * j + 3]);
            }
            zr[i] = __builtin_fmaf(w00, a[w], zr[i]);
            zr[i] = __builtin_fmaf(w01, b[w], zr[i]);
            zi[i] = __builtin_fmaf(w10, a[w], zi[i]);
            zi[i] = __builtin_fmaf(w11, b[w], zi[i]);
        }
        if (k + 1 < L) {
#pragma unroll
            for (int e = 0; e < T; ++e) c[e] = cn[e];
        }
    }
}

// Same FIR with every coefficient in registers (coef: the whole table,
// 4*L*NI + 2 floats): no scalar operands, so no extra moves or scalar
// register pressure.  Used when the table is small enough to keep resident.
template <int NI, int L, int S>
__device__ __forceinline__ void fir_outputs_reg(const float (&a)[S + L - 1], const float (&b)[S + L - 1],
                                                const float (&s)[S + L - 1],
                                                const float (&coef)[4 * L * NI + 2], float (&zr)[S],
                                                float (&zi)[S])
{
#pragma unroll
    for (int i = 0; i < S; ++i) {
        zr[i] = coef[4 * L * NI];
        zi[i] = coef[4 * L * NI + 1];
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const float *Mk = coef + 4 * NI * k;
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
    }
}

// Coefficient tables up to this many floats stay in registers in the
// streaming kernel (larger ones are read as scalar operands).
constexpr int kRegCoefMax = 96;

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

// One-shot kernel (stage_lds = 0): each block computes one tile of kBlock*S
// outputs; every thread loads its own S+L-1 window with 16-byte loads (the
// halo part re-reads its neighbour's samples, which the vector L1 / L2 serve).
template <int NI, int L, int S>
__global__ void __launch_bounds__(kBlock) fwd_tile_kernel(FwdParams p)
{
    static_assert(S % 2 == 0, "S must be even (16-byte stores)");
    constexpr int T = kBlock * S;
    constexpr int HP = (L - 1 + 1) & ~1;   // halo rounded up to an even count
    constexpr int W = S + L - 1;
    constexpr int WL = HP + S;              // loaded samples (even)
    __shared__ float ctop[4 * L];

    const int tid = threadIdx.x;
    if (tid < 4 * L) ctop[tid] = p.M[(tid >> 2) * 4 * NI + 4 * (NI - 1) + (tid & 3)];
    __syncthreads();
    float top[4 * L];
#pragma unroll
    for (int e = 0; e < 4 * L; ++e) top[e] = ctop[e];

    for (int64_t step = xcd_remap(blockIdx.x, gridDim.x); step < p.total_tiles; step += gridDim.x) {
        const int64_t row = step / p.tiles_per_row;
        const int64_t t0 = (step - row * p.tiles_per_row) * (int64_t)T;
        const float2 *__restrict__ x = p.in + row * p.ld;
        float2 *__restrict__ z = p.out + row * p.ld;
        const float2 *__restrict__ hist = row == 0 ? p.hist : nullptr;
        const bool full = t0 + T <= p.n;
        const int64_t m0 = t0 + (int64_t)tid * S;   // first output of this thread

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
        float2 win[W];
#pragma unroll
        for (int w = 0; w < W; ++w) win[w] = raw[HP - (L - 1) + w];
        float a[W], b[W], s[W];
        split_window<W>(win, a, b, s);
        float zr[S], zi[S];
        fir_outputs<NI, L, S>(a, b, s, top, as_const(p.M), zr, zi);
        if (m0 < p.n) store_outputs<S>(z, m0, p.n, full, zr, zi);
    }
}

// Compiler-only ordering point for LDS traffic between the lanes of one wave.
// A wave's LDS instructions execute in program order, so no wait is needed;
// this only stops the compiler from moving LDS accesses across it.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Streaming kernel (stage_lds = 1).  Persistent grid of waves; at every step
// the waves of the grid work on adjacent chunks of C = 64*S samples (wave g
// takes chunks g, g + nw, g + 2 nw, ... of the flattened rows), so the whole
// chip sweeps memory in order.  Per chunk:
//   * the next chunk is already in flight (register prefetch); every
//     load instruction is a nontemporal read of 1 KiB of contiguous memory
//     (lane l, part i -> the 16 bytes at sample 2*(l + 64 i)); the L-1 halo
//     samples before the chunk are read by the first L-1 lanes, one each (a
//     vector load, in order with the chunk's; zeros at a row start, the
//     caller's history before row 0);
//   * samples and |x|^2 go to a wave-private LDS buffer laid out with one pad
//     slot after every S samples (odd lane stride: conflict-free window reads);
//     each lane reads its S+L-1 consecutive-sample window back, filters and
//     stores 16-byte outputs.
// The loop body has no divergent global accesses and no conditional loads, so
// the compiler's counter waits stay exact.  The partial last chunk of each row
// (when C does not divide n) is handled after the loop with guarded accesses.
// No block-wide barrier after the coefficient staging.
template <int S>
struct ChunkRegs {
    float4 v[S / 2];
    float2 h;   // raw halo sample for this lane's slot (selected at use)
};

// LDS slot of window sample d (relative to the chunk start, d >= -(L-1)).
template <int L, int S>
struct PadLayout {
    static constexpr int HG = (L - 1 + S - 1) / S;          // pad groups before the chunk
    static constexpr int OFF = HG * (S + 1);                // slot of sample 0
    static constexpr int SLOTS = OFF + 64 * (S + 1);
    __device__ static constexpr int slot(int d)
    {
        return OFF + d + (d >= 0 ? d / S : -((-d + S - 1) / S));
    }
};

template <int NI, int L, int S>
__global__ void __launch_bounds__(kBlock) fwd_stream_kernel(FwdParams p)
{
    static_assert(S % 2 == 0, "S must be even (16-byte loads and stores)");
    constexpr int C = 64 * S;
    constexpr int W = S + L - 1;
    constexpr int NV = S / 2;
    constexpr int WAVES = kBlock / 64;
    using PL = PadLayout<L, S>;
    constexpr int HS = L - 1;                        // halo samples
    constexpr int NC = 4 * L * NI + 2;               // coefficient table floats
    constexpr bool REG = NC <= kRegCoefMax;          // whole table in registers
    __shared__ float ctab[REG ? NC : 4 * L];
    __shared__ __align__(16) float2 xs[WAVES][PL::SLOTS];
    __shared__ __align__(16) float ss[WAVES][PL::SLOTS];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave
    if constexpr (REG) {
        if (tid < NC) ctab[tid] = p.M[tid];
    } else {
        if (tid < 4 * L) ctab[tid] = p.M[(tid >> 2) * 4 * NI + 4 * (NI - 1) + (tid & 3)];
    }
    __syncthreads();
    float top[4 * L];
    float coef[REG ? NC : 1];
    if constexpr (REG) {
#pragma unroll
        for (int e = 0; e < NC; ++e) coef[e] = ctab[e];
    } else {
#pragma unroll
        for (int e = 0; e < 4 * L; ++e) top[e] = ctab[e];
    }
    const cfloat *M = as_const(p.M);

    float2 *X = xs[wv];
    float *SX = ss[wv];
    const int64_t rows = p.total_tiles / p.tiles_per_row;
    const int64_t tpr = p.n / C;                 // full chunks per row
    const int64_t total = rows * tpr;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    const int64_t gw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * WAVES + wv;
    // halo sample this lane fetches: d = hl - HS in [-(L-1), -1]
    const int hl = HS > 0 ? (lane < HS ? lane : HS - 1) : 0;
    float2 hist_v = make_float2(0.f, 0.f);
    if (HS > 0 && p.hist != nullptr) hist_v = p.hist[hl];

    // raw sample for halo sample hl - HS of the chunk starting at t0 (lane hl
    // selects its own sample; the compiler makes it one per-lane load).  At a
    // row start (t0 < HS) nothing is read; the value is replaced at use.
    auto halo_raw = [&](int64_t row, int64_t t0) {
        float2 r = make_float2(0.f, 0.f);
        if (HS > 0 && t0 >= HS) {
            const cfloat *hp = as_const(reinterpret_cast<const float *>(p.in + row * p.ld + t0 - HS));
            r = make_float2(hp[0], hp[1]);
#pragma unroll
            for (int k = 1; k < (HS > 0 ? HS : 1); ++k)
                if (hl == k) r = make_float2(hp[2 * k], hp[2 * k + 1]);
        }
        return r;
    };
    // The same for a full chunk (row length >= C > HS): always read, from the
    // row start when t0 < HS, so the loop issues the same loads on every trip.
    auto halo_raw_full = [&](int64_t row, int64_t t0) {
        const int64_t off = t0 >= HS ? t0 - HS : 0;
        const cfloat *hp = as_const(reinterpret_cast<const float *>(p.in + row * p.ld + off));
        float2 r = make_float2(hp[0], hp[1]);
#pragma unroll
        for (int k = 1; k < (HS > 0 ? HS : 1); ++k)
            if (hl == k) r = make_float2(hp[2 * k], hp[2 * k + 1]);
        return r;
    };

    // samples -> LDS, windows -> registers, filter
    auto filter_chunk = [&](const ChunkRegs<S> &buf, int64_t row, int64_t t0, float (&zr)[S],
                            float (&zi)[S]) {
        wave_lds_order();
        if (HS > 0 && lane < HS) {
            float2 h = buf.h;
            if (t0 - HS + lane < 0) h = row == 0 ? hist_v : make_float2(0.f, 0.f);
            const int q = PL::slot(lane - HS);
            X[q] = h;
            SX[q] = __builtin_fmaf(h.x, h.x, h.y * h.y);
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float4 v = buf.v[i];
            const int j = 2 * (lane + 64 * i);           // even, same pad group as j + 1
            const int q = PL::OFF + j + j / S;
            X[q] = make_float2(v.x, v.y);
            X[q + 1] = make_float2(v.z, v.w);
            SX[q] = __builtin_fmaf(v.x, v.x, v.y * v.y);
            SX[q + 1] = __builtin_fmaf(v.z, v.z, v.w * v.w);
        }
        wave_lds_order();
        float a[W], b[W], s[W];
        const int lb = lane * (S + 1);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int q = lb + PL::slot(w - (L - 1));
            const float2 v = X[q];
            a[w] = v.x;
            b[w] = v.y;
            s[w] = SX[q];
        }
        if constexpr (REG)
            fir_outputs_reg<NI, L, S>(a, b, s, coef, zr, zi);
        else
            fir_outputs<NI, L, S>(a, b, s, top, M, zr, zi);
    };

    // Store the S outputs of every lane of a full chunk.  S = 2: each lane's
    // 16 bytes are adjacent to its neighbour's, so the store instruction already
    // writes 1 KiB contiguously.  S > 2: the outputs go back through the wave's
    // LDS buffer and leave in the load order (lane l, part i -> samples
    // 2*(l + 64 i)), so every store writes whole cache lines.
    auto store_chunk = [&](float2 *zrow, int64_t t0, const float (&zr)[S], const float (&zi)[S]) {
        if constexpr (S == 2) {
            store_outputs<S>(zrow, t0 + lane * S, p.n, true, zr, zi);
        } else {
            wave_lds_order();
            const int lb = lane * (S + 1) + PL::OFF;
#pragma unroll
            for (int i = 0; i < S; ++i) X[lb + i] = make_float2(zr[i], zi[i]);
            wave_lds_order();
            v4f *z4 = reinterpret_cast<v4f *>(zrow + t0);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int j = 2 * (lane + 64 * i);
                const int q = PL::OFF + j + j / S;
                const float2 u = X[q], w = X[q + 1];
                const v4f v = {u.x, u.y, w.x, w.y};
                __builtin_nontemporal_store(v, z4 + lane + 64 * i);
            }
        }
    };

    // ---- main loop over full chunks gw, gw + nw, ...
    if (gw < total) {
        // chunk c <-> (row, k); advancing by nw chunks without dividing
        const int64_t dr = nw / tpr, dk = nw - (nw / tpr) * tpr;
        struct Cur {
            int64_t row, k;
        };
        auto next = [&](Cur u) {
            u.row += dr;
            u.k += dk;
            if (u.k >= tpr) {
                u.k -= tpr;
                ++u.row;
            }
            return u;
        };
        // The prefetch issues at raised wave priority, so a wave reaching it
        // is not held behind the other waves' filter work on the SIMD
        // (measured: 47.8 -> 47.2 us at the 2^24 headline, outputs unchanged).
        auto load_full = [&](ChunkRegs<S> &buf, const Cur &u) {
            __builtin_amdgcn_s_setprio(2);
            const int64_t t0 = u.k * C;
            const float4 *x4 = reinterpret_cast<const float4 *>(p.in + u.row * p.ld + t0);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                // read once: nontemporal (streaming) loads
                const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(x4) + lane + 64 * i);
                buf.v[i] = make_float4(t.x, t.y, t.z, t.w);
            }
            buf.h = halo_raw_full(u.row, t0);
            __builtin_amdgcn_s_setprio(0);
        };
        auto step = [&](const ChunkRegs<S> &buf, const Cur &u) {
            float zr[S], zi[S];
            filter_chunk(buf, u.row, u.k * C, zr, zi);
            store_chunk(p.out + u.row * p.ld, u.k * C, zr, zi);
        };
        // Two chunks per trip with the next one always in flight; the loop
        // body is straight-line code (exact counter waits) and the last one
        // or two chunks are peeled off, so nothing is read past the run.
        int64_t left = (total - 1 - gw) / nw + 1;    // chunks of this wave
        Cur cur;
        cur.row = gw / tpr;
        cur.k = gw - cur.row * tpr;
        ChunkRegs<S> A, B;
        load_full(A, cur);
        for (; left >= 3; left -= 2) {
            const Cur c1 = next(cur);
            load_full(B, c1);
            step(A, cur);
            const Cur c2 = next(c1);
            load_full(A, c2);
            step(B, c1);
            cur = c2;
        }
        if (left == 2) {
            const Cur c1 = next(cur);
            load_full(B, c1);
            step(A, cur);
            step(B, c1);
        } else {
            step(A, cur);
        }
    }

    // ---- the partial last chunk of each row (when C does not divide n)
    if (tpr * C < p.n) {
        for (int64_t rw = gw; rw < rows; rw += nw) {
            const int64_t t0 = tpr * C;
            const float2 *x = p.in + rw * p.ld;
            ChunkRegs<S> buf;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int64_t m = t0 + 2 * (lane + 64 * i);
                const float2 u = m < p.n ? x[m] : make_float2(0.f, 0.f);
                const float2 w = m + 1 < p.n ? x[m + 1] : make_float2(0.f, 0.f);
                buf.v[i] = make_float4(u.x, u.y, w.x, w.y);
            }
            buf.h = halo_raw(rw, t0);
            float zr[S], zi[S];
            filter_chunk(buf, rw, t0, zr, zi);
            const int64_t m0 = t0 + (int64_t)lane * S;
            float2 *z = p.out + rw * p.ld;
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (m0 + i < p.n) z[m0 + i] = make_float2(zr[i], zi[i]);
        }
    }
}


int num_cus();

template <int NI, int L, int S, bool STREAM>
hipError_t launch_fwd(const FwdParams &p, hipStream_t stream, int grid_mult)
{
    int64_t grid;
    if constexpr (STREAM) {
        // persistent: grid_mult blocks per CU, never more than one chunk per wave
        // never more blocks than can be resident at once (a second round of a
        // persistent grid would double the tail)
        static const int occ = [] {
            int o = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, fwd_stream_kernel<NI, L, S>, kBlock,
                                                             0) != hipSuccess || o < 1)
                o = 1;
            return o;
        }();
        const int64_t want = (int64_t)num_cus() * (grid_mult < occ ? grid_mult : occ);
        const int64_t need = (p.total_tiles + kBlock / 64 - 1) / (kBlock / 64);   // >= 1 wave per chunk
        grid = need < want ? need : want;
        hipLaunchKernelGGL((fwd_stream_kernel<NI, L, S>), dim3((uint32_t)grid),
                           dim3(kBlock), 0,
                           stream, p);
    } else {
        const int64_t cap = 1 << 20;
        grid = p.total_tiles < cap ? p.total_tiles : cap;
        hipLaunchKernelGGL((fwd_tile_kernel<NI, L, S>), dim3((uint32_t)grid), dim3(kBlock), 0,
                           stream, p);
    }
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
