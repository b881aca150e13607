// Least-squares coefficient estimation (section 2.2, Eq. 2) on the GPU: the
// normal equations A = Psi^H Psi, b = Psi^H t of the APH basis, and their
// Cholesky solve.  Used by the indirect-learning loop (postdistorter fitted
// from PA output to PA input, then copied into the predistorter).
//
// Row m of Psi is [psi_p(y_{m-k}) ..., conj(psi_q(y_{m-k})) ..., 1] in the
// section 2.2 stacking (K columns), with zero samples before each row start
// (the first M rows of the zero-filled element matrices of Eq. (2)).
//
// Real formulation.  With the 2K+2 real features of a sample,
//     f = [Re Psi_m (K), Im Psi_m (K), Re t_m, Im t_m],
// the real Gram R = sum_m f f^T carries everything:
//     Re A = R_rr + R_ii,      Im A = R_ri - R_ri^T,
//     Re b = R_r,t_r + R_i,t_i,  Im b = R_r,t_i - R_i,t_r.
// R is a dense contraction over samples, so it runs on the matrix cores:
// v_mfma_f32_16x16x32_bf16 over 16x16 tiles of the upper triangle of R.  The
// basis psi_j of 64 samples at a time (and of the L - 1 before them) is staged
// in LDS once per input sample, each FP32 value as a bf16 high part and the
// bf16 rounding of its remainder, and the tap columns read it shifted; the four cross products of
// every pair of features are summed in FP32 (the dropped terms are ~2^-17 of
// each product, below FP32 accumulation error).  Each block covers one slab
// of 1024..8192 samples (the size depends only on the input shape and the
// number of CUs) and writes its FP32 tiles (each FP32 accumulator adds the
// eight-sample steps of a quarter of the slab -- at most 256 -- or, when the
// basis needs 8 or more column tiles and the tile pairs split into two groups
// of two waves, of half the slab -- at most 512; the partial tiles of the
// waves are summed in FP32); the slabs are summed in FP64 in a fixed order
// (two levels), so the result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <type_traits>
#include <utility>

#include "dpd.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {

typedef float v4f_ls __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_ls __attribute__((ext_vector_type(8)));
typedef unsigned u32x4_ls __attribute__((ext_vector_type(4)));

constexpr int kLsTile = 64;         // samples staged per step
constexpr int kLsSolveMaxK = 1024;  // one wave, at most 16 rows per lane
constexpr int kLsSlabMax = 8192;    // samples per block / FP32 partial (at most)
constexpr int kLsSlabMin = 1024;
constexpr int kLsMaxDp = 192;       // padded real features (2K+2 rounded up to 16): K <= 95
constexpr int kLsMaxNt = kLsMaxDp / 16;
constexpr int kLsWaves = kBlock / 64;
constexpr int kLsGroup = 64;        // slabs per first-level FP64 sum

// Entries of a basis row (roles): Re psi_j, Im psi_j, -Im psi_j for each
// power level j, the constant, a zero and the target (Re, Im).
constexpr int kLsRIm = kMaxNI, kLsRNegIm = 2 * kMaxNI;
constexpr int kLsROne = 3 * kMaxNI, kLsRZero = kLsROne + 1, kLsRT = kLsROne + 2;
constexpr int kLsRoles = kLsRT + 2;
static_assert(kLsRoles <= 32 && kLsRoles <= 3 * kMaxNI + 5, "plan slot table too small");

struct LsParams {
    const float2 *y;        // basis input, rows x ld
    const float2 *t;        // target, same layout
    int64_t n, ld;
    int64_t slabs_per_row;
    int64_t slab;           // samples per block (a multiple of kLsTile)
    float y_scale;          // the basis is built from y_scale * y
    float *partials;        // [slab][pair][256]
    int K, D, Dp, nt, npairs;
    int L, NI;
    int16_t off[kLsMaxDp];  // LDS word of feature f relative to the basis row of the sample
    int8_t slot[kLsRoles];  // LDS row slot of each basis entry
};

// Tile pair q of the upper triangle, row-major over (I <= J), at compile time.
constexpr int ls_pair_i(int q, int nt)
{
    int I = 0;
    while (q >= nt - I) {
        q -= nt - I;
        ++I;
    }
    return I;
}
constexpr int ls_pair_j(int q, int nt)
{
    int I = 0;
    while (q >= nt - I) {
        q -= nt - I;
        ++I;
    }
    return I + q;
}

// A feature as its bf16 high part (low half) and the bf16 rounding of the
// remainder (high half): f = hi + lo to about 2^-16 relative, so the four
// cross products of two features carry FP32-level accuracy.
__device__ __forceinline__ uint32_t ls_pack(float f)
{
    const __bf16 h = (__bf16)f;
    const __bf16 l = (__bf16)(f - (float)h);
    return (uint32_t)__builtin_bit_cast(unsigned short, h) | ((uint32_t)__builtin_bit_cast(unsigned short, l) << 16);
}

typedef float f32x2_ls __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_ls __attribute__((ext_vector_type(2)));

// ls_pack of two values with two packed conversions (round to nearest even).
__device__ __forceinline__ void ls_pack2(float a, float b, uint32_t &wa, uint32_t &wb)
{
    const uint32_t hw = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_ls{a, b}, bf16x2_ls));
    const float ha = __uint_as_float(hw << 16), hb = __uint_as_float(hw & 0xffff0000u);
    const uint32_t lw = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_ls{a - ha, b - hb}, bf16x2_ls));
    wa = __builtin_amdgcn_perm(lw, hw, 0x05040100u);   // (hw & 0xffff) | (lw << 16)
    wb = __builtin_amdgcn_perm(lw, hw, 0x07060302u);   // (hw >> 16) | (lw & 0xffff0000)
}

// One 8-sample step of the pairs Q0, Q0 + 1, ...: a[b] / c[b] are operand
// block b as (hi, lo, hi, lo) per sample and as (hi, hi, lo, lo), so every
// sample contributes hi hi' + lo hi' + hi lo' + lo lo'.  The blocks of each
// pair are compile-time constants (forced).
template <int NT, int Q0, int... U>
__device__ __forceinline__ void ls_gram_step(v4f_ls *acc, const bf16x8_ls *a, const bf16x8_ls *c,
                                             std::integer_sequence<int, U...>)
{
    ((acc[U] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[std::integral_constant<int, ls_pair_i(Q0 + U, NT)>::value],
                                                       c[std::integral_constant<int, ls_pair_j(Q0 + U, NT)>::value],
                                                       acc[U], 0, 0, 0)),
     ...);
}

// Pair groups of the Gram kernel for NT column tiles: one (every wave holds
// all NT (NT + 1) / 2 tile accumulators) while they fit in 128 registers,
// else two (two waves per group).
constexpr int ls_pair_groups(int nt) { return nt * (nt + 1) / 2 * 4 <= 128 ? 1 : 2; }

// The basis of a tile in LDS: one row per input sample (the tile's 64 samples
// and the L - 1 before them), holding psi_j of that sample as packed words
// (Re, Im and -Im of every power level), the constant 1 (0 outside the slab),
// a zero word and the target t, each entry twice (two equal words, so that
// one 64-bit read per sample gives the row-side operand).  Row m of Psi
// repeats the rows of samples m, m-1, ..., m-L+1 (Eq. 2 is Toeplitz in the
// taps), so each Gram column f reads the word off[f] = (L - 1 - k) stride +
// 2 slot(f) relative to row m.  The slot of each entry in a row is chosen per
// basis layout on the host (ls_layout) to spread the matrix phase's reads over
// the LDS banks.
constexpr int kLsBEntries = 3 * kMaxNI + 5;        // slots per row (odd: rows start on rotating banks)
constexpr int kLsBStride = 2 * kLsBEntries;        // words per row
constexpr int kLsRows = kLsTile + kMaxL - 1;

// One 64-sample tile of the matrix phase.  Lane l feeds row / column l % 16
// and samples 2 (l / 16), 2 (l / 16) + 1 of each 8-sample step (four slots
// each); a step's operand blocks are read once and feed every pair; a
// scheduling barrier per step keeps one step's operands in registers.  mid()
// runs first (the next tile's basis goes into the other LDS buffer: kept out
// of the matrix steps, where its branches would make the accumulators move
// between registers).  With MASK the samples at or past vt (the end of the
// slab) contribute nothing: their row-side operands are zeroed.
template <int NT, int Q0, int PW, int GK, bool MASK, typename Mid>
__device__ __forceinline__ void ls_gram_tile(v4f_ls *acc, const uint32_t *Xf, const int *addr, int kw, int g2,
                                             int vt, Mid mid)
{
    mid();   // the next tile's basis, into the other buffer
#pragma unroll
    for (int i = 0; i < kLsTile / 8 / GK; ++i) {
        const int row = 8 * GK * i;   // step kw + GK i, relative to the wave's first step
        bf16x8_ls a[NT], cb[NT];      // blocks no pair of the group uses are never loaded
        bool ok0 = true, ok1 = true;
        if constexpr (MASK) {
            const int m = 8 * (kw + GK * i) + g2;
            ok0 = m < vt;
            ok1 = m + 1 < vt;
        }
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            const uint2 p0 = *reinterpret_cast<const uint2 *>(Xf + addr[b] + row * kLsBStride);
            const uint2 p1 = *reinterpret_cast<const uint2 *>(Xf + addr[b] + (row + 1) * kLsBStride);
            // (hi, lo, hi, lo) against (hi', hi', lo', lo'): the four slots of a
            // sample give hi hi' + lo hi' + hi lo' + lo lo' (the column side
            // by byte permutes written straight into the operand)
            const u32x4_ls av = MASK ? u32x4_ls{ok0 ? p0.x : 0u, ok0 ? p0.y : 0u, ok1 ? p1.x : 0u, ok1 ? p1.y : 0u}
                                     : u32x4_ls{p0.x, p0.y, p1.x, p1.y};
            const u32x4_ls bv = {__builtin_amdgcn_perm(p0.x, p0.x, 0x01000100u), __builtin_amdgcn_perm(p0.y, p0.y, 0x03020302u),
                                 __builtin_amdgcn_perm(p1.x, p1.x, 0x01000100u), __builtin_amdgcn_perm(p1.y, p1.y, 0x03020302u)};
            a[b] = __builtin_bit_cast(bf16x8_ls, av);
            cb[b] = __builtin_bit_cast(bf16x8_ls, bv);
        }
        ls_gram_step<NT, Q0>(acc, a, cb, std::make_integer_sequence<int, PW>{});
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One wave's part of a slab.  The waves of pair group G (GK = 4 / GP of
// them) accumulate the tile pairs [G PP, (G + 1) PP) of the row-major upper
// triangle, each over every GK-th 8-sample step of each 64-sample tile, so
// a step loads each 16-column operand block once for all of its pairs.  All
// four waves build the basis rows of each tile together, one tile ahead into
// the other of two LDS buffers (one barrier per tile): wave w the power levels
// [w lpw, (w + 1) lpw), the last wave also the constant and target words.  At
// the end the GK partial tiles of each pair are summed through LDS (fixed
// order) and written out.  The pair list is a compile-time
// constant: the matrix loop has no conditionals (a guarded accumulation
// becomes a branch whose merge copies every accumulator) and every wave runs
// the same code.
template <int NT, int G>
__device__ __forceinline__ void ls_gram_wave(const LsParams &p, uint32_t (*X)[kLsBStride], int64_t slab, int64_t s0,
                                             int64_t send, const float2 *yr, const float2 *tr)
{
    constexpr int NP = NT * (NT + 1) / 2;
    constexpr int GP = ls_pair_groups(NT);
    constexpr int GK = kLsWaves / GP;
    constexpr int PP = (NP + GP - 1) / GP;
    constexpr int Q0 = G * PP;
    constexpr int PW = NP - Q0 < PP ? NP - Q0 : PP;   // pairs of this group
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kw = wv % GK;                           // this wave's steps: kw, kw + GK, ...
    v4f_ls acc[PW];
#pragma unroll
    for (int u = 0; u < PW; ++u) acc[u] = v4f_ls{0.f, 0.f, 0.f, 0.f};

    // operand addresses (words) of the lane's column in each block, at the
    // wave's first step
    const int g2 = 2 * (lane >> 4), c = lane & 15;
    int addr[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) addr[b] = (8 * kw + g2) * kLsBStride + p.off[16 * b + c];

    // Basis rows: row r holds sample m0 - H + r of tile m0, so the tile's own
    // samples are rows H..H+63 (lane l builds row H + l) and the H rows before
    // them are rows 64..63+H of the previous tile.  Two LDS buffers: tile
    // t + 1 is built into one (its carried rows copied from tile t's) just
    // before the matrix steps of tile t on the other, one barrier per tile.  A
    // lane's sample and target are loaded two tiles ahead of their matrix
    // phase.
    // 32-bit sample indices relative to the slab start: nl samples in the
    // slab, inputs valid from index lo on (the row start, or kMaxL samples
    // back).
    const int H = p.L - 1;
    const bool halo = lane < H;
    const bool last = wv == kLsWaves - 1;
    const int lpw = (p.NI + kLsWaves - 1) / kLsWaves;
    const int j0 = wv * lpw, nj = std::min(p.NI - j0, lpw);
    constexpr int UJ = (kMaxNI + kLsWaves - 1) / kLsWaves;   // levels per wave at most
    // the row slots of this wave's level entries (Re, Im, -Im)
    int sre[UJ], sim[UJ], sng[UJ];
#pragma unroll
    for (int u = 0; u < UJ; ++u) {
        const int j = (j0 + u) & (kMaxNI - 1);   // in range also where u >= nj (unused there)
        sre[u] = p.slot[j];
        sim[u] = p.slot[kLsRIm + j];
        sng[u] = p.slot[kLsRNegIm + j];
    }
    const float2 *ys = yr + s0, *ts = tr + s0;
    const int nl = (int)(send - s0);
    const int lo = s0 >= kMaxL ? -kMaxL : (int)-s0;
    // (zeros as literals: a named zero turns the guarded loads into flat
    // loads through a pointer select, with the zero in scratch memory)
    float2 y0 = make_float2(0.f, 0.f), t0 = y0;
    auto fetch = [&](int m0) {
        const int q = m0 + lane;
        y0 = q < nl ? ys[q] : make_float2(0.f, 0.f);
        if (last) t0 = q < nl ? ts[q] : make_float2(0.f, 0.f);
    };
    auto put = [](uint32_t *x, int e, uint32_t w) {
        x[2 * e] = w;
        x[2 * e + 1] = w;
    };
    // psi_j for j in [j0, j0 + nj) of sample y into row x (nj <= UJ uniform)
    auto levels = [&](uint32_t *x, float2 y) {
        const float vx = p.y_scale * y.x, vy = p.y_scale * y.y;
        const float s2 = __builtin_fmaf(vx, vx, vy * vy);
        float pw = 1.f;
        for (int e = 0; e < j0; ++e) pw *= s2;
#pragma unroll
        for (int u = 0; u < UJ; ++u) {
            if (u < nj) {
                uint32_t wa, wb;
                ls_pack2(pw * vx, pw * vy, wa, wb);
                put(x, sre[u], wa);
                put(x, sim[u], wb);
                put(x, sng[u], wb ^ 0x80008000u);   // -b: both parts negated exactly
                pw *= s2;
            }
        }
    };
    // tile m0 into buffer B (the carried rows from buffer B ^ 1 unless first)
    auto build = [&](int m0, uint32_t (*B)[kLsBStride], const uint32_t (*P)[kLsBStride]) {
        if (m0 > 0 && halo) {
            const uint2 *src = reinterpret_cast<const uint2 *>(P[64 + lane]);
            uint2 *dst = reinterpret_cast<uint2 *>(B[lane]);
#pragma unroll
            for (int u = 0; u < UJ; ++u) {
                if (u < nj) {
                    dst[sre[u]] = src[sre[u]];
                    dst[sim[u]] = src[sim[u]];
                    dst[sng[u]] = src[sng[u]];
                }
            }
        }
        uint32_t *x = B[H + lane];
        levels(x, y0);
        if (last) {
            uint32_t ta, tb;
            ls_pack2(t0.x, t0.y, ta, tb);
            put(x, p.slot[kLsROne], m0 + lane < nl ? ls_pack(1.f) : 0u);
            put(x, p.slot[kLsRZero], 0u);
            put(x, p.slot[kLsRT], ta);
            put(x, p.slot[kLsRT + 1], tb);
        }
        if (m0 + kLsTile < nl) fetch(m0 + kLsTile);
    };
    // the rows before the slab's first tile (zero before the row start)
    if (halo) {
        const int q = lane - H;
        levels(X[lane], q >= lo ? ys[q] : make_float2(0.f, 0.f));
    }
    fetch(0);
    build(0, X, X);
    __syncthreads();
    // whole tiles, then the ragged one (apart, so that the loop carries the
    // accumulators in place)
    int m0 = 0, cur = 0;
    for (; m0 + kLsTile <= nl; m0 += kLsTile, cur ^= 1) {
        uint32_t(*B)[kLsBStride] = X + cur * kLsRows;
        uint32_t(*N)[kLsBStride] = X + (cur ^ 1) * kLsRows;
        const int mn = m0 + kLsTile;
        ls_gram_tile<NT, Q0, PW, GK, false>(acc, &B[0][0], addr, kw, g2, kLsTile, [&]() {
            if (mn < nl) build(mn, N, B);
        });
        __syncthreads();   // tile m0's reads and tile m0 + 64's writes are done
    }
    if (m0 < nl)
        ls_gram_tile<NT, Q0, PW, GK, true>(acc, &X[cur * kLsRows][0], addr, kw, g2, nl - m0, []() {});
    // Sum the GK partial tiles of each pair: the four waves put their
    // accumulators (pair u of their group) in LDS, then the waves of a group
    // each add up 4 / GK of the register slots, in wave order.  Tile element
    // (4 (l / 16) + v, l % 16) is register v of lane l.
    float *buf = reinterpret_cast<float *>(&X[0][0]);   // 4 x 256 floats (kLsRows x kLsBStride >= 1024 words)
    float *out = p.partials + (slab * NP + Q0) * 256;
    for (int u = 0; u < PP; ++u) {
        __syncthreads();   // the matrix reads of the last tile / the previous pair's sums are done
        if (u < PW) {
#pragma unroll
            for (int v = 0; v < 4; ++v) buf[wv * 256 + lane * 4 + v] = acc[u][v];
        }
        __syncthreads();
        if (u < PW) {
            constexpr int VPW = 4 / GK;   // register slots per wave
#pragma unroll
            for (int vv = 0; vv < VPW; ++vv) {
                const int v = kw * VPW + vv;
                float t = 0.f;
#pragma unroll
                for (int w = 0; w < GK; ++w) t += buf[(G * GK + w) * 256 + lane * 4 + v];
                out[u * 256 + (4 * (lane >> 4) + v) * 16 + (lane & 15)] = t;
            }
        }
    }
}

// Normal equations of one slab of samples: the basis of 64 samples at a time
// staged in LDS (two buffers), then the upper triangle of the real Gram on the matrix
// cores, FP32 tiles per slab.  One instance per column-tile count NT.
template <int NT>
__global__ void __launch_bounds__(kBlock) ls_gram_kernel(LsParams p)
{
    static_assert(kLsRows * kLsBStride >= kLsWaves * 256, "LDS tile too small for the final sums");
    __shared__ __align__(16) uint32_t X[2 * kLsRows][kLsBStride];   // two tile buffers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t slab = blockIdx.x;
    const int64_t row = slab / p.slabs_per_row;
    const int64_t s0 = (slab - row * p.slabs_per_row) * p.slab;
    const float2 *yr = p.y + row * p.ld;
    const float2 *tr = p.t + row * p.ld;
    const int64_t send = std::min<int64_t>(s0 + p.slab, p.n);
    if constexpr (ls_pair_groups(NT) == 1) {
        ls_gram_wave<NT, 0>(p, X, slab, s0, send, yr, tr);
    } else {
        if (wv < kLsWaves / 2)
            ls_gram_wave<NT, 0>(p, X, slab, s0, send, yr, tr);
        else
            ls_gram_wave<NT, 1>(p, X, slab, s0, send, yr, tr);
    }
}

__global__ void __launch_bounds__(kBlock) ls_reduce1_kernel(const float *__restrict__ partials, int64_t nslabs,
                                                            int64_t E, double *__restrict__ r1)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= E) return;
    const int64_t g = blockIdx.y;
    const int64_t s1 = std::min<int64_t>(nslabs, (g + 1) * kLsGroup);
    // eight loads in flight at a time, the sum in slab order
    double t = 0.0;
    int64_t sl = g * kLsGroup;
    for (; sl + 8 <= s1; sl += 8) {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = partials[(sl + i) * E + e];
#pragma unroll
        for (int i = 0; i < 8; ++i) t += (double)v[i];
    }
    for (; sl < s1; ++sl) t += (double)partials[sl * E + e];
    r1[g * E + e] = t;
}

// Sum over the 64 lanes of a wave in FP64 (fixed butterfly: every lane gets
// the same total).
__device__ __forceinline__ double ls_wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// v of lane `src` (wave-uniform) in every lane, through scalar registers.
__device__ __forceinline__ double ls_bcast(double v, int src)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Index of the real-Gram entry R[i][j] (either order) in a slab's tile list:
// the upper-triangle element, so R is symmetric by construction.
__device__ __forceinline__ int64_t ls_entry(int i, int j, int nt)
{
    if (i > j) {
        const int t = i;
        i = j;
        j = t;
    }
    const int I = i >> 4, J = j >> 4;
    const int q = I * nt - I * (I - 1) / 2 + (J - I);   // row-major upper-triangle pair
    return (int64_t)q * 256 + (i & 15) * 16 + (j & 15);
}

// Second level and assembly: one wave per output (A row-major, then b).  Lane
// g sums groups g, g + 64, ... of the four real-Gram entries the output needs
// (in group order), a fixed butterfly adds the lanes, and
//   A[a][c] = (R[a][c] + R[K+a][K+c]) + i (R[a][K+c] - R[K+a][c]),
//   b[a]    = (R[a][tr] + R[K+a][ti]) + i (R[a][ti] - R[K+a][tr]),
// tr, ti = 2K, 2K+1.  A[c][a] reads the same entries, so A is Hermitian.
__global__ void __launch_bounds__(kBlock) ls_finish_kernel(const double *__restrict__ r1, int64_t groups, int64_t E,
                                                           int nt, int K, double2 *__restrict__ A,
                                                           double2 *__restrict__ b)
{
    const int64_t o = (int64_t)blockIdx.x * kLsWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (o >= (int64_t)K * K + K) return;   // the whole wave
    int a, c0, c1;                         // rows a, K + a against columns c0, c1
    if (o < (int64_t)K * K) {
        a = (int)(o / K);
        c0 = (int)(o % K);
        c1 = K + c0;
    } else {
        a = (int)(o - (int64_t)K * K);
        c0 = 2 * K;
        c1 = 2 * K + 1;
    }
    const int64_t e[4] = {ls_entry(a, c0, nt), ls_entry(K + a, c1, nt), ls_entry(a, c1, nt),
                          ls_entry(K + a, c0, nt)};
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t g = lane; g < groups; g += 64)
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] += r1[g * E + e[t]];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = ls_wave_sum(v[t]);
    if (lane == 0) {
        const double2 r = make_double2(v[0] + v[1], v[2] - v[3]);
        if (o < (int64_t)K * K)
            A[o] = r;
        else
            b[a] = r;
    }
}

// L y = b, then L^H h = y on the factor F (column-major at stride ld, the
// diagonal in place): one wave, lane l holding rows l, l + 64, ... (R of them)
// in registers; h in complex64, info = 0.
template <int R>
__device__ __forceinline__ void ls_substitute(const double2 *F, int ld, const double2 *__restrict__ b, int K,
                                              float2 *__restrict__ h, int32_t *__restrict__ info, int lane)
{
    int rc[R];   // owned rows clamped into the matrix (loads only)
#pragma unroll
    for (int t = 0; t < R; ++t) rc[t] = min(lane + 64 * t, K - 1);
    double invd[R];   // 1 / L[r][r] of the owned rows
#pragma unroll
    for (int t = 0; t < R; ++t) invd[t] = 1.0 / F[rc[t] * ld + rc[t]].x;
    double2 y[R], f[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int r = lane + 64 * t;
        y[t] = r < K ? b[r] : make_double2(0.0, 0.0);
        f[t] = F[rc[t]];   // column 0
    }
    for (int j = 0; j < K; ++j) {
        double2 fn[R];
        const int jn = min(j + 1, K - 1);
#pragma unroll
        for (int t = 0; t < R; ++t) fn[t] = F[jn * ld + rc[t]];   // L[r][j+1]
        double2 mine = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t == (j >> 6)) mine = make_double2(y[t].x * invd[t], y[t].y * invd[t]);
        const double2 yj = make_double2(ls_bcast(mine.x, j & 63), ls_bcast(mine.y, j & 63));
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int r = lane + 64 * t;
            if (r == j) {
                y[t] = yj;
            } else if (r > j) {
                // y_r -= L[r][j] y_j
                y[t].x -= f[t].x * yj.x - f[t].y * yj.y;
                y[t].y -= f[t].x * yj.y + f[t].y * yj.x;
            }
            f[t] = fn[t];
        }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) f[t] = F[rc[t] * ld + (K - 1)];   // L[K-1][r]
    for (int j = K - 1; j >= 0; --j) {
        double2 fn[R];
        const int jn = max(j - 1, 0);
#pragma unroll
        for (int t = 0; t < R; ++t) fn[t] = F[rc[t] * ld + jn];   // L[j-1][r]
        double2 mine = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t == (j >> 6)) mine = make_double2(y[t].x * invd[t], y[t].y * invd[t]);
        const double2 hj = make_double2(ls_bcast(mine.x, j & 63), ls_bcast(mine.y, j & 63));
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int r = lane + 64 * t;
            if (r == j) {
                y[t] = hj;
            } else if (r < j) {
                // y_r -= conj(L[j][r]) h_j
                y[t].x -= f[t].x * hj.x + f[t].y * hj.y;
                y[t].y -= f[t].x * hj.y - f[t].y * hj.x;
            }
            f[t] = fn[t];
        }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int r = lane + 64 * t;
        if (r < K) h[r] = make_float2((float)y[t].x, (float)y[t].y);
    }
    if (lane == 0) *info = 0;
}

// Cholesky solve of (A + delta I) h = b in FP64 by one wave, delta = ridge *
// mean(Re diag A).  Lane l owns rows l, l + 64, ... (R slots).  The factor is
// stored by columns, F[k ld + r] = L[r][k] (ld = 64 in LDS, where K <= 64,
// else K), zero above the diagonal, so the lanes read one column at
// consecutive addresses and the entries of row j are broadcasts.
// Left-looking: for column j every owned row r >= j forms
//   s_r = A[r][j] - sum_{k<j} L[r][k] conj(L[j][k]),
// G k per step into up to four partial sums.  The diagonal of A + delta I stays in
// its owner's registers and F's diagonal holds zero until L[j][j] is written,
// so the row-j factor of every k >= j reads zero: the last step of a column
// needs no mask.  s_j is the pivot (taken from its owner lane), L[j][j] =
// sqrt(s_j) and the rows below store s_r / L[j][j].  The triangular solves
// sweep columns: once y_j (then h_j) is final its owner broadcasts it and
// every row still open subtracts its multiple, the next column's entries
// already loading.  Loads use row indices clamped into the matrix (every
// value read is finite), so the inner loops have no per-lane branches; only
// rows a lane owns are stored.  info = 0, or j + 1 when the pivot of column
// j is not positive (h is then NaN).
template <bool LDS, int R>
__global__ void __launch_bounds__(64) ls_solve_kernel(const double2 *__restrict__ A, const double2 *__restrict__ b,
                                                      int K, double ridge, double2 *__restrict__ Fg,
                                                      float2 *__restrict__ h, int32_t *__restrict__ info)
{
    extern __shared__ double2 ls_smem[];
    double2 *F = LDS ? ls_smem : Fg;
    const int ld = LDS ? 64 : K;
    const int lane = threadIdx.x;
    int rc[R];   // owned rows clamped into the matrix (loads only)
#pragma unroll
    for (int t = 0; t < R; ++t) rc[t] = min(lane + 64 * t, K - 1);
    double tr = 0.0;
    for (int i = lane; i < K; i += 64) tr += A[(int64_t)i * K + i].x;
    const double delta = ridge * ls_wave_sum(tr) / K;
    double dg[R];   // Re A[r][r] + delta of the owned rows
#pragma unroll
    for (int t = 0; t < R; ++t) dg[t] = A[(int64_t)rc[t] * K + rc[t]].x + delta;
    // F = strict lower triangle of A (row r, column k), zero elsewhere; U
    // columns of loads in flight
    constexpr int U = R <= 2 ? 8 : (R <= 4 ? 4 : 2);
    for (int k0 = 0; k0 < K; k0 += U) {
        double2 v[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int r = lane + 64 * t, k = k0 + u;
                v[u][t] = (k < K && r > k && r < K) ? A[(int64_t)r * K + k] : make_double2(0.0, 0.0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int r = lane + 64 * t, k = k0 + u;
                if (k < K && r < K) F[k * ld + r] = v[u][t];
            }
    }
    __syncthreads();

    // k per step of the column sums (fewer when a lane owns more rows)
    constexpr int G = R == 1 ? 8 : (R == 2 ? 4 : (R == 4 ? 2 : 1));
    for (int j = 0; j < K; ++j) {
        constexpr int P = G >= 4 ? 4 : G;   // partial sums per row
        double2 s[P][R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            s[0][t] = F[j * ld + rc[t]];
            if (lane + 64 * t == j) s[0][t].x += dg[t];
#pragma unroll
            for (int e = 1; e < P; ++e) s[e][t] = make_double2(0.0, 0.0);
        }
        for (int k = 0; k < j; k += G) {
            double2 c[G], a[G][R];
            if (k + G <= K) {   // every column of the step exists
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    c[q] = F[(k + q) * ld + j];                                      // L[j][k]
#pragma unroll
                    for (int t = 0; t < R; ++t) a[q][t] = F[(k + q) * ld + rc[t]];  // L[r][k]
                }
            } else {
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const int kc = min(k + q, K - 1);
                    c[q] = F[kc * ld + j];
#pragma unroll
                    for (int t = 0; t < R; ++t) a[q][t] = F[kc * ld + rc[t]];
                }
            }
            __builtin_amdgcn_sched_barrier(0);   // every load of the step in flight first
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    double2 &acc = s[q % P][t];
                    // acc -= a * conj(c)
                    acc.x = fma(-a[q][t].x, c[q].x, acc.x);
                    acc.x = fma(-a[q][t].y, c[q].y, acc.x);
                    acc.y = fma(-a[q][t].y, c[q].x, acc.y);
                    acc.y = fma(a[q][t].x, c[q].y, acc.y);
                }
        }
        double mine = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
#pragma unroll
            for (int e = 1; e < P; ++e) {
                s[0][t].x += s[e][t].x;
                s[0][t].y += s[e][t].y;
            }
            if (t == (j >> 6)) mine = s[0][t].x;
        }
        const double piv = ls_bcast(mine, j & 63);
        if (!(piv > 0.0)) {
            for (int i = lane; i < K; i += 64) h[i] = make_float2(NAN, NAN);
            if (lane == 0) *info = j + 1;
            return;
        }
        const double d = sqrt(piv), inv = 1.0 / d;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int r = lane + 64 * t;
            if (r == j)
                F[j * ld + r] = make_double2(d, 0.0);
            else if (r > j && r < K)
                F[j * ld + r] = make_double2(s[0][t].x * inv, s[0][t].y * inv);
        }
        __syncthreads();
    }

    ls_substitute<R>(F, ld, b, K, h, info, lane);
}

// The same solve for K <= kLsSolve4MaxK on four waves: F in LDS (column
// stride 64); the sums of column j are split over the waves (lane = row r,
// wave w the columns k = w, w + 4, ... < j, two partial sums each) and added
// up in wave order by every wave after one barrier, so all waves hold the
// same column; wave j mod 4 stores it, and only that wave reads it later (it
// owns k = j), so the column needs no second barrier.  The partial sums
// alternate between two LDS buffers; each lane reads its A entry of column j
// before the barrier.  Wave 0 runs the substitutions at the end.
constexpr int kLsSolve4MaxK = 56;   // F and the partial sums within 64 KiB of LDS
__global__ void __launch_bounds__(256) ls_solve4_kernel(const double2 *__restrict__ A,
                                                        const double2 *__restrict__ b, int K, double ridge,
                                                        float2 *__restrict__ h, int32_t *__restrict__ info)
{
    extern __shared__ double2 ls_smem[];
    double2 *F = ls_smem;             // K columns of 64
    double2 *part = ls_smem + 64 * K; // 2 x 4 x 64 partial sums
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rc = min(lane, K - 1);
    // F = strict lower triangle of A, zero elsewhere (the diagonal included)
    for (int e = tid; e < 64 * K; e += 256) {
        const int k = e >> 6, r = e & 63;
        F[e] = (r < K && r > k) ? A[(int64_t)r * K + k] : make_double2(0.0, 0.0);
    }
    double tr = 0.0;
    for (int i = lane; i < K; i += 64) tr += A[(int64_t)i * K + i].x;
    const double delta = ridge * ls_wave_sum(tr) / K;
    const double dg = A[(int64_t)rc * K + rc].x + delta;   // Re A[r][r] + delta of the lane's row
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        const double2 aj = F[j * 64 + rc];   // A[r][j] (column j is not written before the barrier)
        // -sum_{k = w mod 4, k < j} L[r][k] conj(L[j][k])
        double2 s0 = make_double2(0.0, 0.0), s1 = s0;
        int k = w;
        for (; k + 4 < j; k += 8) {
            const double2 c0 = F[k * 64 + j], a0 = F[k * 64 + rc];
            const double2 c1 = F[(k + 4) * 64 + j], a1 = F[(k + 4) * 64 + rc];
            s0.x = fma(-a0.x, c0.x, s0.x);
            s0.x = fma(-a0.y, c0.y, s0.x);
            s0.y = fma(-a0.y, c0.x, s0.y);
            s0.y = fma(a0.x, c0.y, s0.y);
            s1.x = fma(-a1.x, c1.x, s1.x);
            s1.x = fma(-a1.y, c1.y, s1.x);
            s1.y = fma(-a1.y, c1.x, s1.y);
            s1.y = fma(a1.x, c1.y, s1.y);
        }
        if (k < j) {
            const double2 c0 = F[k * 64 + j], a0 = F[k * 64 + rc];
            s0.x = fma(-a0.x, c0.x, s0.x);
            s0.x = fma(-a0.y, c0.y, s0.x);
            s0.y = fma(-a0.y, c0.x, s0.y);
            s0.y = fma(a0.x, c0.y, s0.y);
        }
        double2 *pj = part + (j & 1) * 256;
        pj[w * 64 + lane] = make_double2(s0.x + s1.x, s0.y + s1.y);
        __syncthreads();
        double2 s = aj;
        if (lane == j) s.x += dg;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            s.x += pj[q * 64 + lane].x;
            s.y += pj[q * 64 + lane].y;
        }
        const double piv = ls_bcast(s.x, j);
        if (!(piv > 0.0)) {   // the same in every wave
            if (w == 0) {
                for (int i = lane; i < K; i += 64) h[i] = make_float2(NAN, NAN);
                if (lane == 0) *info = j + 1;
            }
            return;
        }
        if (w == (j & 3)) {
            const double d = sqrt(piv), inv = 1.0 / d;
            if (lane == j)
                F[j * 64 + lane] = make_double2(d, 0.0);
            else if (lane > j && lane < K)
                F[j * 64 + lane] = make_double2(s.x * inv, s.y * inv);
        }
        // Column j is read again (by other lanes of the wave that stored it)
        // before the next barrier: the LDS accesses of one wave execute in
        // program order, and this keeps the compiler from moving those reads
        // above the stores.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();   // every column stored
    if (w == 0) ls_substitute<1>(F, 64, b, K, h, info, lane);
}

__global__ void __launch_bounds__(kBlock) ls_zero_kernel(double2 *__restrict__ p, int64_t count)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < count) p[e] = make_double2(0.0, 0.0);
}

typedef void (*LsGramKernel)(LsParams);

template <int... P>
static const LsGramKernel *ls_gram_table_of(std::integer_sequence<int, P...>)
{
    static const LsGramKernel t[] = {&ls_gram_kernel<P + 1>...};
    return t;
}

static const LsGramKernel *ls_gram_table()
{
    return ls_gram_table_of(std::make_integer_sequence<int, kLsMaxNt>{});
}

struct LsShape {
    int K, D, Dp, nt, npairs;
};

static LsShape ls_shape(const CoefMap &map)
{
    LsShape s;
    s.K = (map.n_main + map.n_conj) * map.L + 1;
    s.D = 2 * s.K + 2;
    s.Dp = (s.D + 15) / 16 * 16;
    s.nt = s.Dp / 16;
    s.npairs = s.nt * (s.nt + 1) / 2;
    return s;
}

struct LsWs {
    size_t partials, r1, total;
};

// Samples per block: 8192 on large inputs; smaller (down to 1024) when that
// leaves fewer than ~6 blocks per CU, so small fits still fill the chip.
int num_cus();
static int64_t ls_slab(int64_t rows, int64_t n)
{
    const int64_t want = (int64_t)num_cus() * 6;
    int64_t slab = kLsSlabMax;
    while (slab > kLsSlabMin && rows * ((n + slab - 1) / slab) < want) slab /= 2;
    return slab;
}

static LsWs ls_ws(const LsShape &s, int64_t rows, int64_t n)
{
    const int64_t slab = ls_slab(rows, n);
    const int64_t spr = (n + slab - 1) / slab;
    const int64_t nslabs = std::max<int64_t>(rows * spr, 1);
    const int64_t groups = (nslabs + kLsGroup - 1) / kLsGroup;
    const int64_t E = (int64_t)s.npairs * 256;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    LsWs w;
    w.partials = up((size_t)(nslabs * E) * sizeof(float));
    w.r1 = up((size_t)(groups * E) * sizeof(double));
    w.total = w.partials + w.r1;
    return w;
}

// Role and tap of feature f (the column order of the real formulation):
// branch group g = f / L (main groups first) carries power level j with
// main_idx[j] == g (or conj_idx[j] == g - n_main); the conjugate branch takes
// -Im.  Padding columns read the zero entry (tap 0).
static void ls_columns(const CoefMap &map, const LsShape &s, int *role, int *tap)
{
    int level[2 * kMaxNI];
    for (int j = 0; j < map.NI; ++j) {
        if (map.main_idx[j] >= 0) level[map.main_idx[j]] = j;
        if (map.conj_idx[j] >= 0) level[map.n_main + map.conj_idx[j]] = j;
    }
    for (int f = 0; f < s.Dp; ++f) {
        role[f] = kLsRZero;
        tap[f] = 0;
    }
    for (int f = 0; f < s.K - 1; ++f) {
        const int g = f / map.L, k = f % map.L;
        const int j = level[g];
        role[f] = j;
        role[s.K + f] = (g >= map.n_main ? kLsRNegIm : kLsRIm) + j;
        tap[f] = tap[s.K + f] = k;
    }
    role[s.K - 1] = kLsROne;
    role[2 * s.K] = kLsRT;
    role[2 * s.K + 1] = kLsRT + 1;
}

// Feature f of a sample as a word of the LDS basis rows: row offset L - 1 - k
// for tap k, then the slot of its entry.
static void ls_offsets(const CoefMap &map, const LsShape &s, const int8_t *slot, int16_t *off)
{
    int role[kLsMaxDp], tap[kLsMaxDp];
    ls_columns(map, s, role, tap);
    for (int f = 0; f < kLsMaxDp; ++f) off[f] = (int16_t)(2 * ((map.L - 1) * kLsBEntries + slot[kLsRZero]));
    for (int f = 0; f < s.Dp; ++f) off[f] = (int16_t)(2 * ((map.L - 1 - tap[f]) * kLsBEntries + slot[role[f]]));
}

// Slots of the basis entries in an LDS row for one basis layout.  The matrix
// phase reads, per 16-column operand block, 16 entries at once (one per lane,
// rows shifted by each column's tap); a 64-bit LDS read serves 16 lanes per
// cycle over 32 four-byte banks, so distinct entries whose 8-byte units fall
// on the same bank pair (unit mod 16) take a cycle each.  A short
// deterministic local search over the slots minimizes the summed worst
// bank-pair load of the blocks (the odd row length keeps the row-per-lane
// writes conflict-free for any order).
void ls_layout(const CoefMap &map, int8_t *slot)
{
    for (int r = 0; r < kLsRoles; ++r) slot[r] = (int8_t)r;
    const LsShape s = ls_shape(map);
    if (s.Dp > kLsMaxDp) return;
    int role[kLsMaxDp], tap[kLsMaxDp];
    ls_columns(map, s, role, tap);
    auto cost = [&]() {
        int total = 0;
        for (int b = 0; b < s.nt; ++b) {
            int unit[16], load[16] = {0}, worst = 0;
            for (int c = 0; c < 16; ++c) {
                const int f = 16 * b + c;
                unit[c] = (map.L - 1 - tap[f]) * kLsBEntries + slot[role[f]];
                bool seen = false;
                for (int d = 0; d < c; ++d) seen |= unit[d] == unit[c];
                if (!seen) worst = std::max(worst, ++load[unit[c] & 15]);
            }
            total += worst;
        }
        return total;
    };
    int best = cost();
    uint32_t rng = 0x9e3779b9u;
    for (int it = 0; it < 4000 && best > s.nt; ++it) {
        rng = rng * 1664525u + 1013904223u;
        const int r = (int)((rng >> 8) % kLsRoles);
        rng = rng * 1664525u + 1013904223u;
        const int t = (int)((rng >> 8) % kLsBEntries);
        int other = -1;
        for (int q = 0; q < kLsRoles; ++q)
            if (slot[q] == t) other = q;
        const int8_t was = slot[r];
        slot[r] = (int8_t)t;
        if (other >= 0) slot[other] = was;
        const int c = cost();
        if (c <= best) {
            best = c;
        } else {
            if (other >= 0) slot[other] = (int8_t)t;
            slot[r] = was;
        }
    }
}

}  // namespace dpd

using namespace dpd;

DPD_EXPORT dpd_status dpd_ls_ws_size(const dpd_plan *plan, int64_t rows, int64_t n, size_t *bytes)
{
    if (plan == nullptr || bytes == nullptr || rows < 0 || n < 0) return DPD_EINVAL;
    const LsShape s = ls_shape(plan->map);
    if (s.Dp > kLsMaxDp) return DPD_EUNSUPPORTED;
    *bytes = ls_ws(s, rows, n).total;
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_ls_normal(dpd_plan *plan, void *stream, const void *y, const void *t, int64_t rows,
                                    int64_t n, int64_t ld, float y_scale, void *ws, size_t ws_bytes, void *A,
                                    void *b)
{
    if (plan == nullptr || A == nullptr || b == nullptr) return DPD_EINVAL;
    if (rows == 1 && ld < n) ld = n;
    if (n < 0 || rows < 0 || (rows > 1 && ld < n) || !std::isfinite(y_scale)) return DPD_EINVAL;
    const CoefMap &map = plan->map;
    const LsShape s = ls_shape(map);
    if (s.Dp > kLsMaxDp) return DPD_EUNSUPPORTED;
    const LsWs w = ls_ws(s, rows, n);
    if (ws == nullptr || ws_bytes < w.total || (uintptr_t)ws % 256 != 0) return DPD_EINVAL;
    for (const void *q : {y, t, (const void *)A, (const void *)b})
        if ((uintptr_t)q % 8 != 0) return DPD_EINVAL;
    if (rows * n > 0 && (y == nullptr || t == nullptr)) return DPD_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    float *partials = (float *)base;
    double *r1 = (double *)(base + w.partials);
    const int64_t slab = ls_slab(rows, n);
    const int64_t spr = (n + slab - 1) / slab;
    const int64_t nslabs = rows * spr;
    const int64_t E = (int64_t)s.npairs * 256;
    hipError_t e = hipSuccess;
    if (nslabs == 0) {
        // no samples: A = 0, b = 0 (a fill kernel, not a memset: capturable)
        const int64_t kk = (int64_t)s.K * s.K;
        hipLaunchKernelGGL(ls_zero_kernel, dim3((uint32_t)((kk + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           (double2 *)A, kk);
        hipLaunchKernelGGL(ls_zero_kernel, dim3((uint32_t)((s.K + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           (double2 *)b, (int64_t)s.K);
        e = hipGetLastError();
        return e == hipSuccess ? DPD_OK : hip_fail(e);
    }
    LsParams p;
    p.y = (const float2 *)y;
    p.t = (const float2 *)t;
    p.n = n;
    p.ld = ld;
    p.slabs_per_row = spr;
    p.slab = slab;
    p.y_scale = y_scale;
    p.partials = partials;
    p.K = s.K;
    p.D = s.D;
    p.Dp = s.Dp;
    p.nt = s.nt;
    p.npairs = s.npairs;
    p.L = map.L;
    p.NI = map.NI;
    std::call_once(plan->ls_once, [plan]() { ls_layout(plan->map, plan->ls_slot); });
    std::copy(plan->ls_slot, plan->ls_slot + kLsRoles, p.slot);
    ls_offsets(map, s, p.slot, p.off);
    if (nslabs >= ((int64_t)1 << 31)) return DPD_EUNSUPPORTED;
    hipLaunchKernelGGL(ls_gram_table()[s.nt - 1], dim3((uint32_t)nslabs), dim3(kBlock), 0, st, p);
    e = hipGetLastError();
    const int64_t groups = (nslabs + kLsGroup - 1) / kLsGroup;
    const uint32_t eb = (uint32_t)((E + kBlock - 1) / kBlock);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(ls_reduce1_kernel, dim3(eb, (uint32_t)groups), dim3(kBlock), 0, st,
                           (const float *)partials, nslabs, E, r1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        const int64_t outs = (int64_t)s.K * s.K + s.K;
        hipLaunchKernelGGL(ls_finish_kernel, dim3((uint32_t)((outs + kLsWaves - 1) / kLsWaves)), dim3(kBlock), 0, st,
                           (const double *)r1, groups, E, s.nt, s.K, (double2 *)A, (double2 *)b);
        e = hipGetLastError();
    }
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_ls_solve_ws_size(int32_t K, size_t *bytes)
{
    if (K < 1 || bytes == nullptr) return DPD_EINVAL;
    if (K > kLsSolveMaxK) return DPD_EUNSUPPORTED;
    *bytes = (size_t)K * K * sizeof(double2);
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_ls_solve(void *stream, int32_t K, const void *A, const void *b, double ridge, void *ws,
                                   size_t ws_bytes, void *h, void *info)
{
    if (K < 1 || A == nullptr || b == nullptr || h == nullptr || info == nullptr || ws == nullptr) return DPD_EINVAL;
    if (K > kLsSolveMaxK) return DPD_EUNSUPPORTED;
    if (!(ridge >= 0.0) || !std::isfinite(ridge)) return DPD_EINVAL;
    if (ws_bytes < (size_t)K * K * sizeof(double2)) return DPD_EINVAL;
    for (const void *q : {A, b, (const void *)ws})
        if ((uintptr_t)q % 16 != 0) return DPD_EINVAL;
    if ((uintptr_t)h % 8 != 0 || (uintptr_t)info % 4 != 0) return DPD_EINVAL;
    const bool in_lds = K <= 64;   // F at column stride 64: at most 64 KiB of LDS
    const size_t lds = (size_t)K * 64 * sizeof(double2);
    const int slots = (K + 63) / 64;
    const int R = slots <= 1 ? 1 : slots <= 2 ? 2 : slots <= 4 ? 4 : slots <= 8 ? 8 : 16;
    const hipStream_t st = (hipStream_t)stream;
    const double2 *Ad = (const double2 *)A, *bd = (const double2 *)b;
    double2 *F = (double2 *)ws;
    float2 *hd = (float2 *)h;
    int32_t *id = (int32_t *)info;
    if (K <= kLsSolve4MaxK)
        hipLaunchKernelGGL(ls_solve4_kernel, dim3(1), dim3(256), (size_t)(64 * K + 2 * 4 * 64) * sizeof(double2), st,
                           Ad, bd, K, ridge, hd, id);
    else if (in_lds)
        hipLaunchKernelGGL((ls_solve_kernel<true, 1>), dim3(1), dim3(64), lds, st, Ad, bd, K, ridge, F, hd, id);
    else if (R == 2)
        hipLaunchKernelGGL((ls_solve_kernel<false, 2>), dim3(1), dim3(64), 0, st, Ad, bd, K, ridge, F, hd, id);
    else if (R == 4)
        hipLaunchKernelGGL((ls_solve_kernel<false, 4>), dim3(1), dim3(64), 0, st, Ad, bd, K, ridge, F, hd, id);
    else if (R == 8)
        hipLaunchKernelGGL((ls_solve_kernel<false, 8>), dim3(1), dim3(64), 0, st, Ad, bd, K, ridge, F, hd, id);
    else
        hipLaunchKernelGGL((ls_solve_kernel<false, 16>), dim3(1), dim3(64), 0, st, Ad, bd, K, ridge, F, hd, id);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}
