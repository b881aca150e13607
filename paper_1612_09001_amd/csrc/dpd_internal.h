// Internal declarations shared by the host library and the kernel translation
// units of libdpd (not part of the public ABI; the public header is dpd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpd {

// Largest power level NI = (max order + 1) / 2 (orders up to 15) and taps.
constexpr int kMaxNI = 8;
constexpr int kMaxL = 16;
// Specialised (fully unrolled) kernels exist for NI <= kSpecNI, L <= kSpecL.
constexpr int kSpecNI = 8;
constexpr int kSpecL = 8;
constexpr int kBlock = 256;

// Launch variants of the specialised forward kernel:
//   variant = s_index * 2 + stage_lds,   samples per thread = 2 << s_index;
//   stage_lds = 0: one-shot tiles, windows loaded directly;
//   stage_lds = 1: persistent streaming kernel, windows staged through LDS.
constexpr int kNumSIdx = 3;                 // S in {2, 4, 8}
constexpr int kNumFwdVariants = kNumSIdx * 2;

// How the stacked coefficient vector (section 2.2) feeds power level j
// (order 2j+1): index of the main / conjugate branch carrying that order, or -1.
struct CoefMap {
    int32_t L;
    int32_t NI;
    int32_t n_main;
    int32_t n_conj;
    int8_t main_idx[kMaxNI];
    int8_t conj_idx[kMaxNI];
};

// Precombined coefficient table read by every kernel (FP32):
//   for tap k, power level j: 4 floats {m00, m01, m10, m11} at (k*NI + j)*4,
//   the real 2x2 matrix of  w -> h*w + hbar*conj(w):
//     m00 = hr + gr   m01 = gi - hi
//     m10 = hi + gi   m11 = hr - gr
//   then c (2 floats) at 4*L*NI.
__host__ __device__ inline int table_floats(int L, int NI) { return 4 * L * NI + 2; }

struct FwdParams {
    const float2 *in;
    float2 *out;
    int64_t n;             // samples per row
    int64_t ld;            // row stride in samples
    int64_t tiles_per_row;
    int64_t total_tiles;   // rows * tiles_per_row
    const float *M;        // precombined table
    const float2 *hist;    // L-1 samples preceding row 0, or nullptr
};

typedef hipError_t (*FwdLaunch)(const FwdParams &, hipStream_t, int grid_mult);

struct FwdTable {
    FwdLaunch fn[kSpecNI][kSpecL][kNumFwdVariants];
    int tile[kNumFwdVariants];   // samples per tile (one-shot) or per wave chunk (streaming)
};

// Registration hooks, one per power-level translation unit.
void register_fwd_ni1(FwdTable &);
void register_fwd_ni2(FwdTable &);
void register_fwd_ni3(FwdTable &);
void register_fwd_ni4(FwdTable &);
void register_fwd_ni5(FwdTable &);
void register_fwd_ni6(FwdTable &);
void register_fwd_ni7(FwdTable &);
void register_fwd_ni8(FwdTable &);

}  // namespace dpd
