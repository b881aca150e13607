// Cross-lane sums by DPP row operations, shared by the reductions of the
// backward and learning-step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace dpd {

// One DPP step of a lane reduction: x from the lane that CTRL selects (rows
// outside RMASK read zero).
template <int CTRL, int RMASK>
__device__ __forceinline__ float dpp_from(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, RMASK, 0xf, false));
}

// The same for FP64 values: each half of the double moved by its own DPP
// step (rows outside RMASK read zero, i.e. +0.0).
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_from(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, RMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, RMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes, complete in lane 63 (the other lanes hold partial
// sums), by DPP row operations -- no LDS round trips: quad sums (quad_perm
// 1,0,3,2 and 2,3,0,1), 8- and 16-lane sums (row_half_mirror, row_mirror),
// then rows 1 and 3 add rows 0 and 2 (row_bcast:15) and rows 2 and 3 add the
// sum of rows 0..1 (row_bcast:31).  Fixed order: the same inputs give the
// same bits.
template <class T>
__device__ __forceinline__ T wave_sum_to_lane63(T v)
{
    v += dpp_from<0xB1, 0xf>(v);
    v += dpp_from<0x4E, 0xf>(v);
    v += dpp_from<0x141, 0xf>(v);
    v += dpp_from<0x140, 0xf>(v);
    v += dpp_from<0x142, 0xa>(v);
    v += dpp_from<0x143, 0xc>(v);
    return v;
}

// N <= 64 per-lane values v[0..N) summed over the wave, transposed: lane l
// returns the sum of v[l] over all 64 lanes (zero for l >= N); v is
// overwritten.  Six butterfly stages; at the stage of lane stride o the
// registers pair up (i, i + o) and each lane keeps the one its lane bit o
// selects, adding its partner's copy of it, so every stage halves the
// registers still live (at most 63 exchanges instead of N separate
// reductions).  Fixed order: the same inputs give the same bits.
template <int N>
__device__ __forceinline__ float wave_transpose_sum(float (&v)[N], int lane)
{
    static_assert(N >= 1 && N <= 64, "one register per lane and group");
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < o && i < N; ++i) {
            const float other = i + o < N ? v[i + o] : 0.f;
            const float keep = up ? other : v[i];
            const float send = up ? v[i] : other;
            v[i] = keep + __shfl_xor(send, o);
        }
    }
    return v[0];
}

// Calls f(std::integral_constant<int, G>) for G = 0 .. NG-1.
template <int G, int NG>
struct ForEachGroup {
    template <class F>
    __device__ __forceinline__ static void run(F &f)
    {
        f(std::integral_constant<int, G>{});
        ForEachGroup<G + 1, NG>::run(f);
    }
};
template <int NG>
struct ForEachGroup<NG, NG> {
    template <class F>
    __device__ __forceinline__ static void run(F &)
    {
    }
};

// The wave sums of E per-lane accumulators added to FP64 totals held
// transposed (entry 64 g + l in lane l of tot[g]); acc is consumed.
template <int E>
__device__ __forceinline__ void wave_sums_into(float (&acc)[E], double (&tot)[(E + 63) / 64], int lane)
{
    auto one = [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        constexpr int n = E - 64 * g < 64 ? E - 64 * g : 64;
        tot[g] += (double)wave_transpose_sum<n>(*reinterpret_cast<float(*)[n]>(&acc[64 * g]), lane);
    };
    ForEachGroup<0, (E + 63) / 64>::run(one);
}

}  // namespace dpd
