// Cross-lane sums by DPP row operations, shared by the reductions of the
// backward and learning-step kernels.
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace dpd
