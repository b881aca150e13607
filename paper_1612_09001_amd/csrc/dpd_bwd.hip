// Host side of the backward pass (dpd_backward, dpd_backward_ws_size) plus
// the generic backward kernels (any L <= 16) and the FP64 finalisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "dpd.h"
#include "dpd_bwd_kernels.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {

int num_cus();

constexpr int kGenericBlocks = 1024;   // fixed grid of the generic kernels
constexpr int kGroup = 16;             // coefficient-gradient entries per pass

static BwdTable g_bwd;
static std::once_flag g_bwd_once;

static const BwdTable &bwd_table()
{
    std::call_once(g_bwd_once, [] {
        std::memset(&g_bwd, 0, sizeof(g_bwd));
        register_bwd_ni1(g_bwd);
        register_bwd_ni2(g_bwd);
        register_bwd_ni3(g_bwd);
        register_bwd_ni4(g_bwd);
        register_bwd_ni5(g_bwd);
        register_bwd_ni6(g_bwd);
        register_bwd_ni7(g_bwd);
        register_bwd_ni8(g_bwd);
    });
    return g_bwd;
}

// Resident blocks per CU of a specialised backward kernel (cached).
static int bwd_occupancy(int NI, int L, int want)
{
    static int cache[kSpecNI][kSpecL][3] = {};
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    int &o = cache[NI - 1][L - 1][want];
    if (o == 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, bwd_table().kern[NI - 1][L - 1][want],
                                                         kBlock, 0) != hipSuccess || v < 1)
            v = 1;
        o = v;
    }
    return o;
}

// ------------------------------------------------------- generic kernels ---

// dE/dx, one sample per thread, runtime NI and L.
__global__ void __launch_bounds__(kBlock) bwd_dx_generic(BwdParams p, int NI, int L)
{
    const cfloat *M = as_const(p.M);
    const int64_t total = p.rows * p.n;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t row = idx / p.n, m = idx - row * p.n;
        const float2 v = p.x[row * p.ld + m];
        const float a = v.x, b = v.y, s = __builtin_fmaf(a, a, b * b);
        float Pa = 0.f, Pb = 0.f, Q = 0.f;
        for (int j = NI - 1; j >= 0; --j) {
            float ua = 0.f, ub = 0.f;
            for (int k = 0; k < L && m + k < p.n; ++k) {
                const float2 g = p.gz[row * p.ld + m + k];
                const cfloat *Mk = M + 4 * (k * NI + j);
                ua = __builtin_fmaf(Mk[0], g.x, ua);
                ua = __builtin_fmaf(Mk[2], g.y, ua);
                ub = __builtin_fmaf(Mk[1], g.x, ub);
                ub = __builtin_fmaf(Mk[3], g.y, ub);
            }
            Pa = __builtin_fmaf(Pa, s, ua);
            Pb = __builtin_fmaf(Pb, s, ub);
            if (j > 0) Q = __builtin_fmaf(Q, s, (float)j * __builtin_fmaf(a, ua, b * ub));
        }
        p.gx[row * p.ld + m] = make_float2(__builtin_fmaf(2.f * Q, a, Pa), __builtin_fmaf(2.f * Q, b, Pb));
    }
}

// dE/dM entries [g*kGroup, (g+1)*kGroup) for the samples of block b (a
// contiguous range of the flattened rows); one partial per (block, entry).
__global__ void __launch_bounds__(kBlock) bwd_dc_generic(BwdParams p, int NI, int L)
{
    __shared__ double red[kBlock];
    const int E = 4 * L * NI + 2;
    const int64_t total = p.rows * p.n;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < total ? lo + per : total;
    // FP32 sums over at most 64 samples per thread, then FP64
    float acc[kGroup];
    double accd[kGroup];
    for (int q = 0; q < kGroup; ++q) acc[q] = 0.f, accd[q] = 0.0;
    int cnt = 0;
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += kBlock) {
        if (++cnt == 64) {
            for (int q = 0; q < kGroup; ++q) accd[q] += acc[q], acc[q] = 0.f;
            cnt = 0;
        }
        const int64_t row = idx / p.n, m = idx - row * p.n;
        const float2 v = p.x[row * p.ld + m];
        const float s = __builtin_fmaf(v.x, v.x, v.y * v.y);
        for (int q = 0; q < kGroup; ++q) {
            const int e = blockIdx.y * kGroup + q;
            if (e >= E) break;
            if (e >= E - 2) {
                const float2 g = p.gz[row * p.ld + m];
                acc[q] += e == E - 2 ? g.x : g.y;
                continue;
            }
            const int rc = e & 3, jk = e >> 2, k = jk / NI, j = jk - k * NI;
            if (m + k >= p.n) continue;
            const float2 g = p.gz[row * p.ld + m + k];
            float r = 1.f;
            for (int t = 0; t < j; ++t) r *= s;
            const float gc = (rc < 2) ? g.x : g.y;
            const float pc = (rc & 1) ? r * v.y : r * v.x;
            acc[q] = __builtin_fmaf(gc, pc, acc[q]);
        }
    }
    for (int q = 0; q < kGroup; ++q) {
        const int e = blockIdx.y * kGroup + q;
        if (e >= E) break;
        red[threadIdx.x] = accd[q] + (double)acc[q];
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) p.partials[(int64_t)blockIdx.x * E + e] = (float)red[0];
        __syncthreads();
    }
}

// Coefficient-gradient finalisation: block q sums, in FP64, the partials of
// the four entries of table matrix q = k*NI + j (block L*NI: the two entries
// of c) over all nblk producer blocks -- thread t takes producers t, t + 256,
// ... in order, then the DPP lane sum of each wave and the four waves in
// order, so the result is bitwise reproducible -- and applies the chain rule
// through M = [[hr+gr, gi-hi], [hi+gi, hr-gr]] to the main and conjugate
// coefficients of order 2j+1, tap k (section 2.2 layout):
//   u1 = dE/dm00, u4 = dE/dm01, u3 = dE/dm10, u2 = dE/dm11
//   grad h    = (u1 + u2) + j (u3 - u4)
//   grad hbar = (u1 - u2) + j (u3 + u4)
//   grad c    = sum G
__global__ void __launch_bounds__(kBlock) bwd_finalize(const float *__restrict__ partials, int nblk,
                                                       CoefMap map, float2 *__restrict__ gcoef)
{
    __shared__ double red[kBlock / 64][4];
    double u[4];
    dcoef_block_sums(partials, nblk, map, blockIdx.x, red, u);
    if (threadIdx.x != 0) return;
    int idx[2];
    float2 g[2];
    const int c = dcoef_block_grads(map, blockIdx.x, u, idx, g);
    for (int i = 0; i < c; ++i) gcoef[idx[i]] = g[i];
}

static bool spec_ok(const CoefMap &m) { return m.NI <= kSpecNI && m.L <= kSpecL; }

static int64_t spec_grid_cap() { return (int64_t)num_cus() * 8; }

size_t bwd_ws_bytes(const CoefMap &map)
{
    const int64_t E = 4 * map.L * map.NI + 2;
    const int64_t blocks = std::max<int64_t>(spec_grid_cap(), kGenericBlocks);
    return (size_t)(blocks * E * (int64_t)sizeof(float) + 256);
}

hipError_t launch_bwd_finalize(const float *partials, int nblk, const CoefMap &map, float2 *grad_coeffs,
                               hipStream_t st)
{
    hipLaunchKernelGGL(bwd_finalize, dim3((uint32_t)(map.L * map.NI + 1)), dim3(kBlock), 0, st, partials, nblk,
                       map, grad_coeffs);
    return hipGetLastError();
}

}  // namespace dpd

using namespace dpd;

DPD_EXPORT dpd_status dpd_backward_ws_size(const dpd_plan *plan, int64_t rows, int64_t n, size_t *bytes)
{
    if (plan == nullptr || bytes == nullptr || rows < 0 || n < 0) return DPD_EINVAL;
    *bytes = bwd_ws_bytes(plan->map);
    return DPD_OK;
}

static dpd_status backward_impl(dpd_plan *plan, void *stream, const void *coeffs_dev, const void *x,
                                const void *grad_z, void *grad_x, void *grad_coeffs, int64_t rows,
                                int64_t n, int64_t ld, void *ws, size_t ws_bytes)
{
    if (plan == nullptr) return DPD_EINVAL;
    if (rows == 1 && ld < n) ld = n;
    if (n < 0 || rows < 0 || (rows > 1 && ld < n)) return DPD_EINVAL;
    const CoefMap &map = plan->map;
    const hipStream_t st = (hipStream_t)stream;
    const bool want_dx = grad_x != nullptr, want_dc = grad_coeffs != nullptr;
    const bool empty = n == 0 || rows == 0;
    if (!empty && (x == nullptr || grad_z == nullptr)) return DPD_EINVAL;
    for (const void *q : {x, grad_z, (const void *)grad_x, (const void *)grad_coeffs, coeffs_dev})
        if ((uintptr_t)q % 8 != 0) return DPD_EINVAL;
    if (want_dc && (ws == nullptr || ws_bytes < bwd_ws_bytes(map) || (uintptr_t)ws % 4 != 0))
        return DPD_EINVAL;
    if (want_dx && !empty) {
        const size_t span = (size_t)(((rows - 1) * ld + n) * 8);
        auto ov = [&](const void *a, const void *b) {
            const uintptr_t p = (uintptr_t)a, q = (uintptr_t)b;
            return p < q + span && q < p + span;
        };
        if (ov(grad_x, x) || ov(grad_x, grad_z)) return DPD_EINVAL;
    }
    // only dx reads the coefficients: dE/dcoeffs is the correlation of grad_z
    // with the basis of x alone
    const float *table = plan->d_table;
    if (coeffs_dev != nullptr && want_dx) {
        hipError_t e = launch_prep(map, coeffs_dev, plan->d_table_call, st);
        if (e != hipSuccess) return hip_fail(e);
        table = plan->d_table_call;
    }
    if (!want_dx && !want_dc) return DPD_OK;

    BwdParams p;
    p.x = (const float2 *)x;
    p.gz = (const float2 *)grad_z;
    p.gx = (float2 *)grad_x;
    p.partials = (float *)ws;
    p.n = n;
    p.ld = ld;
    p.rows = rows;
    p.M = table;
    int nblk = 0;
    if (!empty) {
        const bool aligned = (uintptr_t)x % 16 == 0 && (uintptr_t)grad_z % 16 == 0 &&
                             (uintptr_t)grad_x % 16 == 0 && (rows == 1 || ld % 2 == 0);
        if (aligned && spec_ok(map)) {
            const int want = want_dx && want_dc ? 2 : (want_dc ? 1 : 0);
            const int64_t C = 64 * kBwdS;
            p.tpr = n / C;
            const int64_t chunks = rows * ((n + C - 1) / C);
            const int64_t cap = (int64_t)num_cus() * std::min(8, bwd_occupancy(map.NI, map.L, want));
            const int64_t grid = std::max<int64_t>(1, std::min(cap, (chunks + 3) / 4));
            hipError_t e = bwd_table().fn[map.NI - 1][map.L - 1][want](p, st, (int)grid);
            if (e != hipSuccess) return hip_fail(e);
            nblk = (int)grid;
        } else {
            p.tpr = 0;
            if (want_dx) {
                const int64_t blocks = std::min<int64_t>((rows * n + kBlock - 1) / kBlock, 1 << 20);
                hipLaunchKernelGGL(bwd_dx_generic, dim3((uint32_t)blocks), dim3(kBlock), 0, st, p,
                                   map.NI, map.L);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(e);
            }
            if (want_dc) {
                const int E = 4 * map.L * map.NI + 2;
                const int groups = (E + kGroup - 1) / kGroup;
                hipLaunchKernelGGL(bwd_dc_generic, dim3(kGenericBlocks, groups), dim3(kBlock), 0, st, p,
                                   map.NI, map.L);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(e);
                nblk = kGenericBlocks;
            }
        }
    }
    if (want_dc) {
        hipLaunchKernelGGL(bwd_finalize, dim3((uint32_t)(map.L * map.NI + 1)), dim3(kBlock), 0, st,
                           (const float *)ws, nblk, map, (float2 *)grad_coeffs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_backward(dpd_plan *plan, void *stream, const void *coeffs_dev, const void *x,
                                   const void *grad_z, void *grad_x, void *grad_coeffs, int64_t rows,
                                   int64_t n, int64_t ld, void *ws, size_t ws_bytes)
{
    return backward_impl(plan, stream, coeffs_dev, x, grad_z, grad_x, grad_coeffs, rows, n, ld, ws, ws_bytes);
}

// ------------------------------------------------------------ no-allocation --
// Fixed device scratch for dpd_backward_noalloc: the per-block FP32 partials of
// the coefficient gradient (at most kMaxBwdScratch bytes; every plan on a
// 256-CU device needs <= 2048 blocks x 514 entries x 4 bytes + 256).  Each GPU
// holds its own copy of the array for the life of the process.  In host code
// the name `scratch` is only a host-side stand-in: its device address comes
// from hipGetSymbolAddress, once per device.
constexpr size_t kMaxBwdScratch = (size_t)17 << 18;   // 4.25 MiB
static __device__ __align__(256) unsigned char scratch[kMaxBwdScratch];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
static dpd_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxScratchDevices) return DPD_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (p == nullptr) return DPD_EHIP;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_backward_noalloc(dpd_plan *plan, void *stream, const void *coeffs_dev, const void *x,
                                           const void *grad_z, void *grad_x, void *grad_coeffs, int64_t rows,
                                           int64_t n, int64_t ld)
{
    if (plan == nullptr) return DPD_EINVAL;
    if (grad_coeffs == nullptr)   // no coefficient gradient: no scratch is used
        return backward_impl(plan, stream, coeffs_dev, x, grad_z, grad_x, nullptr, rows, n, ld, nullptr, 0);
    if (bwd_ws_bytes(plan->map) > kMaxBwdScratch) return DPD_EUNSUPPORTED;
    void *ws = nullptr;
    dpd_status st = scratch_address(&ws);
    if (st != DPD_OK) return st;
    return backward_impl(plan, stream, coeffs_dev, x, grad_z, grad_x, grad_coeffs, rows, n, ld, ws,
                         kMaxBwdScratch);
}
