// Host side of libdpd: argument validation, coefficient precombination,
// kernel selection and the C ABI declared in include/dpd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dpd.h"
#include "dpd_fwd_kernels.h"
#include "dpd_internal.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {

static thread_local int g_last_hip_error = 0;

dpd_status hip_fail(hipError_t e)
{
    g_last_hip_error = (int)e;
    return DPD_EHIP;
}

// ------------------------------------------------------------ validation ---

dpd_status parse_orders(const int32_t *orders, int32_t n, int8_t (&idx)[kMaxNI], int &max_level)
{
    if (n < 0 || n > kMaxNI) return n < 0 ? DPD_EINVAL : DPD_EUNSUPPORTED;
    if (n > 0 && orders == nullptr) return DPD_EINVAL;
    int prev = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int p = orders[i];
        if (p < 1 || (p & 1) == 0 || p <= prev) return DPD_EINVAL;
        if (p > 2 * kMaxNI - 1) return DPD_EUNSUPPORTED;
        idx[(p - 1) / 2] = (int8_t)i;
        max_level = std::max(max_level, (p - 1) / 2 + 1);
        prev = p;
    }
    return DPD_OK;
}

dpd_status make_map(const int32_t *mo, int32_t nm, const int32_t *co, int32_t nc, int32_t L,
                    CoefMap &map)
{
    if (L < 1) return DPD_EINVAL;
    if (L > kMaxL) return DPD_EUNSUPPORTED;
    if (nm < 1) return DPD_EINVAL;
    std::memset(&map, 0, sizeof(map));
    std::memset(map.main_idx, -1, sizeof(map.main_idx));
    std::memset(map.conj_idx, -1, sizeof(map.conj_idx));
    int levels = 0;
    dpd_status st = parse_orders(mo, nm, map.main_idx, levels);
    if (st != DPD_OK) return st;
    st = parse_orders(co, nc, map.conj_idx, levels);
    if (st != DPD_OK) return st;
    map.L = L;
    map.NI = levels;
    map.n_main = nm;
    map.n_conj = nc;
    return DPD_OK;
}

// Precombine (section 2.2 stacking) -> table of real 2x2 matrices (FP32).
// The device kernel prep_coeffs_kernel performs the same float additions.
void precombine_host(const CoefMap &map, const float *raw, std::vector<float> &M)
{
    const int L = map.L, NI = map.NI;
    M.assign(table_floats(L, NI), 0.f);
    for (int k = 0; k < L; ++k)
        for (int j = 0; j < NI; ++j) {
            float hr = 0.f, hi = 0.f, gr = 0.f, gi = 0.f;
            if (map.main_idx[j] >= 0) {
                const float *h = raw + 2 * (map.main_idx[j] * L + k);
                hr = h[0];
                hi = h[1];
            }
            if (map.conj_idx[j] >= 0) {
                const float *g = raw + 2 * ((map.n_main + map.conj_idx[j]) * L + k);
                gr = g[0];
                gi = g[1];
            }
            float *m = &M[4 * (k * NI + j)];
            m[0] = hr + gr;
            m[1] = gi - hi;
            m[2] = hi + gi;
            m[3] = hr - gr;
        }
    const int K = (map.n_main + map.n_conj) * L + 1;
    M[4 * L * NI] = raw[2 * (K - 1)];
    M[4 * L * NI + 1] = raw[2 * (K - 1) + 1];
}

__global__ void prep_coeffs_kernel(const float2 *__restrict__ raw, CoefMap map, float *__restrict__ M,
                                   const int32_t *__restrict__ flag)
{
    if (flag != nullptr && *flag != 0) return;   // conditional form: keep the table
    const int t = threadIdx.x;
    const int L = map.L, NI = map.NI;
    if (t < L * NI) {
        const int k = t / NI, j = t - k * NI;
        float2 h = make_float2(0.f, 0.f), g = make_float2(0.f, 0.f);
        if (map.main_idx[j] >= 0) h = raw[map.main_idx[j] * L + k];
        if (map.conj_idx[j] >= 0) g = raw[(map.n_main + map.conj_idx[j]) * L + k];
        M[4 * t + 0] = h.x + g.x;
        M[4 * t + 1] = g.y - h.y;
        M[4 * t + 2] = h.y + g.y;
        M[4 * t + 3] = h.x - g.x;
    }
    if (t == 0) {
        const int K = (map.n_main + map.n_conj) * L + 1;
        const float2 c = raw[K - 1];
        M[4 * L * NI] = c.x;
        M[4 * L * NI + 1] = c.y;
    }
}

hipError_t launch_prep(const CoefMap &map, const void *raw, float *M, hipStream_t stream,
                       const int32_t *flag)
{
    hipLaunchKernelGGL(prep_coeffs_kernel, dim3(1), dim3(kMaxL * kMaxNI), 0, stream,
                       (const float2 *)raw, map, M, flag);
    return hipGetLastError();
}

// ------------------------------------------------------ generic forward ---
// Any L <= 16, any NI <= 8, 8-byte alignment: one output per thread, runtime
// loops over taps and power levels (the specialised kernels cover the common
// shapes; this one keeps every valid plan usable).
__global__ void __launch_bounds__(kBlock) fwd_generic_kernel(FwdParams p, int NI, int L)
{
    const cfloat *M = as_const(p.M);
    const int64_t total = p.total_tiles;   // rows * n for this kernel
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t row = idx / p.n;
        const int64_t m = idx - row * p.n;
        const float2 *x = p.in + row * p.ld;
        const float2 *hist = row == 0 ? p.hist : nullptr;
        float zr = M[4 * L * NI], zi = M[4 * L * NI + 1];
        for (int k = 0; k < L; ++k) {
            const int64_t t = m - k;
            float2 v = make_float2(0.f, 0.f);
            if (t >= 0)
                v = x[t];
            else if (hist != nullptr && t >= -(int64_t)(L - 1))
                v = hist[(L - 1) + t];
            const float s = __builtin_fmaf(v.x, v.x, v.y * v.y);
            const cfloat *Mk = M + 4 * NI * k;
            float w00 = Mk[4 * (NI - 1) + 0], w01 = Mk[4 * (NI - 1) + 1];
            float w10 = Mk[4 * (NI - 1) + 2], w11 = Mk[4 * (NI - 1) + 3];
            for (int j = NI - 2; j >= 0; --j) {
                w00 = __builtin_fmaf(w00, s, Mk[4 * j + 0]);
                w01 = __builtin_fmaf(w01, s, Mk[4 * j + 1]);
                w10 = __builtin_fmaf(w10, s, Mk[4 * j + 2]);
                w11 = __builtin_fmaf(w11, s, Mk[4 * j + 3]);
            }
            zr = __builtin_fmaf(w00, v.x, zr);
            zr = __builtin_fmaf(w01, v.y, zr);
            zi = __builtin_fmaf(w10, v.x, zi);
            zi = __builtin_fmaf(w11, v.y, zi);
        }
        p.out[row * p.ld + m] = make_float2(zr, zi);
    }
}

// After a streaming call: hist <- last L-1 samples of (hist ++ in).
__global__ void hist_update_kernel(const float2 *__restrict__ in, int64_t n, float2 *hist, int Lm1)
{
    const int i = threadIdx.x;
    float2 v = make_float2(0.f, 0.f);
    if (i < Lm1) {
        const int64_t src = n - Lm1 + i;
        v = src >= 0 ? in[src] : hist[Lm1 + src];
    }
    __syncthreads();
    if (i < Lm1) hist[i] = v;
}

// ------------------------------------------------------- streaming copy ---
// The forward kernel's memory walk without the filter (measurement of the
// practical HBM ceiling of that walk): persistent waves, wave g copies chunks
// g, g + nw, ... of 512 samples with one chunk of register prefetch and
// nontemporal 16-byte loads and stores (1 KiB per instruction); the last
// n mod 512 samples one per lane after the walk.
__global__ void __launch_bounds__(kBlock) copy_walk_kernel(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                          int64_t n)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    constexpr int C = 512, NV = 4;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t total = n / C;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t gw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * (kBlock / 64) + wv;
    auto ld = [&](v4 (&r)[NV], int64_t c) {
        const v4 *x4 = reinterpret_cast<const v4 *>(in + c * C);
#pragma unroll
        for (int i = 0; i < NV; ++i) r[i] = __builtin_nontemporal_load(x4 + lane + 64 * i);
    };
    auto st = [&](const v4 (&r)[NV], int64_t c) {
        v4 *z4 = reinterpret_cast<v4 *>(out + c * C);
#pragma unroll
        for (int i = 0; i < NV; ++i) __builtin_nontemporal_store(r[i], z4 + lane + 64 * i);
    };
    if (gw < total) {
        v4 A[NV], B[NV];
        int64_t c = gw;
        ld(A, c);
        for (; c + 2 * nw < total; c += 2 * nw) {
            ld(B, c + nw);
            st(A, c);
            ld(A, c + 2 * nw);
            st(B, c + nw);
        }
        if (c + nw < total) {
            ld(B, c + nw);
            st(A, c);
            st(B, c + nw);
        } else {
            st(A, c);
        }
    }
    for (int64_t m = total * C + gw * 64 + lane; m < n; m += nw * 64) out[m] = in[m];
}

// --------------------------------------------------------------- tables ---

// Compute units of the current device (cached per device id; concurrent
// first calls store the same value).
int num_cus()
{
    static std::atomic<int> cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int cus = cache[dev].load(std::memory_order_relaxed);
    if (cus == 0) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev].store(cus, std::memory_order_relaxed);
    }
    return cus;
}

static FwdTable g_fwd;
static std::once_flag g_fwd_once;

const FwdTable &fwd_table()
{
    std::call_once(g_fwd_once, [] {
        std::memset(&g_fwd, 0, sizeof(g_fwd));
        register_fwd_ni1(g_fwd);
        register_fwd_ni2(g_fwd);
        register_fwd_ni3(g_fwd);
        register_fwd_ni4(g_fwd);
        register_fwd_ni5(g_fwd);
        register_fwd_ni6(g_fwd);
        register_fwd_ni7(g_fwd);
        register_fwd_ni8(g_fwd);
        for (int v = 0; v < kNumFwdVariants; ++v)
            g_fwd.tile[v] = (v & 1 ? 64 : kBlock) * (2 << (v / 2));
    });
    return g_fwd;
}

int fwd_variant(const dpd_tune &t)
{
    const int sidx = t.samples_per_thread == 2 ? 0 : t.samples_per_thread == 4 ? 1 : 2;
    return sidx * 2 + (t.stage_lds ? 1 : 0);
}

bool valid_tune(const dpd_tune &t)
{
    const bool s_ok = t.samples_per_thread == 2 || t.samples_per_thread == 4 || t.samples_per_thread == 8;
    return s_ok && (t.stage_lds == 0 || t.stage_lds == 1) && t.block == kBlock && t.grid_mult >= 1 &&
           t.grid_mult <= 32;
}

dpd_tune default_tune()
{
    dpd_tune t;
    t.samples_per_thread = 8;
    t.stage_lds = 1;
    t.block = kBlock;
    t.grid_mult = 2;    // persistent blocks per CU (capped at the resident limit)
    return t;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

static size_t span_bytes(int64_t rows, int64_t n, int64_t ld)
{
    if (rows <= 0 || n <= 0) return 0;
    return (size_t)(((rows - 1) * ld + n) * (int64_t)sizeof(float2));
}

// Forward launch for an already-prepared device table M.
dpd_status run_forward(const CoefMap &map, const dpd_tune &tune, const float *M, hipStream_t stream,
                       const void *in, void *out, int64_t rows, int64_t n, int64_t ld,
                       const void *hist)
{
    FwdParams p;
    p.in = (const float2 *)in;
    p.out = (float2 *)out;
    p.n = n;
    p.ld = ld;
    p.M = M;
    p.hist = (const float2 *)hist;
    const bool aligned = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0) &&
                         (rows == 1 || ld % 2 == 0);
    if (aligned && map.NI <= kSpecNI && map.L <= kSpecL) {
        const FwdTable &t = fwd_table();
        const int v = fwd_variant(tune);
        const int64_t T = t.tile[v];
        p.tiles_per_row = (n + T - 1) / T;
        p.total_tiles = p.tiles_per_row * rows;
        hipError_t e = t.fn[map.NI - 1][map.L - 1][v](p, stream, tune.grid_mult);
        return e == hipSuccess ? DPD_OK : hip_fail(e);
    }
    p.tiles_per_row = 0;
    p.total_tiles = rows * n;
    const int64_t blocks = std::min<int64_t>((p.total_tiles + kBlock - 1) / kBlock, 1 << 20);
    hipLaunchKernelGGL(fwd_generic_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, p,
                       map.NI, map.L);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

dpd_status check_io(const void *in, const void *out, int64_t rows, int64_t n, int64_t ld)
{
    if (n < 0 || rows < 0) return DPD_EINVAL;
    if (rows > 1 && ld < n) return DPD_EINVAL;
    if (n == 0 || rows == 0) return DPD_OK;
    if (in == nullptr || out == nullptr) return DPD_EINVAL;
    if ((uintptr_t)in % 8 != 0 || (uintptr_t)out % 8 != 0) return DPD_EINVAL;
    if (overlap(in, span_bytes(rows, n, ld), out, span_bytes(rows, n, ld))) return DPD_EINVAL;
    return DPD_OK;
}

}  // namespace dpd

using namespace dpd;

// ================================================================= C ABI ===

DPD_EXPORT dpd_status dpd_create(const int32_t *main_orders, int32_t n_main, const int32_t *conj_orders,
                                 int32_t n_conj, int32_t L, const float *coeffs_host, dpd_plan **out)
{
    if (out == nullptr || coeffs_host == nullptr) return DPD_EINVAL;
    CoefMap map;
    dpd_status st = make_map(main_orders, n_main, conj_orders, n_conj, L, map);
    if (st != DPD_OK) return st;
    dpd_plan *p = new (std::nothrow) dpd_plan();
    if (p == nullptr) return DPD_ENOMEM;
    p->map = map;
    p->K = (n_main + n_conj) * L + 1;
    p->tune = default_tune();
    p->raw.assign(coeffs_host, coeffs_host + 2 * p->K);
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e);
    }
    const size_t bytes = ((size_t)table_floats(L, map.NI) * sizeof(float) + 255) & ~(size_t)255;
    e = hipMalloc((void **)&p->d_table, 2 * bytes);
    if (e != hipSuccess) {
        delete p;
        return e == hipErrorOutOfMemory ? DPD_ENOMEM : hip_fail(e);
    }
    p->d_table_call = p->d_table + bytes / sizeof(float);
    std::vector<float> M;
    precombine_host(map, p->raw.data(), M);
    e = hipMemcpy(p->d_table, M.data(), M.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->d_table);
        delete p;
        return hip_fail(e);
    }
    *out = p;
    return DPD_OK;
}

// hipFree and hipHostFree wait for the device themselves: the plan's memory
// is released only after every kernel that may read it has finished.
DPD_EXPORT dpd_status dpd_destroy(dpd_plan *plan)
{
    if (plan == nullptr) return DPD_OK;
    hipError_t e = hipSuccess;
    if (plan->d_table) e = hipFree(plan->d_table);
    if (plan->staged) (void)hipEventDestroy(plan->staged);
    if (plan->h_stage) (void)hipHostFree(plan->h_stage);
    delete plan;
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_num_coeffs(const dpd_plan *plan, int32_t *K)
{
    if (plan == nullptr || K == nullptr) return DPD_EINVAL;
    *K = plan->K;
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_set_coeffs(dpd_plan *plan, const float *coeffs_host)
{
    if (plan == nullptr || coeffs_host == nullptr) return DPD_EINVAL;
    std::vector<float> M;
    precombine_host(plan->map, coeffs_host, M);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e);
    e = hipMemcpy(plan->d_table, M.data(), M.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    plan->raw.assign(coeffs_host, coeffs_host + 2 * plan->K);
    return DPD_OK;
}

// Stream-ordered: the precombined table goes through a pinned staging buffer
// of the plan; before refilling it, the host waits only for the previous copy
// out of it (the plan's event), not for the device.
DPD_EXPORT dpd_status dpd_set_coeffs_async(dpd_plan *plan, const float *coeffs_host, void *stream)
{
    if (plan == nullptr || coeffs_host == nullptr) return DPD_EINVAL;
    std::vector<float> M;
    precombine_host(plan->map, coeffs_host, M);
    const size_t bytes = M.size() * sizeof(float);
    hipError_t e = hipSuccess;
    if (plan->h_stage == nullptr) {
        e = hipHostMalloc((void **)&plan->h_stage, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            plan->h_stage = nullptr;
            return e == hipErrorOutOfMemory ? DPD_ENOMEM : hip_fail(e);
        }
        e = hipEventCreateWithFlags(&plan->staged, hipEventDisableTiming);
        if (e != hipSuccess) {
            plan->staged = nullptr;
            return hip_fail(e);
        }
    } else {
        e = hipEventSynchronize(plan->staged);
        if (e != hipSuccess) return hip_fail(e);
    }
    std::memcpy(plan->h_stage, M.data(), bytes);
    const hipStream_t st = (hipStream_t)stream;
    e = hipMemcpyAsync(plan->d_table, plan->h_stage, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(plan->staged, st);
    if (e != hipSuccess) return hip_fail(e);
    plan->raw.assign(coeffs_host, coeffs_host + 2 * plan->K);
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_set_coeffs_device(dpd_plan *plan, const void *coeffs_dev, void *stream)
{
    if (plan == nullptr || coeffs_dev == nullptr || (uintptr_t)coeffs_dev % 8 != 0) return DPD_EINVAL;
    hipError_t e = launch_prep(plan->map, coeffs_dev, plan->d_table, (hipStream_t)stream);
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_set_coeffs_device_if(dpd_plan *plan, const void *coeffs_dev, const int32_t *flag_dev,
                                               void *stream)
{
    if (plan == nullptr || coeffs_dev == nullptr || (uintptr_t)coeffs_dev % 8 != 0) return DPD_EINVAL;
    if (flag_dev == nullptr || (uintptr_t)flag_dev % 4 != 0) return DPD_EINVAL;
    hipError_t e = launch_prep(plan->map, coeffs_dev, plan->d_table, (hipStream_t)stream, flag_dev);
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_set_tune(dpd_plan *plan, const dpd_tune *tune)
{
    if (plan == nullptr || tune == nullptr || !valid_tune(*tune)) return DPD_EINVAL;
    plan->tune = *tune;
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_get_tune(const dpd_plan *plan, dpd_tune *tune)
{
    if (plan == nullptr || tune == nullptr) return DPD_EINVAL;
    *tune = plan->tune;
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_apply_rows(dpd_plan *plan, void *stream, const void *in, void *out,
                                     int64_t rows, int64_t n, int64_t ld)
{
    if (plan == nullptr) return DPD_EINVAL;
    if (rows == 1 && ld < n) ld = n;
    dpd_status st = check_io(in, out, rows, n, ld);
    if (st != DPD_OK || n == 0 || rows == 0) return st;
    return run_forward(plan->map, plan->tune, plan->d_table, (hipStream_t)stream, in, out, rows, n,
                       ld, nullptr);
}

DPD_EXPORT dpd_status dpd_apply(dpd_plan *plan, void *stream, const void *in, void *out, int64_t n)
{
    return dpd_apply_rows(plan, stream, in, out, 1, n, n);
}

DPD_EXPORT dpd_status dpd_apply_coeffs(dpd_plan *plan, void *stream, const void *coeffs_dev,
                                       const void *in, void *out, int64_t rows, int64_t n, int64_t ld)
{
    if (plan == nullptr || coeffs_dev == nullptr || (uintptr_t)coeffs_dev % 8 != 0) return DPD_EINVAL;
    if (rows == 1 && ld < n) ld = n;
    dpd_status st = check_io(in, out, rows, n, ld);
    if (st != DPD_OK) return st;
    hipError_t e = launch_prep(plan->map, coeffs_dev, plan->d_table_call, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    if (n == 0 || rows == 0) return DPD_OK;
    return run_forward(plan->map, plan->tune, plan->d_table_call, (hipStream_t)stream, in, out, rows, n,
                       ld, nullptr);
}

DPD_EXPORT dpd_status dpd_apply_hist(dpd_plan *plan, void *stream, const void *in, void *out,
                                     int64_t n, void *hist)
{
    if (plan == nullptr) return DPD_EINVAL;
    const int Lm1 = plan->map.L - 1;
    if (Lm1 > 0 && (hist == nullptr || (uintptr_t)hist % 8 != 0)) return DPD_EINVAL;
    dpd_status st = check_io(in, out, 1, n, n);
    if (st != DPD_OK || n == 0) return st;
    const size_t hb = (size_t)Lm1 * sizeof(float2);
    if (overlap(hist, hb, in, (size_t)n * 8) || overlap(hist, hb, out, (size_t)n * 8)) return DPD_EINVAL;
    st = run_forward(plan->map, plan->tune, plan->d_table, (hipStream_t)stream, in, out, 1, n, n,
                     Lm1 > 0 ? hist : nullptr);
    if (st != DPD_OK || Lm1 == 0) return st;
    hipLaunchKernelGGL(hist_update_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream,
                       (const float2 *)in, n, (float2 *)hist, Lm1);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_copy(void *stream, const void *in, void *out, int64_t n)
{
    if (n < 0) return DPD_EINVAL;
    if (n == 0) return DPD_OK;
    if (in == nullptr || out == nullptr || (uintptr_t)in % 16 != 0 || (uintptr_t)out % 16 != 0) return DPD_EINVAL;
    if (overlap(in, (size_t)n * 8, out, (size_t)n * 8)) return DPD_EINVAL;
    const int64_t want = (int64_t)num_cus() * 2;      // the forward kernel's persistent grid
    const int64_t need = (n / 512 + 3) / 4;
    const int64_t grid = std::max<int64_t>(1, std::min(want, need));
    hipLaunchKernelGGL(copy_walk_kernel, dim3((uint32_t)grid), dim3(kBlock), 0, (hipStream_t)stream,
                       (const float2 *)in, (float2 *)out, n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT const char *dpd_status_string(dpd_status status)
{
    switch (status) {
    case DPD_OK: return "DPD_OK";
    case DPD_EINVAL: return "DPD_EINVAL: invalid argument";
    case DPD_EUNSUPPORTED: return "DPD_EUNSUPPORTED: order, L or size outside the supported range";
    case DPD_ENOMEM: return "DPD_ENOMEM: allocation failed";
    case DPD_EHIP: return "DPD_EHIP: HIP runtime error (see dpd_last_hip_error)";
    }
    return "unknown dpd_status";
}

DPD_EXPORT int dpd_last_hip_error(void)
{
    return g_last_hip_error;
}

DPD_EXPORT const char *dpd_version(void)
{
    return "libdpd 0.1.0 gfx950";
}
