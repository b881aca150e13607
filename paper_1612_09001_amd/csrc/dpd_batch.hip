// Host side of the batched multi-stream apply (dpd_batch_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dpd.h"
#include "dpd_batch_kernels.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

struct dpd_batch {
    int device = 0;
    int32_t n_streams = 0;
    std::vector<dpd_stream_desc> desc;
    std::vector<dpd::CoefMap> maps;
    std::vector<int32_t> tab;
    std::vector<int32_t> fallback;       // streams run by separate launches
    dpd::BatchChunk *d_chunks = nullptr;  // full chunks, ragged chunks, idle entry
    dpd::BatchPrepJob *d_jobs = nullptr;
    int32_t n_jobs = 0;
    float *d_tables = nullptr;
    float2 *d_idle = nullptr;              // samples the idle entry points at
    int64_t n_full = 0;
    int64_t n_chunks = 0;
    int grid = 0;        // blocks of the streaming kernel
    int tail_grid = 0;   // blocks of the ragged-chunk kernel
    int sidx = 2;
    dpd_tune tune;
    int64_t n_heavy = 0;
    int32_t light_mask = 0;
};

namespace dpd {

int num_cus();

// Precombine every stream's coefficients into its table: one thread per
// table entry (a flat job list built at create), one dependent load.
__global__ void __launch_bounds__(kBlock) batch_prep_kernel(const BatchPrepJob *__restrict__ jobs, int32_t n_jobs,
                                                            float *__restrict__ tables)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_jobs) return;
    const BatchPrepJob jb = jobs[i];
    const float2 h = jb.h != nullptr ? *jb.h : make_float2(0.f, 0.f);
    const float2 g = jb.g != nullptr ? *jb.g : make_float2(0.f, 0.f);
    if (jb.dc) {
        tables[jb.out] = h.x;
        tables[jb.out + 1] = h.y;
    } else {
        *reinterpret_cast<float4 *>(tables + jb.out) = make_float4(h.x + g.x, g.y - h.y, h.y + g.y, h.x - g.x);
    }
}

static BatchTable g_batch;
static std::once_flag g_batch_once;

static const BatchTable &batch_table()
{
    std::call_once(g_batch_once, [] {
        std::memset(&g_batch, 0, sizeof(g_batch));
        register_batch_s2(g_batch);
        register_batch_s4(g_batch);
        register_batch_s8(g_batch);
    });
    return g_batch;
}

static int batch_occupancy(int sidx)
{
    static int cache[kNumSIdx] = {};
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[sidx] == 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, batch_table().kern[sidx], kBlock, 0) !=
                hipSuccess ||
            v < 1)
            v = 1;
        cache[sidx] = v;
    }
    return cache[sidx];
}

static void free_batch(dpd_batch *b)
{
    if (b->d_chunks) (void)hipFree(b->d_chunks);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_tables) (void)hipFree(b->d_tables);
    if (b->d_idle) (void)hipFree(b->d_idle);
    delete b;
}

template <class T>
static hipError_t upload(T **dst, const std::vector<T> &v)
{
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

static dpd_status batch_prep(dpd_batch *b, hipStream_t st)
{
    if (b->n_streams == 0) return DPD_OK;
    if (b->n_jobs == 0) return DPD_OK;
    hipLaunchKernelGGL(batch_prep_kernel, dim3((uint32_t)((b->n_jobs + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       b->d_jobs, b->n_jobs, b->d_tables);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

static dpd_status run_stream(dpd_batch *b, int s, hipStream_t st)
{
    const dpd_stream_desc &d = b->desc[s];
    if (d.n == 0) return DPD_OK;
    return run_forward(b->maps[s], default_tune(), b->d_tables + b->tab[s], st, d.in, d.out, 1, d.n, d.n,
                       nullptr);
}

}  // namespace dpd

using namespace dpd;

DPD_EXPORT dpd_status dpd_batch_create(const dpd_stream_desc *desc, int32_t n_streams, const dpd_tune *tune,
                                       dpd_batch **out)
{
    if (out == nullptr || n_streams < 0 || (n_streams > 0 && desc == nullptr)) return DPD_EINVAL;
    if (desc == nullptr) return DPD_EINVAL;
    dpd_tune t = default_tune();
    if (tune != nullptr) {
        if (!valid_tune(*tune) || tune->stage_lds != 1) return DPD_EINVAL;
        t = *tune;
    }
    dpd_batch *b = new (std::nothrow) dpd_batch();
    if (b == nullptr) return DPD_ENOMEM;
    b->tune = t;
    b->sidx = t.samples_per_thread == 2 ? 0 : (t.samples_per_thread == 4 ? 1 : 2);
    b->n_streams = n_streams;
    b->desc.assign(desc, desc + n_streams);
    std::vector<BatchPrepJob> jobs;
    std::vector<int32_t> order;   // streams in the persistent kernel
    int64_t tab_total = 0;
    for (int32_t s = 0; s < n_streams; ++s) {
        const dpd_stream_desc &d = desc[s];
        int32_t mo[kMaxNI], co[kMaxNI], nm = 0, nc = 0;
        if ((d.main_mask >> kMaxNI) != 0 || (d.conj_mask >> kMaxNI) != 0) {
            free_batch(b);
            return DPD_EUNSUPPORTED;
        }
        for (int j = 0; j < kMaxNI; ++j) {
            if (d.main_mask & (1u << j)) mo[nm++] = 2 * j + 1;
            if (d.conj_mask & (1u << j)) co[nc++] = 2 * j + 1;
        }
        CoefMap map;
        dpd_status st = make_map(mo, nm, co, nc, d.L, map);
        if (st == DPD_OK && (d.n < 0 || d.coeffs_dev == nullptr || (uintptr_t)d.coeffs_dev % 8 != 0))
            st = DPD_EINVAL;
        if (st == DPD_OK) st = check_io(d.in, d.out, 1, d.n, d.n);
        if (st != DPD_OK) {
            free_batch(b);
            return st;
        }
        b->maps.push_back(map);
        b->tab.push_back((int32_t)tab_total);
        {
            // table entries of this stream: matrix (k, j) at 4 (k NI + j), then c
            const float2 *raw = (const float2 *)d.coeffs_dev;
            for (int k = 0; k < map.L; ++k)
                for (int j = 0; j < map.NI; ++j) {
                    BatchPrepJob jb;
                    jb.h = map.main_idx[j] >= 0 ? raw + map.main_idx[j] * map.L + k : nullptr;
                    jb.g = map.conj_idx[j] >= 0 ? raw + (map.n_main + map.conj_idx[j]) * map.L + k : nullptr;
                    jb.out = (int32_t)(tab_total + 4 * (k * map.NI + j));
                    jb.dc = 0;
                    jb.pad_ = 0;
                    jobs.push_back(jb);
                }
            BatchPrepJob jc;
            jc.h = raw + (map.n_main + map.n_conj) * map.L;
            jc.g = nullptr;
            jc.out = (int32_t)(tab_total + 4 * map.L * map.NI);
            jc.dc = 1;
            jc.pad_ = 0;
            jobs.push_back(jc);
        }
        tab_total += (table_floats(map.L, map.NI) + 3) & ~3;
        const bool aligned = (uintptr_t)d.in % 16 == 0 && (uintptr_t)d.out % 16 == 0;
        const bool in_kernel = aligned && map.NI <= kBatchMaxNI && map.L <= kBatchMaxL;
        if (!in_kernel) {
            b->fallback.push_back(s);
            continue;
        }
        if (d.n > 0) order.push_back(s);
    }
    // No stream may write where any stream reads or another one writes
    // (inputs may be shared).  Sorted output ranges overlap iff two neighbours
    // do; each input range is then looked up among them: O(n log n).
    {
        std::vector<std::pair<uintptr_t, uintptr_t>> outs;   // [begin, end) of every output
        for (int32_t s = 0; s < n_streams; ++s)
            if (desc[s].n > 0)
                outs.emplace_back((uintptr_t)desc[s].out, (uintptr_t)desc[s].out + (size_t)desc[s].n * 8);
        std::sort(outs.begin(), outs.end());
        bool bad = false;
        for (size_t i = 1; i < outs.size() && !bad; ++i) bad = outs[i].first < outs[i - 1].second;
        for (int32_t s = 0; s < n_streams && !bad; ++s) {
            if (desc[s].n == 0) continue;
            const uintptr_t lo = (uintptr_t)desc[s].in, hi = lo + (size_t)desc[s].n * 8;
            // the first output ending after lo (ends ascend: the ranges are disjoint and sorted)
            auto it = std::upper_bound(outs.begin(), outs.end(), lo,
                                       [](uintptr_t v, const std::pair<uintptr_t, uintptr_t> &o) { return v < o.second; });
            bad = it != outs.end() && it->first < hi;
        }
        if (bad) {
            free_batch(b);
            return DPD_EINVAL;
        }
    }
    if (tab_total >= (int64_t)1 << 30) {
        free_batch(b);
        return DPD_EUNSUPPORTED;
    }
    // Streams most expensive class first (per-sample cost ~ NI * L), one class
    // together, then stream order; their full chunks in that order, then the
    // ragged last chunks in the same order, then the idle entry.
    auto cls_of = [&](int32_t s) { return (b->maps[s].NI - 1) * kBatchMaxL + (b->maps[s].L - 1); };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const int cx = b->maps[x].NI * b->maps[x].L, cy = b->maps[y].NI * b->maps[y].L;
        return cx != cy ? cx > cy : cls_of(x) < cls_of(y);
    });
    const int64_t C = 64 * (int64_t)t.samples_per_thread;
    std::vector<BatchChunk> chunks;
    auto push = [&](int32_t s, int64_t t0, int64_t valid) {
        const dpd_stream_desc &d = desc[s];
        const CoefMap &m = b->maps[s];
        BatchChunk c;
        c.in = (const float2 *)d.in + t0;
        c.out = (float2 *)d.out + t0;
        c.tab = b->tab[s];
        c.meta = batch_meta(cls_of(s), (int)std::min<int64_t>(t0, kBatchHalo),
                            (table_floats(m.L, m.NI) + 3) / 4);
        c.valid = (int32_t)valid;
        c.pad_ = 0;
        chunks.push_back(c);
    };
    for (int32_t s : order)
        for (int64_t t0 = 0; t0 + C <= desc[s].n; t0 += C) push(s, t0, C);
    b->n_full = (int64_t)chunks.size();
    for (int32_t s : order)
        if (desc[s].n % C != 0) push(s, desc[s].n - desc[s].n % C, desc[s].n % C);
    b->n_chunks = (int64_t)chunks.size();
    const int64_t cap = (int64_t)num_cus() * std::min(t.grid_mult, batch_occupancy(b->sidx));
    const int64_t waves = kBlock / 64;
    b->grid = (int)std::min<int64_t>(cap, (b->n_full + waves - 1) / waves);
    // Heavy and light chunks side by side (batch_kernel): with whole slots of
    // blocks (grid a multiple of the CU count, two or more per CU), the blocks
    // of slot 1 walk the light end of the cost-sorted list and the others the
    // heavy start, split where the cumulative cost max(NI L, 10) reaches 55 %
    // of the total (60 % with two slots).  Measured on the 256-stream
    // workload: 480 -> 449 us with three slots; the cost floor stands for
    // the memory time of a chunk, which the lightest classes are bound by.
    {
        const int ncu = num_cus();
        const int slots = b->grid % ncu == 0 ? b->grid / ncu : 0;
        if (slots >= 2) {
            const double f = slots == 2 ? 0.60 : 0.55;
            auto cost = [](const BatchChunk &c) {
                const int cl = (int)(c.meta & 0xffu);
                return std::max(10.0, (double)((cl / kBatchMaxL + 1) * (cl % kBatchMaxL + 1)));
            };
            double tot = 0.0, cum = 0.0;
            for (int64_t i = 0; i < b->n_full; ++i) tot += cost(chunks[i]);
            int64_t h = 0;
            while (h < b->n_full && cum < f * tot) cum += cost(chunks[h++]);
            b->n_heavy = h;
            b->light_mask = 1 << 1;
        }
    }
    b->tail_grid = (int)std::min<int64_t>(cap, (b->n_chunks - b->n_full + waves - 1) / waves);
    hipError_t e = hipGetDevice(&b->device);
    // zero fills as synchronous host copies: complete on return, so no
    // stream (whatever its flags) can see the buffers before they hold zeros
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_idle, (size_t)C * sizeof(float2));
    if (e == hipSuccess) {
        const std::vector<float2> zeros((size_t)C, make_float2(0.f, 0.f));
        e = hipMemcpy(b->d_idle, zeros.data(), zeros.size() * sizeof(float2), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        BatchChunk idle;
        idle.in = b->d_idle;
        idle.out = b->d_idle;   // never written: the idle entry is only read
        idle.tab = 0;
        idle.meta = batch_meta(0, 0, 1);
        idle.valid = (int32_t)C;
        idle.pad_ = 0;
        chunks.push_back(idle);
        e = upload(&b->d_chunks, chunks);
    }
    if (e == hipSuccess) e = upload(&b->d_jobs, jobs);
    b->n_jobs = (int32_t)jobs.size();
    // + 4 floats: the idle entry reads table floats 0..3
    if (e == hipSuccess) e = upload(&b->d_tables, std::vector<float>((size_t)(tab_total + 4), 0.f));
    if (e != hipSuccess) {
        free_batch(b);
        return e == hipErrorOutOfMemory ? DPD_ENOMEM : hip_fail(e);
    }
    *out = b;
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_batch_apply(dpd_batch *b, void *stream)
{
    if (b == nullptr) return DPD_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    dpd_status s = batch_prep(b, st);
    if (s != DPD_OK) return s;
    if (b->n_chunks > 0) {
        BatchParams bp;
        bp.chunks = b->d_chunks;
        bp.n_full = b->n_full;
        bp.n_chunks = b->n_chunks;
        bp.tables = b->d_tables;
        bp.n_heavy = b->n_heavy;
        bp.ncu = num_cus();
        bp.light_mask = b->light_mask;
        hipError_t e = batch_table().fn[b->sidx](bp, st, b->grid, b->tail_grid);
        if (e != hipSuccess) return hip_fail(e);
    }
    for (int32_t idx : b->fallback) {
        s = run_stream(b, idx, st);
        if (s != DPD_OK) return s;
    }
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_batch_apply_each(dpd_batch *b, void *stream)
{
    if (b == nullptr) return DPD_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    dpd_status s = batch_prep(b, st);
    if (s != DPD_OK) return s;
    for (int32_t i = 0; i < b->n_streams; ++i) {
        s = run_stream(b, i, st);
        if (s != DPD_OK) return s;
    }
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_batch_info(const dpd_batch *b, int64_t *n_tiles, int32_t *n_blocks)
{
    if (b == nullptr || n_tiles == nullptr || n_blocks == nullptr) return DPD_EINVAL;
    *n_tiles = b->n_chunks;
    *n_blocks = b->grid;
    return DPD_OK;
}

// hipFree waits for the device itself, so in-flight batch kernels finish
// before their chunk list and tables are released.
DPD_EXPORT dpd_status dpd_batch_destroy(dpd_batch *b)
{
    if (b == nullptr) return DPD_OK;
    free_batch(b);
    return DPD_OK;
}
