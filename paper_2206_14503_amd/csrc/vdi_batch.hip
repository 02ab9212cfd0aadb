// vdi_batch.hip -- host side of batched compositing: job and tile tables,
// tile sizes per (k, N) bucket from the autotune cache, graph capture, and the
// autotuner that fills the cache.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

namespace {

constexpr int kDefaultTile = 256;
constexpr int kCandidates[] = { 64, 128, 256, 512, 1024 };

int k_bucket(int k) { return k <= 4 ? 0 : (k <= 8 ? 1 : 2); }

struct BatchImpl {
    vdi_ctx* ctx = nullptr;
    int n_jobs = 0;
    CompParams* d_jobs = nullptr;
    uint2* d_tiles = nullptr;
    uint32_t* d_head = nullptr;
    int* d_queue = nullptr;     // per job: [npix] queued pixels, then the counters [n_jobs]
    size_t q_total = 0;         // queue entries before the counters
    uint32_t n_tiles = 0;
    size_t lds = 0;             // depth-disjoint phase
    int grid = 0;
    size_t lds_gen = 0;         // general-merge phase
    int grid_gen = 0;
    double clock_hz = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

size_t queue_counters(const BatchImpl* b) { return b->q_total; }

using TileMap = std::map<std::pair<int, int>, int>;

TileMap read_cache(const char* path, const char* arch)
{
    TileMap m;
    if (!path) return m;
    FILE* f = fopen(path, "r");
    if (!f) return m;
    char a[64];
    int kb, n, tile;
    double ms;
    while (fscanf(f, "%63s %d %d %d %lf", a, &kb, &n, &tile, &ms) == 5)
        if (strcmp(a, arch) == 0 && tile > 0 && tile <= 4096) m[{ kb, n }] = tile;
    fclose(f);
    return m;
}

vdi_status check_job(const vdi_job_t& j, int idx)
{
    if (!j.in || j.k < 1 || j.k > VDI_MAX_INPUTS) return fail(VDI_E_INVALID, "job %d: k=%d or in NULL", idx, j.k);
    const vdi_t& o = j.out;
    if (o.layout != VDI_LAYOUT_REGULAR || o.width <= 0 || o.height <= 0 || o.max_n < 1 || o.max_n > VDI_MAX_N ||
        !o.color || !o.depth || !o.count || !(o.ref_step > 0.0f))
        return fail(VDI_E_INVALID, "job %d: bad output", idx);
    if ((int64_t)o.width * o.height >= ((int64_t)1 << 31)) return fail(VDI_E_UNSUPPORTED, "job %d: too large", idx);
    if (j.tau.mode != VDI_TAU_FIXED && j.tau.mode != VDI_TAU_BISECT)
        return fail(VDI_E_UNSUPPORTED, "job %d: tau mode must be FIXED or BISECT", idx);
    if (j.tau.mode == VDI_TAU_BISECT && (j.tau.iters < 1 || j.tau.iters > 24 || !(j.tau.gamma_max > 1.7320509f)))
        return fail(VDI_E_INVALID, "job %d: bisection parameters", idx);
    int seq_cap = 0;
    for (int r = 0; r < j.k; ++r) {
        const vdi_t& v = j.in[r];
        if (v.width != o.width || v.height != o.height || v.ref_step != o.ref_step)
            return fail(VDI_E_INVALID, "job %d input %d: size or ref_step differs from the output", idx, r);
        if (v.max_n < 1 || v.max_n > VDI_MAX_N || !v.color || !v.depth || !v.count)
            return fail(VDI_E_INVALID, "job %d input %d: bad VDI", idx, r);
        if (v.layout == VDI_LAYOUT_COMPACT && !v.offset) return fail(VDI_E_INVALID, "job %d input %d: offset", idx, r);
        seq_cap += v.max_n;
    }
    if (composite_lds_bytes(j.k, seq_cap) > 160 * 1024) return fail(VDI_E_UNSUPPORTED, "job %d: k*N too large", idx);
    return VDI_OK;
}

int any_compact(const vdi_t* in, int k)
{
    for (int r = 0; r < k; ++r)
        if (in[r].layout == VDI_LAYOUT_COMPACT) return 1;
    return 0;
}

CompParams job_params(vdi_ctx* ctx, const vdi_job_t& j)
{
    CompParams P;
    memset(&P, 0, sizeof P);
    int seq_cap = 0;
    for (int r = 0; r < j.k; ++r) {
        const vdi_t& v = j.in[r];
        P.in[r].color = (const float4*)v.color;
        P.in[r].depth = (const float2*)v.depth;
        P.in[r].count = v.count;
        P.in[r].offset = v.offset;
        P.in[r].max_n = v.max_n;
        P.in[r].compact = v.layout == VDI_LAYOUT_COMPACT;
        P.in[r].capacity = P.in[r].compact ? v.capacity : (uint64_t)v.max_n * (uint64_t)v.width * v.height;
        seq_cap += v.max_n;
    }
    P.k = j.k;
    P.npix = (uint32_t)((size_t)j.out.width * j.out.height);
    P.cache_bound = any_compact(j.in, j.k);
    P.inv_ref = 1.0f / j.out.ref_step;
    P.mode = j.tau.mode;
    P.tau = j.tau.tau;
    P.iters = j.tau.iters;
    P.gmax = j.tau.gamma_max;
    P.out_n = j.out.max_n;
    P.out_color = (float4*)j.out.color;
    P.out_depth = (float2*)j.out.depth;
    P.out_count = j.out.count;
    P.out_gamma = j.out.gamma;
    P.status = ctx->status;
    P.seq_cap = seq_cap;
    return P;
}

void destroy_impl(BatchImpl* b)
{
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->d_jobs) hipFree(b->d_jobs);
    if (b->d_tiles) hipFree(b->d_tiles);
    if (b->d_head) hipFree(b->d_head);
    if (b->d_queue) hipFree(b->d_queue);
    delete b;
}

vdi_status create_impl(vdi_ctx* ctx, const vdi_job_t* jobs, int n_jobs, const TileMap& tiles_by_bucket,
                       int forced_tile, BatchImpl** out)
{
    *out = nullptr;
    if (!ctx || !jobs || n_jobs < 1 || n_jobs > 65535) return fail(VDI_E_INVALID, "bad batch arguments");
    for (int i = 0; i < n_jobs; ++i) {
        vdi_status st = check_job(jobs[i], i);
        if (st != VDI_OK) return st;
    }
    std::vector<CompParams> hp(n_jobs);
    std::vector<double> work(n_jobs);
    std::vector<size_t> q_off(n_jobs);
    size_t lds = 0, lds_gen = 0, q_total = 0;
    for (int i = 0; i < n_jobs; ++i) {
        hp[i] = job_params(ctx, jobs[i]);
        lds_gen = std::max(lds_gen, composite_lds_bytes(hp[i].k, hp[i].seq_cap));
        // compact inputs run at the general merge's occupancy (see launch_composite)
        if (hp[i].k <= kCatMaxInputs)
            lds = std::max(lds, hp[i].cache_bound ? std::max(cat_lds_bytes(hp[i].k),
                                                             composite_lds_bytes(hp[i].k, hp[i].seq_cap))
                                                  : cat_lds_bytes(hp[i].k));
        work[i] = (double)hp[i].k * hp[i].out_n * hp[i].npix;
        q_off[i] = q_total;
        q_total += hp[i].k <= kCatMaxInputs ? hp[i].npix : 0;
    }
    std::vector<int> order(n_jobs);
    for (int i = 0; i < n_jobs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<uint2> tiles;
    for (int j : order) {
        if (hp[j].k > kCatMaxInputs) continue;   // general merge only
        int tile = forced_tile;
        if (tile <= 0) {
            auto it = tiles_by_bucket.find({ k_bucket(hp[j].k), hp[j].out_n });
            tile = it != tiles_by_bucket.end() ? it->second : kDefaultTile;
        }
        // tile size in pixels -> whole 64-pixel blocks (at least one)
        const uint32_t per = std::max<uint32_t>(1u, (uint32_t)tile / 64u);
        const uint32_t nblocks = composite_blocks(hp[j]);
        for (uint32_t b0 = 0; b0 < nblocks; b0 += per) {
            uint32_t nb = std::min<uint32_t>(per, nblocks - b0);
            tiles.push_back(make_uint2((uint32_t)j | (nb << 16), b0));
        }
    }
    BatchImpl* b = new BatchImpl();
    b->ctx = ctx;
    b->n_jobs = n_jobs;
    b->n_tiles = (uint32_t)tiles.size();
    b->lds = lds;
    b->lds_gen = lds_gen;
    b->q_total = q_total;
    // blocks per CU: limited by LDS (160 KiB per CU) and by 7 waves per SIMD
    int per_cu = std::max(1, std::min<int>((int)((160 * 1024) / (lds + 64)), 28));
    b->grid = std::max(1, std::min<int>(ctx->num_cus * per_cu, (int)b->n_tiles));
    int per_cu_gen = std::max(1, std::min<int>((int)((160 * 1024) / (lds_gen + 64)), 28));
    b->grid_gen = ctx->num_cus * per_cu_gen;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0)
        khz = 100000;
    b->clock_hz = (double)khz * 1e3;
    hipError_t e = hipMalloc(&b->d_jobs, sizeof(CompParams) * n_jobs);
    if (e == hipSuccess) e = hipMalloc(&b->d_tiles, sizeof(uint2) * std::max<size_t>(tiles.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_head, 256);
    if (e == hipSuccess) e = hipMalloc(&b->d_queue, sizeof(int) * (q_total + (size_t)n_jobs));
    if (e == hipSuccess) {
        for (int i = 0; i < n_jobs; ++i) {
            hp[i].q_list = b->d_queue + q_off[i];
            hp[i].q_count = b->d_queue + q_total + i;
        }
        e = hipMemcpy(b->d_jobs, hp.data(), sizeof(CompParams) * n_jobs, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(b->d_tiles, tiles.data(), sizeof(uint2) * tiles.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy_impl(b);
        return fail(VDI_E_HIP, "batch setup: %s", hipGetErrorString(e));
    }
    *out = b;
    return VDI_OK;
}

vdi_status run_impl(BatchImpl* b, uint64_t* t_se, hipStream_t s)
{
    launch_batch(b->d_jobs, b->d_tiles, b->n_tiles, b->d_head, b->d_queue + queue_counters(b), (unsigned long long*)t_se,
                 b->n_jobs, b->lds, b->grid, b->lds_gen, b->grid_gen, s);
    return launched();
}

}  // namespace
}  // namespace vdi

using namespace vdi;

extern "C" {

vdi_status vdi_batch_create(vdi_ctx* ctx, const vdi_job_t* jobs, int n_jobs, const char* autotune_cache,
                            vdi_batch** out)
{
    if (!out) return fail(VDI_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(VDI_E_INVALID, "ctx is NULL");
    BatchImpl* b = nullptr;
    vdi_status st = create_impl(ctx, jobs, n_jobs, read_cache(autotune_cache, ctx->arch), 0, &b);
    if (st != VDI_OK) return st;
    *out = (vdi_batch*)b;
    return VDI_OK;
}

vdi_status vdi_batch_run(vdi_batch* batch, uint64_t* t_start_end, void* stream)
{
    if (!batch) return fail(VDI_E_INVALID, "batch is NULL");
    return run_impl((BatchImpl*)batch, t_start_end, (hipStream_t)stream);
}

vdi_status vdi_batch_capture(vdi_batch* batch, uint64_t* t_start_end, void* stream)
{
    if (!batch) return fail(VDI_E_INVALID, "batch is NULL");
    if (!stream) return fail(VDI_E_INVALID, "capture needs a non-default stream");
    BatchImpl* b = (BatchImpl*)batch;
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    VDI_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    launch_batch(b->d_jobs, b->d_tiles, b->n_tiles, b->d_head, b->d_queue + queue_counters(b),
                 (unsigned long long*)t_start_end, b->n_jobs, b->lds, b->grid, b->lds_gen, b->grid_gen, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return fail(VDI_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    VDI_HIP_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return VDI_OK;
}

vdi_status vdi_batch_replay(vdi_batch* batch, void* stream)
{
    if (!batch) return fail(VDI_E_INVALID, "batch is NULL");
    BatchImpl* b = (BatchImpl*)batch;
    if (!b->exec) return fail(VDI_E_INVALID, "batch has no captured graph");
    VDI_HIP_CHECK(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return VDI_OK;
}

vdi_status vdi_batch_info(const vdi_batch* batch, int32_t* n_tiles, int32_t* grid, int32_t* lds_bytes,
                          double* clock_hz)
{
    if (!batch) return fail(VDI_E_INVALID, "batch is NULL");
    const BatchImpl* b = (const BatchImpl*)batch;
    if (n_tiles) *n_tiles = (int32_t)b->n_tiles;
    if (grid) *grid = b->grid;
    if (lds_bytes) *lds_bytes = (int32_t)b->lds;
    if (clock_hz) *clock_hz = b->clock_hz;
    return VDI_OK;
}

vdi_status vdi_batch_destroy(vdi_batch* batch)
{
    if (!batch) return VDI_OK;
    BatchImpl* b = (BatchImpl*)batch;
    hipSetDevice(b->ctx->device);
    hipDeviceSynchronize();
    destroy_impl(b);
    return VDI_OK;
}

vdi_status vdi_autotune(vdi_ctx* ctx, const vdi_job_t* jobs, int n_jobs, const char* cache_path, void* stream)
{
    if (!ctx || !jobs || n_jobs < 1 || !cache_path) return fail(VDI_E_INVALID, "bad autotune arguments");
    hipStream_t s = (hipStream_t)stream;
    std::map<std::pair<int, int>, std::vector<int>> buckets;
    for (int i = 0; i < n_jobs; ++i) {
        vdi_status st = check_job(jobs[i], i);
        if (st != VDI_OK) return st;
        buckets[{ k_bucket(jobs[i].k), jobs[i].out.max_n }].push_back(i);
    }
    FILE* f = fopen(cache_path, "w");
    if (!f) return fail(VDI_E_INVALID, "cannot write %s", cache_path);
    hipEvent_t e0, e1;
    VDI_HIP_CHECK(hipEventCreate(&e0));
    VDI_HIP_CHECK(hipEventCreate(&e1));
    vdi_status result = VDI_OK;
    for (auto& kv : buckets) {
        std::vector<vdi_job_t> sub;
        for (int i : kv.second) sub.push_back(jobs[i]);
        int best_tile = kDefaultTile;
        float best_ms = 1e30f;
        for (int tile : kCandidates) {
            BatchImpl* b = nullptr;
            vdi_status st = create_impl(ctx, sub.data(), (int)sub.size(), TileMap(), tile, &b);
            if (st != VDI_OK) { result = st; break; }
            float ts[3];
            run_impl(b, nullptr, s);
            for (int rep = 0; rep < 3 && st == VDI_OK; ++rep) {
                hipEventRecord(e0, s);
                st = run_impl(b, nullptr, s);
                hipEventRecord(e1, s);
                hipEventSynchronize(e1);
                hipEventElapsedTime(&ts[rep], e0, e1);
            }
            destroy_impl(b);
            if (st != VDI_OK) { result = st; break; }
            std::sort(ts, ts + 3);
            if (ts[1] < best_ms) {
                best_ms = ts[1];
                best_tile = tile;
            }
        }
        if (result != VDI_OK) break;
        fprintf(f, "%s %d %d %d %.4f\n", ctx->arch, kv.first.first, kv.first.second, best_tile, best_ms);
    }
    fclose(f);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return result;
}

}  // extern "C"
