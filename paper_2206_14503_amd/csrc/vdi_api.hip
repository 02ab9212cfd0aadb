// vdi_api.hip -- the C ABI of libvdi: argument checking, scratch memory and
// kernel launches for generation, compositing and rendering.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

static thread_local char g_err[1024];

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

vdi_status fail(vdi_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

vdi_status launched()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VDI_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return VDI_OK;
}

vdi_status ensure_scratch(vdi_ctx* ctx, size_t bytes)
{
    if (ctx->user_ws) {
        if (bytes > ctx->user_ws_bytes)
            return fail(VDI_E_WORKSPACE, "the call needs %zu bytes of workspace, %zu were set", bytes,
                        ctx->user_ws_bytes);
        return VDI_OK;
    }
    if (bytes <= ctx->scratch_bytes) return VDI_OK;
    // growing the library's own scratch: the old block may still be read by
    // work in flight on any stream
    if (ctx->scratch) {
        VDI_HIP_CHECK(hipDeviceSynchronize());
        VDI_HIP_CHECK(hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t sz = std::max(bytes, (size_t)1 << 20);
    VDI_HIP_CHECK(hipMalloc(&ctx->scratch, sz));
    ctx->scratch_bytes = sz;
    return VDI_OK;
}

char* ws_base(vdi_ctx* ctx) { return (char*)(ctx->user_ws ? ctx->user_ws : ctx->scratch); }

// Scratch of vdi_composite_noalloc: a fixed device array (each device holds
// its own copy until the process ends).  Its name is a host-side stand-in in
// host code; the kernels get the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device at context set-up.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void* g_static_ptr[kMaxDevices];

// Device address of `scratch` on `device` (current); VDI_E_HIP if the lookup fails.
static vdi_status static_scratch_ptr(int device, void** ptr)
{
    if (device < 0 || device >= kMaxDevices) return fail(VDI_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VDI_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_static_ptr[device] = p;
    }
    *ptr = g_static_ptr[device];
    return VDI_OK;
}

static Cam to_cam(const vdi_camera_t* c)
{
    Cam k;
    k.ortho = c->ortho;
    for (int a = 0; a < 3; ++a) {
        k.eye[a] = c->eye[a];
        k.fwd[a] = c->fwd[a];
        k.right[a] = c->right[a];
        k.up[a] = c->up[a];
    }
    k.width = c->width;
    k.height = c->height;
    return k;
}

static vdi_status check_vdi(const vdi_t* v, const char* what, bool allow_compact)
{
    if (!v) return fail(VDI_E_INVALID, "%s is NULL", what);
    if (v->width <= 0 || v->height <= 0) return fail(VDI_E_INVALID, "%s: bad size %dx%d", what, v->width, v->height);
    if ((int64_t)v->width * v->height >= ((int64_t)1 << 31))
        return fail(VDI_E_UNSUPPORTED, "%s: more than 2^31 pixels", what);
    if (v->max_n < 1 || v->max_n > VDI_MAX_N)
        return fail(VDI_E_INVALID, "%s: max_n %d outside [1, %d]", what, v->max_n, VDI_MAX_N);
    if (!(v->ref_step > 0.0f)) return fail(VDI_E_INVALID, "%s: ref_step must be > 0", what);
    if (!v->color || !v->depth || !v->count) return fail(VDI_E_INVALID, "%s: color/depth/count must be set", what);
    if (v->layout == VDI_LAYOUT_COMPACT) {
        if (!allow_compact) return fail(VDI_E_INVALID, "%s must use the regular layout", what);
        if (!v->offset) return fail(VDI_E_INVALID, "%s: compact layout needs offset", what);
        // the kernels address entries with 32-bit offsets
        if (v->capacity >= ((uint64_t)1 << 32))
            return fail(VDI_E_UNSUPPORTED, "%s: compact capacity of 2^32 entries or more", what);
    } else if (v->layout != VDI_LAYOUT_REGULAR) {
        return fail(VDI_E_INVALID, "%s: unknown layout %d", what, v->layout);
    } else if ((uint64_t)v->max_n * (uint64_t)v->width * (uint64_t)v->height >= ((uint64_t)1 << 32)) {
        return fail(VDI_E_UNSUPPORTED, "%s: max_n * width * height of 2^32 entries or more", what);
    }
    return VDI_OK;
}

static vdi_status check_tau(const vdi_tau_t* tau, bool allow_learned)
{
    if (!tau) return fail(VDI_E_INVALID, "tau is NULL");
    if (tau->mode == VDI_TAU_FIXED) {
        if (!(tau->tau >= 0.0f)) return fail(VDI_E_INVALID, "fixed tau must be >= 0");
        return VDI_OK;
    }
    if ((tau->mode == VDI_TAU_LEARNED || tau->mode == VDI_TAU_BISECT_SEQ) && !allow_learned)
        return fail(VDI_E_UNSUPPORTED, "tau mode %d is only available for generation", tau->mode);
    if (tau->mode != VDI_TAU_BISECT && tau->mode != VDI_TAU_LEARNED && tau->mode != VDI_TAU_BISECT_SEQ)
        return fail(VDI_E_INVALID, "unknown tau mode %d", tau->mode);
    if (tau->iters < 1 || tau->iters > 24) return fail(VDI_E_INVALID, "iters %d outside [1, 24]", tau->iters);
    if (!(tau->gamma_max > 1.7320509f)) return fail(VDI_E_INVALID, "gamma_max must exceed sqrt(3)");
    return VDI_OK;
}

static GenBricks make_bricks(const vdi_brick_t* bricks, vdi_t* out, int r0, int nb, int total)
{
    GenBricks B;
    memset(&B, 0, sizeof B);
    B.first = r0;
    B.total = total;
    for (int i = 0; i < nb; ++i) {
        const vdi_brick_t& b = bricks[r0 + i];
        GenBrick& g = B.b[i];
        g.data = b.data;
        g.owner = b.owner;
        g.rank = b.rank;
        if (out) {
            vdi_t& o = out[r0 + i];
            g.color = (float4*)o.color;
            g.depth = (float2*)o.depth;
            g.count = o.count;
            g.gamma = o.gamma;
            g.offset = o.offset;
            g.capacity = o.capacity;
        }
        for (int a = 0; a < 3; ++a) {
            g.lo[a] = b.lo[a];
            g.hi[a] = b.hi[a];
            g.dlo[a] = b.data_lo[a];
            g.ddim[a] = b.data_dim[a];
        }
    }
    return B;
}

__global__ void fill_i32_kernel(int* p, int v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static void fill_i32(int* p, int v, size_t n, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

// Scratch layout of the learned path for nb bricks of npix pixels
// (nblk 256-slot blocks per brick).
struct LearnScratch {
    size_t hist, nnt, cmax, y, ry, span, hlist, hcnt, kind, qcnt, qoff, qlist, scan, total;
};
static LearnScratch learn_layout(size_t rays, int nb, size_t nblk)
{
    LearnScratch L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t a = o; o += (bytes + 255) & ~(size_t)255; return a; };
    const size_t nq = (size_t)nb * nblk;
    L.hist = take(rays * 64 * sizeof(uint16_t));
    L.nnt = take(rays * sizeof(int));
    L.cmax = take(rays * sizeof(int));
    L.y = take(rays * sizeof(float));
    L.ry = take(rays * sizeof(float2));
    L.span = take(rays * sizeof(int2));
    L.hlist = take(rays * sizeof(int));
    L.hcnt = take((size_t)nb * sizeof(int));
    L.kind = take(nq * 256);
    L.qcnt = take(kQueues * nq * sizeof(int));
    L.qoff = take(kQueues * (nq + 1) * sizeof(uint32_t));
    L.qlist = take(kQueues * rays * sizeof(int));
    L.scan = take(scan_scratch_bytes(nq));
    L.total = o;
    return L;
}

// Workspace bytes of vdi_generate: the learned path's buffers; for compact
// outputs a gamma plane per brick of a launch and the prefix-sum partials.
static size_t generate_ws_bytes(int k, int width, int height, bool compact, bool learned)
{
    const size_t npix = (size_t)width * height;
    if (learned) {
        const size_t nblk = (size_t)((width + 15) / 16) * (size_t)((height + 15) / 16);
        return learn_layout(npix * (size_t)k, k, nblk).total;
    }
    if (compact) return npix * sizeof(float) * kGenBricksPerLaunch + scan_scratch_bytes(npix) + 256;
    return 0;
}

// Workspace of vdi_mlp_backward: one partial gradient per block of rows.
static size_t mlp_bwd_ws_bytes(int rows)
{
    const size_t nb = ((size_t)rows + mlp_rows_per_block() - 1) / mlp_rows_per_block();
    return nb * mlp_params() * sizeof(float);
}

// Workspace of vdi_composite: the queue of pixels left to the general merge
// ([npix] + counter), the block order of the depth-disjoint pass (order and
// bucket per block), then the ordered general merge's chunk: staging slabs,
// merge orders and list lengths for up to 1.25 GiB of slabs (the queue is
// processed in as many chunks as it takes).  Merged-list capacities above
// kOrderedMaxCap (and the allocation-free entry point) take the general merge
// with its merge sequence in LDS instead, without staging.
struct CompWs {
    size_t qbytes, obytes, grid, total, buf;
    uint32_t chunk;
    int nbuf;          // ordered-merge buffers: 2 or 3 when the queue can span several chunks
};
static CompWs composite_ws(const vdi_ctx* ctx, size_t npix, int k, int seq_cap, bool staged, size_t limit = 0)
{
    CompWs W;
    const size_t nblk = (npix + 63) / 64;
    const size_t lds = composite_lds_bytes(k, seq_cap);
    const int per_cu = std::max(1, std::min<int>((int)((160 * 1024) / (lds + 64)), 28));
    W.grid = std::max<size_t>(1, std::min<size_t>((size_t)ctx->num_cus * per_cu, nblk));
    // counters and queue; staged: the deferral list (pixel, levels, bracket)
    W.qbytes = (((npix + 64) + (staged ? 2 * npix : 0)) * sizeof(int) + (staged ? npix * sizeof(float2) : 0) + 255) &
               ~(size_t)255;
    W.obytes = (2 * nblk * sizeof(uint32_t) + 255) & ~(size_t)255;
    const uint32_t grid = (uint32_t)ctx->num_cus * kResegBlocksPerCU * 64u;
    W.chunk = staged ? ordered_chunk(seq_cap, kStageBudget, (uint32_t)npix, grid) : 0u;
    W.nbuf = W.chunk == 0 ? 0 : (W.chunk < npix ? std::min<int>(kStageBufs, (int)((npix + W.chunk - 1) / W.chunk)) : 1);
    W.buf = W.chunk ? ordered_ws_bytes(seq_cap, W.chunk) : 0;
    W.total = W.qbytes + W.obytes + W.nbuf * W.buf;
    if (limit && W.chunk && W.total > limit && limit > W.qbytes + W.obytes + 2048) {
        // a smaller caller workspace: the largest chunk two buffers of which
        // fit beside the queues (down to 64 entries; below that the call
        // reports VDI_E_WORKSPACE)
        const size_t per_buf = (limit - W.qbytes - W.obytes) / 2 - 1024;
        const uint32_t c = ordered_chunk(seq_cap, per_buf, (uint32_t)npix, grid);
        if (c >= 64) {
            W.chunk = c;
            W.nbuf = c < npix ? 2 : 1;
            W.buf = ordered_ws_bytes(seq_cap, c);
            W.total = W.qbytes + W.obytes + W.nbuf * W.buf;
        }
    }
    return W;
}

// The ordered merge's buffers at base (ordered_ws_bytes(seq_cap, chunk) bytes).
static void composite_ordered(CompParams& P, char* base, uint32_t chunk)
{
    const size_t c = chunk, cap = P.seq_cap;
    P.chunk = chunk;
    P.stage_c = (float4*)base;
    P.stage_d = (float2*)(base + c * cap * sizeof(float4));
    char* q = base + c * cap * (sizeof(float4) + sizeof(float2));
    P.seq = (uint16_t*)q;
    q += (c * cap * sizeof(uint16_t) + 255) & ~(size_t)255;
    P.qtot = (int*)q;
    q += (c * sizeof(int) + 255) & ~(size_t)255;
    P.ghat = (float*)q;
    q += (c * sizeof(float) + 255) & ~(size_t)255;
    P.feat = P.mlp_wb ? (uint16_t*)q : nullptr;
}

static vdi_status generate_learned(vdi_ctx* ctx, const vdi_brick_t* bricks, int k, const GenParams& P,
                                   const vdi_tau_t* tau, vdi_t* out, int dtype, hipStream_t s)
{
    const size_t npix = (size_t)P.cam.width * P.cam.height;
    const size_t rays = npix * (size_t)k;
    if (rays >= ((size_t)1 << 31)) return fail(VDI_E_UNSUPPORTED, "too many brick-rays for the learned path");
    if (k > kGenBricksPerLaunch)
        return fail(VDI_E_UNSUPPORTED, "the learned path takes at most %d bricks per call", kGenBricksPerLaunch);
    const size_t nblk = (size_t)((P.cam.width + 15) / 16) * (size_t)((P.cam.height + 15) / 16);
    const size_t nq = (size_t)k * nblk;
    LearnScratch Ls = learn_layout(rays, k, nblk);
    vdi_status st = ensure_scratch(ctx, generate_ws_bytes(k, P.cam.width, P.cam.height, false, true));
    if (st != VDI_OK) return st;
    char* base = ws_base(ctx);
    LearnBufs Lb;
    memset(&Lb, 0, sizeof Lb);
    Lb.hist = (uint16_t*)(base + Ls.hist);
    Lb.nnt = (int*)(base + Ls.nnt);
    Lb.cmax = (int*)(base + Ls.cmax);
    Lb.y = (const float*)(base + Ls.y);
    // the generation path keeps each served ray's first-scan bracket and
    // levels (the count at the smallest threshold is for the features only)
    Lb.bracket = (float2*)(base + Ls.ry);
    Lb.level = (int*)(base + Ls.cmax);
    Lb.span = (int2*)(base + Ls.span);
    Lb.hist_list = (int*)(base + Ls.hlist);
    Lb.hist_count = (int*)(base + Ls.hcnt);
    Lb.kind = (uint8_t*)(base + Ls.kind);
    Lb.qcnt = (int*)(base + Ls.qcnt);
    Lb.qoff = (uint32_t*)(base + Ls.qoff);
    Lb.qlist = (int*)(base + Ls.qlist);
    Lb.nblk = (int)nblk;
    Lb.stats = ctx->status + 4;
    Lb.s_ref = tau->feature_scale;
    Lb.blocks_per_brick = std::max(1, ctx->num_cus * 8 / k);
    const vdi_mlp_t* mlp = (const vdi_mlp_t*)tau->mlp;
    if (tau->y) Lb.y = tau->y;
    void* scan_scratch = base + Ls.scan;
    GenBricks B = make_bricks(bricks, out, 0, k, k);
    auto phase = [&](int ph) { launch_learned(ph, dtype, P, B, k, Lb, s); return launched(); };
    // list q in slot order: scan its per-block counts, then place its rays
    auto order = [&](int q) {
        launch_scan(Lb.qcnt + (size_t)q * nq, Lb.qoff + (size_t)q * (nq + 1), nq, scan_scratch, s);
        vdi_status e = launched();
        if (e != VDI_OK) return e;
        launch_compact(q, P, k, Lb, s);
        return launched();
    };
    fill_i32(Lb.hist_count, 0, (size_t)k, s);
    fill_i32(Lb.qcnt, 0, kQueues * nq, s);
    if ((st = phase(0)) != VDI_OK) return st;
    if ((st = order(Q_SERVED)) != VDI_OK) return st;
    if ((st = order(Q_SHORT)) != VDI_OK) return st;
    if (!tau->y) {
        // per brick: the served rays' compacted histograms; y scattered back to pixel order
        for (int r = 0; r < k; ++r) {
            launch_mlp_fwd(mlp->w_bf16, mlp->w_f32, Lb.hist + (size_t)r * npix * 64, (int)npix, Lb.hist_count + r,
                           Lb.hist_list + (size_t)r * npix, ctx->num_cus * 3, (float*)(base + Ls.y) + (size_t)r * npix,
                           nullptr, s);
            if ((st = launched()) != VDI_OK) return st;
        }
    }
    if ((st = phase(1)) != VDI_OK) return st;   // the steered rest of the bisection, and the write
    return phase(4);                            // all-feasible lists
}

// Checks the arguments of a composite and fills its parameter block (all
// but the scratch pointers).
static vdi_status composite_params(vdi_ctx* ctx, const vdi_t* in, int k, const vdi_tau_t* tau, vdi_t* out,
                                   CompParams& P)
{
    if (!ctx || !in || !out) return fail(VDI_E_INVALID, "NULL argument");
    if (k < 1 || k > VDI_MAX_INPUTS) return fail(VDI_E_INVALID, "k=%d outside [1, %d]", k, VDI_MAX_INPUTS);
    if (!tau) return fail(VDI_E_INVALID, "tau is NULL");
    if (tau->mode == VDI_TAU_BISECT_SEQ) return fail(VDI_E_UNSUPPORTED, "BISECT_SEQ is only available for generation");
    vdi_status st = check_tau(tau, tau->mode == VDI_TAU_LEARNED);
    if (st != VDI_OK) return st;
    const vdi_mlp_t* mlp = (const vdi_mlp_t*)tau->mlp;
    if (tau->mode == VDI_TAU_LEARNED && (!mlp || !mlp->w_bf16 || !mlp->w_f32))
        return fail(VDI_E_INVALID, "learned compositing needs tau->mlp");
    if ((st = check_vdi(out, "out", false)) != VDI_OK) return st;
    memset(&P, 0, sizeof P);
    int seq_cap = 0;
    for (int r = 0; r < k; ++r) {
        if ((st = check_vdi(&in[r], "in", true)) != VDI_OK) return st;
        if (in[r].width != out->width || in[r].height != out->height)
            return fail(VDI_E_INVALID, "in[%d] is %dx%d, out %dx%d", r, in[r].width, in[r].height, out->width,
                        out->height);
        if (in[r].ref_step != out->ref_step) return fail(VDI_E_INVALID, "in[%d].ref_step differs from out", r);
        P.in[r].color = (const float4*)in[r].color;
        P.in[r].depth = (const float2*)in[r].depth;
        P.in[r].count = in[r].count;
        P.in[r].offset = in[r].offset;
        P.in[r].max_n = in[r].max_n;
        P.in[r].compact = in[r].layout == VDI_LAYOUT_COMPACT;
        P.in[r].capacity = P.in[r].compact ? in[r].capacity
                                           : (uint64_t)in[r].max_n * (uint64_t)in[r].width * in[r].height;
        seq_cap += in[r].max_n;
    }
    P.k = k;
    P.npix = (uint32_t)((size_t)out->width * out->height);
    P.cache_bound = 0;
    for (int r = 0; r < k; ++r)
        if (in[r].layout == VDI_LAYOUT_COMPACT) P.cache_bound = 1;
    P.inv_ref = 1.0f / out->ref_step;
    P.mode = tau->mode;
    P.tau = tau->tau;
    P.iters = tau->iters;
    P.gmax = tau->gamma_max;
    P.out_n = out->max_n;
    P.out_color = (float4*)out->color;
    P.out_depth = (float2*)out->depth;
    P.out_count = out->count;
    P.out_gamma = out->gamma;
    P.status = ctx->status;
    P.seq_cap = seq_cap;
    P.num_cus = ctx->num_cus;
    P.feat_out = tau->features;
    if (tau->mode == VDI_TAU_LEARNED) {
        P.mode = VDI_TAU_BISECT;
        P.mlp_wb = mlp->w_bf16;
        P.mlp_wf = mlp->w_f32;
    }
    return VDI_OK;
}

// The composite's queue ([64] counter words, then [npix] pixels), with
// `staged` the deferral list after it ([npix] pixels, [npix] levels, [npix]
// brackets; its counter the second word), and the block order ([nblk]
// order, [nblk] bucket) at base; qbytes as composite_ws gives.
static void composite_queues(CompParams& P, char* base, size_t qbytes, bool staged)
{
    P.q_count = (int*)base;
    P.q_list = (int*)base + 64;
    if (staged) {
        P.dq_count = (int*)base + 1;
        P.dq_pix = P.q_list + P.npix;
        P.dq_lv = P.dq_pix + P.npix;
        P.dq_br = (float2*)(P.dq_lv + P.npix);
    }
    // slot-major inputs only: a block of compact inputs reads one stretch of
    // each input, next to its neighbours' stretches, and loses that locality
    // out of image order (measured slower)
    P.order = P.cache_bound ? nullptr : (uint32_t*)(base + qbytes);
    P.bucket = (uint32_t*)(base + qbytes) + composite_blocks(P);
}

}  // namespace vdi

using namespace vdi;

extern "C" {

const char* vdi_last_error(void) { return g_err; }

vdi_status vdi_ctx_create(vdi_ctx** out, int device)
{
    if (!out) return fail(VDI_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    VDI_HIP_CHECK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(VDI_E_INVALID, "device %d of %d", device, n);
    VDI_HIP_CHECK(hipSetDevice(device));
    hipDeviceProp_t prop;
    VDI_HIP_CHECK(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(VDI_E_UNSUPPORTED, "libvdi is built for gfx950, device is %s", prop.gcnArchName);
    void* sptr = nullptr;
    vdi_status sst = static_scratch_ptr(device, &sptr);
    if (sst != VDI_OK) return sst;
    vdi_ctx* c = new vdi_ctx();
    c->device = device;
    c->static_scratch = sptr;
    c->aux = nullptr;
    for (int i = 0; i < 7; ++i) c->ev[i] = nullptr;
    hipError_t es = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    for (int i = 0; i < 7 && es == hipSuccess; ++i) es = hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming);
    if (es != hipSuccess) {
        for (int i = 0; i < 7; ++i)
            if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        delete c;
        return fail(VDI_E_HIP, "stream/event creation failed: %s", hipGetErrorString(es));
    }
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    c->user_ws = nullptr;
    c->user_ws_bytes = 0;
    c->num_cus = prop.multiProcessorCount;
    snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    hipError_t e = hipMalloc(&c->status, 64);
    if (e == hipSuccess) e = hipMemset(c->status, 0, 64);
    if (e != hipSuccess) {
        for (int i = 0; i < 7; ++i) (void)hipEventDestroy(c->ev[i]);
        (void)hipStreamDestroy(c->aux);
        delete c;
        return fail(VDI_E_HIP, "status allocation failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return VDI_OK;
}

vdi_status vdi_ctx_destroy(vdi_ctx* ctx)
{
    if (!ctx) return VDI_OK;
    // teardown: errors are not reported (the context is gone either way)
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->status) (void)hipFree(ctx->status);
    for (int i = 0; i < 7; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    delete ctx;
    return VDI_OK;
}

vdi_status vdi_workspace_size(vdi_ctx* ctx, const vdi_shape_t* shape, size_t* bytes)
{
    if (!ctx || !shape || !bytes) return fail(VDI_E_INVALID, "NULL argument");
    *bytes = 0;
    switch (shape->op) {
    case VDI_OP_GENERATE: {
        if (shape->width <= 0 || shape->height <= 0 || shape->k < 1) return fail(VDI_E_INVALID, "bad width/height/k");
        const bool learned = shape->tau_mode == VDI_TAU_LEARNED;
        const bool compact = shape->layout == VDI_LAYOUT_COMPACT;
        if (learned && compact) return fail(VDI_E_UNSUPPORTED, "learned thresholds need the regular layout");
        *bytes = generate_ws_bytes(shape->k, shape->width, shape->height, compact, learned);
        return VDI_OK;
    }
    case VDI_OP_COMPOSITE: {
        if (shape->width <= 0 || shape->height <= 0 || shape->k < 1 || shape->k > VDI_MAX_INPUTS)
            return fail(VDI_E_INVALID, "bad width/height/k");
        if (shape->in_max_n_sum < shape->k || shape->in_max_n_sum > shape->k * VDI_MAX_N)
            return fail(VDI_E_INVALID, "in_max_n_sum %d outside [k, k*%d]", shape->in_max_n_sum, VDI_MAX_N);
        if (composite_lds_bytes(shape->k, shape->in_max_n_sum) > 160 * 1024)
            return fail(VDI_E_UNSUPPORTED, "merged list capacity %d too large", shape->in_max_n_sum);
        *bytes = composite_ws(ctx, (size_t)shape->width * shape->height, shape->k, shape->in_max_n_sum, true).total;
        return VDI_OK;
    }
    case VDI_OP_MLP_BACKWARD:
        if (shape->rows <= 0) return fail(VDI_E_INVALID, "rows must be > 0");
        *bytes = mlp_bwd_ws_bytes(shape->rows);
        return VDI_OK;
    default:
        return fail(VDI_E_INVALID, "unknown op %d", shape->op);
    }
}

vdi_status vdi_ctx_set_workspace(vdi_ctx* ctx, void* workspace, size_t bytes)
{
    if (!ctx) return fail(VDI_E_INVALID, "ctx is NULL");
    if (workspace && ((uintptr_t)workspace & 255) != 0) return fail(VDI_E_INVALID, "workspace must be 256-byte aligned");
    VDI_HIP_CHECK(hipSetDevice(ctx->device));
    VDI_HIP_CHECK(hipDeviceSynchronize());
    if (workspace && ctx->scratch) {
        VDI_HIP_CHECK(hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    ctx->user_ws = workspace;
    ctx->user_ws_bytes = workspace ? bytes : 0;
    return VDI_OK;
}

vdi_status vdi_ctx_reserve_workspace(vdi_ctx* ctx, size_t bytes)
{
    if (!ctx) return fail(VDI_E_INVALID, "ctx is NULL");
    if (ctx->user_ws) return fail(VDI_E_INVALID, "the context uses a caller workspace");
    VDI_HIP_CHECK(hipSetDevice(ctx->device));
    return ensure_scratch(ctx, bytes);
}

vdi_status vdi_ctx_device_status(vdi_ctx* ctx, int32_t* flags, void* stream)
{
    if (!ctx || !flags) return fail(VDI_E_INVALID, "ctx/flags is NULL");
    hipStream_t s = (hipStream_t)stream;
    VDI_HIP_CHECK(hipStreamSynchronize(s));
    int32_t v = 0;
    VDI_HIP_CHECK(hipMemcpy(&v, ctx->status, sizeof v, hipMemcpyDeviceToHost));
    VDI_HIP_CHECK(hipMemset(ctx->status, 0, sizeof v));
    *flags = v;
    return VDI_OK;
}

vdi_status vdi_generate(vdi_ctx* ctx, const vdi_brick_t* bricks, int k, const vdi_camera_t* cam,
                        const vdi_tf_t* tf, float step, const vdi_tau_t* tau, vdi_t* out, void* stream)
{
    if (!ctx || !bricks || !cam || !tf || !out) return fail(VDI_E_INVALID, "NULL argument");
    if (k < 1) return fail(VDI_E_INVALID, "k must be >= 1");
    if (cam->width <= 0 || cam->height <= 0) return fail(VDI_E_INVALID, "camera size");
    if (!tf->rgba || tf->entries < 2 || tf->entries > VDI_MAX_TF)
        return fail(VDI_E_INVALID, "transfer function needs 2..%d entries", VDI_MAX_TF);
    if (!(step > 0.0f)) return fail(VDI_E_INVALID, "step must be > 0");
    vdi_status st = check_tau(tau, true);
    if (st != VDI_OK) return st;
    if (tau->mode == VDI_TAU_LEARNED) {
        const vdi_mlp_t* mlp = (const vdi_mlp_t*)tau->mlp;
        if (!tau->y && (!mlp || !mlp->w_bf16 || !mlp->w_f32))
            return fail(VDI_E_INVALID, "learned mode needs tau->mlp or tau->y");
        if (!(tau->feature_scale > 0.0f)) return fail(VDI_E_INVALID, "learned mode needs feature_scale > 0");
        if (!(1.7320508f / step < 65535.0f))
            return fail(VDI_E_UNSUPPORTED, "step too small for the learned path (histogram bins count to 65535)");
    }
    const int dtype = bricks[0].dtype;
    if (dtype != VDI_F32 && dtype != VDI_F16) return fail(VDI_E_INVALID, "brick dtype %d", dtype);
    for (int r = 0; r < k; ++r) {
        const vdi_brick_t& b = bricks[r];
        if (!b.data) return fail(VDI_E_INVALID, "brick %d: data is NULL", r);
        if (b.dtype != dtype) return fail(VDI_E_INVALID, "bricks must share one dtype");
        if (b.owner && (b.rank < 0 || b.rank > 255)) return fail(VDI_E_INVALID, "brick %d: rank must be 0..255", r);
        if (b.owner && tau->mode != VDI_TAU_BISECT && tau->mode != VDI_TAU_BISECT_SEQ)
            return fail(VDI_E_UNSUPPORTED, "brick %d: owner maps need a bisection threshold mode", r);
        for (int a = 0; a < 3; ++a) {
            if (b.full_dim[a] != bricks[0].full_dim[a] || b.full_dim[a] < 1)
                return fail(VDI_E_INVALID, "brick %d: full_dim mismatch", r);
            int n = b.full_dim[a];
            if (b.lo[a] < 0 || b.hi[a] > n || b.lo[a] >= b.hi[a])
                return fail(VDI_E_INVALID, "brick %d: owned box axis %d is [%d,%d) of %d", r, a, b.lo[a], b.hi[a], n);
            int need_lo = std::max(b.lo[a] - 1, 0), need_hi = std::min(b.hi[a] + 1, n);
            if (b.data_lo[a] > need_lo || b.data_lo[a] + b.data_dim[a] < need_hi || b.data_dim[a] < 1)
                return fail(VDI_E_INVALID, "brick %d: data box axis %d does not cover the owned box plus one voxel", r, a);
        }
        if ((int64_t)b.data_dim[0] * b.data_dim[1] * b.data_dim[2] * (b.dtype == VDI_F16 ? 2 : 4) >=
            ((int64_t)1 << 32))
            return fail(VDI_E_UNSUPPORTED, "brick %d: data box of 4 GiB or more; split the volume into more bricks", r);
        st = check_vdi(&out[r], "out", true);
        if (st != VDI_OK) return st;
        if (out[r].width != cam->width || out[r].height != cam->height)
            return fail(VDI_E_INVALID, "out[%d] is %dx%d, camera %dx%d", r, out[r].width, out[r].height, cam->width,
                        cam->height);
        if (out[r].ref_step != out[0].ref_step) return fail(VDI_E_INVALID, "outputs must share ref_step");
        if (out[r].layout != out[0].layout) return fail(VDI_E_INVALID, "outputs must share one layout");
        if (out[r].max_n != out[0].max_n) return fail(VDI_E_INVALID, "outputs must share max_n");
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t npix = (size_t)cam->width * cam->height;
    const bool compact = out[0].layout == VDI_LAYOUT_COMPACT;
    const bool learned = tau->mode == VDI_TAU_LEARNED;
    if (learned && compact) return fail(VDI_E_UNSUPPORTED, "learned thresholds need the regular layout");

    GenParams P;
    memset(&P, 0, sizeof P);
    P.cam = to_cam(cam);
    for (int a = 0; a < 3; ++a) P.n[a] = bricks[0].full_dim[a];
    P.step = step;
    P.l_step = step / out[0].ref_step;
    P.mode = tau->mode;
    P.tau = tau->tau;
    P.iters = tau->iters;
    P.gmax = tau->gamma_max;
    P.max_n = out[0].max_n;
    P.tf_entries = tf->entries;
    P.tf = (const float4*)tf->rgba;
    P.status = ctx->status;

    // compact outputs without a gamma plane borrow scratch for it
    size_t gamma_bytes = 0;
    if (compact) {
        gamma_bytes = npix * sizeof(float) * kGenBricksPerLaunch;
        st = ensure_scratch(ctx, generate_ws_bytes(k, cam->width, cam->height, true, false));
        if (st != VDI_OK) return st;
    }
    if (learned) return generate_learned(ctx, bricks, k, P, tau, out, dtype, s);
    for (int r0 = 0; r0 < k; r0 += kGenBricksPerLaunch) {
        int nb = std::min(k - r0, kGenBricksPerLaunch);
        GenBricks B;
        memset(&B, 0, sizeof B);
        B.first = r0;
        B.total = k;
        for (int i = 0; i < nb; ++i) {
            const vdi_brick_t& b = bricks[r0 + i];
            vdi_t& o = out[r0 + i];
            GenBrick& g = B.b[i];
            g.data = b.data;
            g.owner = b.owner;
            g.rank = b.rank;
            g.color = (float4*)o.color;
            g.depth = (float2*)o.depth;
            g.count = o.count;
            g.gamma = o.gamma;
            if (compact && !g.gamma) g.gamma = (float*)ws_base(ctx) + (size_t)i * npix;
            g.offset = o.offset;
            g.capacity = o.capacity;
            for (int a = 0; a < 3; ++a) {
                g.lo[a] = b.lo[a];
                g.hi[a] = b.hi[a];
                g.dlo[a] = b.data_lo[a];
                g.ddim[a] = b.data_dim[a];
            }
        }
        if (!compact) {
            launch_generate(0, dtype, P, B, nb, s);
            if ((st = launched()) != VDI_OK) return st;
            continue;
        }
        // compact (Sec. 4): search -> prefix sum of counts -> write at offsets
        launch_generate(1, dtype, P, B, nb, s);
        if ((st = launched()) != VDI_OK) return st;
        void* scan_scratch = ws_base(ctx) + gamma_bytes;
        for (int i = 0; i < nb; ++i) {
            launch_scan(out[r0 + i].count, out[r0 + i].offset, npix, scan_scratch, s);
            if ((st = launched()) != VDI_OK) return st;
        }
        launch_generate(2, dtype, P, B, nb, s);
        if ((st = launched()) != VDI_OK) return st;
    }
    return VDI_OK;
}

vdi_status vdi_composite(vdi_ctx* ctx, const vdi_t* in, int k, const vdi_tau_t* tau, vdi_t* out, void* stream)
{
    CompParams P;
    vdi_status st = composite_params(ctx, in, k, tau, out, P);
    if (st != VDI_OK) return st;
    if (composite_lds_bytes(k, P.seq_cap) > 160 * 1024)
        return fail(VDI_E_UNSUPPORTED, "merged list capacity %d too large", P.seq_cap);
    const CompWs W = composite_ws(ctx, P.npix, k, P.seq_cap, true, ctx->user_ws ? ctx->user_ws_bytes : 0);
    if ((st = ensure_scratch(ctx, W.total)) != VDI_OK) return st;
    char* base = ws_base(ctx);
    composite_queues(P, base, W.qbytes, W.chunk != 0);
    // the ordered merge's buffers after the queue and the block order
    char* obase = base + W.qbytes + W.obytes;
    if (W.chunk) composite_ordered(P, obase, W.chunk);
    if (W.nbuf >= 2) {
        CompParams Pb[kStageBufs];
        OrderedSync sync;
        sync.aux = ctx->aux;
        for (int i = 0; i < 7; ++i) sync.ev[i] = ctx->ev[i];
        sync.nbuf = W.nbuf;
        sync.B[0] = &P;
        for (int b = 1; b < W.nbuf; ++b) {
            Pb[b] = P;
            composite_ordered(Pb[b], obase + b * W.buf, W.chunk);
            sync.B[b] = &Pb[b];
        }
        launch_composite(P, (int)W.grid, (hipStream_t)stream, &sync);
    } else {
        launch_composite(P, (int)W.grid, (hipStream_t)stream);
    }
    return launched();
}

vdi_status vdi_composite_noalloc(vdi_ctx* ctx, const vdi_t* in, int k, const vdi_tau_t* tau, vdi_t* out,
                                 void* stream)
{
    CompParams P;
    vdi_status st = composite_params(ctx, in, k, tau, out, P);
    if (st != VDI_OK) return st;
    // no staging slabs: the general merge keeps its merge sequence in LDS
    if (composite_lds_bytes(k, P.seq_cap) > 160 * 1024)
        return fail(VDI_E_UNSUPPORTED, "merged list capacity %d too large for the merge sequence in LDS", P.seq_cap);
    const CompWs W = composite_ws(ctx, P.npix, k, P.seq_cap, false);
    const size_t need = W.qbytes + W.obytes;
    if (need > kStaticScratchBytes)
        return fail(VDI_E_UNSUPPORTED, "%u pixels need %zu bytes of scratch, more than the fixed %zu", P.npix, need,
                    kStaticScratchBytes);
    composite_queues(P, (char*)ctx->static_scratch, W.qbytes, false);
    launch_composite(P, (int)W.grid, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_render_original_view(vdi_ctx* ctx, const vdi_t* v, float* rgba, void* stream)
{
    if (!ctx || !rgba) return fail(VDI_E_INVALID, "NULL argument");
    vdi_status st = check_vdi(v, "vdi", true);
    if (st != VDI_OK) return st;
    uint32_t npix = (uint32_t)((size_t)v->width * v->height);
    const bool compact = v->layout == VDI_LAYOUT_COMPACT;
    uint64_t cap = compact ? v->capacity : (uint64_t)v->max_n * npix;
    launch_render((const float4*)v->color, (const float2*)v->depth, v->count, compact ? v->offset : nullptr, cap,
                  v->max_n, npix, 1.0f / v->ref_step, (float4*)rgba, ctx->status, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_render_novel_view(vdi_ctx* ctx, const vdi_t* v, const vdi_camera_t* vdi_cam, const vdi_camera_t* view,
                                 float step, float* rgba, void* stream)
{
    if (!ctx || !vdi_cam || !view || !rgba) return fail(VDI_E_INVALID, "NULL argument");
    vdi_status st = check_vdi(v, "vdi", true);
    if (st != VDI_OK) return st;
    if (vdi_cam->width != v->width || vdi_cam->height != v->height)
        return fail(VDI_E_INVALID, "vdi_cam is %dx%d, the VDI %dx%d", vdi_cam->width, vdi_cam->height, v->width,
                    v->height);
    if (view->width <= 0 || view->height <= 0) return fail(VDI_E_INVALID, "bad view size");
    if (!(step > 0.0f)) return fail(VDI_E_INVALID, "step must be > 0");
    if (!(1.7320508f / step < 16777216.0f)) return fail(VDI_E_UNSUPPORTED, "step too small");
    NovelParams N;
    N.view = to_cam(view);
    N.vcam = to_cam(vdi_cam);
    N.color = (const float4*)v->color;
    N.depth = (const float2*)v->depth;
    N.count = v->count;
    const bool compact = v->layout == VDI_LAYOUT_COMPACT;
    N.offset = compact ? v->offset : nullptr;
    N.npix = (uint32_t)((size_t)v->width * v->height);
    N.capacity = compact ? v->capacity : (uint64_t)v->max_n * N.npix;
    N.max_n = v->max_n;
    N.step = step;
    N.l = step / v->ref_step;
    N.rgba = (float4*)rgba;
    N.status = ctx->status;
    launch_novel(N, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_debug_rays(vdi_ctx* ctx, const vdi_camera_t* cam, float step, float* o, float* d, float* tn,
                          float* tf, int32_t* nsamples, void* stream)
{
    if (!ctx || !cam || !o || !d || !tn || !tf || !nsamples) return fail(VDI_E_INVALID, "NULL argument");
    if (cam->width <= 0 || cam->height <= 0 || !(step > 0.0f)) return fail(VDI_E_INVALID, "bad camera or step");
    launch_rays(to_cam(cam), step, o, d, tn, tf, nsamples, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_tau_features(vdi_ctx* ctx, const vdi_brick_t* bricks, int k, const vdi_camera_t* cam,
                            const vdi_tf_t* tf, float step, float ref_step, int max_n, const vdi_tau_t* tau,
                            uint16_t* hist, int32_t* nnt, int32_t* cmax, void* stream)
{
    if (!ctx || !bricks || !cam || !tf || !tau || !hist || !nnt || !cmax) return fail(VDI_E_INVALID, "NULL argument");
    if (k < 1 || cam->width <= 0 || cam->height <= 0) return fail(VDI_E_INVALID, "bad k or camera");
    if (!tf->rgba || tf->entries < 2 || tf->entries > VDI_MAX_TF) return fail(VDI_E_INVALID, "transfer function");
    if (!(step > 0.0f) || !(ref_step > 0.0f)) return fail(VDI_E_INVALID, "step and ref_step must be > 0");
    if (!(1.7320508f / step < 65535.0f))
        return fail(VDI_E_UNSUPPORTED, "step too small for the histogram (bins count to 65535)");
    if (max_n < 1 || max_n > VDI_MAX_N) return fail(VDI_E_INVALID, "max_n");
    if (tau->iters < 1 || tau->iters > 24 || !(tau->gamma_max > 1.7320509f) || !(tau->feature_scale > 0.0f))
        return fail(VDI_E_INVALID, "tau: iters, gamma_max or feature_scale");
    const int dtype = bricks[0].dtype;
    for (int r = 0; r < k; ++r) {
        const vdi_brick_t& b = bricks[r];
        if (!b.data || b.dtype != dtype) return fail(VDI_E_INVALID, "brick %d: data/dtype", r);
        if (b.owner) return fail(VDI_E_UNSUPPORTED, "brick %d: owner maps are not supported by the learned path", r);
        for (int a = 0; a < 3; ++a) {
            int n = b.full_dim[a];
            if (n != bricks[0].full_dim[a] || b.lo[a] < 0 || b.hi[a] > n || b.lo[a] >= b.hi[a])
                return fail(VDI_E_INVALID, "brick %d: owned box", r);
            int need_lo = std::max(b.lo[a] - 1, 0), need_hi = std::min(b.hi[a] + 1, n);
            if (b.data_lo[a] > need_lo || b.data_lo[a] + b.data_dim[a] < need_hi)
                return fail(VDI_E_INVALID, "brick %d: data box", r);
        }
        if ((int64_t)b.data_dim[0] * b.data_dim[1] * b.data_dim[2] * (b.dtype == VDI_F16 ? 2 : 4) >=
            ((int64_t)1 << 32))
            return fail(VDI_E_UNSUPPORTED, "brick %d: data box of 4 GiB or more; split the volume into more bricks", r);
    }
    GenParams P;
    memset(&P, 0, sizeof P);
    P.cam = to_cam(cam);
    for (int a = 0; a < 3; ++a) P.n[a] = bricks[0].full_dim[a];
    P.step = step;
    P.l_step = step / ref_step;
    P.mode = VDI_TAU_BISECT;
    P.iters = tau->iters;
    P.gmax = tau->gamma_max;
    P.max_n = max_n;
    P.tf_entries = tf->entries;
    P.tf = (const float4*)tf->rgba;
    P.status = ctx->status;
    LearnBufs Lb;
    memset(&Lb, 0, sizeof Lb);
    Lb.hist = hist;
    Lb.nnt = nnt;
    Lb.cmax = cmax;
    Lb.s_ref = tau->feature_scale;
    hipStream_t s = (hipStream_t)stream;
    for (int r0 = 0; r0 < k; r0 += kGenBricksPerLaunch) {
        int nb = std::min(k - r0, kGenBricksPerLaunch);
        GenBricks B = make_bricks(bricks, nullptr, r0, nb, k);
        launch_learned(0, dtype, P, B, nb, Lb, s);
        vdi_status st = launched();
        if (st != VDI_OK) return st;
    }
    return VDI_OK;
}

static vdi_status check_mlp(const vdi_mlp_t* mlp)
{
    if (!mlp || !mlp->w_bf16 || !mlp->w_f32) return fail(VDI_E_INVALID, "mlp weights are NULL");
    if (((uintptr_t)mlp->w_bf16 & 15) != 0) return fail(VDI_E_INVALID, "mlp->w_bf16 must be 16-byte aligned");
    return VDI_OK;
}

vdi_status vdi_mlp_forward(vdi_ctx* ctx, const vdi_mlp_t* mlp, const uint16_t* x, int rows, float* y, float* acts,
                           void* stream)
{
    if (!ctx || !x || !y) return fail(VDI_E_INVALID, "NULL argument");
    vdi_status st = check_mlp(mlp);
    if (st != VDI_OK) return st;
    if (rows < 0) return fail(VDI_E_INVALID, "rows < 0");
    if (((uintptr_t)x & 7) != 0) return fail(VDI_E_INVALID, "x must be 8-byte aligned");
    if (rows == 0) return VDI_OK;
    launch_mlp_fwd(mlp->w_bf16, mlp->w_f32, x, rows, nullptr, nullptr, ctx->num_cus * 3, y, acts, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_mlp_backward(vdi_ctx* ctx, const vdi_mlp_t* mlp, const uint16_t* x, const float* acts,
                            const float* dy, int rows, float* grad, void* stream)
{
    if (!ctx || !x || !acts || !dy || !grad) return fail(VDI_E_INVALID, "NULL argument");
    vdi_status st = check_mlp(mlp);
    if (st != VDI_OK) return st;
    if (rows <= 0) return fail(VDI_E_INVALID, "rows must be > 0");
    st = ensure_scratch(ctx, mlp_bwd_ws_bytes(rows));
    if (st != VDI_OK) return st;
    launch_mlp_bwd(mlp->w_bf16, x, acts, dy, rows, (float*)ws_base(ctx), grad, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_mlp_adam(vdi_ctx* ctx, vdi_mlp_t* mlp, const float* grad, float* m, float* v, int step, float lr,
                        float beta1, float beta2, float eps, void* stream)
{
    if (!ctx || !grad || !m || !v) return fail(VDI_E_INVALID, "NULL argument");
    vdi_status st = check_mlp(mlp);
    if (st != VDI_OK) return st;
    if (step < 1) return fail(VDI_E_INVALID, "step must be >= 1");
    launch_mlp_adam(mlp->w_f32, mlp->w_bf16, grad, m, v, lr, beta1, beta2, eps, step, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_mlp_mse(vdi_ctx* ctx, const float* y, const float* gamma, int rows, float scale, float* dy,
                       double* loss_part, void* stream)
{
    if (!ctx || !y || !gamma || !dy) return fail(VDI_E_INVALID, "NULL argument");
    if (rows <= 0) return fail(VDI_E_INVALID, "rows must be > 0");
    launch_mlp_mse(y, gamma, rows, scale, dy, loss_part, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_mlp_pack(vdi_ctx* ctx, vdi_mlp_t* mlp, void* stream)
{
    if (!ctx) return fail(VDI_E_INVALID, "NULL argument");
    vdi_status st = check_mlp(mlp);
    if (st != VDI_OK) return st;
    launch_mlp_pack(mlp->w_f32, mlp->w_bf16, (hipStream_t)stream);
    return launched();
}

vdi_status vdi_learned_stats(vdi_ctx* ctx, int64_t* stats, void* stream)
{
    if (!ctx || !stats) return fail(VDI_E_INVALID, "NULL argument");
    VDI_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    int32_t v[kLearnStats];
    VDI_HIP_CHECK(hipMemcpy(v, ctx->status + 4, sizeof v, hipMemcpyDeviceToHost));
    VDI_HIP_CHECK(hipMemset(ctx->status + 4, 0, sizeof v));
    for (int i = 0; i < kLearnStats; ++i) stats[i] = v[i];
    return VDI_OK;
}

vdi_status vdi_debug_mfma(vdi_ctx* ctx, const uint16_t* A, const uint16_t* B, float* D, void* stream)
{
    if (!ctx || !A || !B || !D) return fail(VDI_E_INVALID, "NULL argument");
    launch_mfma_probe(A, B, D, (hipStream_t)stream);
    return launched();
}

}  // extern "C"
