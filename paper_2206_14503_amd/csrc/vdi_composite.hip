// vdi_composite.hip -- per-pixel k-way depth merge and re-segmentation of
// sub-VDIs (Sec. 5.2, supplementary Algorithm S1).
//
// One lane per pixel, one wavefront per block.  The lane first merges the k
// front-to-back sorted input lists by front depth (ties: lower input index)
// into a merge sequence of (input, slot) pairs kept in LDS; every later pass
// (the threshold bisection and the final write) replays that sequence and
// reads the supersegments straight from the inputs, so the inputs are read
// from HBM once and re-read from cache.
#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

namespace {

constexpr int kWave = 64;

struct CSeg {
    float c0, c1, c2;  // premultiplied colour
    float A;           // accumulated opacity
    float T;           // transmittance
    float f, b, bt;    // front, back (incl. trailing gap/transparent), back of last non-transparent
    int open;
};

struct COut {
    float4* color;
    float2* depth;
    uint32_t pix, npix;
    int limit;
};

template <bool WRITE>
__device__ inline void c_close(CSeg& S, int& count, const COut& o, float inv_ref)
{
    if (WRITE && count < o.limit) {
        float invA = 1.0f / S.A;
        float len = (S.bt - S.f) * inv_ref;
        float a = -expm1f(logf(S.T) / len);
        size_t slot = (size_t)count * o.npix + o.pix;
        o.color[slot] = make_float4(S.c0 * invA, S.c1 * invA, S.c2 * invA, a);
        o.depth[slot] = make_float2(S.f, S.bt);
    }
    ++count;
    S.open = 0;
}

// Eq. 1 test of the open supersegment against an element with per-unit
// premultiplied colour (e0, e1, e2).
__device__ inline float c_dist2(const CSeg& S, float inv_ref, float e0, float e1, float e2)
{
    float L = (S.b - S.f) * inv_ref;
    float aS = -expm1f(logf(S.T) / L);
    float sc = aS / S.A;
    float d0 = S.c0 * sc - e0, d1 = S.c1 * sc - e1, d2 = S.c2 * sc - e2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

template <bool WRITE>
__device__ inline void c_step(CSeg& S, int& count, const COut& o, float inv_ref, float g2, int cap, float fe,
                              float be, float4 c)
{
    // empty space before the element is a transparent sample (Alg. S1)
    if (S.open && fe > S.b) {
        bool may_close = cap <= 0 || count < cap - 1;
        if (may_close && g2 < c_dist2(S, inv_ref, 0.0f, 0.0f, 0.0f)) c_close<WRITE>(S, count, o, inv_ref);
        else S.b = fe;
    }
    const bool transparent = (c.w == 0.0f);
    float l = (be - fe) * inv_ref;
    float lg = l * log1pf(-c.w);
    float Te = expf(lg);          // Eq. 2: 1 - alpha~ = (1 - a)^l
    float at = -expm1f(lg);
    if (S.open) {
        bool may_close = cap <= 0 || count < cap - 1;
        if (may_close && g2 < c_dist2(S, inv_ref, c.x * c.w, c.y * c.w, c.z * c.w)) {
            c_close<WRITE>(S, count, o, inv_ref);
        } else {
            float w = S.T * at;
            S.c0 = fmaf(w, c.x, S.c0);
            S.c1 = fmaf(w, c.y, S.c1);
            S.c2 = fmaf(w, c.z, S.c2);
            S.A += w;
            S.T *= Te;
            S.b = be;
            if (!transparent) S.bt = be;
        }
    }
    if (!S.open && !transparent) {
        S.open = 1;
        S.f = fe;
        S.b = S.bt = be;
        S.c0 = c.x * at;
        S.c1 = c.y * at;
        S.c2 = c.z * at;
        S.A = at;
        S.T = Te;
    }
}

struct Lds {
    uint16_t* seq;     // [seq_cap][64]: input << 8 | slot
    float* front;      // [k][64]
    uint32_t* ebase;   // [k][64]: element index of slot 0
    uint16_t* cur;     // [k][64]
    uint16_t* cnt;     // [k][64]
};

__device__ inline uint32_t elem_index(const CompParams& P, const Lds& L, int r, int s, int t)
{
    uint32_t stride = P.in[r].compact ? 1u : P.npix;
    return L.ebase[r * kWave + t] + (uint32_t)s * stride;
}

template <bool WRITE>
__device__ int c_pass(const CompParams& P, const Lds& L, int t, int total, float gamma, int cap, int limit,
                      const COut& o)
{
    const float g2 = gamma * gamma;
    CSeg S;
    S.open = 0;
    S.c0 = S.c1 = S.c2 = S.A = 0.0f;
    S.T = 1.0f;
    S.f = S.b = S.bt = 0.0f;
    int count = 0;
    for (int i = 0; i < total; ++i) {
        uint32_t rs = L.seq[i * kWave + t];
        int r = (int)(rs >> 8), s = (int)(rs & 255u);
        uint32_t e = elem_index(P, L, r, s, t);
        float4 c = P.in[r].color[e];
        float2 fb = P.in[r].depth[e];
        c_step<WRITE>(S, count, o, P.inv_ref, g2, cap, fb.x, fb.y, c);
        if (!WRITE && count > limit) return count;
    }
    if (S.open) c_close<WRITE>(S, count, o, P.inv_ref);
    return count;
}

}  // namespace

__global__ __launch_bounds__(64) void composite_kernel(CompParams P)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int t = threadIdx.x;
    Lds L;
    L.seq = (uint16_t*)lds_raw;
    L.front = (float*)(lds_raw + (size_t)2 * kWave * P.seq_cap);
    L.ebase = (uint32_t*)(L.front + kWave * P.k);
    L.cur = (uint16_t*)(L.ebase + kWave * P.k);
    L.cnt = L.cur + kWave * P.k;

    const uint32_t p = blockIdx.x * kWave + t;
    if (p >= P.npix) return;

    // ---- load counts, validate, set up the merge cursors
    int total = 0;
    bool bad = false;
    for (int r = 0; r < P.k; ++r) {
        const CompInput& in = P.in[r];
        int c = in.count[p];
        if (c < 0 || c > in.max_n) { bad = true; c = 0; }
        uint32_t eb = in.compact ? in.offset[p] : p;
        uint64_t last = in.compact ? (uint64_t)eb + (uint64_t)c : (uint64_t)c * P.npix;
        if (last > in.capacity) { bad = true; c = 0; }
        L.ebase[r * kWave + t] = eb;
        L.cur[r * kWave + t] = 0;
        L.cnt[r * kWave + t] = (uint16_t)c;
        float f = __builtin_inff();
        if (c > 0) {
            float2 fb = in.depth[eb];
            if (!(fb.x < fb.y) || !isfinite(fb.x) || !isfinite(fb.y)) bad = true;
            f = fb.x;
        }
        L.front[r * kWave + t] = f;
        total += c;
    }

    // ---- k-way merge by (front depth, input index)
    for (int i = 0; i < total && !bad; ++i) {
        float best = __builtin_inff();
        int rb = -1;
        for (int r = 0; r < P.k; ++r) {
            float f = L.front[r * kWave + t];
            if (f < best) { best = f; rb = r; }
        }
        if (rb < 0) { bad = true; break; }
        int s = L.cur[rb * kWave + t];
        L.seq[i * kWave + t] = (uint16_t)((rb << 8) | s);
        ++s;
        L.cur[rb * kWave + t] = (uint16_t)s;
        float nf = __builtin_inff();
        if (s < L.cnt[rb * kWave + t]) {
            float2 fb = P.in[rb].depth[elem_index(P, L, rb, s, t)];
            if (!(fb.x < fb.y) || !(fb.x >= best) || !isfinite(fb.y)) bad = true;
            nf = fb.x;
        }
        L.front[rb * kWave + t] = nf;
    }
    if (bad) {
        atomicOr(P.status, 2);
        total = 0;
    }

    COut o{P.out_color, P.out_depth, p, P.npix, P.out_n};
    int count;
    float gm = 0.0f;
    if (total <= P.out_n) {
        // pass-through: the merged list already fits
        for (int i = 0; i < total; ++i) {
            uint32_t rs = L.seq[i * kWave + t];
            int r = (int)(rs >> 8), s = (int)(rs & 255u);
            uint32_t e = elem_index(P, L, r, s, t);
            size_t slot = (size_t)i * P.npix + p;
            P.out_color[slot] = P.in[r].color[e];
            P.out_depth[slot] = P.in[r].depth[e];
        }
        count = total;
    } else if (P.mode == VDI_TAU_FIXED) {
        gm = P.tau;
        count = c_pass<true>(P, L, t, total, gm, P.out_n, 1 << 30, o);
    } else {
        float lo = 0.0f, hi = P.gmax;
        for (int it = 0; it < P.iters; ++it) {
            float m = 0.5f * (lo + hi);
            int c = c_pass<false>(P, L, t, total, m, 0, P.out_n, o);
            if (c <= P.out_n) hi = m;
            else lo = m;
        }
        gm = hi;
        count = c_pass<true>(P, L, t, total, gm, 0, 1 << 30, o);
    }
    if (count > P.out_n) count = P.out_n;
    for (int j = count; j < P.out_n; ++j) {
        size_t slot = (size_t)j * P.npix + p;
        P.out_color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        P.out_depth[slot] = make_float2(0.0f, 0.0f);
    }
    P.out_count[p] = count;
    if (P.out_gamma) P.out_gamma[p] = gm;
}

void launch_composite(const CompParams& P, hipStream_t s)
{
    size_t lds = (size_t)kWave * (2 * (size_t)P.seq_cap + 4 * P.k + 4 * P.k + 2 * P.k + 2 * P.k);
    dim3 grid((P.npix + kWave - 1) / kWave);
    hipLaunchKernelGGL(composite_kernel, grid, dim3(kWave), lds, s, P);
}

// ---------------------------------------------------------------- rendering

// Sec. 2.3: front-to-back over of the stored supersegments, each with its
// total opacity 1-(1-a)^((b-f)/ref).
__global__ __launch_bounds__(256) void render_kernel(const float4* __restrict__ color,
                                                     const float2* __restrict__ depth,
                                                     const int* __restrict__ count,
                                                     const uint32_t* __restrict__ offset, uint64_t capacity,
                                                     int max_n, uint32_t npix, float inv_ref,
                                                     float4* __restrict__ rgba, int* status)
{
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    int c = count[p];
    uint32_t base = offset ? offset[p] : p;
    uint32_t stride = offset ? 1u : npix;
    uint64_t last = offset ? (uint64_t)base + (uint64_t)(c > 0 ? c : 0) : (uint64_t)(c > 0 ? c : 0) * npix;
    if (c < 0 || c > max_n || last > capacity) {
        atomicOr(status, 2);
        c = 0;
    }
    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, A = 0.0f;
    for (int j = 0; j < c; ++j) {
        size_t e = (size_t)base + (size_t)j * stride;
        float4 s = color[e];
        float2 fb = depth[e];
        float Aj = -expm1f((fb.y - fb.x) * inv_ref * log1pf(-s.w));
        float w = (1.0f - A) * Aj;
        C0 = fmaf(w, s.x, C0);
        C1 = fmaf(w, s.y, C1);
        C2 = fmaf(w, s.z, C2);
        A += w;
    }
    rgba[p] = make_float4(C0, C1, C2, A);
}

void launch_render(const float4* color, const float2* depth, const int* count, const uint32_t* offset,
                   uint64_t capacity, int max_n, uint32_t npix, float inv_ref, float4* rgba, int* status,
                   hipStream_t s)
{
    dim3 grid((npix + 255) / 256);
    hipLaunchKernelGGL(render_kernel, grid, dim3(256), 0, s, color, depth, count, offset, capacity, max_n, npix,
                       inv_ref, rgba, status);
}

}  // namespace vdi
