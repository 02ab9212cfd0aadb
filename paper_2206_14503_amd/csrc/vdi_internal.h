// vdi_internal.h -- device-side building blocks shared by the libvdi kernels.
//
// Geometry, sample positions, trilinear reconstruction and the
// transfer-function coordinate are evaluated in fp32 with a fixed operation
// order (the ray setup with separate multiplies and adds, no contraction; the
// sample position and the trilinear blend with explicit fused multiply-adds):
// their results decide integers (sample counts, brick ownership, voxel and
// table cells, transparency), which must come out the same on every run and
// on any other implementation that follows the same order.  Everything after
// the transfer-function lookup is free fp32 arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/vdi.h"

// Library context: one per device.
struct vdi_ctx {
    int device;
    int* status;          // device words: [0] flags, [4..7] learned-path counters
    void* scratch;        // library-owned scratch: grown on demand, kept until destroy
    size_t scratch_bytes;
    void* user_ws;        // caller-owned workspace (vdi_ctx_set_workspace); when set, ops use it
    size_t user_ws_bytes; // and never allocate
    void* static_scratch; // device address of the fixed scratch array on this device
    hipStream_t aux;      // second stream of the ordered general merge (fork/join with the caller's)
    hipEvent_t ev[7];     // its fork/join and chunk events
    int num_cus;
    char arch[64];
};

namespace vdi {

// ---------------------------------------------------------------- host plumbing

void set_error(const char* fmt, ...);
vdi_status fail(vdi_status st, const char* fmt, ...);
vdi_status launched();                       // VDI_E_HIP if the last launch failed
// Workspace of an op: the caller's (VDI_E_WORKSPACE if smaller than bytes) or
// the library's own, grown when too small; ws_base() is its start.
vdi_status ensure_scratch(struct ::vdi_ctx* ctx, size_t bytes);
char* ws_base(struct ::vdi_ctx* ctx);

#define VDI_HIP_CHECK(expr)                                                          \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::vdi::set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
            return VDI_E_HIP;                                                        \
        }                                                                            \
    } while (0)

// ---------------------------------------------------------------- camera and rays

struct Cam {
    int ortho;
    float eye[3], fwd[3], right[3], up[3];
    int width, height;
};

struct Ray {
    float o[3], d[3];
    float tn, tf;
    int hit;
};

// One ray per pixel through the shared camera (Sec. 2.4, Sec. 5.1).
__device__ inline Ray make_ray(const Cam& c, int x, int y)
{
#pragma clang fp contract(off)
    Ray r;
    float sx = (float)(2 * x + 1) / (float)c.width - 1.0f;
    float sy = 1.0f - (float)(2 * y + 1) / (float)c.height;
    if (c.ortho) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float t1 = sx * c.right[a];
            float t2 = sy * c.up[a];
            float s = c.eye[a] + t1;
            r.o[a] = s + t2;
            r.d[a] = c.fwd[a];
        }
    } else {
        float v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float t1 = sx * c.right[a];
            float t2 = sy * c.up[a];
            float s = c.fwd[a] + t1;
            v[a] = s + t2;
            r.o[a] = c.eye[a];
        }
        float xx = v[0] * v[0];
        float yy = v[1] * v[1];
        float zz = v[2] * v[2];
        float n2 = xx + yy;
        n2 = n2 + zz;
        float nrm = __builtin_sqrtf(n2);
#pragma unroll
        for (int a = 0; a < 3; ++a) r.d[a] = v[a] / nrm;
    }
    // slab test against the world box [0,1]^3
    float tn = 0.0f, tf = __builtin_inff();
    int hit = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.d[a] == 0.0f) {
            if (r.o[a] < 0.0f || r.o[a] > 1.0f) hit = 0;
            continue;
        }
        float ta = (0.0f - r.o[a]) / r.d[a];
        float tb = (1.0f - r.o[a]) / r.d[a];
        float lo = ta < tb ? ta : tb;
        float hi = ta < tb ? tb : ta;
        if (lo > tn) tn = lo;
        if (hi < tf) tf = hi;
    }
    if (!(tn < tf)) hit = 0;
    r.tn = tn;
    r.tf = tf;
    r.hit = hit;
    return r;
}

// Distance of the midpoint of sample k from the ray origin (one fused
// multiply-add, the same single rounding on every implementation).
__device__ inline float sample_t(const Ray& r, int k, float step)
{
    float kk = (float)k + 0.5f;
    return __builtin_fmaf(kk, step, r.tn);
}

__device__ inline float sample_coord(const Ray& r, float t, int a)
{
    return __builtin_fmaf(t, r.d[a], r.o[a]);
}

// Number of samples of the ray: midpoints strictly before the exit.
__device__ inline int ray_samples(const Ray& r, float step)
{
    if (!r.hit) return 0;
    float est = (r.tf - r.tn) / step - 0.5f;
    int k = est > 0.0f ? (int)ceilf(est) : 0;
    if (k > (1 << 24)) k = 1 << 24;
    while (k > 0 && !(sample_t(r, k - 1, step) < r.tf)) --k;
    while (sample_t(r, k, step) < r.tf) ++k;
    return k;
}

// clamp for lo <= hi (one max and one min)
__device__ inline int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// clampi for lo <= hi (then the clamp is the median of the three) in one
// instruction; lo is wave-uniform.
__device__ inline int clamp_med3(int v, int lo, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(v), "s"(lo), "v"(hi));
    return r;
}

// Voxel index along axis a of the sample point (decides brick ownership).
__device__ inline int voxel_of(float p, int n)
{
#pragma clang fp contract(off)
    float g = p * (float)n;
    return clampi((int)floorf(g), 0, n - 1);
}

// ---------------------------------------------------------------- ownership
//
// Along a ray, each coordinate of the sample point is monotone in the sample
// index (rounding is monotone), so each clamped voxel index is monotone and
// the samples a box brick owns form one run [k0, k1).  Each of the six face
// predicates is monotone; its switching index is found from the analytic
// plane crossing and then corrected against the exact predicate.

struct OwnTest {
    const Ray* r;
    float step;
    int axis, n, bound;
    bool ge;   // predicate: voxel >= bound (else voxel < bound)
    __device__ bool operator()(int k) const
    {
        float t = sample_t(*r, k, step);
        int v = voxel_of(sample_coord(*r, t, axis), n);
        return ge ? v >= bound : v < bound;
    }
};

// First k in [0, ns] where a predicate that is monotone over [0, ns) becomes
// `want` (ns if never).  `rising` tells whether it goes false->true.
template <typename Pred>
__device__ inline int first_switch(const Pred& pred, int ns, int guess, bool rising)
{
    // predicate value `target` after the switch
    int k = clampi(guess, 0, ns);
    if (rising) {
        while (k > 0 && pred(k - 1)) --k;
        while (k < ns && !pred(k)) ++k;
    } else {
        while (k > 0 && !pred(k - 1)) --k;
        while (k < ns && pred(k)) ++k;
    }
    return k;
}

// Owned run [k0, k1) of brick box [lo, hi) among the ns samples of the ray.
__device__ inline void owned_run(const Ray& r, float step, int ns, const int n[3], const int lo[3],
                                 const int hi[3], int& k0, int& k1)
{
    k0 = 0;
    k1 = ns;
    if (ns <= 0) { k1 = 0; return; }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float d = r.d[a];
        if (d == 0.0f) {
            float t = sample_t(r, 0, step);
            int v = voxel_of(sample_coord(r, t, a), n[a]);
            if (v < lo[a] || v >= hi[a]) { k0 = 0; k1 = 0; return; }
            continue;
        }
        // sample index whose midpoint lies on the plane x_a = P/n
        auto guess = [&](int P) {
            float tp = ((float)P / (float)n[a] - r.o[a]) / d;
            float kf = (tp - r.tn) / step - 0.5f;
            kf = fminf(fmaxf(kf, -1.0f), (float)ns + 1.0f);
            return (int)ceilf(kf);
        };
        OwnTest geLo{&r, step, a, n[a], lo[a], true};
        OwnTest ltHi{&r, step, a, n[a], hi[a], false};
        int b, e;
        if (d > 0.0f) {
            // voxel index non-decreasing: >= lo rises, < hi falls
            b = lo[a] > 0 ? first_switch(geLo, ns, guess(lo[a]), true) : 0;
            e = hi[a] < n[a] ? first_switch(ltHi, ns, guess(hi[a]), false) : ns;
        } else {
            // voxel index non-increasing: < hi rises, >= lo falls
            b = hi[a] < n[a] ? first_switch(ltHi, ns, guess(hi[a]), true) : 0;
            e = lo[a] > 0 ? first_switch(geLo, ns, guess(lo[a]), false) : ns;
        }
        k0 = max(k0, b);
        k1 = min(k1, e);
    }
    if (k1 < k0) k1 = k0;
}

// ---------------------------------------------------------------- reconstruction

// a + w (b - a) with one fused multiply-add.
__device__ inline float lerp_exact(float a, float b, float w)
{
    float d = b - a;
    return __builtin_fmaf(w, d, a);
}

struct BrickGeo {
    float nf[3];    // global volume dims
    int dlo[3];     // global index of the first data voxel
    int clo[3];     // index range of the clamped stencil, relative to dlo:
    int chi[3];     //   clamp(clamp(i, 0, n-1) - dlo, 0, ddim-1) = clamp(i - dlo, clo, chi)
    uint32_t sx2;   // 1 if the x extent allows paired loads (ddim[0] >= 2)
    int xmax;       // ddim[0] - 2: last x of a paired load
    uint32_t sy, sz;  // element strides of y and z
    const uint8_t* own;  // optional rank per voxel of the whole volume (non-convex domains)
    int rank;
    int vn[3];           // global volume dims (voxel index of a sample)
};

// Geometry of a brick whose data box starts at global voxel dlo with extent
// ddim, inside a volume of n voxels (the two boxes intersect).
__device__ inline BrickGeo make_geo(const int n[3], const int dlo[3], const int ddim[3])
{
    BrickGeo g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.nf[a] = (float)n[a];
        g.dlo[a] = dlo[a];
        g.clo[a] = -dlo[a] > 0 ? -dlo[a] : 0;
        g.chi[a] = (n[a] - 1 - dlo[a]) < (ddim[a] - 1) ? (n[a] - 1 - dlo[a]) : (ddim[a] - 1);
    }
    g.sx2 = ddim[0] >= 2 ? 1u : 0u;
    g.xmax = ddim[0] - 2;
    g.sy = (uint32_t)ddim[0];
    g.sz = (uint32_t)ddim[0] * (uint32_t)ddim[1];
    g.own = nullptr;
    g.rank = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) g.vn[a] = n[a];
    return g;
}

// Whether the brick's owner map gives sample k of ray r to it (the voxel of
// the sample point decides, as for box ownership).
__device__ inline bool owns_sample(const BrickGeo& g, const Ray& r, float step, int k)
{
    const float t = sample_t(r, k, step);
    const int vx = voxel_of(sample_coord(r, t, 0), g.vn[0]);
    const int vy = voxel_of(sample_coord(r, t, 1), g.vn[1]);
    const int vz = voxel_of(sample_coord(r, t, 2), g.vn[2]);
    return g.own[((size_t)vz * (size_t)g.vn[1] + (size_t)vy) * (size_t)g.vn[0] + (size_t)vx] == (uint8_t)g.rank;
}

// Two x-adjacent voxels (p[0], p[1]) with one load (4-byte or 2-byte
// alignment; gfx950 allows unaligned dword loads from global memory).
typedef float vdi_f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef unsigned short vdi_h2u __attribute__((ext_vector_type(2), aligned(2)));

// Loads at a 32-bit byte offset from a wave-uniform base (a brick's data
// occupies less than 4 GiB; checked on the host).
template <typename VT> __device__ inline void load_pair(const VT* base, uint32_t i, float& a, float& b);
template <> __device__ inline void load_pair<float>(const float* base, uint32_t i, float& a, float& b)
{
    vdi_f2u v = *(const vdi_f2u*)((const char*)base + i * 4u);
    a = v.x;
    b = v.y;
}
template <> __device__ inline void load_pair<__half>(const __half* base, uint32_t i, float& a, float& b)
{
    vdi_h2u v = *(const vdi_h2u*)((const char*)base + i * 2u);
    a = __half2float(__ushort_as_half(v.x));
    b = __half2float(__ushort_as_half(v.y));
}
template <typename VT> __device__ inline float load_one(const VT* base, uint32_t i);
template <> __device__ inline float load_one<float>(const float* base, uint32_t i)
{
    return *(const float*)((const char*)base + i * 4u);
}
template <> __device__ inline float load_one<__half>(const __half* base, uint32_t i)
{
    return __half2float(*(const __half*)((const char*)base + i * 2u));
}

// Trilinear reconstruction on the global voxel grid from a halo'd brick, in
// two halves so that loops can issue the loads of a later sample before
// blending an earlier one.  Each of the four x-rows of the 2x2x2 stencil is
// read with one paired load at xb = min(x0, dx-2), which stays inside the row
// also at clamped edges; every index is clamped to the data box, so the loads
// stay in bounds for any position.
struct Taps {
    float a[4], b[4];   // rows (y0,z0), (y1,z0), (y0,z1), (y1,z1): voxels xb, xb+1
    float w[3];         // blend weights; w[0] is 0 where both x taps are one voxel
    bool hi;            // both x taps are voxel xb+1 (the data box's last x)
};

// PAIRED: the brick's data box is at least two voxels wide in x (g.sx2); a
// loop over samples picks the variant once, outside the loop.
template <typename VT, bool PAIRED>
__device__ inline Taps trilinear_fetch(const VT* data, const BrickGeo& g, const float p[3])
{
#pragma clang fp contract(off)
    Taps t;
    int i0[3], i1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float u = __builtin_fmaf(p[a], g.nf[a], -0.5f);
        float f = floorf(u);
        t.w[a] = u - f;
        int ii = (int)f - g.dlo[a];
        i0[a] = clamp_med3(ii, g.clo[a], g.chi[a]);
        i1[a] = clamp_med3(ii + 1, g.clo[a], g.chi[a]);
    }
    // 24-bit multiplies: indices and strides are below 2^24 and every product
    // below 2^30 (the data box is under 4 GiB)
    const uint32_t y0 = __umul24((uint32_t)i0[1], g.sy), y1 = __umul24((uint32_t)i1[1], g.sy);
    const uint32_t z0 = __umul24((uint32_t)i0[2], g.sz), z1 = __umul24((uint32_t)i1[2], g.sz);
    const uint32_t r00 = y0 + z0, r10 = y1 + z0, r01 = y0 + z1, r11 = y1 + z1;
    if (PAIRED) {
        const int xb = i0[0] < g.xmax ? i0[0] : g.xmax;
        // x0 is voxel xb, else xb + 1 (the data box's last voxel, x1 = x0);
        // x1 is voxel xb + 1 unless clamped onto x0.  Where both taps are one
        // voxel the row's value is that voxel: weight 0 on the lerp based at
        // it (the blend bases the lerp at b where `hi`)
        t.hi = i0[0] != xb;
        t.w[0] = (i0[0] == xb && i1[0] != xb) ? t.w[0] : 0.0f;
        load_pair<VT>(data, r00 + xb, t.a[0], t.b[0]);
        load_pair<VT>(data, r10 + xb, t.a[1], t.b[1]);
        load_pair<VT>(data, r01 + xb, t.a[2], t.b[2]);
        load_pair<VT>(data, r11 + xb, t.a[3], t.b[3]);
    } else {
        t.w[0] = 0.0f;
        t.hi = false;
        t.a[0] = t.b[0] = load_one<VT>(data, r00);
        t.a[1] = t.b[1] = load_one<VT>(data, r10);
        t.a[2] = t.b[2] = load_one<VT>(data, r01);
        t.a[3] = t.b[3] = load_one<VT>(data, r11);
    }
    return t;
}

// The x lerps are a + w (b - a) with one rounding, as every lerp of the
// reconstruction; a row whose taps are one voxel v gives exactly v (weight 0
// on base v).
__device__ inline float lerp_x(const Taps& t, int row)
{
    const float d = t.b[row] - t.a[row];
    return __builtin_fmaf(t.w[0], d, t.hi ? t.b[row] : t.a[row]);
}

__device__ inline float trilinear_blend(const Taps& t)
{
#pragma clang fp contract(off)
    float c00 = lerp_x(t, 0);
    float c10 = lerp_x(t, 1);
    float c01 = lerp_x(t, 2);
    float c11 = lerp_x(t, 3);
    float c0 = lerp_exact(c00, c10, t.w[1]);
    float c1 = lerp_exact(c01, c11, t.w[1]);
    return lerp_exact(c0, c1, t.w[2]);
}

template <typename VT>
__device__ inline float trilinear(const VT* data, const BrickGeo& g, const float p[3])
{
    return g.sx2 ? trilinear_blend(trilinear_fetch<VT, true>(data, g, p))
                 : trilinear_blend(trilinear_fetch<VT, false>(data, g, p));
}

// Transfer-function cell and weight of scalar s.
__device__ inline void tf_coord(float s, int entries, int& cell, float& w)
{
#pragma clang fp contract(off)
    float sc = fminf(fmaxf(s, 0.0f), 1.0f);
    float q = sc * (float)(entries - 1);
    int i = (int)floorf(q);
    if (i > entries - 2) i = entries - 2;
    cell = i;
    w = q - (float)i;
}

// The transfer function as the kernels stage it: per cell i (0 <= i <
// entries - 1) its lower row and the difference to the row above.
struct TfCell {
    float4 lo, d;
};

// Cells of the rows tf[0 .. entries), by the threads of a block (stride n).
__device__ inline void tf_stage(TfCell* cells, const float4* tf, int entries, int t, int n)
{
    for (int i = t; i < entries - 1; i += n) {
        const float4 lo = tf[i], hi = tf[i + 1];
        cells[i].lo = lo;
        cells[i].d = make_float4(hi.x - lo.x, hi.y - lo.y, hi.z - lo.z, hi.w - lo.w);
    }
}

__device__ inline float4 tf_lookup(const TfCell* tf, int entries, float s)
{
    int i;
    float w;
    tf_coord(s, entries, i, w);
    const TfCell c = tf[i];
    return make_float4(fmaf(w, c.d.x, c.lo.x), fmaf(w, c.d.y, c.lo.y), fmaf(w, c.d.z, c.lo.z),
                       fmaf(w, c.d.w, c.lo.w));
}

// ---------------------------------------------------------------- fast math
//
// Hardware log2/exp2/reciprocal (about 1 ulp).  Quantities that are small
// differences from 1 use forms that keep their relative accuracy.

__device__ inline float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// log2(1 - a) for a in [0, 1], accurate also for tiny a (the rounding of
// u = 1 - a is undone by the factor a / (1 - u)).  Written without branches:
// every lane evaluates all forms and selects.
__device__ inline float log2_1m(float a)
{
    const float u = 1.0f - a;
    const float lu = hw_log2(u);
    const float d = 1.0f - u;                                   // exact
    const float r = lu * (a * hw_rcp(d));
    const float tiny = -a * 1.4426950408889634f;               // a below half an ulp of 1
    return a >= 0.5f ? lu : (u == 1.0f ? tiny : r);            // 1 - a exact for a >= 1/2
}

// 1 - 2^y for y <= 0, accurate also for y near 0 (the rounding of u = 2^y is
// undone by the factor y / log2(u)).  Without branches.
__device__ inline float one_minus_exp2(float y)
{
    const float u = hw_exp2(y);
    const float r = (1.0f - u) * (y * hw_rcp(hw_log2(u)));
    const float tiny = -y * 0.6931471805599453f;
    return u == 1.0f ? tiny : (u == 0.0f ? 1.0f : r);
}

// ---------------------------------------------------------------- global loads

// Loads through pointers the compiler cannot prove global (e.g. read from an
// LDS table), issued as global rather than flat loads.
typedef float vdi_gf4 __attribute__((ext_vector_type(4)));
typedef float vdi_gf2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) vdi_gf4* vdi_gp4;
typedef const __attribute__((address_space(1))) vdi_gf2* vdi_gp2;

__device__ inline float4 gload(const float4* p, uint32_t i)
{
    vdi_gf4 v = ((vdi_gp4)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline float2 gload(const float2* p, uint32_t i)
{
    vdi_gf2 v = ((vdi_gp2)p)[i];
    return make_float2(v.x, v.y);
}

// ---------------------------------------------------------------- queues

// Add `inc` (0 or 1 per lane) to *ctr with one atomic per wavefront; returns
// this lane's position among the wave's incrementing lanes plus the old value
// (meaningful for lanes with inc == 1).
__device__ inline int wave_append(int* ctr, bool inc)
{
    const unsigned long long m = __ballot(inc);
    const int n = __popcll(m);
    const int lane = threadIdx.x & 63;
    const int leader = m ? (__ffsll((long long)m) - 1) : 0;
    int base = 0;
    if (n && lane == leader) base = atomicAdd(ctr, n);
    base = __shfl(base, leader, 64);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    return base + rank;
}

// Add the number of lanes with `inc` to *ctr (one atomic per wavefront).
__device__ inline void wave_count(int* ctr, bool inc)
{
    const unsigned long long m = __ballot(inc);
    const int lane = threadIdx.x & 63;
    const int leader = m ? (__ffsll((long long)m) - 1) : 0;
    if (m && lane == leader) atomicAdd(ctr, __popcll(m));
}

// ---------------------------------------------------------------- misc

// fp32 -> bf16 bits, round to nearest even.
__device__ inline uint16_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float gamma_sq(float g) { return g * g; }

}  // namespace vdi
