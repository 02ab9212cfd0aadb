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
    void* scratch;        // grown on demand, kept until destroy
    size_t scratch_bytes;
    int num_cus;
    char arch[64];
};

namespace vdi {

// ---------------------------------------------------------------- host plumbing

void set_error(const char* fmt, ...);
vdi_status fail(vdi_status st, const char* fmt, ...);
vdi_status launched();                       // VDI_E_HIP if the last launch failed
vdi_status ensure_scratch(struct ::vdi_ctx* ctx, size_t bytes);

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

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

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

template <typename VT> __device__ inline float load_voxel(const VT* p, size_t i);
template <> __device__ inline float load_voxel<float>(const float* p, size_t i) { return p[i]; }
template <> __device__ inline float load_voxel<__half>(const __half* p, size_t i) { return __half2float(p[i]); }

// a + w (b - a) with one fused multiply-add.
__device__ inline float lerp_exact(float a, float b, float w)
{
    float d = b - a;
    return __builtin_fmaf(w, d, a);
}

struct BrickGeo {
    int n[3];       // global volume dims
    int dlo[3];     // global index of the first data voxel
    int ddim[3];    // data box dims
};

// Two x-adjacent voxels (p[0], p[1]) with one load (4-byte or 2-byte
// alignment; gfx950 allows unaligned dword loads from global memory).
typedef float vdi_f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef unsigned short vdi_h2u __attribute__((ext_vector_type(2), aligned(2)));

template <typename VT> __device__ inline void load_pair(const VT* p, float& a, float& b);
template <> __device__ inline void load_pair<float>(const float* p, float& a, float& b)
{
    vdi_f2u v = *(const vdi_f2u*)p;
    a = v.x;
    b = v.y;
}
template <> __device__ inline void load_pair<__half>(const __half* p, float& a, float& b)
{
    vdi_h2u v = *(const vdi_h2u*)p;
    a = __half2float(__ushort_as_half(v.x));
    b = __half2float(__ushort_as_half(v.y));
}

// Trilinear reconstruction on the global voxel grid from a halo'd brick.
// Each of the four x-rows of the 2x2x2 stencil is read with one paired load
// at xb = min(x0, dx-2), which stays inside the row also at clamped edges.
template <typename VT>
__device__ inline float trilinear(const VT* data, const BrickGeo& g, const float p[3])
{
#pragma clang fp contract(off)
    int i0[3], i1[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float u = __builtin_fmaf(p[a], (float)g.n[a], -0.5f);
        float f = floorf(u);
        w[a] = u - f;
        int ii = (int)f;
        i0[a] = clampi(clampi(ii, 0, g.n[a] - 1) - g.dlo[a], 0, g.ddim[a] - 1);
        i1[a] = clampi(clampi(ii + 1, 0, g.n[a] - 1) - g.dlo[a], 0, g.ddim[a] - 1);
    }
    // 32-bit offsets: a brick's data holds fewer than 2^31 voxels (checked on the host)
    const uint32_t sy = (uint32_t)g.ddim[0], sz = (uint32_t)g.ddim[0] * (uint32_t)g.ddim[1];
    const uint32_t r00 = i0[1] * sy + i0[2] * sz, r10 = i1[1] * sy + i0[2] * sz;
    const uint32_t r01 = i0[1] * sy + i1[2] * sz, r11 = i1[1] * sy + i1[2] * sz;
    float v000, v100, v010, v110, v001, v101, v011, v111;
    if (g.ddim[0] >= 2) {
        const int xb = i0[0] < g.ddim[0] - 2 ? i0[0] : g.ddim[0] - 2;
        const bool s0 = i0[0] == xb, s1 = i1[0] == xb;
        float a, b;
        load_pair<VT>(data + r00 + xb, a, b);
        v000 = s0 ? a : b;
        v100 = s1 ? a : b;
        load_pair<VT>(data + r10 + xb, a, b);
        v010 = s0 ? a : b;
        v110 = s1 ? a : b;
        load_pair<VT>(data + r01 + xb, a, b);
        v001 = s0 ? a : b;
        v101 = s1 ? a : b;
        load_pair<VT>(data + r11 + xb, a, b);
        v011 = s0 ? a : b;
        v111 = s1 ? a : b;
    } else {
        v000 = v100 = load_voxel(data, r00);
        v010 = v110 = load_voxel(data, r10);
        v001 = v101 = load_voxel(data, r01);
        v011 = v111 = load_voxel(data, r11);
    }
    float c00 = lerp_exact(v000, v100, w[0]);
    float c10 = lerp_exact(v010, v110, w[0]);
    float c01 = lerp_exact(v001, v101, w[0]);
    float c11 = lerp_exact(v011, v111, w[0]);
    float c0 = lerp_exact(c00, c10, w[1]);
    float c1 = lerp_exact(c01, c11, w[1]);
    return lerp_exact(c0, c1, w[2]);
}

// Transfer-function cell and weight of scalar s.
__device__ inline void tf_coord(float s, int entries, int& cell, float& w)
{
#pragma clang fp contract(off)
    float sc = s < 0.0f ? 0.0f : (s > 1.0f ? 1.0f : s);
    float q = sc * (float)(entries - 1);
    int i = (int)floorf(q);
    if (i > entries - 2) i = entries - 2;
    cell = i;
    w = q - (float)i;
}

__device__ inline float4 tf_lookup(const float4* tf, int entries, float s)
{
    int i;
    float w;
    tf_coord(s, entries, i, w);
    float4 lo = tf[i], hi = tf[i + 1];
    return make_float4(fmaf(w, hi.x - lo.x, lo.x), fmaf(w, hi.y - lo.y, lo.y),
                       fmaf(w, hi.z - lo.z, lo.z), fmaf(w, hi.w - lo.w, lo.w));
}

// ---------------------------------------------------------------- fast math
//
// Hardware log2/exp2/reciprocal (about 1 ulp).  Quantities that are small
// differences from 1 use forms that keep their relative accuracy.

__device__ inline float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// log2(1 - a) for a in [0, 1], accurate also for tiny a.
__device__ inline float log2_1m(float a)
{
    float u = 1.0f - a;
    if (a >= 0.5f) return hw_log2(u);                 // 1 - a exact here
    if (u == 1.0f) return -a * 1.4426950408889634f;   // a below half an ulp of 1
    float d = 1.0f - u;                               // exact
    return hw_log2(u) * (a * hw_rcp(d));
}

// 1 - 2^y for y <= 0, accurate also for y near 0.
__device__ inline float one_minus_exp2(float y)
{
    float u = hw_exp2(y);
    if (u == 1.0f) return -y * 0.6931471805599453f;
    if (u == 0.0f) return 1.0f;
    return (1.0f - u) * (y * hw_rcp(hw_log2(u)));
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
