// vdi_novel.hip -- a VDI rendered from a viewpoint other than the one it was
// generated from (the paper evaluates VDIs rendered at viewpoint deviations,
// Sec. 7; the rendering itself is prior work it cites).
//
// The VDI is read as the piecewise-constant field it encodes: supersegment j
// of pixel q fills the part of q's view frustum between its front and back
// depths with its colour and per-ref-step opacity; outside every supersegment
// the field is empty.  A ray of the new view is sampled like a generation ray
// (midpoints of its grid from the entry into [0,1]^3, fp32 positions).  Each
// sample is projected into the VDI camera in fp64 with a fixed operation
// order (its pixel and its depth: distance from the eye for a perspective
// camera, along fwd for an orthographic one), looked up in that pixel's list
// and composited front to back with opacity 1 - (1 - a)^(step/ref) (Eq. 2).
//
// One lane per ray, 16x16-pixel blocks.  A lane keeps the depth interval it
// last found in a pixel's list (a supersegment, or the gap between two), so
// the samples that stay in it skip the search.
#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

namespace {

struct Proj {
    double e[3], f[3], r[3], u[3];
    double ff, irr, iuu;   // |fwd|^2, 1/|right|^2, 1/|up|^2
    int ortho, W, H;
};

__device__ inline double dot3d(const double a[3], const double b[3])
{
#pragma clang fp contract(off)
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ inline Proj make_proj(const Cam& c)
{
    Proj P;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        P.e[a] = c.eye[a];
        P.f[a] = c.fwd[a];
        P.r[a] = c.right[a];
        P.u[a] = c.up[a];
    }
    P.ff = dot3d(P.f, P.f);
    P.irr = 1.0 / dot3d(P.r, P.r);
    P.iuu = 1.0 / dot3d(P.u, P.u);
    P.ortho = c.ortho;
    P.W = c.width;
    P.H = c.height;
    return P;
}

// Pixel q of the VDI camera that point p falls in and its depth (squared for
// a perspective camera, whose direction through screen point (sx, sy) is
// fwd + sx right + sy up); false outside the image or not in front of the eye.
__device__ inline bool project(const Proj& P, const float p[3], int& q, double& depth)
{
#pragma clang fp contract(off)
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = (double)p[a] - P.e[a];
    const double vf = dot3d(v, P.f), vr = dot3d(v, P.r), vu = dot3d(v, P.u);
    double sx, sy;
    if (P.ortho) {
        sx = vr * P.irr;
        sy = vu * P.iuu;
        depth = vf;
    } else {
        if (!(vf > 0.0)) return false;
        const double w = P.ff / vf;
        sx = (vr * w) * P.irr;
        sy = (vu * w) * P.iuu;
        depth = dot3d(v, v);
    }
    const double fx = floor(((sx + 1.0) * 0.5) * (double)P.W);
    const double fy = floor(((1.0 - sy) * 0.5) * (double)P.H);
    if (!(fx >= 0.0 && fx < (double)P.W && fy >= 0.0 && fy < (double)P.H)) return false;
    q = (int)fy * P.W + (int)fx;
    return true;
}

}  // namespace

__global__ __launch_bounds__(256) void novel_kernel(NovelParams N)
{
    const int x = blockIdx.x * 16 + (threadIdx.x & 15);
    const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= N.view.width || y >= N.view.height) return;
    const Proj P = make_proj(N.vcam);
    const Ray r = make_ray(N.view, x, y);
    const int ns = ray_samples(r, N.step);
    const uint32_t stride = N.offset ? 1u : N.npix;
    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
    // the depth interval [lo, hi) of pixel cq last looked up: a supersegment
    // (inside, with its colour, sample opacity and transmittance) or a gap
    int cq = -1;
    double lo = 0.0, hi = 0.0;
    bool inside = false;
    float4 col = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float alpha = 0.0f, te = 1.0f;
    for (int k = 0; k < ns; ++k) {
        const float t = sample_t(r, k, N.step);
        const float p[3] = { sample_coord(r, t, 0), sample_coord(r, t, 1), sample_coord(r, t, 2) };
        int q;
        double d;
        if (!project(P, p, q, d)) continue;
        if (q != cq || !(lo <= d && d < hi)) {
            cq = q;
            int c = N.count[q];
            const uint32_t base = N.offset ? N.offset[q] : (uint32_t)q;
            const uint64_t last = N.offset ? (uint64_t)base + (uint64_t)(c > 0 ? c : 0)
                                           : (uint64_t)(c > 0 ? c : 0) * N.npix;
            if (c < 0 || c > N.max_n || last > N.capacity) {
                atomicOr(N.status, 2);
                c = 0;
            }
            // fronts are non-decreasing: the last supersegment with front <= d
            int a = 0, b = c;
            while (a < b) {
                const int m = (a + b) >> 1;
                const double f = N.depth[(size_t)base + (size_t)m * stride].x;
                if ((P.ortho ? f : f * f) <= d) a = m + 1;
                else b = m;
            }
            const int j = a - 1;
            double jb = -__builtin_inf();   // back of supersegment j (or -inf)
            if (j >= 0) {
                const size_t e = (size_t)base + (size_t)j * stride;
                const float2 fb = N.depth[e];
                const double f = fb.x, bk = fb.y;
                jb = P.ortho ? bk : bk * bk;
                if (d < jb) {
                    inside = true;
                    lo = P.ortho ? f : f * f;
                    hi = jb;
                    col = N.color[e];
                    const float lg = N.l * log2_1m(col.w);
                    alpha = one_minus_exp2(lg);
                    te = hw_exp2(lg);
                }
            }
            if (j < 0 || !(d < jb)) {
                // the gap up to the next front
                inside = false;
                lo = j >= 0 ? jb : -__builtin_inf();
                if (a < c) {
                    const double f = N.depth[(size_t)base + (size_t)a * stride].x;
                    hi = P.ortho ? f : f * f;
                } else {
                    hi = __builtin_inf();
                }
            }
        }
        if (inside) {
            const float w = T * alpha;
            C0 = fmaf(w, col.x, C0);
            C1 = fmaf(w, col.y, C1);
            C2 = fmaf(w, col.z, C2);
            T *= te;
        }
    }
    N.rgba[(size_t)y * N.view.width + x] = make_float4(C0, C1, C2, 1.0f - T);
}

void launch_novel(const NovelParams& N, hipStream_t s)
{
    dim3 grid((N.view.width + 15) / 16, (N.view.height + 15) / 16);
    hipLaunchKernelGGL(novel_kernel, grid, dim3(256), 0, s, N);
}

}  // namespace vdi
