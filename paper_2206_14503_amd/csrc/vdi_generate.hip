// vdi_generate.hip -- sub-VDI generation on one brick per grid z-slice
// (Sec. 5.1), with the Eq. 1 termination criterion, the per-ray bisection of
// the threshold (Sec. 2.4) and regular or compact output (Sec. 4).
//
// Launch shape: a 256-thread block covers a 16x16 pixel tile, each wavefront
// an 8x8 ray tile, so the 64 rays of a wave sample neighbouring voxels of the
// brick at every step.  The transfer function is staged in LDS.
#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

// Segmenter state over a brick's owned sample run (all samples share the
// length step; indices are sample numbers).
struct GenSeg {
    float c0, c1, c2;   // premultiplied colour
    float A;            // accumulated opacity (added up, exact for thin segments)
    float T;            // transmittance (multiplied, exact for thick segments)
    int kf, kb, kbt;    // first sample, one past the last, one past the last non-transparent
    int open;
};

struct GenOut {
    float4* color;
    float2* depth;
    uint32_t base;      // first slot index of this list (compact) or pixel index (regular)
    uint32_t stride;    // slot stride: 1 (compact) or P (regular)
    uint32_t limit;     // slots that may be written
};

template <bool WRITE>
__device__ inline void gen_close(GenSeg& S, int& count, const GenOut& o, const Ray& r, float step,
                                 float l_step)
{
    if (WRITE && (uint32_t)count < o.limit) {
        float invA = 1.0f / S.A;
        float len = (float)(S.kbt - S.kf) * l_step;
        float a = -expm1f(logf(S.T) / len);
        size_t slot = (size_t)o.base + (size_t)count * o.stride;
        o.color[slot] = make_float4(S.c0 * invA, S.c1 * invA, S.c2 * invA, a);
        float f = r.tn + (float)S.kf * step;
        float b = r.tn + (float)S.kbt * step;
        o.depth[slot] = make_float2(f, b);
    }
    ++count;
    S.open = 0;
}

// One pass of the segmenter over samples [k0, k1) at threshold gamma.
// Returns the supersegment count; a pass that is only counting stops as soon
// as the count exceeds `limit` (its outcome "infeasible" is then decided).
// cap > 0 saturates after cap-1 closes (fixed-threshold mode).
template <typename VT, bool WRITE>
__device__ int gen_pass(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int k0,
                        int k1, const float4* tf, int entries, float gamma, int cap, int limit, const GenOut& o,
                        int* n_opaque_out)
{
    const float g2 = gamma * gamma;
    GenSeg S;
    S.open = 0;
    S.c0 = S.c1 = S.c2 = 0.0f;
    S.A = 0.0f;
    S.T = 1.0f;
    S.kf = S.kb = S.kbt = 0;
    int count = 0, n_opaque = 0;
    const bool unit = (l_step == 1.0f);
    for (int k = k0; k < k1; ++k) {
        float t = sample_t(r, k, step);
        float p[3] = { sample_coord(r, t, 0), sample_coord(r, t, 1), sample_coord(r, t, 2) };
        float s = trilinear<VT>(data, g, p);
        float4 c = tf_lookup(tf, entries, s);
        const bool transparent = (c.w == 0.0f);
        n_opaque += transparent ? 0 : 1;
        // Eq. 2 / length-adjusted opacity of the sample
        float at = unit ? c.w : -expm1f(l_step * log1pf(-c.w));
        if (S.open) {
            float L = (float)(k - S.kf) * l_step;
            float aS = -expm1f(logf(S.T) / L);
            float sc = aS / S.A;
            float d0 = S.c0 * sc - c.x * c.w;
            float d1 = S.c1 * sc - c.y * c.w;
            float d2 = S.c2 * sc - c.z * c.w;
            float dd = d0 * d0 + d1 * d1 + d2 * d2;
            bool may_close = cap <= 0 || count < cap - 1;
            if (may_close && g2 < dd) {
                gen_close<WRITE>(S, count, o, r, step, l_step);
                if (!WRITE && count > limit) break;
            } else {
                float w = S.T * at;
                S.c0 = fmaf(w, c.x, S.c0);
                S.c1 = fmaf(w, c.y, S.c1);
                S.c2 = fmaf(w, c.z, S.c2);
                S.A += w;
                S.T *= unit ? (1.0f - c.w) : expf(l_step * log1pf(-c.w));
                S.kb = k + 1;
                if (!transparent) S.kbt = k + 1;
            }
        }
        if (!S.open && !transparent) {
            S.open = 1;
            S.kf = k;
            S.kb = S.kbt = k + 1;
            S.c0 = c.x * at;
            S.c1 = c.y * at;
            S.c2 = c.z * at;
            S.A = at;
            S.T = unit ? (1.0f - c.w) : expf(l_step * log1pf(-c.w));
        }
    }
    if (S.open) gen_close<WRITE>(S, count, o, r, step, l_step);
    if (n_opaque_out) *n_opaque_out = n_opaque;
    return count;
}

// Threshold for one brick-ray and the count it yields.
template <typename VT>
__device__ void gen_search(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int k0,
                           int k1, const float4* tf, int entries, const GenParams& P, float& gamma_out,
                           int& count_out, bool need_count)
{
    GenOut none{nullptr, nullptr, 0, 0, 0};
    if (P.mode == VDI_TAU_FIXED) {
        gamma_out = P.tau;
        count_out = need_count ? gen_pass<VT, false>(data, g, r, step, l_step, k0, k1, tf, entries, P.tau,
                                                     P.max_n, 1 << 30, none, nullptr)
                               : -1;
        return;
    }
    float lo = 0.0f, hi = P.gmax;
    int hi_count = -1;
    for (int it = 0; it < P.iters; ++it) {
        float m = 0.5f * (lo + hi);
        int n_opaque = 0;
        int c = gen_pass<VT, false>(data, g, r, step, l_step, k0, k1, tf, entries, m, 0, P.max_n, none,
                                    it == 0 ? &n_opaque : nullptr);
        if (c <= P.max_n) {
            hi = m;
            hi_count = c;
            // every supersegment starts at a non-transparent sample, so a run
            // with at most N of them is feasible at every threshold: the
            // remaining halvings all move the upper bracket
            if (it == 0 && n_opaque <= P.max_n) {
                for (int j = 1; j < P.iters; ++j) hi *= 0.5f;
                hi_count = (P.iters > 1) ? -1 : c;
                break;
            }
        } else {
            lo = m;
        }
    }
    gamma_out = hi;
    if (need_count && hi_count < 0)
        hi_count = gen_pass<VT, false>(data, g, r, step, l_step, k0, k1, tf, entries, hi, 0, 1 << 30, none,
                                       nullptr);
    count_out = hi_count;
}

// kind: 0 = search + regular write, 1 = search only (count + gamma), 2 = compact write
template <typename VT, int KIND>
__global__ __launch_bounds__(256) void gen_kernel(GenParams P, GenBricks B)
{
    __shared__ float4 tf_s[VDI_MAX_TF];
    for (int i = threadIdx.x; i < P.tf_entries; i += blockDim.x) tf_s[i] = P.tf[i];
    __syncthreads();

    const GenBrick& br = B.b[blockIdx.z];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (x >= P.cam.width || y >= P.cam.height) return;
    const uint32_t pix = (uint32_t)y * (uint32_t)P.cam.width + (uint32_t)x;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;

    BrickGeo g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.n[a] = P.n[a];
        g.dlo[a] = br.dlo[a];
        g.ddim[a] = br.ddim[a];
    }
    const VT* data = (const VT*)br.data;
    Ray r = make_ray(P.cam, x, y);
    int ns = ray_samples(r, P.step);
    int k0 = 0, k1 = 0;
    if (ns > 0) owned_run(r, P.step, ns, P.n, br.lo, br.hi, k0, k1);

    const float empty_gamma = P.mode == VDI_TAU_FIXED ? P.tau : ldexpf(P.gmax, -P.iters);
    if (KIND == 1) {
        float gm = empty_gamma;
        int c = 0;
        if (k1 > k0) gen_search<VT>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, P, gm, c, true);
        br.count[pix] = c;
        br.gamma[pix] = gm;
        return;
    }
    if (KIND == 2) {
        int c = br.count[pix];
        float gm = br.gamma[pix];
        uint32_t off = br.offset[pix];
        uint32_t lim = 0;
        if ((uint64_t)off + (uint64_t)c <= br.capacity) lim = (uint32_t)c;
        else if (c > 0) atomicOr(P.status, 1);
        GenOut o{br.color, br.depth, off, 1, lim};
        if (c > 0 && lim > 0) {
            int cap = P.mode == VDI_TAU_FIXED ? P.max_n : 0;
            gen_pass<VT, true>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gm, cap, 1 << 30, o,
                               nullptr);
        }
        return;
    }
    // KIND 0: search, then write the regular slots and zero the rest
    float gm = empty_gamma;
    int c = 0;
    GenOut o{br.color, br.depth, pix, npix, (uint32_t)P.max_n};
    if (k1 > k0) {
        gen_search<VT>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, P, gm, c, false);
        int cap = P.mode == VDI_TAU_FIXED ? P.max_n : 0;
        c = gen_pass<VT, true>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gm, cap, 1 << 30, o,
                               nullptr);
    }
    for (int j = c; j < P.max_n; ++j) {
        size_t slot = (size_t)j * npix + pix;
        br.color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        br.depth[slot] = make_float2(0.0f, 0.0f);
    }
    br.count[pix] = c < P.max_n ? c : P.max_n;
    if (br.gamma) br.gamma[pix] = gm;
}

template <typename VT>
static void launch_gen(int kind, const GenParams& P, const GenBricks& B, int nb, hipStream_t s)
{
    dim3 grid((P.cam.width + 15) / 16, (P.cam.height + 15) / 16, nb);
    if (kind == 0) hipLaunchKernelGGL((gen_kernel<VT, 0>), grid, dim3(256), 0, s, P, B);
    if (kind == 1) hipLaunchKernelGGL((gen_kernel<VT, 1>), grid, dim3(256), 0, s, P, B);
    if (kind == 2) hipLaunchKernelGGL((gen_kernel<VT, 2>), grid, dim3(256), 0, s, P, B);
}

void launch_generate(int kind, int dtype, const GenParams& P, const GenBricks& B, int nb, hipStream_t s)
{
    if (dtype == VDI_F16) launch_gen<__half>(kind, P, B, nb, s);
    else launch_gen<float>(kind, P, B, nb, s);
}

// ---------------------------------------------------------------- rays (diagnostic)

__global__ void rays_kernel(Cam cam, float step, float* o, float* d, float* tn, float* tf, int* ns)
{
    int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= cam.width) return;
    size_t p = (size_t)y * cam.width + x;
    Ray r = make_ray(cam, x, y);
    for (int a = 0; a < 3; ++a) {
        o[3 * p + a] = r.o[a];
        d[3 * p + a] = r.d[a];
    }
    tn[p] = r.tn;
    tf[p] = r.tf;
    ns[p] = r.hit ? ray_samples(r, step) : -1;
}

void launch_rays(const Cam& cam, float step, float* o, float* d, float* tn, float* tf, int* ns, hipStream_t s)
{
    dim3 grid((cam.width + 255) / 256, cam.height);
    hipLaunchKernelGGL(rays_kernel, grid, dim3(256), 0, s, cam, step, o, d, tn, tf, ns);
}

}  // namespace vdi
