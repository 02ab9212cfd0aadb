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
    float T;            // transmittance (multiplied)
    float lT;           // log2 of the transmittance (added up)
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
        float a = one_minus_exp2(S.lT / len);
        size_t slot = (size_t)o.base + (size_t)count * o.stride;
        o.color[slot] = make_float4(S.c0 * invA, S.c1 * invA, S.c2 * invA, a);
        float f = r.tn + (float)S.kf * step;
        float b = r.tn + (float)S.kbt * step;
        o.depth[slot] = make_float2(f, b);
    }
    ++count;
    S.open = 0;
}

template <typename VT>
__device__ inline float4 gen_sample(const VT* data, const BrickGeo& g, const Ray& r, float step, int k,
                                    const float4* tf, int entries)
{
    float t = sample_t(r, k, step);
    float p[3] = { sample_coord(r, t, 0), sample_coord(r, t, 1), sample_coord(r, t, 2) };
    float s = trilinear<VT>(data, g, p);
    return tf_lookup(tf, entries, s);
}

__device__ inline void gen_seg_init(GenSeg& S)
{
    S.open = 0;
    S.c0 = S.c1 = S.c2 = 0.0f;
    S.A = 0.0f;
    S.T = 1.0f;
    S.lT = 0.0f;
    S.kf = S.kb = S.kbt = 0;
}

// A classified sample prepared once and shared by every segmenter state.
struct GenSample {
    float4 c;        // colour and per-step opacity a
    float at;        // opacity over the sample's length (Eq. 2 / length-adjusted)
    float Te;        // 1 - at
    float lg;        // log2(1 - at)
    float e0, e1, e2;  // per-step premultiplied colour (Eq. 1 operand)
    bool transparent;
};

__device__ inline GenSample gen_prep(float4 c, float l_step, bool unit)
{
    GenSample q;
    q.c = c;
    q.transparent = (c.w == 0.0f);
    float lg1 = log2_1m(c.w);
    q.lg = unit ? lg1 : l_step * lg1;
    q.at = unit ? c.w : one_minus_exp2(q.lg);
    q.Te = unit ? 1.0f - c.w : hw_exp2(q.lg);
    q.e0 = c.x * c.w;
    q.e1 = c.y * c.w;
    q.e2 = c.z * c.w;
    return q;
}

// One sample through the segmenter (Eq. 1 test, then merge or close/open).
// The test gamma < |C a_S / A - e| is evaluated as gamma^2 A^2 < |C a_S - e A|^2
// (A > 0), with a_S = 1 - 2^(log2(T) / L) the open supersegment's per-step
// opacity.
template <bool WRITE>
__device__ inline void gen_step(GenSeg& S, int& count, const GenOut& o, const Ray& r, float step, float l_step,
                                float g2, int cap, int k, const GenSample& q)
{
    if (S.open) {
        float L = (float)(S.kb - S.kf) * l_step;
        float aS = 1.0f - hw_exp2(S.lT * hw_rcp(L));
        float d0 = S.c0 * aS - q.e0 * S.A;
        float d1 = S.c1 * aS - q.e1 * S.A;
        float d2 = S.c2 * aS - q.e2 * S.A;
        float dd = d0 * d0 + d1 * d1 + d2 * d2;
        bool may_close = cap <= 0 || count < cap - 1;
        if (may_close && g2 * (S.A * S.A) < dd) {
            gen_close<WRITE>(S, count, o, r, step, l_step);
        } else {
            float w = S.T * q.at;
            S.c0 = fmaf(w, q.c.x, S.c0);
            S.c1 = fmaf(w, q.c.y, S.c1);
            S.c2 = fmaf(w, q.c.z, S.c2);
            S.A += w;
            S.T *= q.Te;
            S.lT += q.lg;
            S.kb = k + 1;
            if (!q.transparent) S.kbt = k + 1;
        }
    }
    if (!S.open && !q.transparent) {
        S.open = 1;
        S.kf = k;
        S.kb = S.kbt = k + 1;
        S.c0 = q.c.x * q.at;
        S.c1 = q.c.y * q.at;
        S.c2 = q.c.z * q.at;
        S.A = q.at;
        S.T = q.Te;
        S.lT = q.lg;
    }
}

// One pass of the segmenter over samples [k0, k1) at threshold gamma.
// Returns the supersegment count.  With EARLY the pass stops as soon as the
// count exceeds `limit` (its outcome "more than limit" is then decided).
// cap > 0 saturates after cap-1 closes (fixed-threshold mode).
template <typename VT, bool WRITE, bool EARLY = !WRITE>
__device__ int gen_pass(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int k0,
                        int k1, const float4* tf, int entries, float gamma, int cap, int limit, const GenOut& o,
                        int* n_opaque_out)
{
    const float g2 = gamma * gamma;
    GenSeg S;
    gen_seg_init(S);
    int count = 0, n_opaque = 0;
    const bool unit = (l_step == 1.0f);
    for (int k = k0; k < k1; ++k) {
        const GenSample q = gen_prep(gen_sample<VT>(data, g, r, step, k, tf, entries), l_step, unit);
        n_opaque += q.transparent ? 0 : 1;
        gen_step<WRITE>(S, count, o, r, step, l_step, g2, cap, k, q);
        if (EARLY && count > limit) break;
    }
    if (S.open) gen_close<WRITE>(S, count, o, r, step, l_step);
    if (n_opaque_out) *n_opaque_out = n_opaque;
    return count;
}

// One counting scan over samples [k0, k1) carrying NC segmenter states
// (thresholds g[]): the sample (position, trilinear taps, classification) is
// computed once and fed to every state.  A state freezes once its count
// exceeds `limit`; the scan ends when all are frozen.  n_opaque counts the
// non-transparent samples seen (complete only if the scan ran to the end).
template <typename VT, int NC>
__device__ void gen_scan(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int k0, int k1,
                         const float4* tf, int entries, const float* gam, int limit, int* counts, int* n_opaque_out)
{
    GenSeg S[NC];
    int cnt[NC];
    float g2[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        gen_seg_init(S[c]);
        cnt[c] = 0;
        g2[c] = gam[c] * gam[c];
    }
    GenOut none{nullptr, nullptr, 0, 0, 0};
    const bool unit = (l_step == 1.0f);
    int n_opaque = 0;
    for (int k = k0; k < k1; ++k) {
        const GenSample q = gen_prep(gen_sample<VT>(data, g, r, step, k, tf, entries), l_step, unit);
        n_opaque += q.transparent ? 0 : 1;
        bool live = false;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            if (cnt[j] <= limit) {
                gen_step<false>(S[j], cnt[j], none, r, step, l_step, g2[j], 0, k, q);
                live |= cnt[j] <= limit;
            }
        }
        if (!live) break;
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        if (S[j].open && cnt[j] <= limit) gen_close<false>(S[j], cnt[j], none, r, step, l_step);
        counts[j] = cnt[j];
    }
    if (n_opaque_out) *n_opaque_out = n_opaque;
}

// Threshold for one brick-ray and the count it yields.  The bisection runs
// two levels per scan (midpoint m and both next-level midpoints) and replays
// the sequential decisions, which it reproduces exactly.
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
    int level = 0;
    while (level < P.iters) {
        float m = 0.5f * (lo + hi);
        if (level + 2 <= P.iters) {
            float g3[3] = { m, 0.5f * (lo + m), 0.5f * (m + hi) };
            int c3[3];
            int n_opaque = 0;
            gen_scan<VT, 3>(data, g, r, step, l_step, k0, k1, tf, entries, g3, P.max_n, c3, &n_opaque);
            // every supersegment starts at a non-transparent sample, so a run
            // with at most N of them is feasible at every threshold: all
            // halvings move the upper bracket
            if (level == 0 && c3[0] <= P.max_n && c3[1] <= P.max_n && n_opaque <= P.max_n) {
                hi = ldexpf(P.gmax, -P.iters);
                hi_count = -1;
                break;
            }
            if (c3[0] <= P.max_n) {
                hi = m;
                hi_count = c3[0];
                if (c3[1] <= P.max_n) {
                    hi = g3[1];
                    hi_count = c3[1];
                } else {
                    lo = g3[1];
                }
            } else {
                lo = m;
                if (c3[2] <= P.max_n) {
                    hi = g3[2];
                    hi_count = c3[2];
                } else {
                    lo = g3[2];
                }
            }
            level += 2;
        } else {
            int c1[1];
            gen_scan<VT, 1>(data, g, r, step, l_step, k0, k1, tf, entries, &m, P.max_n, c1, nullptr);
            if (c1[0] <= P.max_n) {
                hi = m;
                hi_count = c1[0];
            } else {
                lo = m;
            }
            level += 1;
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

// ---------------------------------------------------------------- learned threshold
//
// The regressor of the learned path needs per brick-ray features: a 64-bin
// histogram of the sample opacities (bin j: a in (j/64, (j+1)/64], the opacity
// from the transfer function in the same fixed-order fp32 as the oracle, so
// bins agree exactly), the number of non-transparent samples and the count at
// the smallest threshold the bisection can return (saturating at N+1).

__device__ inline float tf_alpha_exact(const float4* tf, int entries, float s)
{
    int i;
    float w;
    tf_coord(s, entries, i, w);
    return lerp_exact(tf[i].w, tf[i + 1].w, w);
}

template <typename VT>
__global__ __launch_bounds__(256) void features_kernel(GenParams P, GenBricks B, LearnBufs Lb)
{
    __shared__ float4 tf_s[VDI_MAX_TF];
    __shared__ uint16_t hs[64][256];
    for (int i = threadIdx.x; i < P.tf_entries; i += blockDim.x) tf_s[i] = P.tf[i];
    for (int j = 0; j < 64; ++j) hs[j][threadIdx.x] = 0;
    __syncthreads();

    const GenBrick& br = B.b[blockIdx.z];
    const int brick = B.first + blockIdx.z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (x >= P.cam.width || y >= P.cam.height) return;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;
    const size_t ray = (size_t)brick * npix + (uint32_t)y * (uint32_t)P.cam.width + (uint32_t)x;

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

    const float gmin = ldexpf(P.gmax, -P.iters);
    const float g2 = gmin * gmin;
    const bool unit = (P.l_step == 1.0f);
    GenOut none{nullptr, nullptr, 0, 0, 0};
    GenSeg S;
    gen_seg_init(S);
    int count = 0, m = 0;
    for (int k = k0; k < k1; ++k) {
        float t = sample_t(r, k, P.step);
        float p[3] = { sample_coord(r, t, 0), sample_coord(r, t, 1), sample_coord(r, t, 2) };
        float sv = trilinear<VT>(data, g, p);
        float a32 = tf_alpha_exact(tf_s, P.tf_entries, sv);
        if (a32 > 0.0f) {
            int j = (int)ceilf(64.0f * a32) - 1;
            j = j > 63 ? 63 : (j < 0 ? 0 : j);
            hs[j][threadIdx.x] += 1;
            ++m;
        }
        if (count <= P.max_n) {
            const GenSample q = gen_prep(tf_lookup(tf_s, P.tf_entries, sv), P.l_step, unit);
            gen_step<false>(S, count, none, r, P.step, P.l_step, g2, 0, k, q);
        }
    }
    if (S.open && count <= P.max_n) gen_close<false>(S, count, none, r, P.step, P.l_step);
    Lb.nnt[ray] = m;
    Lb.cmax[ray] = count;
    uint32_t* hrow = (uint32_t*)(Lb.hist + ray * 64);
    for (int j = 0; j < 64; j += 2) {
        float f0 = (float)hs[j][threadIdx.x] / Lb.s_ref;
        float f1 = (float)hs[j + 1][threadIdx.x] / Lb.s_ref;
        hrow[j / 2] = (uint32_t)bf16_bits(f0) | ((uint32_t)bf16_bits(f1) << 16);
    }
}

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

// Generation at the regressed threshold, with the acceptance test; rays
// that fail it are queued (per brick) for the plain bisection.
template <typename VT>
__global__ __launch_bounds__(256) void learned_kernel(GenParams P, GenBricks B, LearnBufs Lb)
{
    __shared__ float4 tf_s[VDI_MAX_TF];
    for (int i = threadIdx.x; i < P.tf_entries; i += blockDim.x) tf_s[i] = P.tf[i];
    __syncthreads();

    const GenBrick& br = B.b[blockIdx.z];
    const int brick = B.first + blockIdx.z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (x >= P.cam.width || y >= P.cam.height) return;
    const uint32_t pix = (uint32_t)y * (uint32_t)P.cam.width + (uint32_t)x;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;
    const size_t ray = (size_t)brick * npix + pix;

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

    const float gmin = ldexpf(P.gmax, -P.iters);
    const int m = Lb.nnt[ray];
    GenOut o{br.color, br.depth, pix, npix, (uint32_t)P.max_n};
    float gm = gmin;
    int c = 0;
    int kind = 0;   // 0 kept, 1 all-feasible shortcut, 2 fallback, 3 empty
    if (k1 <= k0 || m == 0) {
        kind = 3;
    } else if (m <= P.max_n) {
        // every threshold is feasible: the bisection would return its lower end
        c = gen_pass<VT, true, false>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gmin, 0, 1 << 30,
                                      o, nullptr);
        kind = 1;
    } else {
        // the regressed threshold and four neighbours (x 2^{-1/2, -1/4, 1/4, 1/2})
        // share one sampling scan; the in-band candidate with the largest
        // count is kept (ties: the one listed first)
        const float lg_hi = log2f(P.gmax), lg_lo = lg_hi - (float)P.iters;
        const float yv = Lb.y[ray];
        const float dl[5] = { 0.0f, -0.25f, 0.25f, -0.5f, 0.5f };
        float g5[5];
        int c5[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) g5[j] = exp2f(fminf(fmaxf(yv + dl[j], lg_lo), lg_hi));
        gen_scan<VT, 5>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, g5, P.max_n, c5, nullptr);
        const int target = min(P.max_n, Lb.cmax[ray]);
        const int lo = target - (int)floorf(Lb.tol * (float)target + 1e-6f);
        int best = -1;
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if (c5[j] <= P.max_n && c5[j] >= lo && (best < 0 || c5[j] > c5[best])) best = j;
        if (best < 0) {
            kind = 2;
        } else {
            gm = g5[best];
            c = gen_pass<VT, true, false>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gm, 0, 1 << 30,
                                          o, nullptr);
        }
    }
    // every active lane of the wave reaches this point (lanes of pixels
    // outside the image returned at the top and take no part in the ballots)
    const int pos = wave_append(&Lb.fb_count[brick], kind == 2);
    if (kind == 2) Lb.fb_list[(size_t)brick * npix + pos] = (int)pix;
#pragma unroll
    for (int q = 0; q < 4; ++q) wave_append(&Lb.stats[q], kind == q);
    if (kind == 2) return;
    for (int j = c; j < P.max_n; ++j) {
        size_t slot = (size_t)j * npix + pix;
        br.color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        br.depth[slot] = make_float2(0.0f, 0.0f);
    }
    br.count[pix] = c;
    if (br.gamma) br.gamma[pix] = gm;
}

// Plain bisection for the queued rays of each brick.
template <typename VT>
__global__ __launch_bounds__(256) void fallback_kernel(GenParams P, GenBricks B, LearnBufs Lb)
{
    __shared__ float4 tf_s[VDI_MAX_TF];
    for (int i = threadIdx.x; i < P.tf_entries; i += blockDim.x) tf_s[i] = P.tf[i];
    __syncthreads();
    const GenBrick& br = B.b[blockIdx.z];
    const int brick = B.first + blockIdx.z;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint32_t)Lb.fb_count[brick]) return;
    const uint32_t pix = (uint32_t)Lb.fb_list[(size_t)brick * npix + idx];
    const int x = (int)(pix % (uint32_t)P.cam.width), y = (int)(pix / (uint32_t)P.cam.width);

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
    float gm = ldexpf(P.gmax, -P.iters);
    int c = 0;
    GenOut o{br.color, br.depth, pix, npix, (uint32_t)P.max_n};
    if (k1 > k0) {
        gen_search<VT>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, P, gm, c, false);
        c = gen_pass<VT, true>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gm, 0, 1 << 30, o, nullptr);
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
static void launch_learned_t(int phase, const GenParams& P, const GenBricks& B, int nb, const LearnBufs& L,
                             hipStream_t s)
{
    dim3 grid((P.cam.width + 15) / 16, (P.cam.height + 15) / 16, nb);
    if (phase == 0) hipLaunchKernelGGL(features_kernel<VT>, grid, dim3(256), 0, s, P, B, L);
    if (phase == 1) hipLaunchKernelGGL(learned_kernel<VT>, grid, dim3(256), 0, s, P, B, L);
    if (phase == 2) {
        size_t npix = (size_t)P.cam.width * P.cam.height;
        dim3 g2((unsigned)((npix + 255) / 256), 1, nb);
        hipLaunchKernelGGL(fallback_kernel<VT>, g2, dim3(256), 0, s, P, B, L);
    }
}

void launch_learned(int phase, int dtype, const GenParams& P, const GenBricks& B, int nb, const LearnBufs& L,
                    hipStream_t s)
{
    if (dtype == VDI_F16) launch_learned_t<__half>(phase, P, B, nb, L, s);
    else launch_learned_t<float>(phase, P, B, nb, L, s);
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
