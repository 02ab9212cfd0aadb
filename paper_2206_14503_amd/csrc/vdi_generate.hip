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
    float nL;           // samples covered, as a float (kb - kf)
    int kf, kbt;        // first sample, one past the last non-transparent
    bool open;
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
    S.open = false;
}

// Stencil loads of sample k, issued now and blended later.
template <typename VT, bool PAIRED>
__device__ inline Taps gen_fetch(const VT* data, const BrickGeo& g, const Ray& r, float step, int k)
{
    float t = sample_t(r, k, step);
    float p[3] = { sample_coord(r, t, 0), sample_coord(r, t, 1), sample_coord(r, t, 2) };
    return trilinear_fetch<VT, PAIRED>(data, g, p);
}

// Calls body(k, value) for the samples k of [k0, k1) in order until it
// returns false.  The stencil loads run SLOTS samples ahead: SLOTS stencil
// slots in rotation (the loop unrolled by SLOTS), each refilled with the
// sample SLOTS places on right after its blend, so no slot is copied and a
// sample's loads overlap the work on the samples before it.  A load past the
// run re-reads its last sample (every stencil index is clamped to the
// brick's data box, so it stays in bounds).
template <typename VT, bool PAIRED, int SLOTS, typename F>
__device__ inline void for_samples_t(const VT* data, const BrickGeo& g, const Ray& r, float step, int k0, int k1,
                                     F& body)
{
    static_assert(SLOTS == 2 || SLOTS == 3, "two or three stencil slots");
    const int kl = k1 - 1;
    Taps t0 = gen_fetch<VT, PAIRED>(data, g, r, step, k0);
    Taps t1 = gen_fetch<VT, PAIRED>(data, g, r, step, min(k0 + 1, kl));
    Taps t2;
    if (SLOTS == 3) t2 = gen_fetch<VT, PAIRED>(data, g, r, step, min(k0 + 2, kl));
    for (int k = k0;;) {
        float v = trilinear_blend(t0);
        t0 = gen_fetch<VT, PAIRED>(data, g, r, step, min(k + SLOTS, kl));
        if (!body(k, v) || ++k >= k1) break;
        v = trilinear_blend(t1);
        t1 = gen_fetch<VT, PAIRED>(data, g, r, step, min(k + SLOTS, kl));
        if (!body(k, v) || ++k >= k1) break;
        if (SLOTS == 3) {
            v = trilinear_blend(t2);
            t2 = gen_fetch<VT, PAIRED>(data, g, r, step, min(k + SLOTS, kl));
            if (!body(k, v) || ++k >= k1) break;
        }
    }
}

template <typename VT, int SLOTS = 3, typename F>
__device__ inline void for_samples(const VT* data, const BrickGeo& g, const Ray& r, float step, int k0, int k1,
                                   F&& body)
{
    if (k1 <= k0) return;
    if (g.sx2) for_samples_t<VT, true, SLOTS>(data, g, r, step, k0, k1, body);
    else for_samples_t<VT, false, SLOTS>(data, g, r, step, k0, k1, body);
}

__device__ inline void gen_seg_init(GenSeg& S)
{
    S.open = false;
    S.c0 = S.c1 = S.c2 = 0.0f;
    S.A = 0.0f;
    S.T = 1.0f;
    S.lT = 0.0f;
    S.nL = 1.0f;
    S.kf = S.kbt = 0;
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
// opacity.  The state update is written as selects: a closed state's fields
// are don't-cares (its test result is masked by `open`), so every lane runs
// the same instruction stream whatever its decisions.
template <bool WRITE>
__device__ inline void gen_step(GenSeg& S, int& count, const GenOut& o, const Ray& r, float step, float l_step,
                                float g2, int cap, int k, const GenSample& q)
{
    const float aS = 1.0f - hw_exp2(S.lT * hw_rcp(S.nL * l_step));
    const float d0 = S.c0 * aS - q.e0 * S.A;
    const float d1 = S.c1 * aS - q.e1 * S.A;
    const float d2 = S.c2 * aS - q.e2 * S.A;
    const float dd = d0 * d0 + d1 * d1 + d2 * d2;
    const bool may_close = cap <= 0 || count < cap - 1;
    const bool close = S.open & may_close & (g2 * (S.A * S.A) < dd);
    if (WRITE && close) gen_close<true>(S, count, o, r, step, l_step);
    else count += close ? 1 : 0;
    const bool merge = S.open & !close;
    const float w = S.T * q.at;
    S.c0 = merge ? fmaf(w, q.c.x, S.c0) : q.c.x * q.at;
    S.c1 = merge ? fmaf(w, q.c.y, S.c1) : q.c.y * q.at;
    S.c2 = merge ? fmaf(w, q.c.z, S.c2) : q.c.z * q.at;
    S.A = merge ? S.A + w : q.at;
    S.T = merge ? S.T * q.Te : q.Te;
    S.lT = merge ? S.lT + q.lg : q.lg;
    S.nL = merge ? S.nL + 1.0f : 1.0f;
    S.kf = merge ? S.kf : k;
    S.kbt = (merge & q.transparent) ? S.kbt : k + 1;
    S.open = merge | !q.transparent;
}

// One pass of the segmenter over samples [k0, k1) at threshold gamma.
// Returns the supersegment count.  With EARLY the pass stops as soon as the
// count exceeds `limit` (its outcome "more than limit" is then decided).
// cap > 0 saturates after cap-1 closes (fixed-threshold mode).
template <typename VT, bool WRITE, bool EARLY = !WRITE, bool MASK = false>
__device__ int gen_pass(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int k0,
                        int k1, const TfCell* tf, int entries, float gamma, int cap, int limit, const GenOut& o,
                        int* n_opaque_out)
{
    const float g2 = gamma * gamma;
    GenSeg S;
    gen_seg_init(S);
    int count = 0, n_opaque = 0;
    const bool unit = (l_step == 1.0f);
    for_samples<VT>(data, g, r, step, k0, k1, [&](int k, float v) {
        if (MASK && g.own && !owns_sample(g, r, step, k)) {
            // the ray is outside the domain: an open supersegment ends here
            if (S.open) gen_close<WRITE>(S, count, o, r, step, l_step);
            return !(EARLY && count > limit);
        }
        const GenSample q = gen_prep(tf_lookup(tf, entries, v), l_step, unit);
        n_opaque += q.transparent ? 0 : 1;
        gen_step<WRITE>(S, count, o, r, step, l_step, g2, cap, k, q);
        return !(EARLY && count > limit);
    });
    if (S.open) gen_close<WRITE>(S, count, o, r, step, l_step);
    if (n_opaque_out) *n_opaque_out = n_opaque;
    return count;
}

// One counting scan over samples [k0, k1) carrying NC segmenter states
// (thresholds g[]): the sample (position, trilinear taps, classification) is
// computed once and fed to every state.  A state freezes once its count
// exceeds `limit`; the scan ends when all are frozen.  n_opaque counts the
// non-transparent samples seen (complete only if the scan ran to the end).
// kspan (optional) receives the first non-transparent sample seen, one past
// the last one, and whether the scan ran to k1 (1) or stopped early (0).
template <typename VT, int NC, bool MASK = false>
__device__ void gen_scan(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int k0, int k1,
                         const TfCell* tf, int entries, const float* gam, int limit, int* counts, int* n_opaque_out,
                         int* kspan = nullptr)
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
    int kf = k1, ke = k0, kdone = k0;
    // many states: two stencil slots, to keep the states in registers
    for_samples<VT, (NC >= 6 ? 2 : 3)>(data, g, r, step, k0, k1, [&](int k, float v) {
        if (MASK && g.own && !owns_sample(g, r, step, k)) {
            // outside the domain: every open supersegment ends here
            bool live = false;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                if (S[j].open) gen_close<false>(S[j], cnt[j], none, r, step, l_step);
                live |= cnt[j] <= limit;
            }
            if (kspan) kdone = k + 1;
            return live;
        }
        const GenSample q = gen_prep(tf_lookup(tf, entries, v), l_step, unit);
        n_opaque += q.transparent ? 0 : 1;
        if (kspan) {
            kf = q.transparent ? kf : min(kf, k);
            ke = q.transparent ? ke : k + 1;
            kdone = k + 1;
        }
        // a frozen state (count above limit) keeps stepping: its count only
        // grows, so its outcome stays decided
        bool live = false;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            gen_step<false>(S[j], cnt[j], none, r, step, l_step, g2[j], 0, k, q);
            live |= cnt[j] <= limit;
        }
        return live;
    });
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        if (S[j].open && cnt[j] <= limit) gen_close<false>(S[j], cnt[j], none, r, step, l_step);
        counts[j] = cnt[j];
    }
    if (n_opaque_out) *n_opaque_out = n_opaque;
    if (kspan) {
        kspan[0] = kf;
        kspan[1] = ke;
        kspan[2] = kdone == k1 ? 1 : 0;
    }
}

// Levels of the bisection the first scan speculates on.
constexpr int kGeoLevels = 6;

// The bisection's levels after `level` from bracket [lo, hi]: two per scan
// (the midpoint m and both of the next level's), the last alone if one is
// left.  hi_count receives the count at the final hi where a scan measured it.
template <typename VT, bool MASK = false>
__device__ __forceinline__ void search_rest(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step,
                                            int k0, int k1, const TfCell* tf, int entries, const GenParams& P,
                                            float& lo, float& hi, int level, int& hi_count)
{
    while (level < P.iters) {
        float m = 0.5f * (lo + hi);
        if (level + 2 <= P.iters) {
            float g3[3] = { m, 0.5f * (lo + m), 0.5f * (m + hi) };
            int c3[3];
            gen_scan<VT, 3, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, g3, P.max_n, c3, nullptr);
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
            gen_scan<VT, 1, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, &m, P.max_n, c1, nullptr);
            if (c1[0] <= P.max_n) {
                hi = m;
                hi_count = c1[0];
            } else {
                lo = m;
            }
            level += 1;
        }
    }
}


// Threshold for one brick-ray and the count it yields.  While every level is
// feasible, the bisection's midpoints are gmax/2, gmax/4, ...: the first scan
// carries states at the first kGeoLevels of them and replays the decisions up
// to (and including) the first infeasible one.  The remaining levels run two
// per scan (the midpoint m and both next-level midpoints).  Both reproduce
// the sequential decisions exactly.
template <typename VT, bool MASK = false>
__device__ __forceinline__ void gen_search(const VT* data, const BrickGeo& g, const Ray& r, float step, float l_step, int& k0,
                           int& k1, const TfCell* tf, int entries, const GenParams& P, float& gamma_out,
                           int& count_out, bool need_count)
{
    GenOut none{nullptr, nullptr, 0, 0, 0};
    if (P.mode == VDI_TAU_FIXED) {
        gamma_out = P.tau;
        count_out = need_count ? gen_pass<VT, false, true, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, P.tau,
                                                     P.max_n, 1 << 30, none, nullptr)
                               : -1;
        return;
    }
    float lo = 0.0f, hi = P.gmax;
    int hi_count = -1;
    int level = 0;
    if (P.mode == VDI_TAU_BISECT_SEQ) {
        // one midpoint per pass, in the order the halvings visit them
        for (; level < P.iters; ++level) {
            float m = 0.5f * (lo + hi);
            int c1[1];
            gen_scan<VT, 1, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, &m, P.max_n, c1, nullptr);
            if (c1[0] <= P.max_n) {
                hi = m;
                hi_count = c1[0];
            } else {
                lo = m;
            }
        }
    } else {
        float gg[kGeoLevels];
        int cg[kGeoLevels];
#pragma unroll
        for (int l = 0; l < kGeoLevels; ++l) gg[l] = ldexpf(P.gmax, -(l + 1));
        int n_opaque = 0;
        int ks[3];
        gen_scan<VT, kGeoLevels, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, gg, P.max_n, cg, &n_opaque, ks);
        // later passes (and the caller's write) cover [first non-transparent
        // sample, one past the last): before it every state stays closed and
        // untouched, after it neither the count nor the stored lists change
        // (a trailing close emits the supersegment the end would emit)
        if (n_opaque > 0) {
            k0 = ks[0];
            if (ks[2]) k1 = ks[1];
        }
        if (n_opaque <= P.max_n) {
            // every supersegment starts at a non-transparent sample, so a run
            // with at most N of them is feasible at every threshold: all
            // halvings move the upper bracket
            gamma_out = ldexpf(P.gmax, -P.iters);
            count_out = -1;
            if (need_count)
                count_out = gen_pass<VT, false, true, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, gamma_out, 0, 1 << 30,
                                                none, nullptr);
            return;
        }
        const int lim = kGeoLevels < P.iters ? kGeoLevels : P.iters;
        for (int l = 0; l < lim; ++l) {
            const float m = 0.5f * (lo + hi);   // == gg[l] while every level so far was feasible
            ++level;
            if (cg[l] <= P.max_n) {
                hi = m;
                hi_count = cg[l];
            } else {
                lo = m;
                break;
            }
        }
    }
    search_rest<VT, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, P, lo, hi, level, hi_count);
    gamma_out = hi;
    if (need_count && hi_count < 0)
        hi_count = gen_pass<VT, false, true, MASK>(data, g, r, step, l_step, k0, k1, tf, entries, hi, 0, 1 << 30, none,
                                       nullptr);
    count_out = hi_count;
}

// kind: 0 = search + regular write, 1 = search only (count + gamma), 2 = compact write
template <typename VT, int KIND, bool MASK>
__global__ __launch_bounds__(256) void gen_kernel(GenParams P, GenBricks B)
{
    extern __shared__ TfCell tf_s[];   // P.tf_entries - 1 cells, sized at launch
    tf_stage(tf_s, P.tf, P.tf_entries, threadIdx.x, blockDim.x);
    __syncthreads();

    const GenBrick& br = B.b[blockIdx.z];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (x >= P.cam.width || y >= P.cam.height) return;
    const uint32_t pix = (uint32_t)y * (uint32_t)P.cam.width + (uint32_t)x;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;

    BrickGeo g = make_geo(P.n, br.dlo, br.ddim);
    if (MASK) {
        g.own = br.owner;
        g.rank = br.rank;
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
        if (k1 > k0) gen_search<VT, MASK>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, P, gm, c, true);
        if (MASK && c > P.max_n) {
            // more domain entries than N: the list keeps the first N
            atomicOr(P.status, 4);
            c = P.max_n;
        }
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
            gen_pass<VT, true, false, MASK>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gm, cap, 1 << 30, o,
                               nullptr);
        }
        return;
    }
    // KIND 0: search, then write the regular slots and zero the rest
    float gm = empty_gamma;
    int c = 0;
    GenOut o{br.color, br.depth, pix, npix, (uint32_t)P.max_n};
    if (k1 > k0) {
        gen_search<VT, MASK>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, P, gm, c, false);
        int cap = P.mode == VDI_TAU_FIXED ? P.max_n : 0;
        c = gen_pass<VT, true, false, MASK>(data, g, r, P.step, P.l_step, k0, k1, tf_s, P.tf_entries, gm, cap, 1 << 30, o,
                               nullptr);
    }
    for (int j = c; j < P.max_n; ++j) {
        size_t slot = (size_t)j * npix + pix;
        br.color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        br.depth[slot] = make_float2(0.0f, 0.0f);
    }
    // more domain entries than N (owner maps): the list keeps the first N
    if (MASK && c > P.max_n) atomicOr(P.status, 4);
    br.count[pix] = c < P.max_n ? c : P.max_n;
    if (br.gamma) br.gamma[pix] = gm;
}

// Dynamic LDS of the generation kernels: the transfer function's cells, and
// for bricks whose data box exceeds one XCD's 4 MB L2, at least a third of a
// CU's 160 KB, which holds each CU to two 256-thread blocks (two waves per
// SIMD).  The registers allow three: on bricks that fit in L2 (64^3 volumes)
// three were 20% faster; on 64 MB bricks 2% faster on an FHD frame but 12%
// slower on a grazing view, where more resident waves evict each other's
// stencil lines.
template <typename VT>
static size_t tf_lds(const GenParams& P, const GenBricks& B, int nb)
{
    const size_t cells = sizeof(TfCell) * (size_t)(P.tf_entries - 1);
    size_t box = 0;
    for (int i = 0; i < nb; ++i)
        box = std::max(box, sizeof(VT) * (size_t)B.b[i].ddim[0] * B.b[i].ddim[1] * B.b[i].ddim[2]);
    const size_t two_blocks = (size_t)160 * 1024 / 3 + 1024;
    return box > ((size_t)4 << 20) ? std::max(cells, two_blocks) : cells;
}

template <typename VT>
static void launch_gen(int kind, const GenParams& P, const GenBricks& B, int nb, hipStream_t s)
{
    dim3 grid((P.cam.width + 15) / 16, (P.cam.height + 15) / 16, nb);
    bool mask = false;
    for (int i = 0; i < nb; ++i) mask |= B.b[i].owner != nullptr;
    const size_t lds = tf_lds<VT>(P, B, nb);
    if (mask) {
        if (kind == 0) hipLaunchKernelGGL((gen_kernel<VT, 0, true>), grid, dim3(256), lds, s, P, B);
        if (kind == 1) hipLaunchKernelGGL((gen_kernel<VT, 1, true>), grid, dim3(256), lds, s, P, B);
        if (kind == 2) hipLaunchKernelGGL((gen_kernel<VT, 2, true>), grid, dim3(256), lds, s, P, B);
        return;
    }
    if (kind == 0) hipLaunchKernelGGL((gen_kernel<VT, 0, false>), grid, dim3(256), lds, s, P, B);
    if (kind == 1) hipLaunchKernelGGL((gen_kernel<VT, 1, false>), grid, dim3(256), lds, s, P, B);
    if (kind == 2) hipLaunchKernelGGL((gen_kernel<VT, 2, false>), grid, dim3(256), lds, s, P, B);
}

void launch_generate(int kind, int dtype, const GenParams& P, const GenBricks& B, int nb, hipStream_t s)
{
    if (dtype == VDI_F16) launch_gen<__half>(kind, P, B, nb, s);
    else launch_gen<float>(kind, P, B, nb, s);
}

// ---------------------------------------------------------------- learned threshold
//
// The regressor of the learned path reads per brick-ray features: a 64-bin
// histogram of the sample opacities (bin j: a in (j/64, (j+1)/64], the opacity
// from the transfer function in the same fixed-order fp32 as the oracle, so
// bins agree exactly).  On the generation path the feature pass is also the
// bisection's first scan (the states at gmax/2 ... gmax/2^6 of the all-feasible
// path): the regressed threshold then steers the scans that settle the
// remaining levels, and every ray ends with the bisection's own result.

// Writes a finished list's unused slots, count and threshold.
__device__ inline void finish_list(const GenBrick& br, uint32_t pix, uint32_t npix, int max_n, int c, float gm)
{
    for (int j = c; j < max_n; ++j) {
        size_t slot = (size_t)j * npix + pix;
        br.color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        br.depth[slot] = make_float2(0.0f, 0.0f);
    }
    br.count[pix] = c;
    if (br.gamma) br.gamma[pix] = gm;
}

struct RayRun {
    Ray r;
    int k0, k1;
};

// A listed ray of the learned path: its samples from the first to the last
// non-transparent one, as the feature scan found them (before that span every
// segmenter state stays closed and untouched, after it neither a count nor a
// stored list changes).
__device__ inline RayRun listed_ray(const GenParams& P, const LearnBufs& Lb, size_t ray, int x, int y)
{
    RayRun q;
    q.r = make_ray(P.cam, x, y);
    const int2 sp = Lb.span[ray];
    q.k0 = sp.x;
    q.k1 = sp.y;
    return q;
}

// Slot of pixel (x, y) in the launch order of the 2D generation kernels
// (16x16 blocks, four 8x8 wavefront tiles each), and back.
__device__ inline uint32_t slot_of(int x, int y, int gx)
{
    const uint32_t blk = (uint32_t)(y >> 4) * (uint32_t)gx + (uint32_t)(x >> 4);
    const uint32_t wave = (uint32_t)(((y >> 3) & 1) * 2 + ((x >> 3) & 1));
    const uint32_t lane = (uint32_t)((y & 7) * 8 + (x & 7));
    return (blk << 8) + wave * 64u + lane;
}

__device__ inline void pixel_of_slot(uint32_t slot, int gx, int& x, int& y)
{
    const uint32_t blk = slot >> 8, t = slot & 255u, wave = t >> 6, lane = t & 63u;
    x = (int)((blk % (uint32_t)gx) * 16u + (wave & 1u) * 8u + (lane & 7u));
    y = (int)((blk / (uint32_t)gx) * 16u + (wave >> 1) * 8u + (lane >> 3));
}

// Rays of brick `brick` on list q: [begin, end) of Lb.qlist + q * lstride.
struct ListSpan {
    const int* list;
    uint32_t begin, end;
};

__device__ inline ListSpan list_span(const LearnBufs& Lb, int q, int brick, int nb_total, uint32_t npix)
{
    const uint32_t* off = Lb.qoff + (size_t)q * ((size_t)nb_total * Lb.nblk + 1);
    ListSpan s;
    s.list = Lb.qlist + (size_t)q * (size_t)nb_total * npix;
    s.begin = off[(size_t)brick * Lb.nblk];
    s.end = off[(size_t)(brick + 1) * Lb.nblk];
    return s;
}

// Feature pass.  SEARCH (generation): the sampling scan also carries the
// bisection's first scan (kGeoLevels states on the all-feasible path, as the
// plain search's) and keeps the bracket its decisions leave; empty lists are
// finished here, lists with at most N non-transparent samples go on the
// all-feasible list, the others on the regressor's list.  Without SEARCH
// (features only): the count at the smallest threshold instead.
template <typename VT, bool SEARCH>
__global__ __launch_bounds__(256) void features_kernel(GenParams P, GenBricks B, LearnBufs Lb)
{
    extern __shared__ TfCell tf_s[];   // P.tf_entries - 1 cells, sized at launch
    // bins 2i and 2i+1 of a lane share one 32-bit word (low and high half), so
    // consecutive lanes update consecutive words (no bank conflicts)
    __shared__ uint32_t hs[32][256];
    tf_stage(tf_s, P.tf, P.tf_entries, threadIdx.x, blockDim.x);
    for (int j = 0; j < 32; ++j) hs[j][threadIdx.x] = 0u;
    __syncthreads();

    const GenBrick& br = B.b[blockIdx.z];
    const int brick = B.first + blockIdx.z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    const uint32_t blk = blockIdx.y * gridDim.x + blockIdx.x;
    const size_t slot = (size_t)brick * ((size_t)Lb.nblk << 8) + ((size_t)blk << 8) + threadIdx.x;
    if (x >= P.cam.width || y >= P.cam.height) {
        if (Lb.kind) Lb.kind[slot] = 0;
        return;
    }
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;
    const size_t ray = (size_t)brick * npix + (uint32_t)y * (uint32_t)P.cam.width + (uint32_t)x;

    const BrickGeo g = make_geo(P.n, br.dlo, br.ddim);
    const VT* data = (const VT*)br.data;
    Ray r = make_ray(P.cam, x, y);
    int ns = ray_samples(r, P.step);
    int k0 = 0, k1 = 0;
    if (ns > 0) owned_run(r, P.step, ns, P.n, br.lo, br.hi, k0, k1);

    const float gmin = ldexpf(P.gmax, -P.iters);
    const bool unit = (P.l_step == 1.0f);
    GenOut none{nullptr, nullptr, 0, 0, 0};
    constexpr int NS = SEARCH ? kGeoLevels : 1;
    GenSeg S[NS];
    int cnt[NS];
    float g2[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        gen_seg_init(S[c]);
        cnt[c] = 0;
        const float gc = SEARCH ? ldexpf(P.gmax, -(c + 1)) : gmin;
        g2[c] = gc * gc;
    }
    int m = 0;
    int kf = k1, ke = k0;
    bool live = true;   // SEARCH: some state's count is still at most N
    for_samples<VT, (SEARCH ? 2 : 3)>(data, g, r, P.step, k0, k1, [&](int k, float v) {
        const float4 cs = tf_lookup(tf_s, P.tf_entries, v);
        const float a32 = cs.w;   // the transfer function's opacity, as in the histogram's definition
        kf = a32 > 0.0f ? min(kf, k) : kf;
        ke = a32 > 0.0f ? k + 1 : ke;
        if (a32 > 0.0f) {
            int j = (int)ceilf(64.0f * a32) - 1;
            j = j > 63 ? 63 : (j < 0 ? 0 : j);
            hs[j >> 1][threadIdx.x] += (j & 1) ? 0x10000u : 1u;
            ++m;
        }
        if (SEARCH) {
            // every state steps while one is live (a frozen one's count only
            // grows, its decision stays made); once all are frozen, where the
            // plain search's scan ends, only the histogram goes on
            if (live) {
                const GenSample q = gen_prep(cs, P.l_step, unit);
                live = false;
#pragma unroll
                for (int c = 0; c < NS; ++c) {
                    gen_step<false>(S[c], cnt[c], none, r, P.step, P.l_step, g2[c], 0, k, q);
                    live |= cnt[c] <= P.max_n;
                }
            }
        } else if (cnt[0] <= P.max_n) {
            const GenSample q = gen_prep(cs, P.l_step, unit);
            gen_step<false>(S[0], cnt[0], none, r, P.step, P.l_step, g2[0], 0, k, q);
        }
        return true;
    });
#pragma unroll
    for (int c = 0; c < NS; ++c)
        if (S[c].open && cnt[c] <= P.max_n) gen_close<false>(S[c], cnt[c], none, r, P.step, P.l_step);
    Lb.nnt[ray] = m;
    if (!SEARCH) Lb.cmax[ray] = cnt[0];
    size_t row = ray;
    if (SEARCH) {
        // empty lists are finished here; lists with at most N non-transparent
        // samples (every threshold feasible) go on the list of writes at the
        // smallest threshold, the others on the regressor's list with the
        // first scan's bracket (both counted per 256-slot block); the served
        // rays' histogram rows are compacted per brick in order of arrival
        const uint32_t pix = (uint32_t)(ray - (size_t)brick * npix);
        const bool empty = k1 <= k0 || m == 0;
        const bool served = !empty && m > P.max_n;
        const bool shortcut = !empty && !served;
        Lb.kind[slot] = served ? (uint8_t)(1 + Q_SERVED) : (shortcut ? (uint8_t)(1 + Q_SHORT) : (uint8_t)0);
        const int nb_total = B.total;
        wave_count(&Lb.qcnt[(size_t)Q_SERVED * nb_total * Lb.nblk + (size_t)brick * Lb.nblk + blk], served);
        wave_count(&Lb.qcnt[(size_t)Q_SHORT * nb_total * Lb.nblk + (size_t)brick * Lb.nblk + blk], shortcut);
        wave_append(&Lb.stats[LEARN_EMPTY], empty);
        const int pos = wave_append(&Lb.hist_count[brick], served);
        if (empty) finish_list(br, pix, npix, P.max_n, 0, gmin);
        else Lb.span[ray] = make_int2(kf, ke);
        if (!served) return;
        // the first scan's decisions, up to and including the first infeasible level
        float lo = 0.0f, hi = P.gmax;
        int level = 0;
        const int lim = kGeoLevels < P.iters ? kGeoLevels : P.iters;
#pragma unroll
        for (int l = 0; l < NS; ++l) {
            if (l < lim && (l == 0 || lo == 0.0f)) {
                const float mid = 0.5f * (lo + hi);
                ++level;
                if (cnt[l] <= P.max_n) hi = mid;
                else lo = mid;
            }
        }
        Lb.level[ray] = level;
        Lb.bracket[ray] = make_float2(lo, hi);
        Lb.hist_list[(size_t)brick * npix + pos] = (int)pix;
        row = (size_t)brick * npix + (size_t)pos;
    }
    uint32_t* hrow = (uint32_t*)(Lb.hist + row * 64);
    for (int j = 0; j < 64; j += 2) {
        const uint32_t pair = hs[j >> 1][threadIdx.x];
        float f0 = (float)(pair & 0xffffu) / Lb.s_ref;
        float f1 = (float)(pair >> 16) / Lb.s_ref;
        hrow[j / 2] = (uint32_t)bf16_bits(f0) | ((uint32_t)bf16_bits(f1) << 16);
    }
}

// Levels of the bisection the regressed threshold's scan speculates on.
constexpr int kPredLevels = 5;

// The rest of a served ray's bisection.  From the first scan's bracket, one
// scan carries the midpoints of the next levels along the path toward the
// regressed threshold 2^y (predicted feasible iff the midpoint is at least
// it), and its decisions are replayed up to the first one the prediction got
// wrong; any levels left run as in the plain search, then the write at the
// result.  The result is the bisection's whatever y is.
template <typename VT>
__global__ __launch_bounds__(256) void learned_kernel(GenParams P, GenBricks B, LearnBufs Lb)
{
    extern __shared__ TfCell tf_s[];   // P.tf_entries - 1 cells, sized at launch
    tf_stage(tf_s, P.tf, P.tf_entries, threadIdx.x, blockDim.x);
    __syncthreads();

    const GenBrick& br = B.b[blockIdx.z];
    const int brick = B.first + blockIdx.z;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;
    const ListSpan ls = list_span(Lb, Q_SERVED, brick, B.total, npix);
    const BrickGeo g = make_geo(P.n, br.dlo, br.ddim);
    const VT* data = (const VT*)br.data;
    for (uint32_t idx = ls.begin + blockIdx.x * blockDim.x + threadIdx.x; idx < ls.end;
         idx += gridDim.x * blockDim.x) {
        const uint32_t pix = (uint32_t)ls.list[idx];
        const size_t ray = (size_t)brick * npix + pix;
        const int x = (int)(pix % (uint32_t)P.cam.width), y = (int)(pix / (uint32_t)P.cam.width);
        const RayRun q = listed_ray(P, Lb, ray, x, y);
        const float2 br0 = Lb.bracket[ray];
        float lo = br0.x, hi = br0.y;
        int level = Lb.level[ray];
        const float gp = exp2f(Lb.y[ray]);
        float gg[kPredLevels];
        bool pf[kPredLevels];
        int cg[kPredLevels];
        float plo = lo, phi = hi;
#pragma unroll
        for (int l = 0; l < kPredLevels; ++l) {
            const float m = 0.5f * (plo + phi);
            gg[l] = m;
            pf[l] = !(gp > m);
            plo = pf[l] ? plo : m;
            phi = pf[l] ? m : phi;
        }
        const int nl = min(kPredLevels, P.iters - level);
        if (nl > 0) {
            gen_scan<VT, kPredLevels>(data, g, q.r, P.step, P.l_step, q.k0, q.k1, tf_s, P.tf_entries, gg, P.max_n,
                                      cg, nullptr);
            for (int l = 0; l < nl; ++l) {
                const float m = 0.5f * (lo + hi);
                ++level;
                const bool feasible = cg[l] <= P.max_n;
                if (feasible) hi = m;
                else lo = m;
                if (feasible != pf[l]) break;
            }
        }
        wave_append(&Lb.stats[LEARN_KEPT], level >= P.iters);
        wave_append(&Lb.stats[LEARN_REFINED], level < P.iters);
        int hc = -1;
        search_rest<VT>(data, g, q.r, P.step, P.l_step, q.k0, q.k1, tf_s, P.tf_entries, P, lo, hi, level, hc);
        GenOut o{br.color, br.depth, pix, npix, (uint32_t)P.max_n};
        const int c = gen_pass<VT, true, false>(data, g, q.r, P.step, P.l_step, q.k0, q.k1, tf_s, P.tf_entries, hi, 0,
                                                1 << 30, o, nullptr);
        finish_list(br, pix, npix, P.max_n, c < P.max_n ? c : P.max_n, hi);
    }
}

// Lists with at most N non-transparent samples: the bisection's result is the
// smallest threshold (every threshold is feasible), written directly.
template <typename VT>
__global__ __launch_bounds__(256) void shortcut_kernel(GenParams P, GenBricks B, LearnBufs Lb)
{
    extern __shared__ TfCell tf_s[];   // P.tf_entries - 1 cells, sized at launch
    tf_stage(tf_s, P.tf, P.tf_entries, threadIdx.x, blockDim.x);
    __syncthreads();
    const GenBrick& br = B.b[blockIdx.z];
    const int brick = B.first + blockIdx.z;
    const uint32_t npix = (uint32_t)P.cam.width * (uint32_t)P.cam.height;
    const ListSpan ls = list_span(Lb, Q_SHORT, brick, B.total, npix);
    const BrickGeo g = make_geo(P.n, br.dlo, br.ddim);
    const VT* data = (const VT*)br.data;
    const float gmin = ldexpf(P.gmax, -P.iters);
    for (uint32_t idx = ls.begin + blockIdx.x * blockDim.x + threadIdx.x; idx < ls.end;
         idx += gridDim.x * blockDim.x) {
        const uint32_t pix = (uint32_t)ls.list[idx];
        const int x = (int)(pix % (uint32_t)P.cam.width), y = (int)(pix / (uint32_t)P.cam.width);
        const RayRun q = listed_ray(P, Lb, (size_t)brick * npix + pix, x, y);
        GenOut o{br.color, br.depth, pix, npix, (uint32_t)P.max_n};
        const int c = gen_pass<VT, true, false>(data, g, q.r, P.step, P.l_step, q.k0, q.k1, tf_s, P.tf_entries, gmin,
                                                0, 1 << 30, o, nullptr);
        wave_append(&Lb.stats[LEARN_SHORTCUT], true);
        finish_list(br, pix, npix, P.max_n, c, gmin);
    }
}

// Rays of list q in slot order: block b of brick z places its rays at the
// scanned offset of (z, b) plus their rank among the block's slots.
__global__ __launch_bounds__(256) void compact_kernel(int q, int width, int height, int nb_total, LearnBufs Lb)
{
    __shared__ int wsum[4];
    const int brick = blockIdx.y;
    const uint32_t blk = blockIdx.x;
    const int gx = (width + 15) / 16;
    const uint32_t npix = (uint32_t)width * (uint32_t)height;
    const size_t slot = (size_t)brick * ((size_t)Lb.nblk << 8) + ((size_t)blk << 8) + threadIdx.x;
    const bool on = Lb.kind[slot] == (uint8_t)(1 + q);
    const unsigned long long m = __ballot(on);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int rank = __popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) rank += wsum[w];
    if (!on) return;
    const uint32_t* off = Lb.qoff + (size_t)q * ((size_t)nb_total * Lb.nblk + 1);
    const uint32_t pos = off[(size_t)brick * Lb.nblk + blk] + (uint32_t)rank;
    int x, y;
    pixel_of_slot(((uint32_t)blk << 8) + threadIdx.x, gx, x, y);
    Lb.qlist[(size_t)q * (size_t)nb_total * npix + pos] = y * width + x;
}

void launch_compact(int q, const GenParams& P, int nb, const LearnBufs& L, hipStream_t s)
{
    dim3 grid((unsigned)L.nblk, (unsigned)nb);
    hipLaunchKernelGGL(compact_kernel, grid, dim3(256), 0, s, q, P.cam.width, P.cam.height, nb, L);
}

template <typename VT>
static void launch_learned_t(int phase, const GenParams& P, const GenBricks& B, int nb, const LearnBufs& L,
                             hipStream_t s)
{
    dim3 grid((P.cam.width + 15) / 16, (P.cam.height + 15) / 16, nb);
    if (phase == 0) {
        if (L.hist_list) hipLaunchKernelGGL((features_kernel<VT, true>), grid, dim3(256), tf_lds<VT>(P, B, nb), s, P, B, L);
        else hipLaunchKernelGGL((features_kernel<VT, false>), grid, dim3(256), tf_lds<VT>(P, B, nb), s, P, B, L);
        return;
    }
    // list-driven: grid-stride over each brick's span of the list, enough
    // blocks to fill the device whatever the list length turns out to be
    size_t npix = (size_t)P.cam.width * P.cam.height;
    unsigned bx = (unsigned)std::min<size_t>((npix + 255) / 256, (size_t)L.blocks_per_brick);
    dim3 g2(bx, 1, nb);
    if (phase == 1) hipLaunchKernelGGL(learned_kernel<VT>, g2, dim3(256), tf_lds<VT>(P, B, nb), s, P, B, L);
    if (phase == 4) hipLaunchKernelGGL(shortcut_kernel<VT>, g2, dim3(256), tf_lds<VT>(P, B, nb), s, P, B, L);
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
