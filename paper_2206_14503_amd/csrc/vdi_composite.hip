// vdi_composite.hip -- per-pixel k-way depth merge and re-segmentation of
// sub-VDIs (Sec. 5.2, supplementary Algorithm S1).
//
// One lane per pixel, one wavefront per block.  The lane first merges the k
// front-to-back sorted input lists by front depth (ties: lower input index)
// into a merge sequence of (input, slot) pairs kept in LDS.  Every later scan
// replays that sequence and reads the supersegments from the inputs (HBM the
// first time, cache afterwards), with the next element's load issued before
// the current one is processed.
//
// The per-pixel threshold bisection (Sec. 2.4, run again in compositing) is
// evaluated two levels per scan: one scan carries three segmenter states, for
// the midpoint m and for both midpoints of the next level, and the sequential
// decisions are then replayed from their counts.  The result is identical to
// B one-threshold scans, with about half as many scans over the data.
#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

namespace {

constexpr int kWave = 64;

struct CSeg {
    float c0, c1, c2;  // premultiplied colour
    float A;           // accumulated opacity
    float T;           // transmittance
    float lT;          // log2 of the transmittance
    float f, b, bt;    // front, back (incl. trailing gap/transparent), back of last non-transparent
    bool open;
    int count;
};

// An element prepared once per scan and shared by all segmenter states.
struct CElem {
    float f, b;
    float r, g, bl;    // un-premultiplied colour
    float e0, e1, e2;  // per-step premultiplied colour (Eq. 1 operand)
    float at;          // total opacity over its length (Eq. 2)
    float Te;          // 1 - at
    float lg;          // log2(1 - at)
    bool transparent;
};

__device__ inline CElem prep(float4 c, float2 fb, float inv_ref)
{
    CElem e;
    e.f = fb.x;
    e.b = fb.y;
    e.r = c.x;
    e.g = c.y;
    e.bl = c.z;
    e.e0 = c.x * c.w;
    e.e1 = c.y * c.w;
    e.e2 = c.z * c.w;
    e.transparent = (c.w == 0.0f);
    float lg = (fb.y - fb.x) * inv_ref * log2_1m(c.w);   // log2 of (1 - a)^l
    e.lg = lg;
    e.Te = hw_exp2(lg);
    e.at = e.transparent ? 0.0f : one_minus_exp2(lg);
    return e;
}

struct COut {
    float4* color;
    float2* depth;
    uint32_t pix, npix;
    int limit;
};

__device__ inline void seg_reset(CSeg& S)
{
    S.open = false;
    S.count = 0;
    S.c0 = S.c1 = S.c2 = S.A = 0.0f;
    S.T = 1.0f;
    S.lT = 0.0f;
    S.f = S.b = S.bt = 0.0f;
}

template <bool WRITE>
__device__ inline void c_close(CSeg& S, const COut& o, float inv_ref)
{
    if (WRITE && S.count < o.limit) {
        float invA = 1.0f / S.A;
        float len = (S.bt - S.f) * inv_ref;
        float a = one_minus_exp2(S.lT / len);
        size_t slot = (size_t)S.count * o.npix + o.pix;
        o.color[slot] = make_float4(S.c0 * invA, S.c1 * invA, S.c2 * invA, a);
        o.depth[slot] = make_float2(S.f, S.bt);
    }
    ++S.count;
    S.open = false;
}

// Per-step opacity a_S = 1 - 2^(log2(T) / L) of the open supersegment
// extended to depth b, over L = (b - f) / ref.
__device__ inline float seg_alpha(const CSeg& S, float b, float inv_ref)
{
    return 1.0f - hw_exp2(S.lT * hw_rcp((b - S.f) * inv_ref));
}

// Eq. 1 test: gamma < |C a_S / A - e|, evaluated as
// gamma^2 A^2 < |C a_S - e A|^2 (A > 0).
__device__ inline bool c_exceeds(const CSeg& S, float aS, float g2, float e0, float e1, float e2)
{
    float d0 = S.c0 * aS - e0 * S.A, d1 = S.c1 * aS - e1 * S.A, d2 = S.c2 * aS - e2 * S.A;
    return g2 * (S.A * S.A) < d0 * d0 + d1 * d1 + d2 * d2;
}

// The gap's Eq. 1 test (the empty space's operand is zero):
// gamma^2 A^2 < a_S^2 |C|^2.
__device__ inline bool c_exceeds_gap(const CSeg& S, float aS, float g2)
{
    const float c2 = S.c0 * S.c0 + S.c1 * S.c1 + S.c2 * S.c2;
    return g2 * (S.A * S.A) < (aS * aS) * c2;
}

// One element through the segmenter: the empty space before it (a
// transparent stretch, Alg. S1), then the element itself.  a0 is the open
// supersegment's a_S over its current extent (the gap test's), a1 its a_S
// extended to the element's front (the element test's; a1 = a0 where there
// is no gap).  The state update is written as selects; a closed state's
// fields are don't-cares.
template <bool WRITE>
__device__ inline void c_step(CSeg& S, const COut& o, float inv_ref, float g2, int cap, const CElem& e, float a0,
                              float a1)
{
    // gap [S.b, e.f): closes the open supersegment, or extends it.  The
    // conditions use non-short-circuit & so both tests run unconditionally.
    const bool gap = S.open & (e.f > S.b);
    const bool close_g = gap & (cap <= 0 || S.count < cap - 1) & c_exceeds_gap(S, a0, g2);
    if (WRITE && close_g) c_close<true>(S, o, inv_ref);
    else S.count += close_g ? 1 : 0;
    const bool open1 = S.open & !close_g;
    const float b1 = fmaxf(S.b, e.f);   // = e.f after a gap, else S.b (don't-care when closed)
    // the element
    const bool close = open1 & (cap <= 0 || S.count < cap - 1) & c_exceeds(S, a1, g2, e.e0, e.e1, e.e2);
    if (WRITE && close) {
        S.b = b1;
        c_close<true>(S, o, inv_ref);
    } else {
        S.count += close ? 1 : 0;
    }
    const bool merge = open1 & !close;
    const float w = S.T * e.at;
    S.c0 = merge ? fmaf(w, e.r, S.c0) : e.r * e.at;
    S.c1 = merge ? fmaf(w, e.g, S.c1) : e.g * e.at;
    S.c2 = merge ? fmaf(w, e.bl, S.c2) : e.bl * e.at;
    S.A = merge ? S.A + w : e.at;
    S.T = merge ? S.T * e.Te : e.Te;
    S.lT = merge ? S.lT + e.lg : e.lg;
    S.f = merge ? S.f : e.f;
    S.b = e.b;
    S.bt = (merge & e.transparent) ? S.bt : e.b;
    S.open = merge | !e.transparent;
}

struct InLds {
    const float4* color;
    const float2* depth;
    uint32_t stride;   // slot stride: npix (regular) or 1 (compact)
    uint32_t pad;
};

// Per-lane LDS arrays, lane-minor ([row][64]) so consecutive lanes hit
// consecutive banks.  The merge sequence stores one input id per element
// (4 bits when k <= 16, else 8 bits); the slot of each element is recovered
// during a scan from per-input cursors.
struct Lds {
    const InLds* in;   // [k], shared by the block
    uint8_t* seq;      // [seq bytes][64]
    float* front;      // [k][64]  front depth of each input's current element
    float* next;       // [k][64]  front depth of the element after it
    uint32_t* ebase;   // [k][64]  element index of slot 0
    uint8_t* cur;      // [k][64]  cursor (slot of the next element) per input
    uint8_t* cnt;      // [k][64]  list length per input
    bool nib;          // 4-bit ids
};

__device__ inline int seq_bytes(int k, int seq_cap) { return k <= 16 ? (seq_cap + 1) / 2 : seq_cap; }

__device__ inline Lds lds_layout(unsigned char* lds_raw, int k, int seq_cap)
{
    Lds L;
    L.in = (const InLds*)lds_raw;
    unsigned char* q = lds_raw + sizeof(InLds) * kMaxInputs;
    const int sb = (seq_bytes(k, seq_cap) + 3) & ~3;
    L.seq = q;
    q += (size_t)sb * kWave;
    L.front = (float*)q;
    q += (size_t)4 * k * kWave;
    L.next = (float*)q;
    q += (size_t)4 * k * kWave;
    L.ebase = (uint32_t*)q;
    q += (size_t)4 * k * kWave;
    L.cur = q;
    q += (size_t)k * kWave;
    L.cnt = q;
    L.nib = k <= 16;
    return L;
}

struct Src {
    const float4* c;
    const float2* d;
    uint32_t e;
    bool join;   // first element of a list that follows another (depth-disjoint reader)
};

// Sequential reader of a lane's merge sequence (general merge).
struct SeqReader {
    const Lds* L;
    int t;
    int k;
    int i;
    __device__ void reset()
    {
        i = 0;
        for (int r = 0; r < k; ++r) L->cur[r * kWave + t] = 0;
    }
    __device__ Src next()
    {
        uint32_t b = L->seq[(L->nib ? (i >> 1) : i) * kWave + t];
        int r = L->nib ? (int)((i & 1) ? (b >> 4) : (b & 15u)) : (int)b;
        ++i;
        uint32_t s = L->cur[r * kWave + t];
        L->cur[r * kWave + t] = (uint8_t)(s + 1);
        const InLds in = L->in[r];
        return Src{in.color, in.depth, L->ebase[r * kWave + t] + s * in.stride, false};
    }
};

// Reader of a lane's merged list staged in global memory: element i at
// [i * 64 + t], so the 64 lanes of a scan step read consecutive addresses.
struct StageReader {
    const float4* c;
    const float2* d;
    uint32_t t, e;
    __device__ void reset() { e = t; }
    __device__ Src next()
    {
        Src q{c, d, e, false};
        e += kWave;
        return q;
    }
};

// Per-lane LDS of the depth-disjoint path: two words per input.  During
// set-up they hold each list's first front and last back; afterwards its
// count and the element index of its slot 0.
struct CatLds {
    const InLds* in;
    float* a;   // [k][64]
    float* b;   // [k][64]
};

__device__ inline CatLds cat_layout(unsigned char* lds_raw, int k)
{
    CatLds L;
    L.in = (const InLds*)lds_raw;
    L.a = (float*)(lds_raw + sizeof(InLds) * kMaxInputs);
    L.b = L.a + (size_t)k * kWave;
    return L;
}

// Reader of depth-disjoint lists: the non-empty inputs in the order `ord`
// (4-bit input ids, first list in the low bits), each list slot by slot.
struct CatReader {
    CatLds L;
    int t;
    uint64_t ord;
    int ne;        // lists in ord (1..16)
    int li;        // position in ord of the current list
    int s, c;      // slot in it and its count
    uint32_t e, stride;
    const float4* color;
    const float2* depth;
    __device__ void open(int pos)
    {
        // past the last list nothing more is read: the count becomes
        // unreachable (the words read are those of a valid list, unused)
        const bool past = pos >= ne;
        const int r = (int)((ord >> (4 * (past ? 0 : pos))) & 15u);
        li = pos;
        s = 0;
        const int cr = __float_as_int(L.a[r * kWave + t]);
        c = past ? 0x7fffffff : cr;
        e = __float_as_uint(L.b[r * kWave + t]);
        const InLds in = L.in[r];
        stride = in.stride;
        color = in.color;
        depth = in.depth;
    }
    __device__ void reset() { open(0); }
    __device__ Src next()
    {
        Src q{color, depth, e, s == 0 && li > 0};
        if (++s == c) {
            open(li + 1);
        } else {
            e += stride;
        }
        return q;
    }
};

// Validation of the next element of a merged list: finite depths, f < b,
// fronts non-decreasing; where a depth-disjoint reader joins two lists the
// front must increase strictly (equal fronts would merge by input index,
// which the concatenation does not follow).
__device__ inline bool elem_ok(float2 fb, float prev_f, bool join)
{
    return isfinite(fb.x) & isfinite(fb.y) & (fb.x < fb.y) & (join ? fb.x > prev_f : fb.x >= prev_f);
}

// One scan of the merged list carrying NC segmenter states (thresholds g[]).
// Counting scans (WRITE false) freeze a state once its count exceeds
// `limit` and stop when every state is frozen, unless VALIDATE: then every
// element is visited and checked (finite depths, f < b, fronts
// non-decreasing) up to the first violation, which ends the scan and is
// reported in *bad.
// Elements a scan keeps in flight ahead of the one it processes: the staged
// slabs are streamed from memory, where one element ahead leaves a wavefront
// waiting on every load; the other readers gather through the cache.
template <typename R> struct ScanDepth { static constexpr int D = 1; };
template <> struct ScanDepth<StageReader> { static constexpr int D = 4; };

template <int NC, bool WRITE, bool VALIDATE, typename R>
__device__ void c_scan(R rd, int total, float inv_ref, const float* gam, int cap, int limit, const COut& o,
                       int* counts, bool* bad)
{
    constexpr int D = ScanDepth<R>::D;
    CSeg S[NC];
    float g2[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        seg_reset(S[c]);
        g2[c] = gam[c] * gam[c];
    }
    bool ok = true;
    if (total > 0) {
        rd.reset();
        // ring of the next D elements (slot j holds element i0 + j)
        float4 rc[D];
        float2 rf[D];
        bool rj[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            rc[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            rf[j] = make_float2(0.0f, 1.0f);
            rj[j] = false;
            if (j < total) {
                const Src src = rd.next();
                rc[j] = gload(src.c, src.e);
                rf[j] = gload(src.d, src.e);
                rj[j] = src.join;
            }
        }
        float prev_f = -__builtin_inff();
        bool stop = false;
        for (int i0 = 0; i0 < total && !stop; i0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int i = i0 + j;
                if (i < total && !stop) {
                    const float4 cc = rc[j];
                    const float2 fc = rf[j];
                    const bool jc = rj[j];
                    if (i + D < total) {
                        const Src nx = rd.next();
                        rc[j] = gload(nx.c, nx.e);
                        rf[j] = gload(nx.d, nx.e);
                        rj[j] = nx.join;
                    }
                    if (VALIDATE) {
                        ok &= elem_ok(fc, prev_f, jc);
                        prev_f = fc.x;
                    }
                    CElem e = prep(cc, fc, inv_ref);
                    // a_S of every state; the one extended to the element's
                    // front differs only after a gap, which most lanes see in
                    // few steps, so it is computed only where some state of
                    // the lane has one
                    float a0[NC], a1[NC];
                    bool gap = false;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        a0[c] = seg_alpha(S[c], S[c].b, inv_ref);
                        a1[c] = a0[c];
                        gap |= S[c].open & (e.f > S[c].b);
                    }
                    if (gap) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) a1[c] = seg_alpha(S[c], fmaxf(S[c].b, e.f), inv_ref);
                    }
                    // a frozen state (count above limit) keeps stepping: its
                    // count only grows, so its outcome stays decided
                    bool live = false;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        c_step<WRITE>(S[c], o, inv_ref, g2[c], cap, e, a0[c], a1[c]);
                        live |= WRITE || S[c].count <= limit;
                    }
                    // a failed validation decides the pass (its counts are unused)
                    stop = VALIDATE ? !ok : !live;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (S[c].open && (WRITE || S[c].count <= limit)) c_close<WRITE>(S[c], o, inv_ref);
        counts[c] = S[c].count;
    }
    if (VALIDATE) *bad = !ok;
}

}  // namespace


// Pixel of lane t in block `blk` (64 consecutive pixels); false past the image.
__device__ inline bool block_pixel(const CompParams& P, uint32_t blk, int t, uint32_t& p)
{
    p = blk * 64u + (uint32_t)t;
    return p < P.npix;
}

// The input table of a job in LDS (thread t < k writes entry t).
__device__ inline void setup_inputs(const CompParams& P, unsigned char* lds_raw, int t)
{
    InLds* in_tab = (InLds*)lds_raw;
    if (t < P.k) {
        in_tab[t].color = P.in[t].color;
        in_tab[t].depth = P.in[t].depth;
        in_tab[t].stride = P.in[t].compact ? 1u : P.npix;
        in_tab[t].pad = 0;
    }
}

// Output of an invalid pixel: status flag 2, an empty list.
__device__ inline void reject_pixel(const CompParams& P, uint32_t p)
{
    atomicOr(P.status, 2);
    for (int j = 0; j < P.out_n; ++j) {
        size_t slot = (size_t)j * P.npix + p;
        P.out_color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        P.out_depth[slot] = make_float2(0.0f, 0.0f);
    }
    P.out_count[p] = 0;
    if (P.out_gamma) P.out_gamma[p] = 0.0f;
}

// Levels of the compositing bisection its first scan speculates on.  With a
// predicted threshold (the staged general merge) the scan follows the path
// toward it for four levels: a wavefront runs as many scans as its slowest
// lane, and with four levels the predicted path holds for nearly every lane
// of the dense interleaved frames, so the wave's lanes go on together with
// three two-level scans; six levels save a scan on most lanes but their rare
// mispredicted lanes cost their waves two more (measured 8% slower on the
// 16 x 20 frame).  Without one (depth-disjoint lists) it follows the
// all-feasible path gmax/2, gmax/4, ... for six levels: on the FHD frame the
// composited threshold has median 2^-3.9, so the first infeasible level is
// mostly the fifth (6% faster than four levels there, 2% slower on the large
// frame's shorter lists).  The general merge without staging (batches, the
// allocation-free entry point) has no prediction and interleaved lists,
// whose thresholds are large: four levels on the all-feasible path.
template <typename R> struct FirstLevels { static constexpr int L = 4; };
template <> struct FirstLevels<CatReader> { static constexpr int L = 6; };

// The rest of the bisection from bracket [lo, hi] after `level` levels:
// scans of two levels (the midpoint m and both of the next level's), one of
// a single level if one is left, then the write at the result (returned in
// gm).  Returns the count of the written list.
template <typename R>
__device__ int bisect_finish(const CompParams& P, const R& rd0, int total, uint32_t p, float lo, float hi, int level,
                             float& gm)
{
    COut o{P.out_color, P.out_depth, p, P.npix, P.out_n};
    while (level + 2 <= P.iters) {
        float m = 0.5f * (lo + hi);
        float g3[3] = { m, 0.5f * (lo + m), 0.5f * (m + hi) };
        int c3[3];
        c_scan<3, false, false>(rd0, total, P.inv_ref, g3, 0, P.out_n, o, c3, nullptr);
        if (c3[0] <= P.out_n) {
            hi = m;
            if (c3[1] <= P.out_n) hi = g3[1];
            else lo = g3[1];
        } else {
            lo = m;
            if (c3[2] <= P.out_n) hi = g3[2];
            else lo = g3[2];
        }
        level += 2;
    }
    if (level < P.iters) {
        float m = 0.5f * (lo + hi);
        int c1[1];
        c_scan<1, false, false>(rd0, total, P.inv_ref, &m, 0, P.out_n, o, c1, nullptr);
        if (c1[0] <= P.out_n) hi = m;
        else lo = m;
    }
    gm = hi;
    int c1[1];
    c_scan<1, true, false>(rd0, total, P.inv_ref, &gm, 0, 1 << 30, o, c1, nullptr);
    return c1[0];
}

// A finished list's zero-filled tail, count and threshold.
__device__ inline void finish_pixel(const CompParams& P, uint32_t p, int count, float gm)
{
    if (count > P.out_n) count = P.out_n;
    for (int j = count; j < P.out_n; ++j) {
        size_t slot = (size_t)j * P.npix + p;
        P.out_color[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        P.out_depth[slot] = make_float2(0.0f, 0.0f);
    }
    P.out_count[p] = count;
    if (P.out_gamma) P.out_gamma[p] = gm;
}

// Re-segmentation of pixel p's merged list (read through rd, `total`
// elements): pass-through when it fits (R17), else the fixed threshold or the
// bisection, then the zero-filled tail.  The bisection's first scan carries
// the midpoints of its first levels along the path toward `ghat` (a predicted
// threshold; 0 or NaN: the all-feasible path), and its decisions are replayed
// up to the first one the prediction got wrong; later scans carry two levels.
// The result is the bisection's whatever ghat is.  With `defer`, a pixel
// whose first scan left the predicted path before its last level goes on the
// deferral list with its bracket instead (it would keep its wavefront busy
// for more scans than its wave-mates need).  With VALIDATE the first pass
// checks the elements and returns false, with the pixel's output incomplete,
// if one fails.
template <bool VALIDATE, typename R>
__device__ bool resegment(const CompParams& P, const R& rd0, int total, uint32_t p, float ghat = 0.0f,
                          bool defer = false)
{
    COut o{P.out_color, P.out_depth, p, P.npix, P.out_n};
    int count;
    float gm = 0.0f;
    bool bad = false;
    if (total <= P.out_n) {
        // pass-through: the merged list already fits
        R rd = rd0;
        rd.reset();
        float prev_f = -__builtin_inff();
        bool ok = true;
        for (int i = 0; i < total; ++i) {
            Src src = rd.next();
            size_t slot = (size_t)i * P.npix + p;
            const float4 c = gload(src.c, src.e);
            const float2 fb = gload(src.d, src.e);
            if (VALIDATE) {
                ok &= elem_ok(fb, prev_f, src.join);
                prev_f = fb.x;
                if (!ok) break;
            }
            P.out_color[slot] = c;
            P.out_depth[slot] = fb;
        }
        bad = !ok;
        count = total;
    } else if (P.mode == VDI_TAU_FIXED) {
        gm = P.tau;
        int c1[1];
        c_scan<1, true, VALIDATE>(rd0, total, P.inv_ref, &gm, P.out_n, 1 << 30, o, c1, &bad);
        count = c1[0];
    } else {
        float lo = 0.0f, hi = P.gmax;
        int level = 0;
        // first scan: the midpoints of the first levels along the predicted
        // path (predicted feasible iff the midpoint is at least ghat),
        // replayed up to the first level decided otherwise (this scan also
        // validates the list)
        constexpr int L = FirstLevels<R>::L;
        float gg[L];
        bool pf[L];
        int cg[L];
        float plo = 0.0f, phi = P.gmax;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const float m = 0.5f * (plo + phi);
            gg[l] = m;
            pf[l] = !(ghat > m);
            plo = pf[l] ? plo : m;
            phi = pf[l] ? m : phi;
        }
        c_scan<L, false, VALIDATE>(rd0, total, P.inv_ref, gg, 0, P.out_n, o, cg, &bad);
        const int lim = L < P.iters ? L : P.iters;
        for (int l = 0; l < lim && !bad; ++l) {
            const float m = 0.5f * (lo + hi);
            ++level;
            const bool feasible = cg[l] <= P.out_n;
            if (feasible) hi = m;
            else lo = m;
            if (feasible != pf[l]) break;
        }
        if (defer) {
            const bool dfr = !bad && level < lim;
            const int pos = wave_append(P.dq_count, dfr);
            if (dfr) {
                P.dq_pix[pos] = (int)p;
                P.dq_br[pos] = make_float2(lo, hi);
                P.dq_lv[pos] = level;
                return true;
            }
        }
        count = 0;
        if (!bad) count = bisect_finish(P, rd0, total, p, lo, hi, level, gm);
    }
    if (VALIDATE && bad) return false;
    finish_pixel(P, p, count, gm);
    return true;
}

// The depth-disjoint reader's per-list words of pixel p: count and element
// index of slot 0.
__device__ inline void cat_words(const CompParams& P, const CatLds& L, int t, uint32_t p)
{
    for (int r = 0; r < P.k; ++r) {
        const CompInput& in = P.in[r];
        L.a[r * kWave + t] = __int_as_float(in.count[p]);
        L.b[r * kWave + t] = __uint_as_float(in.compact ? in.offset[p] : p);
    }
}

// Depth-disjoint path for pixel p (lane t): when every front of a list lies
// below the first front of the list after it in order of first front, the
// merge by (front, input) is the lists' concatenation in that order, so no
// merge sequence is stored.  The first scan checks this (fronts increasing
// across each join) together with the elements themselves; on a failure it
// returns false and the pixel takes the general merge, which validates it
// and rewrites its whole output.
__device__ bool composite_pixel_cat(const CompParams& P, unsigned char* lds_raw, int t, uint32_t p)
{
    const CatLds L = cat_layout(lds_raw, P.k);
    // ---- counts (validated) and first front of every list
    int total = 0;
    for (int r = 0; r < P.k; ++r) {
        const CompInput& in = P.in[r];
        int c = in.count[p];
        const uint32_t eb = in.compact ? in.offset[p] : p;
        const uint64_t last = in.compact ? (uint64_t)eb + (uint64_t)(c > 0 ? c : 0) : (uint64_t)(c > 0 ? c : 0) * P.npix;
        if (c < 0 || c > in.max_n || last > in.capacity) {
            reject_pixel(P, p);
            return true;
        }
        float f0 = __builtin_inff();
        if (c > 0) {
            f0 = gload(in.depth, eb).x;
            // a non-finite front: the general merge validates (and rejects) the pixel
            if (!isfinite(f0)) return false;
        }
        L.a[r * kWave + t] = f0;   // +inf marks an empty list
        total += c;
    }
    // ---- order by (first front, input)
    uint64_t ord = 0;
    int ne = 0;
    for (int r = 0; r < P.k; ++r) {
        const float fr = L.a[r * kWave + t];
        if (fr == __builtin_inff()) continue;
        int rank = 0;
        for (int q = 0; q < P.k; ++q) {
            const float fq = L.a[q * kWave + t];
            rank += (fq < fr || (fq == fr && q < r)) ? 1 : 0;
        }
        ord |= (uint64_t)r << (4 * rank);
        ++ne;
    }
    // ---- lists that interleave in depth (some front of a list at or above
    // the first front of the list after it): the general merge
    float prev_last = -__builtin_inff();
    for (int i = 0; i < ne; ++i) {
        const int r = (int)((ord >> (4 * i)) & 15u);
        const CompInput& in = P.in[r];
        const uint32_t eb = in.compact ? in.offset[p] : p;
        const int c = in.count[p];
        if (!(L.a[r * kWave + t] > prev_last)) return false;
        prev_last = gload(in.depth, eb + (uint32_t)(c - 1) * (in.compact ? 1u : P.npix)).x;
    }
    // ---- the reader's per-list words: count and element index of slot 0
    cat_words(P, L, t, p);
    CatReader rd{L, t, ord, ne, 0, 0, 0, 0u, 0u, nullptr, nullptr};
    return resegment<true>(P, rd, total, p);
}

// General path for pixel p (lane t): k-way merge of the lists by (front,
// input) into an LDS merge sequence, then re-segmentation replaying it.
__device__ void composite_pixel(const CompParams& P, unsigned char* lds_raw, int t, uint32_t p)
{
    const Lds L = lds_layout(lds_raw, P.k, P.seq_cap);
    const SeqReader rd{&L, t, P.k, 0};

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
        const uint32_t stride = in.compact ? 1u : P.npix;
        L.ebase[r * kWave + t] = eb;
        L.cur[r * kWave + t] = 0;
        L.cnt[r * kWave + t] = (uint8_t)c;
        float f0 = __builtin_inff(), f1 = __builtin_inff();
        if (c > 0) {
            float2 fb = in.depth[eb];
            if (!(fb.x < fb.y) || !isfinite(fb.x) || !isfinite(fb.y)) bad = true;
            f0 = fb.x;
        }
        if (c > 1) f1 = in.depth[eb + stride].x;
        L.front[r * kWave + t] = f0;
        L.next[r * kWave + t] = f1;
        total += c;
    }

    // ---- k-way merge by (front depth, input index).  Each input keeps its
    // current and next front depth in LDS; the load for the one after is
    // issued when an input advances and only needed when it advances again.
    uint32_t pending = 0;
    for (int i = 0; i < total && !bad; ++i) {
        float best = __builtin_inff();
        int rb = -1;
        for (int r = 0; r < P.k; ++r) {
            float f = L.front[r * kWave + t];
            if (f < best) { best = f; rb = r; }
        }
        if (rb < 0) { bad = true; break; }
        if (L.nib) {
            if (i & 1) L.seq[(i >> 1) * kWave + t] = (uint8_t)(pending | ((uint32_t)rb << 4));
            else pending = (uint32_t)rb;
        } else {
            L.seq[i * kWave + t] = (uint8_t)rb;
        }
        const int s = L.cur[rb * kWave + t] + 1;       // slot now at the front of input rb
        L.cur[rb * kWave + t] = (uint8_t)s;
        const int c = L.cnt[rb * kWave + t];
        const InLds inr = L.in[rb];
        const uint32_t eb = L.ebase[rb * kWave + t];
        float nf = L.next[rb * kWave + t];
        if (s < c) {
            // validate the element now at the front: sorted, f < b
            float2 fb = gload(inr.depth, eb + (uint32_t)s * inr.stride);
            if (!(fb.x < fb.y) || !(fb.x >= best) || !isfinite(fb.y)) bad = true;
        }
        float nn = __builtin_inff();
        if (s + 1 < c) nn = gload(inr.depth, eb + (uint32_t)(s + 1) * inr.stride).x;
        L.front[rb * kWave + t] = nf;
        L.next[rb * kWave + t] = nn;
    }
    if (L.nib && (total & 1) && !bad) L.seq[(total >> 1) * kWave + t] = (uint8_t)pending;
    if (bad) {
        reject_pixel(P, p);
        return;
    }
    resegment<false>(P, rd, total, p);
}

// ---------------------------------------------------------------- ordered general merge
//
// The queue of pixels the depth-disjoint path left (or every pixel when k is
// above its limit) is processed in chunks, each by three kernels:
//   1. merge_order_kernel: per tile of 8 entries (consecutive pixels when the
//      queue holds whole blocks) the depths are read in whole lines into LDS
//      and validated; each entry's lists are merged by (front, input) in LDS
//      by a tree of pairwise merges (inputs 2i and 2i+1, then pairs of
//      those, ...), each pairwise merge cut into equal output ranges for its
//      threads by a co-rank search (merge path); the merge order and the
//      depths in that order (the staged depth rows) are written out;
//   2. merge_stage_kernel: per tile, the colours are read in whole lines into
//      LDS and written to the staging slab in merge order, in whole lines
//      (the 8 entries are adjacent columns of a slab row), with the
//      threshold-prediction features;
//   3. composite_staged_kernel: one lane per entry, the re-segmentation scans
//      over the slab (each scan step of a wavefront reads whole rows).
// Per-lane gathers from the inputs' slot-major planes, where a lane's 16
// bytes come with a line its neighbours need at other times, are avoided.

constexpr int kStageTile = 8;     // entries per merge_stage_kernel block
constexpr int kStageBatch = 8;    // loads a merge_stage_kernel thread keeps in flight
constexpr int kStageLanes = 32;   // threads per entry in the merge (256 / kStageTile)
// Threshold prediction: consecutive-operand distances binned by log2 over
// [kPredLo, kPredHi).
constexpr int kPredBins = 64;
constexpr float kPredLo = -8.0f, kPredHi = 1.0f;

// First slot of input r in an entry's row of merged-list capacity (the
// inputs' max_n in order).
__device__ inline int input_base(const CompParams& P, int r)
{
    int b = 0;
    for (int q = 0; q < r; ++q) b += P.in[q].max_n;
    return b;
}

// LDS of merge_stage_kernel besides the tile's elements.
struct StageLds {
    int cntS[kStageTile][kMaxInputs];
    uint32_t ebS[kStageTile][kMaxInputs];
    int preS[kStageTile][kMaxInputs + 1];   // exclusive prefix of the counts (merge positions)
    int baseS[kMaxInputs];
    uint8_t rinS[kOrderedMaxCap];
    int totS[kStageTile];
    int badS[kStageTile];
    uint32_t histS[kStageTile * kPredBins];
};

// LDS row pitches of the order kernel.  The merge's threads read the fronts
// of one entry at scattered element rows, so each entry's fronts (and backs)
// are a row of their own, padded so that the 8 entries' rows start in
// different banks (in rows of the 8 entries' fronts, an entry's fronts would
// all fall in one or two banks).
__host__ __device__ inline int front_pitch(int cap) { return cap + 8; }   // floats
__host__ __device__ inline int merge_pitch(int cap) { return cap + 2; }   // uint16

// Merge of the sorted runs A = src[a0, a1) and B = src[a1, b1) (element rows
// of one entry, whose fronts are F[row]; an element of A precedes one of B on
// equal fronts: A holds the lower inputs) into dst[a0, b1): thread j of `tpm`
// writes the outputs [d0, d1) of the merged run, starting where a co-rank
// search over A places output d0.
__device__ inline void merge_path(const uint16_t* src, uint16_t* dst, const float* F, int a0, int a1, int b1, int j,
                                  int tpm)
{
    const int a = a1 - a0, b = b1 - a1, n = a + b;
    const int d0 = (int)(((long long)j * n) / tpm), d1 = (int)(((long long)(j + 1) * n) / tpm);
    if (d0 >= d1) return;
    // i = how many of the first d0 outputs come from A
    int lo = max(0, d0 - b), hi = min(d0, a);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        // A[mid] before B[d0 - mid - 1]: more than mid outputs come from A
        if (F[src[a0 + mid]] <= F[src[a1 + d0 - mid - 1]]) lo = mid + 1;
        else hi = mid;
    }
    int ia = lo, ib = d0 - lo;
    float fa = ia < a ? F[src[a0 + ia]] : 0.0f;
    float fb = ib < b ? F[src[a1 + ib]] : 0.0f;
    for (int d = d0; d < d1; ++d) {
        const bool take_a = ia < a && (ib >= b || fa <= fb);
        if (take_a) {
            dst[a0 + d] = src[a0 + ia];
            ++ia;
            if (ia < a) fa = F[src[a0 + ia]];
        } else {
            dst[a0 + d] = src[a1 + ib];
            ++ib;
            if (ib < b) fb = F[src[a1 + ib]];
        }
    }
}

// One tile of 8 chunk entries by a block of 256 threads: the counts
// (validated), the inputs' bases and each entry's count prefix.  Entries past
// the queue have no elements (length -1).
__device__ void tile_setup(const CompParams& P, uint32_t e0, uint32_t le0, StageLds& S, uint32_t nq)
{
    const int t = threadIdx.x;
    if (t < kStageTile) S.badS[t] = 0;
    if (t < P.k) {
        const int b = input_base(P, t);
        S.baseS[t] = b;
        for (int s_ = 0; s_ < P.in[t].max_n; ++s_) S.rinS[b + s_] = (uint8_t)t;
    }
    __syncthreads();   // the flags are clear before any count sets one
    if (t < kStageTile * P.k) {
        const int q = t / P.k, r = t - q * P.k;
        const uint32_t le = le0 + q;
        int c = 0;
        uint32_t eb = 0;
        if (le < P.chunk && e0 + le < nq) {
            const uint32_t p = (uint32_t)P.q_list[e0 + le];
            const CompInput& in = P.in[r];
            c = in.count[p];
            eb = in.compact ? in.offset[p] : p;
            const uint64_t last = in.compact ? (uint64_t)eb + (uint64_t)(c > 0 ? c : 0)
                                             : (uint64_t)(c > 0 ? c : 0) * P.npix;
            if (c < 0 || c > in.max_n || last > in.capacity) {
                atomicOr(&S.badS[q], 1);
                c = 0;
            }
        }
        S.cntS[q][r] = c;
        S.ebS[q][r] = eb;
    }
    __syncthreads();
    if (t < kStageTile) {
        const uint32_t le = le0 + t;
        int acc = 0;
        for (int r = 0; r < P.k; ++r) {
            S.preS[t][r] = acc;
            acc += S.cntS[t][r];
        }
        S.preS[t][P.k] = acc;
        S.totS[t] = (le < P.chunk && e0 + le < nq) ? acc : -1;
    }
    __syncthreads();
}

// The tile's elements into LDS, (slot row, entry) with the entry fastest, so
// the 8 entries of a row read whole lines of each slot-major plane; each
// thread keeps kStageBatch loads in flight.  COLOR (the staging kernel):
// the colours at Ec[row * 8 + entry]; else (the order kernel) the fronts and
// backs at Fx/Bk[entry * fp + row].
template <bool COLOR>
__device__ void tile_load(const CompParams& P, const StageLds& S, float4* Ec, float* Fx, float* Bk, int fp)
{
    const int t = threadIdx.x;
    const int n_el = P.seq_cap * kStageTile;
    for (int b0 = 0; b0 < n_el; b0 += 256 * kStageBatch) {
        float4 c[kStageBatch];
        float2 d[kStageBatch];
        bool v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int idx = b0 + t + 256 * u;
            v[u] = false;
            if (idx < n_el) {
                const int q = idx & 7, rs = idx >> 3;
                const int r = S.rinS[rs];
                const int s_ = rs - S.baseS[r];
                if (s_ < S.cntS[q][r]) {
                    const CompInput& in = P.in[r];
                    const uint32_t e = S.ebS[q][r] + (uint32_t)s_ * (in.compact ? 1u : P.npix);
                    if (COLOR) c[u] = gload(in.color, e);
                    else d[u] = gload(in.depth, e);
                    v[u] = true;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            if (v[u]) {
                const int idx = b0 + t + 256 * u;
                if (COLOR) {
                    Ec[idx] = c[u];
                } else {
                    const int at = (idx & 7) * fp + (idx >> 3);
                    Fx[at] = d[u].x;
                    Bk[at] = d[u].y;
                }
            }
        }
    }
    __syncthreads();
}

// Merge order of one tile: validation (finite depths, f < b, fronts
// non-decreasing along each list), then each entry's lists merged in LDS by
// a tree of pairwise merges (at level l the runs are the merged lists of
// 2^(l-1) consecutive inputs; each run pair, lower inputs first, is merged by
// kStageLanes / (number of pairs) threads of its entry).  Writes the merged
// element rows (input base + slot) and the entries' lengths (-1: rejected).
__device__ void merge_order_tile(const CompParams& P, uint32_t e0, uint32_t tile, unsigned char* lds_raw,
                                 StageLds& S, uint32_t nq)
{
    const int t = threadIdx.x;
    const int cap = P.seq_cap;
    const int fp = front_pitch(cap), mp = merge_pitch(cap);
    float* Fx = (float*)lds_raw;                                  // [8][fp] fronts
    float* Bk = Fx + (size_t)kStageTile * fp;                     // [8][fp] backs
    uint16_t* mb0 = (uint16_t*)(Bk + (size_t)kStageTile * fp);    // [8][mp]
    uint16_t* mb1 = mb0 + (size_t)kStageTile * mp;
    const uint32_t le0 = tile * kStageTile;
    tile_setup(P, e0, le0, S, nq);
    tile_load<false>(P, S, nullptr, Fx, Bk, fp);
    const int n_el = cap * kStageTile;
    for (int idx = t; idx < n_el; idx += 256) {
        const int q = idx & 7, rs = idx >> 3;
        const int r = S.rinS[rs];
        const int s_ = rs - S.baseS[r];
        if (s_ < S.cntS[q][r]) {
            const float f = Fx[q * fp + rs], b = Bk[q * fp + rs];
            bool ok = isfinite(f) & isfinite(b) & (f < b);
            if (s_ > 0) ok &= f >= Fx[q * fp + rs - 1];
            if (!ok) atomicOr(&S.badS[q], 1);
            mb0[q * mp + S.preS[q][r] + s_] = (uint16_t)rs;
        }
    }
    __syncthreads();
    uint16_t* src = mb0;
    {
        const int q = t / kStageLanes, j = t - q * kStageLanes;
        int kp = 1;
        while (kp < P.k) kp <<= 1;
        uint16_t* dst = mb1;
        for (int w = 1; w < kp; w <<= 1) {   // w: inputs per run before this level
            const int pairs = kp / (2 * w);
            const int tpm = kStageLanes / pairs;
            const int m = j / tpm, jj = j - m * tpm;
            const int r0 = m * 2 * w;
            const int a0 = S.preS[q][min(r0, P.k)], a1 = S.preS[q][min(r0 + w, P.k)];
            const int b1 = S.preS[q][min(r0 + 2 * w, P.k)];
            if (S.totS[q] > 0) merge_path(src + q * mp, dst + q * mp, Fx + q * fp, a0, a1, b1, jj, tpm);
            __syncthreads();
            uint16_t* tmp = src;
            src = dst;
            dst = tmp;
        }
    }
    if (t < kStageTile) {
        const uint32_t le = le0 + t;
        if (S.totS[t] >= 0) {
            P.qtot[le] = S.badS[t] ? -1 : S.totS[t];
            if (S.badS[t]) reject_pixel(P, (uint32_t)P.q_list[e0 + le]);
        }
    }
    // the merged rows out (row i of the 8 entries in one 16-byte run), and
    // the staged depths in merge order
    uint16_t* seq = P.seq + (size_t)(le0 >> 3) * cap * 8;
    const size_t slab = (size_t)(le0 >> 6) * cap * 64 + (le0 & 63);
    for (int idx = t; idx < n_el; idx += 256) {
        const int q = idx & 7, i = idx >> 3;
        if (i < S.totS[q]) {
            const int row = src[q * mp + i];
            seq[idx] = (uint16_t)row;
            P.stage_d[slab + (size_t)i * 64 + q] = make_float2(Fx[q * fp + row], Bk[q * fp + row]);
        }
    }
    __syncthreads();   // the next tile reuses the LDS
}

// Staging of one tile: the elements into LDS in whole lines, then out to the
// staging rows in merge order (row i of the 8 entries are adjacent columns of
// a slab row), with the distances between consecutive elements' per-step
// premultiplied colours (the Eq. 1 operands) binned by log2 for the
// threshold prediction.
__device__ void merge_stage_tile(const CompParams& P, uint32_t e0, uint32_t tile, unsigned char* lds_raw,
                                 StageLds& S, uint32_t nq)
{
    const int t = threadIdx.x;
    const int cap = P.seq_cap;
    float4* Ec = (float4*)lds_raw;                         // [cap][8]
    uint16_t* rowS = (uint16_t*)(lds_raw + (size_t)cap * kStageTile * sizeof(float4));  // [cap][8]
    uint32_t* histS = S.histS;
    int* totS = S.totS;
    const uint32_t le0 = tile * kStageTile;
    tile_setup(P, e0, le0, S, nq);
    // lengths as the order kernel found them (-1: rejected or past the queue)
    if (t < kStageTile) {
        const uint32_t le = le0 + t;
        totS[t] = (le < P.chunk && e0 + le < nq) ? P.qtot[le] : -1;
    }
    for (int i = t; i < kStageTile * kPredBins; i += 256) histS[i] = 0u;
    tile_load<true>(P, S, Ec, nullptr, nullptr, 0);
    int tmax = 0;
#pragma unroll
    for (int q = 0; q < kStageTile; ++q) tmax = max(tmax, totS[q]);
    const int n_out = tmax * kStageTile;
    const uint16_t* seq = P.seq + (size_t)(le0 >> 3) * cap * 8;
    for (int b0 = 0; b0 < n_out; b0 += 256 * kStageBatch) {
        uint16_t row[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int idx = b0 + t + 256 * u;
            const int q = idx & 7, i = idx >> 3;
            row[u] = (idx < n_out && i < totS[q]) ? seq[idx] : (uint16_t)0xffffu;
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int idx = b0 + t + 256 * u;
            if (idx < n_out) rowS[idx] = row[u];
        }
    }
    __syncthreads();
    const size_t slab = (size_t)(le0 >> 6) * cap * 64 + (le0 & 63);
    for (int idx = t; idx < n_out; idx += 256) {
        const int rs = rowS[idx];
        if (rs == 0xffff) continue;
        const int q = idx & 7, i = idx >> 3;
        const float4 c = Ec[rs * kStageTile + q];
        P.stage_c[slab + (size_t)i * 64 + q] = c;
        if (i > 0) {
            const float4 c0 = Ec[rowS[idx - kStageTile] * kStageTile + q];
            const float d0 = c.x * c.w - c0.x * c0.w, d1 = c.y * c.w - c0.y * c0.w, d2 = c.z * c.w - c0.z * c0.w;
            const float l2 = 0.5f * hw_log2(d0 * d0 + d1 * d1 + d2 * d2);
            const float x = (l2 - kPredLo) * (kPredBins / (kPredHi - kPredLo));
            const int bin = x > 0.0f ? min((int)x, kPredBins - 1) : 0;
            atomicAdd(&histS[q * kPredBins + bin], 1u);
        }
    }
    __syncthreads();
    // features: the histogram over the out_n (the MLP's input, and an
    // optional per-pixel copy)
    if (P.feat || P.feat_out) {
        const float inv_n = 1.0f / (float)P.out_n;
        for (int idx = t; idx < kStageTile * kPredBins; idx += 256) {
            const int q = idx / kPredBins, b = idx - q * kPredBins;
            if (totS[q] > P.out_n) {
                const uint16_t v = bf16_bits((float)histS[idx] * inv_n);
                if (P.feat) P.feat[(size_t)(le0 + q) * kPredBins + b] = v;
                if (P.feat_out) P.feat_out[(size_t)P.q_list[e0 + le0 + q] * kPredBins + b] = v;
            }
        }
    }
    // predicted threshold: the out_n-th largest distance (a supersegment
    // ends roughly where consecutive operands differ by more than gamma),
    // interpolated inside its bin; with the MLP, its output replaces it
    if (t < kStageTile && totS[t] > P.out_n && P.ghat && !P.mlp_wb) {
        uint32_t cum = 0;
        float lg = kPredLo;
        for (int b = kPredBins - 1; b >= 0; --b) {
            const uint32_t c = histS[t * kPredBins + b];
            if (cum + c >= (uint32_t)P.out_n) {
                const float frac = ((float)(P.out_n - cum) - 0.5f) / (float)c;
                lg = kPredLo + ((float)(b + 1) - frac) * ((kPredHi - kPredLo) / kPredBins);
                break;
            }
            cum += c;
        }
        P.ghat[le0 + t] = hw_exp2(lg);
    }
    __syncthreads();   // the next tile reuses the LDS
}

// Persistent: blocks take tiles of 8 chunk entries until the chunk or the
// queue ends.  At most 72 VGPRs (seven waves per SIMD): the order kernel runs
// beside the re-segmentation and staging kernels of other chunks, and at 80
// it found no room beside them (the dense 16 x 20 composite took 38.3 ms
// instead of 34.0).
__global__ __launch_bounds__(256, 7) void merge_order_kernel(CompParams P, uint32_t e0)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ StageLds S;
    const uint32_t nq = (uint32_t)*P.q_count;
    const uint32_t tiles = P.chunk / kStageTile;
    for (uint32_t tl = blockIdx.x; tl < tiles && e0 + tl * kStageTile < nq; tl += gridDim.x)
        merge_order_tile(P, e0, tl, lds_raw, S, nq);
}

__global__ __launch_bounds__(256) void merge_stage_kernel(CompParams P, uint32_t e0)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ StageLds S;
    const uint32_t nq = (uint32_t)*P.q_count;
    const uint32_t tiles = P.chunk / kStageTile;
    for (uint32_t tl = blockIdx.x; tl < tiles && e0 + tl * kStageTile < nq; tl += gridDim.x)
        merge_stage_tile(P, e0, tl, lds_raw, S, nq);
}

// Persistent, one wavefront per group of 64 chunk entries at a time:
// re-segmentation over the slab.
__global__ __launch_bounds__(64) void composite_staged_kernel(CompParams P, uint32_t e0)
{
    const int t = threadIdx.x;
    const uint32_t nq = (uint32_t)*P.q_count;
    const uint32_t groups = P.chunk / 64;
    for (uint32_t g = blockIdx.x; g < groups && e0 + g * 64 < nq; g += gridDim.x) {
        const uint32_t le = g * 64 + t;
        if (e0 + le >= nq) continue;
        const int tot = P.qtot[le];
        if (tot < 0) continue;
        const uint32_t p = (uint32_t)P.q_list[e0 + le];
        const size_t slab = (size_t)g * P.seq_cap * 64;
        const StageReader rd{P.stage_c + slab, P.stage_d + slab, (uint32_t)t, (uint32_t)t};
        if (P.rs_br) {
            // the deferred round: the rest of the bisection from the bracket
            const float2 br = P.rs_br[e0 + le];
            float gm;
            const int c = bisect_finish(P, rd, tot, p, br.x, br.y, P.rs_lv[e0 + le], gm);
            finish_pixel(P, p, c, gm);
            continue;
        }
        const float gh = P.ghat ? (P.mlp_wb ? hw_exp2(P.ghat[le]) : P.ghat[le]) : 0.0f;
        resegment<false>(P, rd, tot, p, gh, P.dq_count != nullptr);
    }
}

// All pixels by the general merge (k above the depth-disjoint path's limit),
// grid-stride over the 64-pixel blocks.
__global__ __launch_bounds__(64) void composite_kernel(CompParams P)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int t = threadIdx.x;
    setup_inputs(P, lds_raw, t);
    __syncthreads();
    const uint32_t nblk = composite_blocks(P);
    for (uint32_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        uint32_t p;
        if (!block_pixel(P, blk, t, p)) continue;
        composite_pixel(P, lds_raw, t, p);
    }
}

// Every pixel to the general merge's queue (k above the depth-disjoint
// path's limit).
__global__ void queue_all_kernel(CompParams P)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.npix) P.q_list[i] = (int)i;
    if (i == 0) *P.q_count = (int)P.npix;
    if (i == 0 && P.dq_count) *P.dq_count = 0;
}

// Depth-disjoint path over all pixels; the others are queued.
__global__ __launch_bounds__(64) void composite_cat_kernel(CompParams P)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int t = threadIdx.x;
    setup_inputs(P, lds_raw, t);
    __syncthreads();
    uint32_t p;
    const uint32_t blk = P.order ? P.order[blockIdx.x] : blockIdx.x;
    if (!block_pixel(P, blk, t, p)) return;
    const bool done = composite_pixel_cat(P, lds_raw, t, p);
    const int pos = wave_append(P.q_count, !done);
    if (!done) P.q_list[pos] = (int)p;
}

// General merge over the queued pixels (grid-stride).
__global__ __launch_bounds__(64) void composite_queue_kernel(CompParams P, uint32_t first)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int t = threadIdx.x;
    setup_inputs(P, lds_raw, t);
    __syncthreads();
    const uint32_t n = (uint32_t)*P.q_count;
    for (uint32_t idx = first + blockIdx.x * kWave + t; idx < n; idx += gridDim.x * kWave)
        composite_pixel(P, lds_raw, t, (uint32_t)P.q_list[idx]);
}

// ---------------------------------------------------------------- batched (persistent)
//
// One launch composites many jobs of different size, k and N.  The jobs'
// pixels are cut into tiles (tile size chosen per (k, N) bucket); blocks pull
// tile indices from a device counter until the queue is empty, so every block
// exits once all tiles are taken.  Per job, the earliest tile start and the
// latest tile end are recorded with the device's constant-rate clock.

__global__ __launch_bounds__(64) void batch_kernel(const CompParams* __restrict__ jobs,
                                                   const uint2* __restrict__ tiles, uint32_t n_tiles,
                                                   uint32_t* head, unsigned long long* t_start_end)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ uint32_t s_tile;
    const int t = threadIdx.x;
    int cur_job = -1;
    for (;;) {
        if (t == 0) s_tile = atomicAdd(head, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        __syncthreads();
        if (tile >= n_tiles) break;
        const uint2 td = tiles[tile];          // x: job | blocks << 16, y: first 64-pixel block
        const int job = (int)(td.x & 0xffffu);
        const uint32_t nblk = td.x >> 16;      // blocks in the tile
        const CompParams& P = jobs[job];
        if (job != cur_job) {
            setup_inputs(P, lds_raw, t);
            cur_job = job;
        }
        __syncthreads();
        if (t == 0 && t_start_end) atomicMin(&t_start_end[2 * job], (unsigned long long)wall_clock64());
        for (uint32_t blk = td.y; blk < td.y + nblk; ++blk) {
            uint32_t p;
            if (block_pixel(P, blk, t, p)) {
                const bool done = composite_pixel_cat(P, lds_raw, t, p);
                const int pos = wave_append(P.q_count, !done);
                if (!done) P.q_list[pos] = (int)p;
            }
        }
        if (t == 0 && t_start_end) atomicMax(&t_start_end[2 * job + 1], (unsigned long long)wall_clock64());
        __syncthreads();
    }
}

// Second phase of a batch: the general merge for every job's queued pixels
// (all pixels of jobs with more inputs than the depth-disjoint path takes).
// Every block walks the jobs in order; within a job, a grid-stride loop.
__global__ __launch_bounds__(64) void batch_queue_kernel(const CompParams* __restrict__ jobs, int n_jobs,
                                                         unsigned long long* t_start_end)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int t = threadIdx.x;
    for (int j = 0; j < n_jobs; ++j) {
        const CompParams& P = jobs[j];
        const bool all = P.k > kCatMaxInputs;
        const uint32_t n = all ? P.npix : (uint32_t)*P.q_count;
        if (blockIdx.x * kWave >= n) continue;   // uniform in the block
        __syncthreads();                         // the previous job's table is no longer read
        setup_inputs(P, lds_raw, t);
        __syncthreads();
        if (t == 0 && t_start_end && all) atomicMin(&t_start_end[2 * j], (unsigned long long)wall_clock64());
        for (uint32_t idx = blockIdx.x * kWave + t; idx < n; idx += gridDim.x * kWave)
            composite_pixel(P, lds_raw, t, all ? idx : (uint32_t)P.q_list[idx]);
        __syncthreads();
        if (t == 0 && t_start_end) atomicMax(&t_start_end[2 * j + 1], (unsigned long long)wall_clock64());
    }
}

__global__ void fill_i32n_kernel(int* p, int v, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long lo_val, unsigned long long hi_val, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (i & 1) ? hi_val : lo_val;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v) { p[threadIdx.x] = v; }

void launch_batch(const CompParams* jobs, const uint2* tiles, uint32_t n_tiles, uint32_t* head, int* q_counts,
                  unsigned long long* t_se, int n_jobs, size_t lds_cat, int grid_cat, size_t lds_gen, int grid_gen,
                  hipStream_t s)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(1), 0, s, head, 0u);
    hipLaunchKernelGGL(fill_i32n_kernel, dim3((n_jobs + 255) / 256), dim3(256), 0, s, q_counts, 0, n_jobs);
    if (t_se)
        hipLaunchKernelGGL(fill_u64_kernel, dim3((2 * n_jobs + 255) / 256), dim3(256), 0, s, t_se, ~0ull, 0ull,
                           2 * n_jobs);
    if (n_tiles)
        hipLaunchKernelGGL(batch_kernel, dim3(grid_cat), dim3(kWave), lds_cat, s, jobs, tiles, n_tiles, head, t_se);
    hipLaunchKernelGGL(batch_queue_kernel, dim3(grid_gen), dim3(kWave), lds_gen, s, jobs, n_jobs, t_se);
}

size_t composite_lds_bytes(int k, int seq_cap)
{
    const size_t sb = ((size_t)(k <= 16 ? (seq_cap + 1) / 2 : seq_cap) + 3) & ~(size_t)3;
    return sizeof(InLds) * kMaxInputs + (size_t)kWave * (sb + 14 * (size_t)k);
}

size_t cat_lds_bytes(int k) { return sizeof(InLds) * kMaxInputs + (size_t)kWave * 8 * (size_t)k; }

// ---------------------------------------------------------------- block order
//
// A wavefront lasts as long as its longest merged list, and the blocks of
// long lists cluster in the image.  Dispatched in image order, the last of
// them start late and run on a nearly empty device; dispatched longest
// first, the short ones fill in behind them.  Blocks are bucketed by their
// longest merged list (bucket 0: lists that pass through, then steps of 8
// elements) and the order lists the buckets from the longest down.

__device__ inline uint32_t order_bucket(const CompParams& P, uint32_t blk)
{
    const uint32_t p = blk * 64u + (threadIdx.x & 63u);
    int tot = 0;
    if (p < P.npix)
        for (int r = 0; r < P.k; ++r) tot += max(0, min(P.in[r].count[p], P.in[r].max_n));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot = max(tot, __shfl_xor(tot, o));
    const int b = tot <= P.out_n ? 0 : 1 + ((tot - P.out_n - 1) >> 3);
    return (uint32_t)min(b, kOrderBuckets - 1);
}

__global__ __launch_bounds__(64) void order_count_kernel(CompParams P)
{
    const uint32_t b = order_bucket(P, blockIdx.x);
    if (threadIdx.x == 0) P.bucket[blockIdx.x] = b;
}

// One block: a counting sort of the blocks by bucket, longest bucket first
// (LDS counters; the order within a bucket is arbitrary).
__global__ __launch_bounds__(1024) void order_sort_kernel(CompParams P, uint32_t blocks)
{
    __shared__ uint32_t cnt[kOrderBuckets];
    const uint32_t t = threadIdx.x;
    if (t < kOrderBuckets) cnt[t] = 0u;
    __syncthreads();
    for (uint32_t i = t; i < blocks; i += blockDim.x) atomicAdd(&cnt[P.bucket[i]], 1u);
    __syncthreads();
    if (t == 0) {
        uint32_t o = 0;
        for (int b = kOrderBuckets - 1; b >= 0; --b) {
            const uint32_t c = cnt[b];
            cnt[b] = o;
            o += c;
        }
    }
    __syncthreads();
    for (uint32_t i = t; i < blocks; i += blockDim.x) P.order[atomicAdd(&cnt[P.bucket[i]], 1u)] = i;
}

uint32_t ordered_chunk(int seq_cap, size_t bytes, uint32_t npix, uint32_t grid)
{
    if (seq_cap > kOrderedMaxCap) return 0;
    const size_t per = (size_t)seq_cap * (sizeof(float4) + sizeof(float2) + sizeof(uint16_t)) + sizeof(int) +
                       sizeof(float) + kPredBins * sizeof(uint16_t);
    size_t c = bytes / per;
    const size_t all = ((size_t)npix + 63) & ~(size_t)63;
    c = std::min(c, all) & ~(size_t)63;
    if (grid && c >= grid && c < all) c = c / grid * grid;
    if (c == 0) return 0;
    // chunks of equal size (no short last chunk, whose re-segmentation takes
    // as long as a full chunk's with little else on the device)
    const size_t n = ((size_t)npix + c - 1) / c;
    c = std::min(c, ((((size_t)npix + n - 1) / n) + 63) & ~(size_t)63);
    return (uint32_t)c;
}

size_t ordered_ws_bytes(int seq_cap, uint32_t chunk)
{
    const size_t c = chunk;
    const size_t stage = c * seq_cap * (sizeof(float4) + sizeof(float2));
    const size_t seq = (c * seq_cap * sizeof(uint16_t) + 255) & ~(size_t)255;
    const size_t tot = (c * sizeof(int) + 255) & ~(size_t)255;
    const size_t gh = (c * sizeof(float) + 255) & ~(size_t)255;
    const size_t ft = c * kPredBins * sizeof(uint16_t);
    return stage + seq + tot + gh + ft;
}

// Dynamic LDS of merge_order_kernel (the tile's fronts and backs and the two
// merge buffers of element rows) and of merge_stage_kernel (the tile's
// elements and the merged rows).
static size_t order_lds_bytes(int seq_cap)
{
    return (size_t)kStageTile * (2 * sizeof(float) * front_pitch(seq_cap) + 2 * sizeof(uint16_t) * merge_pitch(seq_cap));
}
static size_t stage_lds_bytes(int seq_cap)
{
    return (size_t)seq_cap * kStageTile * (sizeof(float4) + sizeof(uint16_t));
}

// Grids of the persistent ordered-merge kernels: enough blocks to fill the
// device (and no more than the chunk has work for).
static unsigned ord_grid(const CompParams& P, uint32_t units, int per_cu)
{
    return std::max(1u, std::min(units, (unsigned)(P.num_cus * per_cu)));
}

static void launch_order_stage(const CompParams& P, uint32_t e0, hipStream_t s, bool alone = false)
{
    const uint32_t c = P.chunk;
    // four order blocks per CU (as many as LDS holds, 37 KB each) and two
    // staging blocks (52 KB each; three were slower beside the
    // re-segmentation: 34.6 ms against 32.9 ms on the 16 x 20 frame), three
    // for the first chunk, which nothing runs beside
    const unsigned g1 = ord_grid(P, c / kStageTile, 4), g2 = ord_grid(P, c / kStageTile, alone ? 3 : 2);
    hipLaunchKernelGGL(merge_order_kernel, dim3(g1), dim3(256), order_lds_bytes(P.seq_cap), s, P, e0);
    hipLaunchKernelGGL(merge_stage_kernel, dim3(g2), dim3(256), stage_lds_bytes(P.seq_cap), s, P, e0);
    // the MLP's log2 threshold for the chunk's entries of the queue
    if (P.mlp_wb)
        launch_mlp_fwd(P.mlp_wb, P.mlp_wf, P.feat, (int)c, P.q_count, nullptr, P.num_cus * 3, P.ghat, nullptr, s,
                       (int)e0);
}

// Re-segmentation of a staged chunk.
static void launch_resegment(const CompParams& P, uint32_t e0, hipStream_t s)
{
    const uint32_t c = P.chunk;
    // two waves per SIMD: the order and staging kernels of the next chunk run
    // beside these on the second stream and need registers of their own
    // (four waves here leave them none: 6% slower on the 16 x 20 frame)
    hipLaunchKernelGGL(composite_staged_kernel, dim3(ord_grid(P, c / 64, kResegBlocksPerCU)), dim3(64), 0, s, P, e0);
}

// Deferred pixels beyond the deferred round's one chunk: the general merge
// with its merge sequence in LDS, from the start (no staging, no bracket).
static void launch_overflow(const CompParams& D, hipStream_t s)
{
    CompParams O = D;
    O.rs_br = nullptr;
    O.rs_lv = nullptr;
    const size_t lds = composite_lds_bytes(O.k, O.seq_cap);
    hipLaunchKernelGGL(composite_queue_kernel, dim3((unsigned)(O.num_cus * 2)), dim3(kWave), lds, s, O, O.chunk);
}

// Parameters of the deferred round: the deferral list as the queue, the
// brackets as the entries' starting points, no further deferral.
static CompParams deferred_round(const CompParams& P)
{
    CompParams D = P;
    D.q_list = P.dq_pix;
    D.q_count = P.dq_count;
    D.rs_br = P.dq_br;
    D.rs_lv = P.dq_lv;
    D.dq_count = nullptr;
    D.dq_pix = nullptr;
    D.dq_br = nullptr;
    D.dq_lv = nullptr;
    return D;
}

// The ordered general merge over the queue, chunk by chunk (every kernel
// reads the queue length on the device; entries past it exit at once).  With
// several buffers, chunks c + 1 (and c + 2) are ordered and staged on the
// second stream while chunk c is re-segmented.
static void launch_ordered(const CompParams& P, hipStream_t s, const OrderedSync* sync)
{
    const uint32_t c = P.chunk;
    const uint32_t n = (P.npix + c - 1) / c;
    // the queue in up to n chunks, then (with deferral) one chunk of the
    // deferral list (every kernel reads its round's length on the device;
    // deferred pixels are a few per hundred, and any beyond that chunk are
    // composited again from the start by the general merge without staging)
    const uint32_t total = n + (P.dq_count ? 1u : 0u);
    if (!sync || sync->nbuf < 2) {
        for (uint32_t i = 0; i < n; ++i) {
            launch_order_stage(P, i * c, s);
            launch_resegment(P, i * c, s);
        }
        if (P.dq_count) {
            const CompParams D = deferred_round(P);
            launch_order_stage(D, 0, s);
            launch_resegment(D, 0, s);
            launch_overflow(D, s);
        }
        return;
    }
    // per buffer: the queue's chunks, the deferred round, and the last chunk
    // of the queue, which defers nothing: its mispredicted lanes finish in
    // their wavefronts, so the deferral list is complete when the chunk
    // before it is, and the deferred round runs beside the last chunk
    const int nb = sync->nbuf;
    CompParams D[kStageBufs], L[kStageBufs];
    for (int b = 0; b < nb; ++b) {
        D[b] = P.dq_count ? deferred_round(*sync->B[b]) : *sync->B[b];
        L[b] = *sync->B[b];
        L[b].dq_count = nullptr;
    }
    hipStream_t aux = sync->aux;
    const hipEvent_t* staged = sync->ev + 1;
    const hipEvent_t* done = sync->ev + 1 + kStageBufs;
    // fork: the second stream starts after the caller's work so far
    (void)hipEventRecord(sync->ev[0], s);
    (void)hipStreamWaitEvent(aux, sync->ev[0], 0);
    for (uint32_t i = 0; i < total; ++i) {
        const int b = (int)(i % (uint32_t)nb);
        const bool rd = i >= n;
        const CompParams& B = rd ? D[b] : (i + 1 == n && P.dq_count ? L[b] : *sync->B[b]);
        // staging chunk i into buffer b waits until chunk i - nb (same
        // buffer) has been re-segmented; the deferred round also until the
        // last chunk that defers (n - 2) has: the list is then complete
        if (i >= (uint32_t)nb) (void)hipStreamWaitEvent(aux, done[b], 0);
        if (rd && n >= 2 && i - (uint32_t)nb != n - 2)
            (void)hipStreamWaitEvent(aux, done[(n - 2) % (uint32_t)nb], 0);
        const uint32_t e0 = (rd ? 0u : i) * c;
        launch_order_stage(B, e0, aux, i == 0);
        if (rd) {
            // the deferred round: on the second stream, beside the last chunk
            launch_resegment(B, e0, aux);
            launch_overflow(B, aux);
            continue;
        }
        (void)hipEventRecord(staged[b], aux);
        // re-segmenting chunk i waits for its staging
        (void)hipStreamWaitEvent(s, staged[b], 0);
        launch_resegment(B, e0, s);
        (void)hipEventRecord(done[b], s);
    }
    // join: the second stream's work precedes everything after this call
    (void)hipEventRecord(sync->ev[0], aux);
    (void)hipStreamWaitEvent(s, sync->ev[0], 0);
}

void launch_composite(const CompParams& P, int grid_general, hipStream_t s, const OrderedSync* sync)
{
    const size_t lds = composite_lds_bytes(P.k, P.seq_cap);
    const unsigned blocks = composite_blocks(P);
    const unsigned g2 = std::max(1u, std::min(blocks, (unsigned)grid_general));
    if (P.k > kCatMaxInputs) {
        if (P.chunk) {
            hipLaunchKernelGGL(queue_all_kernel, dim3((P.npix + 255) / 256), dim3(256), 0, s, P);
            launch_ordered(P, s, sync);
        } else {
            hipLaunchKernelGGL(composite_kernel, dim3(blocks), dim3(kWave), lds, s, P);
        }
        return;
    }
    // the queue's counter, and the deferral list's in the word after it
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(P.dq_count ? 2 : 1), 0, s, (uint32_t*)P.q_count, 0u);
    // Compact inputs: each lane walks its own contiguous list, reading 16 of
    // every 128 bytes per step, so a line is reused over eight steps only if
    // it stays cached; fewer resident waves (the general merge's LDS
    // footprint) keep it cached, and measured faster.  Slot-major inputs use
    // whole lines per step and prefer full occupancy.
    const size_t lds_cat = P.cache_bound ? std::max(composite_lds_bytes(P.k, P.seq_cap), cat_lds_bytes(P.k))
                                         : cat_lds_bytes(P.k);
    if (P.order) {
        hipLaunchKernelGGL(order_count_kernel, dim3(blocks), dim3(kWave), 0, s, P);
        hipLaunchKernelGGL(order_sort_kernel, dim3(1), dim3(1024), 0, s, P, blocks);
    }
    hipLaunchKernelGGL(composite_cat_kernel, dim3(blocks), dim3(kWave), lds_cat, s, P);
    if (P.chunk)
        launch_ordered(P, s, sync);
    else
        hipLaunchKernelGGL(composite_queue_kernel, dim3(g2), dim3(kWave), lds, s, P, 0u);
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
        float Aj = one_minus_exp2((fb.y - fb.x) * inv_ref * log2_1m(s.w));
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
