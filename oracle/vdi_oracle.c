/*
 * vdi_oracle.c -- plain, slow, fp64 CPU reference for VDI generation,
 * compositing, original-view rendering and direct volume rendering.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path: it is written directly from the paper's definitions,
 * one step at a time, without blocking, fusion or early exits.
 *
 * Paper: Gupta et al., "Parallel Compositing of Volumetric Depth Images for
 * Interactive Visualization of Distributed Volumes at High Frame Rates"
 * (arXiv 2206.14503).
 *
 * Precision.  Everything is fp64 except the steps whose result is an integer
 * decision that the GPU must take identically (which sample a brick owns,
 * how many samples a ray has, the voxel and transfer-function cells a sample
 * falls in, whether a sample is transparent).  Those are evaluated in fp32
 * with a fixed operation order, exactly as the kernels do: the ray (origin,
 * direction, entry/exit; separate multiplies and adds), the sample position,
 * the trilinear blend (fused multiply-adds, C fmaf) and the transfer-function
 * coordinate.  From the
 * transfer-function lookup on, the arithmetic is fp64.
 *
 * Readings of the paper where it is silent or garbled (all shared with the
 * kernels):
 *  - world box [0,1]^3, voxel centres at (i+1/2)/n, clamp-to-edge;
 *  - sample k covers [t0 + k*step, t0 + (k+1)*step) and is taken at its
 *    midpoint; t0 is the ray's entry into the whole volume, so every brick
 *    sees the same sample grid;
 *  - a brick owns a sample iff floor(p*n) (clamped) lies in its box;
 *  - transfer function: linear interpolation between entries at s=i/(E-1);
 *  - Eq. 1 compares per-unit-length premultiplied RGB colours, strictly
 *    (gamma < distance);
 *  - the open supersegment's per-unit opacity is 1 - T^(1/L) (the exponent in
 *    the supplementary algorithm is read as 1/l_s), each element is
 *    accumulated with its length-corrected opacity (Eq. 2);
 *  - a close and an open can happen on the same element; gaps between
 *    elements are transparent elements (compositing only);
 *  - a supersegment stores front f, back of its last non-transparent element,
 *    un-premultiplied RGB and per-ref-step opacity 1 - T^(ref/(b-f));
 *  - bisection over gamma in [0, 2] for B halvings, feasible iff
 *    count <= N, result = upper bracket;
 *  - composite passes the merged list through unchanged when it already has
 *    at most N entries;
 *  - fixed-threshold mode saturates: after N-1 closes no further close.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Inputs                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t ortho;
    float eye[3], fwd[3], right[3], up[3];
    int32_t width, height;
} orc_camera;

typedef struct {
    const void *data;   /* whole volume, [nz][ny][nx], x fastest */
    int32_t dtype;      /* 0 = fp32, 1 = fp16 (IEEE binary16 bits) */
    int32_t n[3];       /* nx, ny, nz */
} orc_volume;

enum { ORC_FIXED = 0, ORC_BISECT = 1 };

/* IEEE binary16 -> float, written out from the format definition. */
static float half_to_float(uint16_t h)
{
    int sign = (h >> 15) & 1, expo = (h >> 10) & 31, mant = h & 1023;
    double v;
    if (expo == 0)
        v = ldexp((double)mant, -24);
    else if (expo == 31)
        v = mant ? NAN : INFINITY;
    else
        v = ldexp((double)(mant | 1024), expo - 25);
    return (float)(sign ? -v : v);
}

static float voxel(const orc_volume *vol, int x, int y, int z)
{
    size_t i = ((size_t)z * vol->n[1] + y) * vol->n[0] + x;
    if (vol->dtype == 1)
        return half_to_float(((const uint16_t *)vol->data)[i]);
    return ((const float *)vol->data)[i];
}

/* ------------------------------------------------------------------------ */
/* Rays (fp32, fixed order): one ray per pixel through the shared camera      */
/* (Sec. 2.4: one list per viewport pixel; Sec. 5.1: all PEs share the camera) */
/* ------------------------------------------------------------------------ */

typedef struct { float o[3], d[3], tn, tf; int hit; } orc_ray;

static orc_ray make_ray(const orc_camera *c, int i, int j)
{
    orc_ray r;
    float sx = (float)(2 * i + 1) / (float)c->width - 1.0f;
    float sy = 1.0f - (float)(2 * j + 1) / (float)c->height;
    if (c->ortho) {
        for (int a = 0; a < 3; ++a) {
            float t1 = sx * c->right[a];
            float t2 = sy * c->up[a];
            float s = c->eye[a] + t1;
            r.o[a] = s + t2;
            r.d[a] = c->fwd[a];
        }
    } else {
        float v[3];
        for (int a = 0; a < 3; ++a) {
            float t1 = sx * c->right[a];
            float t2 = sy * c->up[a];
            float s = c->fwd[a] + t1;
            v[a] = s + t2;
            r.o[a] = c->eye[a];
        }
        float xx = v[0] * v[0], yy = v[1] * v[1], zz = v[2] * v[2];
        float n2 = xx + yy;
        n2 = n2 + zz;
        float nrm = sqrtf(n2);
        for (int a = 0; a < 3; ++a) r.d[a] = v[a] / nrm;
    }
    /* slab test against the world box [0,1]^3 */
    float tn = 0.0f, tf = INFINITY;
    r.hit = 1;
    for (int a = 0; a < 3; ++a) {
        if (r.d[a] == 0.0f) {
            if (r.o[a] < 0.0f || r.o[a] > 1.0f) r.hit = 0;
            continue;
        }
        float ta = (0.0f - r.o[a]) / r.d[a];
        float tb = (1.0f - r.o[a]) / r.d[a];
        float lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
        if (lo > tn) tn = lo;
        if (hi < tf) tf = hi;
    }
    if (!(tn < tf)) r.hit = 0;
    r.tn = tn;
    r.tf = tf;
    return r;
}

/* Midpoint of sample k (fp32, fixed order, fused multiply-adds); returns 0
 * once past the exit. */
static int sample_point(const orc_ray *r, int k, float step, float p[3])
{
    float kk = (float)k + 0.5f;
    float t = fmaf(kk, step, r->tn);
    if (!(t < r->tf)) return 0;
    for (int a = 0; a < 3; ++a) p[a] = fmaf(t, r->d[a], r->o[a]);
    return 1;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Voxel that contains p: decides brick ownership. */
static void voxel_of(const orc_volume *vol, const float p[3], int v[3])
{
    for (int a = 0; a < 3; ++a) {
        float g = p[a] * (float)vol->n[a];
        v[a] = clampi((int)floorf(g), 0, vol->n[a] - 1);
    }
}

/* a + w (b - a) with one fused multiply-add */
static float lerpf32(float a, float b, float w)
{
    float d = b - a;
    return fmaf(w, d, a);
}

/* Trilinear reconstruction at p on the global voxel grid (fp32, fixed order). */
static float trilinear(const orc_volume *vol, const float p[3])
{
    int i0[3], i1[3];
    float w[3];
    for (int a = 0; a < 3; ++a) {
        float u = fmaf(p[a], (float)vol->n[a], -0.5f);
        float f = floorf(u);
        w[a] = u - f;
        int ii = (int)f;
        i0[a] = clampi(ii, 0, vol->n[a] - 1);
        i1[a] = clampi(ii + 1, 0, vol->n[a] - 1);
    }
    float c00 = lerpf32(voxel(vol, i0[0], i0[1], i0[2]), voxel(vol, i1[0], i0[1], i0[2]), w[0]);
    float c10 = lerpf32(voxel(vol, i0[0], i1[1], i0[2]), voxel(vol, i1[0], i1[1], i0[2]), w[0]);
    float c01 = lerpf32(voxel(vol, i0[0], i0[1], i1[2]), voxel(vol, i1[0], i0[1], i1[2]), w[0]);
    float c11 = lerpf32(voxel(vol, i0[0], i1[1], i1[2]), voxel(vol, i1[0], i1[1], i1[2]), w[0]);
    float c0 = lerpf32(c00, c10, w[1]);
    float c1 = lerpf32(c01, c11, w[1]);
    return lerpf32(c0, c1, w[2]);
}

/* Transfer-function cell and weight (fp32, fixed order). */
static void tf_coord(float s, int entries, int *cell, float *w)
{
    float sc = s < 0.0f ? 0.0f : (s > 1.0f ? 1.0f : s);
    float q = sc * (float)(entries - 1);
    int i = (int)floorf(q);
    if (i > entries - 2) i = entries - 2;
    *cell = i;
    *w = q - (float)i;
}

/* Classified sample: colour and per-ref-step opacity in fp64. */
typedef struct { double rgb[3]; double a; float a32; } orc_class;

static orc_class classify(const float *tf, int entries, float s)
{
    orc_class c;
    int i;
    float w;
    tf_coord(s, entries, &i, &w);
    const float *lo = tf + 4 * i, *hi = tf + 4 * (i + 1);
    for (int ch = 0; ch < 3; ++ch)
        c.rgb[ch] = (double)lo[ch] + (double)w * ((double)hi[ch] - (double)lo[ch]);
    c.a = (double)lo[3] + (double)w * ((double)hi[3] - (double)lo[3]);
    c.a32 = lerpf32(lo[3], hi[3], w);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Elements and the segmenter                                               */
/* ------------------------------------------------------------------------ */

/* An element is a sample (generation) or a sub-supersegment (compositing):
 * front/back depth along the ray, un-premultiplied colour and opacity per
 * reference step.  Its own length in reference steps is l = (b-f)/ref. */
typedef struct { double f, b, rgb[3], a; } orc_elem;

typedef struct { double f, b, rgb[3], a; } orc_sseg;

/* Near-tie decisions.  An implementation that evaluates the Eq. 1 distance
 * in fp32 can take the other branch of a decision whose fp64 distance lies
 * within its rounding error of gamma.  Such a decision is a near tie when
 * |d - gamma| < tie * max(1, L / 128), L the number of elements the open
 * supersegment holds (the fp32 error of its accumulated colour grows with L).
 * A run can force the outcomes of its first near ties (to enumerate every
 * outcome a near tie admits); it records the natural outcome of each. */
#define ORC_MAXNEAR 12

typedef struct {
    double gamma;
    int cap;            /* >0: saturate after cap-1 closes (fixed mode) */
    int gaps;           /* insert transparent gap elements (compositing) */
    double ref;
    int count_limit;    /* decisions are recorded only while count <= limit */
    double tie;         /* near-tie band (0: none) */
    const signed char *force;   /* outcomes (1 = close) of the first nforce near ties */
    int nforce;
    /* outputs */
    orc_sseg *out;       /* may be NULL */
    int max_out;
    int count;
    double margin;      /* min |distance - gamma| over recorded decisions */
    int nnear;          /* near ties met */
    signed char natural[ORC_MAXNEAR];   /* their outcomes at the fp64 distance */
} orc_segrun;

static orc_segrun segrun(double gamma, int cap, int gaps, double ref, int limit, double tie, orc_sseg *out,
                         int max_out)
{
    orc_segrun R;
    memset(&R, 0, sizeof R);
    R.gamma = gamma;
    R.cap = cap;
    R.gaps = gaps;
    R.ref = ref;
    R.count_limit = limit;
    R.tie = tie;
    R.out = out;
    R.max_out = max_out;
    return R;
}

/* 1 - 2^y for y <= 0, accurate also for y near 0 (expm1); 1 at y = -inf. */
static double one_minus_pow2(double y)
{
    return -expm1(y * 0.69314718055994530942);
}

/* log2(1 - a) for a in [0, 1], accurate also for small a (log1p); -inf at a = 1. */
static double log2_1m(double a)
{
    return log1p(-a) / 0.69314718055994530942;
}

typedef struct {
    int open;
    double f, b, bt;
    double C[3];        /* premultiplied colour accumulated front to back */
    double lT;          /* log2 of the transmittance of the open supersegment
                           (the product of its elements' Eq. 2 factors, in log
                           form so that it holds transmittances below fp64's
                           range; -inf when an element is opaque) */
    int nel;            /* elements it holds */
} orc_state;

static void seg_close(orc_state *S, orc_segrun *R)
{
    if (R->out && R->count < R->max_out) {
        orc_sseg *o = &R->out[R->count];
        double A = one_minus_pow2(S->lT);
        o->f = S->f;
        o->b = S->bt;
        for (int ch = 0; ch < 3; ++ch) o->rgb[ch] = A > 0.0 ? S->C[ch] / A : 0.0;
        /* opacity per reference step over the stored extent [f, bt] */
        o->a = one_minus_pow2(S->lT * (R->ref / (S->bt - S->f)));
    }
    R->count += 1;
    S->open = 0;
}

/* One element through the segmenter (Eq. 1 criterion, Eq. 2 length correction,
 * supplementary algorithm S1 as read above). */
static void seg_step(orc_state *S, orc_segrun *R, const orc_elem *e)
{
    int transparent = (e->a == 0.0);
    double l = (e->b - e->f) / R->ref;
    /* Eq. 2: the element's transmittance (1 - a)^l (as log2, l log2(1 - a)),
     * and its opacity one minus that.  The transmittance is kept as computed,
     * not as 1 - opacity, which rounds to 0 once (1 - a)^l is below half an
     * ulp of 1. */
    double le = transparent ? 0.0 : l * log2_1m(e->a);
    double at = one_minus_pow2(le);
    if (S->open) {
        double L = (S->b - S->f) / R->ref;
        double A = one_minus_pow2(S->lT);
        double aS = one_minus_pow2(S->lT / L);
        double d2 = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            double repS = A > 0.0 ? S->C[ch] / A * aS : 0.0;
            double repE = e->rgb[ch] * e->a;
            d2 += (repS - repE) * (repS - repE);
        }
        double d = sqrt(d2);
        int may_close = R->cap <= 0 || R->count < R->cap - 1;
        int close = may_close && R->gamma < d;
        if (may_close && R->count <= R->count_limit) {
            double m = fabs(d - R->gamma);
            if (m < R->margin) R->margin = m;
            double band = R->tie * (S->nel > 128 ? S->nel / 128.0 : 1.0);
            if (m < band) {
                int i = R->nnear++;
                if (i < ORC_MAXNEAR) {
                    R->natural[i] = (signed char)close;
                    if (i < R->nforce) close = R->force[i];
                }
            }
        }
        if (close) {
            seg_close(S, R);
        } else {
            double T = exp2(S->lT);
            for (int ch = 0; ch < 3; ++ch) S->C[ch] += T * e->rgb[ch] * at;
            S->lT += le;
            S->b = e->b;
            if (!transparent) S->bt = e->b;
            S->nel += 1;
        }
    }
    if (!S->open && !transparent) {
        S->open = 1;
        S->f = e->f;
        S->b = S->bt = e->b;
        for (int ch = 0; ch < 3; ++ch) S->C[ch] = e->rgb[ch] * at;
        S->lT = le;
        S->nel = 1;
    }
}

static void seg_run(const orc_elem *e, int n, orc_segrun *R)
{
    orc_state S;
    memset(&S, 0, sizeof S);
    R->count = 0;
    R->margin = INFINITY;
    R->nnear = 0;
    for (int i = 0; i < n; ++i) {
        if (S.open && e[i].f > S.b) {
            if (R->gaps) {
                /* compositing: the empty space before the element is a
                 * transparent sample */
                orc_elem g = { S.b, e[i].f, { 0.0, 0.0, 0.0 }, 0.0 };
                seg_step(&S, R, &g);
            } else {
                /* generation: the ray left the brick; the supersegment ends */
                seg_close(&S, R);
            }
        }
        seg_step(&S, R, &e[i]);
    }
    if (S.open) seg_close(&S, R);
}

/* Per-ray threshold search by bisection (Sec. 2.4): B halvings of [0, gmax];
 * a midpoint is feasible iff it yields at most N supersegments. */
static double bisect(const orc_elem *e, int n, int max_n, int iters, double gmax, int gaps,
                     double ref, double *margin)
{
    double lo = 0.0, hi = gmax, mg = INFINITY;
    for (int it = 0; it < iters; ++it) {
        double m = 0.5 * (lo + hi);
        orc_segrun R = segrun(m, 0, gaps, ref, max_n, 0.0, NULL, 0);
        seg_run(e, n, &R);
        if (R.margin < mg) mg = R.margin;
        if (R.count <= max_n) hi = m; else lo = m;
    }
    *margin = mg;
    return hi;
}

/* ------------------------------------------------------------------------ */
/* Outcomes under near ties                                                 */
/* ------------------------------------------------------------------------ */

#define ORC_MAXLEAF 32   /* outcomes of one pass */
#define ORC_MAXPATH 8    /* bisection paths */

typedef struct { signed char f[ORC_MAXNEAR]; int n; } orc_forcing;

/* Every outcome of one pass (the run template R0) when each near-tie decision
 * may go either way: a depth-first walk over the near ties, the first leaf
 * being the run with every decision at its fp64 outcome.  Leaf i's count goes
 * to counts[i] and, when lists != NULL, its supersegments to
 * lists[i * R0.max_out ...].  Returns the number of leaves, negated when the
 * walk is incomplete (more than ORC_MAXNEAR near ties on a path or more than
 * ORC_MAXLEAF leaves). */
static int pass_outcomes(const orc_elem *e, int n, orc_segrun R0, orc_sseg *lists, int *counts, double *margin)
{
    orc_forcing stack[ORC_MAXLEAF];
    int sp = 0, nl = 0, incomplete = 0;
    stack[sp].n = 0;
    sp = 1;
    while (sp > 0) {
        orc_forcing F = stack[--sp];
        if (nl == ORC_MAXLEAF) { incomplete = 1; break; }
        orc_segrun R = R0;
        R.force = F.f;
        R.nforce = F.n;
        R.out = lists ? lists + (size_t)nl * (size_t)R0.max_out : NULL;
        seg_run(e, n, &R);
        if (nl == 0 && margin) *margin = R.margin;
        counts[nl++] = R.count;
        if (R.nnear > ORC_MAXNEAR) incomplete = 1;
        int m = R.nnear < ORC_MAXNEAR ? R.nnear : ORC_MAXNEAR;
        /* the other outcome at each near tie past the forced ones, pushed
         * last-first so that the walk visits them in path order */
        for (int i = m - 1; i >= F.n; --i) {
            if (sp == ORC_MAXLEAF) { incomplete = 1; break; }
            orc_forcing G;
            G.n = i + 1;
            for (int j = 0; j < F.n; ++j) G.f[j] = F.f[j];
            for (int j = F.n; j < i; ++j) G.f[j] = R.natural[j];
            G.f[i] = (signed char)!R.natural[i];
            stack[sp++] = G;
        }
    }
    return incomplete ? -nl : nl;
}

/* Thresholds the bisection reaches when every near tie of its passes may go
 * either way: paths split where a pass admits both a feasible and an
 * infeasible count.  gammas[0] is the fp64 path's result.  Returns the number
 * of paths, negated when incomplete.  *margin: the fp64 path's minimum
 * |d - gamma| over its recorded decisions. */
static int bisect_paths(const orc_elem *e, int n, int max_n, int iters, double gmax, int gaps, double ref,
                        double tie, double *gammas, double *margin)
{
    double plo[ORC_MAXPATH], phi[ORC_MAXPATH];
    int np = 1, incomplete = 0;
    int counts[ORC_MAXLEAF];
    plo[0] = 0.0;
    phi[0] = gmax;
    double mg = INFINITY;
    for (int it = 0; it < iters; ++it) {
        int np0 = np;
        for (int p = 0; p < np0; ++p) {
            double m = 0.5 * (plo[p] + phi[p]), pm = INFINITY;
            orc_segrun R0 = segrun(m, 0, gaps, ref, max_n, tie, NULL, 0);
            int nl = pass_outcomes(e, n, R0, NULL, counts, &pm);
            if (nl < 0) { incomplete = 1; nl = -nl; }
            if (p == 0 && pm < mg) mg = pm;
            int feas = counts[0] <= max_n, other = 0;
            for (int i = 1; i < nl; ++i)
                if ((counts[i] <= max_n) != feas) other = 1;
            if (other) {
                if (np < ORC_MAXPATH) {
                    /* the second path takes the other feasibility */
                    plo[np] = feas ? m : plo[p];
                    phi[np] = feas ? phi[p] : m;
                    ++np;
                } else {
                    incomplete = 1;
                }
            }
            if (feas) phi[p] = m; else plo[p] = m;
        }
    }
    for (int p = 0; p < np; ++p) gammas[p] = phi[p];
    *margin = mg;
    return incomplete ? -np : np;
}

/* Alternative outcomes of the lists computed under near ties (beside the
 * fp64 outcome, which goes to the regular outputs).  Entry i: list `ray`,
 * its count, threshold and first max_n supersegments (zero-filled). */
typedef struct {
    int32_t *ray;
    int32_t *count;
    float *gamma;
    float *color;       /* [cap][max_n][4] */
    float *depth;       /* [cap][max_n][2] */
    int32_t cap;
    int32_t n;          /* entries wanted (may exceed cap: then the call fails) */
} orc_alts;

static int same_list(const orc_sseg *a, const orc_sseg *b, int n)
{
    for (int j = 0; j < n; ++j) {
        if ((float)a[j].f != (float)b[j].f || (float)a[j].b != (float)b[j].b || (float)a[j].a != (float)b[j].a)
            return 0;
        for (int ch = 0; ch < 3; ++ch)
            if ((float)a[j].rgb[ch] != (float)b[j].rgb[ch]) return 0;
    }
    return 1;
}

static void put_alt(orc_alts *A, int ray, int count, double gamma, const orc_sseg *s, int max_n)
{
    int i;
#pragma omp atomic capture
    i = A->n++;
    if (i >= A->cap) return;
    A->ray[i] = ray;
    A->count[i] = count;
    A->gamma[i] = (float)gamma;
    int c = count < max_n ? count : max_n;
    for (int j = 0; j < max_n; ++j) {
        float *co = A->color + ((size_t)i * max_n + j) * 4;
        float *de = A->depth + ((size_t)i * max_n + j) * 2;
        if (j < c) {
            for (int ch = 0; ch < 3; ++ch) co[ch] = (float)s[j].rgb[ch];
            co[3] = (float)s[j].a;
            de[0] = (float)s[j].f;
            de[1] = (float)s[j].b;
        } else {
            memset(co, 0, 4 * sizeof(float));
            memset(de, 0, 2 * sizeof(float));
        }
    }
}

/* Threshold and list(s) of one stream: the fp64 outcome in (*gamma, *count,
 * s[0 .. max_out)) and, in A (when not NULL), every other outcome the near ties
 * admit.  mode FIXED: Seg(gamma = tau) saturating at max_out; BISECT: the
 * bisection over Seg.  Returns the number of distinct outcomes (1: the list
 * is decided), negated when the enumeration was incomplete.  work: room for
 * ORC_MAXLEAF * max_out supersegments. */
static int segment_outcomes(const orc_elem *e, int n, int mode, double tau, int max_out, int iters, int gaps,
                            double ref, double tie, orc_sseg *s, orc_sseg *work, int ray, orc_alts *A,
                            double *gamma, int *count, double *margin)
{
    double gammas[ORC_MAXPATH], mg = INFINITY;
    int np = 1, incomplete = 0;
    if (mode == ORC_FIXED) {
        gammas[0] = tau;
    } else {
        np = bisect_paths(e, n, max_out, iters, 2.0, gaps, ref, tie, gammas, &mg);
        if (np < 0) { incomplete = 1; np = -np; }
    }
    int counts[ORC_MAXLEAF], nout = 0;
    for (int p = 0; p < np; ++p) {
        double fm = INFINITY;
        orc_segrun R0 = segrun(gammas[p], mode == ORC_FIXED ? max_out : 0, gaps, ref, max_out, tie, NULL, max_out);
        int nl = pass_outcomes(e, n, R0, work, counts, &fm);
        if (nl < 0) { incomplete = 1; nl = -nl; }
        if (p == 0 && fm < mg) mg = fm;
        for (int i = 0; i < nl; ++i) {
            const orc_sseg *li = work + (size_t)i * max_out;
            int ci = counts[i] < max_out ? counts[i] : max_out;
            if (p == 0 && i == 0) {
                memcpy(s, li, sizeof(orc_sseg) * (size_t)ci);
                *gamma = gammas[0];
                *count = counts[0];
                nout = 1;
                continue;
            }
            /* distinct from the fp64 outcome and from earlier leaves of this path */
            int dup = gammas[p] == *gamma && counts[i] == *count && same_list(li, s, ci);
            for (int q = 0; q < i && !dup; ++q)
                dup = counts[q] == counts[i] && same_list(work + (size_t)q * max_out, li, ci);
            if (dup) continue;
            ++nout;
            if (A) put_alt(A, ray, counts[i], gammas[p], li, max_out);
        }
    }
    *margin = mg;
    return incomplete ? -nout : nout;
}

/* ------------------------------------------------------------------------ */
/* Sample streams                                                           */
/* ------------------------------------------------------------------------ */

static int brick_owns(const int32_t *lo, const int32_t *hi, const int v[3])
{
    for (int a = 0; a < 3; ++a)
        if (v[a] < lo[a] || v[a] >= hi[a]) return 0;
    return 1;
}

/* Number of samples of a ray inside the volume. */
static int ray_samples(const orc_ray *r, float step)
{
    if (!r->hit) return 0;
    float p[3];
    int k = 0;
    while (sample_point(r, k, step, p)) ++k;
    return k;
}

/* Owned sample stream of one brick along one ray.  A brick owns a sample
 * whose voxel lies in its box [lo, hi) and, when an owner map is given (one
 * rank per voxel, x fastest: arbitrary, possibly non-convex domains, Sec. 5.3),
 * carries the brick's rank there.  Returns the element count; *contiguous is
 * cleared if the owned samples are not one run (the segmenter then ends the
 * open supersegment at each discontinuity: a supersegment must end where the
 * ray leaves the domain, Sec. 5.3). */
static int brick_stream(const orc_volume *vol, const int32_t *lo, const int32_t *hi, const uint8_t *owner,
                        int rank, const orc_ray *r, const float *tf, int entries, float step,
                        orc_elem *e, int cap, int *contiguous, float *a32_out)
{
    int ns = ray_samples(r, step), n = 0, last = -2;
    *contiguous = 1;
    for (int k = 0; k < ns; ++k) {
        float p[3];
        int v[3];
        sample_point(r, k, step, p);
        voxel_of(vol, p, v);
        if (!brick_owns(lo, hi, v)) continue;
        if (owner && owner[((size_t)v[2] * vol->n[1] + v[1]) * vol->n[0] + v[0]] != rank) continue;
        if (last >= 0 && k != last + 1) *contiguous = 0;
        last = k;
        if (n >= cap) break;
        orc_class c = classify(tf, entries, trilinear(vol, p));
        e[n].f = (double)r->tn + (double)k * (double)step;
        e[n].b = (double)r->tn + (double)(k + 1) * (double)step;
        for (int ch = 0; ch < 3; ++ch) e[n].rgb[ch] = c.rgb[ch];
        e[n].a = c.a;
        if (a32_out) a32_out[n] = c.a32;
        ++n;
    }
    return n;
}

static int max_samples(float step)
{
    /* a ray crosses the unit box over at most sqrt(3) world units */
    return (int)(1.7320509 / step) + 4;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                    */
/* ------------------------------------------------------------------------ */

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Generation (Sec. 5.1): for every brick and every requested pixel, the
 * owned sample stream is cut into supersegments, with a fixed threshold
 * (saturating at N) or with the per-ray bisection threshold.
 * Outputs, regular layout over the requested pixels (npix of them):
 *   color [nb][max_n][npix][4], depth [nb][max_n][npix][2] (zero beyond count),
 *   count [nb][npix], gamma [nb][npix], margin [nb][npix] (may be NULL),
 *   contiguous [nb][npix] (may be NULL).
 * Near ties (tie > 0, see above): nout [nb][npix] (may be NULL) receives the
 * number of distinct outcomes of each list (1: decided; negative: the
 * enumeration was incomplete) and alts (may be NULL) the outcomes beside the
 * fp64 one, with ray = r * npix + q.
 * owner (may be NULL): rank of every voxel [nz][ny][nx], ranks [nb] the
 * bricks' ranks (bisection only).  The count is what the segmenter emits:
 * with an owner map a ray can enter a domain more often than N times, and the
 * stored list then holds the first max_n supersegments.
 * Returns 0, -1 on bad arguments, -3 if alts is too small (alts->n then holds
 * the number of entries needed). */
int orc_generate(const void *vol_data, int vol_dtype, const int32_t *n,
                 const int32_t *brick_lo, const int32_t *brick_hi, int nb,
                 const orc_camera *cam, const float *tf, int entries,
                 float step, float ref, int mode, float tau, int max_n, int iters,
                 const int32_t *pixels, int npix,
                 float *color, float *depth, int32_t *count, float *gamma,
                 double *margin, int32_t *contiguous, const uint8_t *owner, const int32_t *ranks,
                 double tie, int32_t *nout, orc_alts *alts, int nthreads)
{
    if (!vol_data || !n || nb <= 0 || !cam || !tf || entries < 2 || max_n <= 0 || npix < 0)
        return -1;
    if (owner && (!ranks || mode == ORC_FIXED)) return -1;
    orc_volume vol = { vol_data, vol_dtype, { n[0], n[1], n[2] } };
    int cap = max_samples(step);
    set_threads(nthreads);
    size_t P = (size_t)npix;
    if (alts) alts->n = 0;
#pragma omp parallel
    {
        orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)cap);
        orc_sseg *s = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)max_n);
        orc_sseg *work = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)max_n * ORC_MAXLEAF);
#pragma omp for schedule(dynamic, 64)
        for (long long job = 0; job < (long long)nb * npix; ++job) {
            int r = (int)(job / npix);
            size_t q = (size_t)(job % npix);
            int pix = pixels ? pixels[q] : (int)q;
            orc_ray ray = make_ray(cam, pix % cam->width, pix / cam->width);
            int contig;
            int ne = ray.hit ? brick_stream(&vol, brick_lo + 3 * r, brick_hi + 3 * r, owner, owner ? ranks[r] : 0,
                                            &ray, tf, entries, step, e, cap, &contig, NULL) : 0;
            if (!ray.hit) contig = 1;
            double g, mg;
            int cnt;
            int no = segment_outcomes(e, ne, mode, tau, max_n, iters, 0, ref, tie, s, work, (int)job, alts, &g,
                                      &cnt, &mg);
            int c = cnt < max_n ? cnt : max_n;
            for (int j = 0; j < max_n; ++j) {
                size_t o = ((size_t)r * max_n + j) * P + q;
                if (j < c) {
                    for (int ch = 0; ch < 3; ++ch) color[4 * o + ch] = (float)s[j].rgb[ch];
                    color[4 * o + 3] = (float)s[j].a;
                    depth[2 * o] = (float)s[j].f;
                    depth[2 * o + 1] = (float)s[j].b;
                } else {
                    memset(color + 4 * o, 0, 4 * sizeof(float));
                    memset(depth + 2 * o, 0, 2 * sizeof(float));
                }
            }
            count[(size_t)r * P + q] = cnt;
            if (gamma) gamma[(size_t)r * P + q] = (float)g;
            if (margin) margin[(size_t)r * P + q] = mg;
            if (contiguous) contiguous[(size_t)r * P + q] = contig;
            if (nout) nout[(size_t)r * P + q] = no;
        }
        free(e);
        free(s);
        free(work);
    }
    if (alts && alts->n > alts->cap) return -3;
    return 0;
}

/* Compositing (Sec. 5.2): merge the k depth-sorted lists of a pixel by front
 * depth (equal fronts: lower input index first), then either pass the merged
 * list through (at most N entries) or re-segment it, treating each
 * sub-supersegment as a sample of its own length and the gaps between them
 * as transparent samples, with the threshold found by the per-ray bisection
 * (or fixed, saturating at N).
 * Inputs: k regular lists over the same npix pixels, color_k [in_n][npix][4],
 * depth_k [in_n][npix][2], count_k [npix].
 * Outputs: color [out_n][npix][4], depth [out_n][npix][2], count, gamma,
 * margin (may be NULL), order [npix][k*in_n] (may be NULL): merged order as
 * rank*65536 + slot, -1 padded; nout and alts as for generation (ray = q).
 * Returns 0; -1 on bad arguments; -2 if an input list is not sorted by front
 * depth, has f >= b, or a count outside [0, in_n]; -3 if alts is too small. */
int orc_composite(int k, const float *const *colors, const float *const *depths,
                  const int32_t *const *counts, int in_n, int npix, float ref,
                  int mode, float tau, int out_n, int iters,
                  float *color, float *depth, int32_t *count, float *gamma,
                  double *margin, int32_t *order, double tie, int32_t *nout, orc_alts *alts, int nthreads)
{
    if (k <= 0 || in_n <= 0 || out_n <= 0 || npix < 0) return -1;
    set_threads(nthreads);
    size_t P = (size_t)npix;
    int bad = 0;
    if (alts) alts->n = 0;
#pragma omp parallel
    {
        int cap = k * in_n;
        orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)cap);
        int32_t *rk = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
        orc_sseg *s = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)out_n);
        orc_sseg *work = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)out_n * ORC_MAXLEAF);
#pragma omp for schedule(dynamic, 64)
        for (long long qq = 0; qq < npix; ++qq) {
            size_t q = (size_t)qq;
            int n = 0, ok = 1;
            for (int r = 0; r < k; ++r) {
                int c = counts[r][q];
                if (c < 0 || c > in_n) { ok = 0; break; }
                for (int j = 0; j < c; ++j) {
                    size_t o = (size_t)j * P + q;
                    double f = depths[r][2 * o], b = depths[r][2 * o + 1];
                    if (!(f < b)) ok = 0;
                    if (j > 0 && f < depths[r][2 * (o - P)]) ok = 0;
                    /* insertion into the merged list: after every entry whose
                     * (front, rank) key is not larger */
                    int pos = n;
                    while (pos > 0 && (e[pos - 1].f > f || (e[pos - 1].f == f && (rk[pos - 1] >> 16) > r)))
                        --pos;
                    memmove(e + pos + 1, e + pos, sizeof(orc_elem) * (size_t)(n - pos));
                    memmove(rk + pos + 1, rk + pos, sizeof(int32_t) * (size_t)(n - pos));
                    e[pos].f = f;
                    e[pos].b = b;
                    for (int ch = 0; ch < 3; ++ch) e[pos].rgb[ch] = colors[r][4 * o + ch];
                    e[pos].a = colors[r][4 * o + 3];
                    rk[pos] = r * 65536 + j;
                    ++n;
                }
            }
            if (!ok) {
#pragma omp atomic write
                bad = 1;
                n = 0;
            }
            if (order)
                for (int j = 0; j < cap; ++j) order[q * (size_t)cap + j] = j < n ? rk[j] : -1;
            double g = 0.0, mg = INFINITY;
            int c, no = 1;
            if (n <= out_n) {
                /* pass-through */
                for (int j = 0; j < n; ++j) {
                    s[j].f = e[j].f;
                    s[j].b = e[j].b;
                    for (int ch = 0; ch < 3; ++ch) s[j].rgb[ch] = e[j].rgb[ch];
                    s[j].a = e[j].a;
                }
                c = n;
            } else {
                int cnt;
                no = segment_outcomes(e, n, mode, tau, out_n, iters, 1, ref, tie, s, work, (int)q, alts, &g, &cnt,
                                      &mg);
                c = cnt < out_n ? cnt : out_n;
            }
            for (int j = 0; j < out_n; ++j) {
                size_t o = (size_t)j * P + q;
                if (j < c) {
                    for (int ch = 0; ch < 3; ++ch) color[4 * o + ch] = (float)s[j].rgb[ch];
                    color[4 * o + 3] = (float)s[j].a;
                    depth[2 * o] = (float)s[j].f;
                    depth[2 * o + 1] = (float)s[j].b;
                } else {
                    memset(color + 4 * o, 0, 4 * sizeof(float));
                    memset(depth + 2 * o, 0, 2 * sizeof(float));
                }
            }
            count[q] = c;
            if (gamma) gamma[q] = (float)g;
            if (margin) margin[q] = mg;
            if (nout) nout[q] = no;
        }
        free(e);
        free(rk);
        free(s);
        free(work);
    }
    if (bad) return -2;
    if (alts && alts->n > alts->cap) return -3;
    return 0;
}

/* Rendering from the viewpoint of generation (Sec. 2.3): each stored
 * supersegment contributes its total opacity 1-(1-a)^((b-f)/ref), composited
 * front to back with the over operator.  Output premultiplied RGBA [npix][4]. */
int orc_render_ov(const float *color, const float *depth, const int32_t *count, int max_n,
                  int npix, float ref, double *rgba, int nthreads)
{
    if (max_n <= 0 || npix < 0) return -1;
    set_threads(nthreads);
    size_t P = (size_t)npix;
#pragma omp parallel for schedule(static)
    for (long long qq = 0; qq < npix; ++qq) {
        size_t q = (size_t)qq;
        double C[3] = { 0, 0, 0 }, A = 0.0;
        int c = count[q] < max_n ? count[q] : max_n;
        for (int j = 0; j < c; ++j) {
            size_t o = (size_t)j * P + q;
            double a = color[4 * o + 3];
            double len = ((double)depth[2 * o + 1] - (double)depth[2 * o]) / ref;
            double Aj = 1.0 - pow(1.0 - a, len);
            for (int ch = 0; ch < 3; ++ch) C[ch] += (1.0 - A) * color[4 * o + ch] * Aj;
            A += (1.0 - A) * Aj;
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * q + ch] = C[ch];
        rgba[4 * q + 3] = A;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rendering a VDI from another viewpoint                                     */
/* ------------------------------------------------------------------------ */

/* A VDI read as the piecewise-constant field it encodes: supersegment j of
 * pixel q fills the part of q's view frustum between its front and back
 * depths with its colour and per-ref-step opacity; outside every
 * supersegment the field is empty.  A ray of the new view is sampled on the
 * generation grid convention (midpoints of [tn + k step, tn + (k+1) step),
 * fp32 positions); sample point p lies in the VDI pixel whose frustum
 * contains it and at the depth the VDI's depths measure (distance from the
 * eye for a perspective VDI camera, distance along fwd from the image plane
 * for an orthographic one).  These integer decisions are taken in fp64 with
 * a fixed operation order, no fused operations. */
typedef struct {
    double e[3], f[3], r[3], u[3];
    double ff, irr, iuu;     /* |fwd|^2, 1/|right|^2, 1/|up|^2 */
    int ortho, W, H;
} orc_proj;

static double dot3(const double a[3], const double b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

static orc_proj make_proj(const orc_camera *c)
{
    orc_proj P;
    for (int a = 0; a < 3; ++a) {
        P.e[a] = c->eye[a];
        P.f[a] = c->fwd[a];
        P.r[a] = c->right[a];
        P.u[a] = c->up[a];
    }
    P.ff = dot3(P.f, P.f);
    P.irr = 1.0 / dot3(P.r, P.r);
    P.iuu = 1.0 / dot3(P.u, P.u);
    P.ortho = c->ortho;
    P.W = c->width;
    P.H = c->height;
    return P;
}

/* Pixel q of the VDI camera that point p falls in, and its depth (squared for
 * a perspective camera).  Returns 0 outside the image or not in front of the
 * eye.  The camera's direction through screen point (sx, sy) is
 * fwd + sx right + sy up (fwd, right, up orthogonal). */
static int project(const orc_proj *P, const float p[3], int *q, double *depth)
{
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = (double)p[a] - P->e[a];
    const double vf = dot3(v, P->f), vr = dot3(v, P->r), vu = dot3(v, P->u);
    double sx, sy;
    if (P->ortho) {
        sx = vr * P->irr;
        sy = vu * P->iuu;
        *depth = vf;
    } else {
        if (!(vf > 0.0)) return 0;
        const double w = P->ff / vf;
        sx = (vr * w) * P->irr;
        sy = (vu * w) * P->iuu;
        *depth = dot3(v, v);
    }
    const double fx = floor(((sx + 1.0) * 0.5) * (double)P->W);
    const double fy = floor(((1.0 - sy) * 0.5) * (double)P->H);
    if (!(fx >= 0.0 && fx < (double)P->W && fy >= 0.0 && fy < (double)P->H)) return 0;
    *q = (int)fy * P->W + (int)fx;
    return 1;
}

/* The VDI (regular layout, or compact when offset != NULL) rendered from
 * camera `view`: front-to-back emission-absorption over the samples of each
 * ray, a sample inside supersegment (rgb, a) taking colour rgb and opacity
 * 1 - (1 - a)^(step/ref) (Eq. 2), a sample outside every supersegment
 * nothing.  The supersegment of a sample is the first in list order whose
 * [front, back) holds its depth.  Output premultiplied RGBA [view pixels][4]. */
int orc_novel_view(const float *color, const float *depth, const int32_t *count, const uint32_t *offset,
                   int max_n, int width, int height, float ref, const orc_camera *vcam, const orc_camera *view,
                   float step, double *rgba, int nthreads)
{
    if (max_n <= 0 || width <= 0 || height <= 0 || vcam->width != width || vcam->height != height) return -1;
    if (!(step > 0.0f) || !(ref > 0.0f)) return -1;
    set_threads(nthreads);
    const orc_proj P = make_proj(vcam);
    const size_t NP = (size_t)width * (size_t)height;
    const long long nout = (long long)view->width * view->height;
    const double l = (double)step / (double)ref;
#pragma omp parallel for schedule(dynamic, 64)
    for (long long pix = 0; pix < nout; ++pix) {
        orc_ray ray = make_ray(view, (int)(pix % view->width), (int)(pix / view->width));
        const int ns = ray_samples(&ray, step);
        double C[3] = { 0, 0, 0 }, T = 1.0;
        for (int k = 0; k < ns; ++k) {
            float p[3];
            sample_point(&ray, k, step, p);
            int q;
            double d;
            if (!project(&P, p, &q, &d)) continue;
            const int c = count[q] < max_n ? count[q] : max_n;
            for (int j = 0; j < c; ++j) {
                const size_t o = offset ? (size_t)offset[q] + (size_t)j : (size_t)j * NP + (size_t)q;
                const double f = depth[2 * o], b = depth[2 * o + 1];
                const int inside = P.ortho ? (f <= d && d < b) : (f * f <= d && d < b * b);
                if (!inside) continue;
                const double alpha = 1.0 - pow(1.0 - (double)color[4 * o + 3], l);
                for (int ch = 0; ch < 3; ++ch) C[ch] += T * (double)color[4 * o + ch] * alpha;
                T *= 1.0 - alpha;
                break;
            }
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * pix + ch] = C[ch];
        rgba[4 * pix + 3] = 1.0 - T;
    }
    return 0;
}

/* Direct volume rendering of the whole volume (Sec. 2.1, emission-absorption,
 * front to back, no early termination) on the same sample grid.
 * Output premultiplied RGBA [npix][4]. */
int orc_dvr(const void *vol_data, int vol_dtype, const int32_t *n, const orc_camera *cam,
            const float *tf, int entries, float step, float ref, const int32_t *pixels, int npix,
            double *rgba, int nthreads)
{
    if (!vol_data || !n || !cam || !tf || npix < 0) return -1;
    orc_volume vol = { vol_data, vol_dtype, { n[0], n[1], n[2] } };
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (long long qq = 0; qq < npix; ++qq) {
        size_t q = (size_t)qq;
        int pix = pixels ? pixels[q] : (int)q;
        orc_ray ray = make_ray(cam, pix % cam->width, pix / cam->width);
        int ns = ray_samples(&ray, step);
        double C[3] = { 0, 0, 0 }, T = 1.0;
        for (int k = 0; k < ns; ++k) {
            float p[3];
            sample_point(&ray, k, step, p);
            orc_class c = classify(tf, entries, trilinear(&vol, p));
            double alpha = 1.0 - pow(1.0 - c.a, (double)step / (double)ref);
            for (int ch = 0; ch < 3; ++ch) C[ch] += T * c.rgb[ch] * alpha;
            T *= 1.0 - alpha;
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * q + ch] = C[ch];
        rgba[4 * q + 3] = 1.0 - T;
    }
    return 0;
}

/* Segmenter on explicit elements, for unit tests.  elems [n][6] = f, b, r, g, b, a.
 * mode FIXED: threshold gamma, saturating at cap (cap<=0: none);
 * mode BISECT: threshold from bisection with max_n/iters.
 * out [max_out][6]; returns the count; *gamma_used, *margin written. */
int orc_seg(const double *elems, int n, int mode, double gamma, int cap, int max_n, int iters,
            int gaps, double ref, double *out, int max_out, double *gamma_used, double *margin)
{
    orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)(n > 0 ? n : 1));
    orc_sseg *s = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)(max_out > 0 ? max_out : 1));
    for (int i = 0; i < n; ++i) {
        e[i].f = elems[6 * i];
        e[i].b = elems[6 * i + 1];
        for (int ch = 0; ch < 3; ++ch) e[i].rgb[ch] = elems[6 * i + 2 + ch];
        e[i].a = elems[6 * i + 5];
    }
    double g = gamma, mg = INFINITY;
    if (mode == ORC_BISECT) g = bisect(e, n, max_n, iters, 2.0, gaps, ref, &mg);
    orc_segrun R = segrun(g, mode == ORC_FIXED ? cap : 0, gaps, ref,
                          mode == ORC_FIXED ? (cap > 0 ? cap : n) : max_n, 0.0, s, max_out);
    seg_run(e, n, &R);
    if (R.margin < mg) mg = R.margin;
    int c = R.count < max_out ? R.count : max_out;
    for (int j = 0; j < c; ++j) {
        out[6 * j] = s[j].f;
        out[6 * j + 1] = s[j].b;
        for (int ch = 0; ch < 3; ++ch) out[6 * j + 2 + ch] = s[j].rgb[ch];
        out[6 * j + 5] = s[j].a;
    }
    if (gamma_used) *gamma_used = g;
    if (margin) *margin = mg;
    free(e);
    free(s);
    return R.count;
}

/* Every outcome of one explicit stream under near ties (for unit tests):
 * elems [n][6] as for orc_seg; mode FIXED (gamma, saturating at max_n) or
 * BISECT (max_n, iters).  Outcome i: counts[i], gammas[i] and lists
 * [i][max_n][6]; outcome 0 is the fp64 one.  Returns the number of outcomes
 * (at most max_outcomes are stored), negated when the enumeration was cut
 * short. */
int orc_seg_outcomes(const double *elems, int n, int mode, double gamma, int max_n, int iters, int gaps,
                     double ref, double tie, int32_t *counts, double *gammas, double *lists, int max_outcomes)
{
    orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)(n > 0 ? n : 1));
    orc_sseg *s = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)max_n);
    orc_sseg *work = (orc_sseg *)malloc(sizeof(orc_sseg) * (size_t)max_n * ORC_MAXLEAF);
    int cap = ORC_MAXLEAF * ORC_MAXPATH;
    float *ac = (float *)malloc(sizeof(float) * (size_t)cap * max_n * 4);
    float *ad = (float *)malloc(sizeof(float) * (size_t)cap * max_n * 2);
    int32_t *ar = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *acnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    float *ag = (float *)malloc(sizeof(float) * (size_t)cap);
    orc_alts A = { ar, acnt, ag, ac, ad, cap, 0 };
    for (int i = 0; i < n; ++i) {
        e[i].f = elems[6 * i];
        e[i].b = elems[6 * i + 1];
        for (int ch = 0; ch < 3; ++ch) e[i].rgb[ch] = elems[6 * i + 2 + ch];
        e[i].a = elems[6 * i + 5];
    }
    double g, mg;
    int cnt;
    int no = segment_outcomes(e, n, mode, gamma, max_n, iters, gaps, ref, tie, s, work, 0, &A, &g, &cnt, &mg);
    int tot = no < 0 ? -no : no;
    for (int i = 0; i < tot && i < max_outcomes; ++i) {
        double *o = lists + (size_t)i * max_n * 6;
        if (i == 0) {
            counts[0] = cnt;
            gammas[0] = g;
            int c = cnt < max_n ? cnt : max_n;
            for (int j = 0; j < max_n; ++j) {
                o[6 * j] = j < c ? s[j].f : 0.0;
                o[6 * j + 1] = j < c ? s[j].b : 0.0;
                for (int ch = 0; ch < 3; ++ch) o[6 * j + 2 + ch] = j < c ? s[j].rgb[ch] : 0.0;
                o[6 * j + 5] = j < c ? s[j].a : 0.0;
            }
        } else {
            counts[i] = acnt[i - 1];
            gammas[i] = ag[i - 1];
            for (int j = 0; j < max_n; ++j) {
                const float *co = ac + ((size_t)(i - 1) * max_n + j) * 4, *de = ad + ((size_t)(i - 1) * max_n + j) * 2;
                o[6 * j] = de[0];
                o[6 * j + 1] = de[1];
                for (int ch = 0; ch < 3; ++ch) o[6 * j + 2 + ch] = co[ch];
                o[6 * j + 5] = co[3];
            }
        }
    }
    free(e); free(s); free(work); free(ac); free(ad); free(ar); free(acnt); free(ag);
    return no;
}

/* Per-pixel sample streams for tests: number of samples of each ray and the
 * brick-owned element list of one pixel. */
int orc_ray_info(const orc_camera *cam, int pix, float step, float *o, float *d, float *tn, float *tf)
{
    orc_ray r = make_ray(cam, pix % cam->width, pix / cam->width);
    for (int a = 0; a < 3; ++a) { o[a] = r.o[a]; d[a] = r.d[a]; }
    *tn = r.tn;
    *tf = r.tf;
    return r.hit ? ray_samples(&r, step) : -1;
}

int orc_stream(const void *vol_data, int vol_dtype, const int32_t *n, const int32_t *lo, const int32_t *hi,
               const orc_camera *cam, const float *tf, int entries, float step, int pix,
               double *elems, int cap, float *a32)
{
    orc_volume vol = { vol_data, vol_dtype, { n[0], n[1], n[2] } };
    orc_ray r = make_ray(cam, pix % cam->width, pix / cam->width);
    if (!r.hit) return 0;
    orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)cap);
    int contig;
    int ne = brick_stream(&vol, lo, hi, NULL, 0, &r, tf, entries, step, e, cap, &contig, a32);
    for (int i = 0; i < ne; ++i) {
        elems[6 * i] = e[i].f;
        elems[6 * i + 1] = e[i].b;
        for (int ch = 0; ch < 3; ++ch) elems[6 * i + 2 + ch] = e[i].rgb[ch];
        elems[6 * i + 5] = e[i].a;
    }
    free(e);
    return contig ? ne : -ne - 1;
}

/* Trilinear value at an explicit fp32 point (tests pin the reconstruction). */
double orc_trilinear(const void *vol_data, int vol_dtype, const int32_t *n, const float *p)
{
    orc_volume vol = { vol_data, vol_dtype, { n[0], n[1], n[2] } };
    return (double)trilinear(&vol, p);
}

/* Classified colour/opacity at a scalar value (tests pin the lookup). */
void orc_classify(const float *tf, int entries, float s, double *rgba)
{
    orc_class c = classify(tf, entries, s);
    for (int ch = 0; ch < 3; ++ch) rgba[ch] = c.rgb[ch];
    rgba[3] = c.a;
}

/* ------------------------------------------------------------------------ */
/* Learned-threshold features (not in the paper: the extension that replaces */
/* the per-ray search by a regression from an opacity histogram)            */
/* ------------------------------------------------------------------------ */

/* bf16 round-to-nearest-even of an fp32 value (returned as float). */
static float bf16_round(float x)
{
    union { float f; uint32_t u; } v = { x };
    if ((v.u & 0x7f800000u) == 0x7f800000u) return x;
    uint32_t lsb = (v.u >> 16) & 1u;
    v.u = (v.u + 0x7fffu + lsb) & 0xffff0000u;
    return v.f;
}

/* Per brick-ray features over the owned samples:
 *   hist [nb][npix][64]: bin j counts non-transparent samples whose fp32
 *       opacity a lies in ((j)/64, (j+1)/64], i.e. j = min(63, ceil(64a)-1),
 *       divided by s_ref and rounded to bf16;
 *   nnt  [nb][npix]: number of non-transparent samples;
 *   cmax [nb][npix]: supersegment count at the smallest threshold the
 *       bisection can return, gmax * 2^-iters. */
int orc_features(const void *vol_data, int vol_dtype, const int32_t *n,
                 const int32_t *brick_lo, const int32_t *brick_hi, int nb,
                 const orc_camera *cam, const float *tf, int entries, float step, float ref,
                 int iters, float gmax, float s_ref, const int32_t *pixels, int npix,
                 float *hist, int32_t *nnt, int32_t *cmax, int nthreads)
{
    if (!vol_data || !n || nb <= 0 || !cam || !tf || npix < 0 || !(s_ref > 0.0f)) return -1;
    orc_volume vol = { vol_data, vol_dtype, { n[0], n[1], n[2] } };
    int cap = max_samples(step);
    set_threads(nthreads);
    double gmin = ldexp((double)gmax, -iters);
#pragma omp parallel
    {
        orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)cap);
        float *a32 = (float *)malloc(sizeof(float) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (long long job = 0; job < (long long)nb * npix; ++job) {
            int r = (int)(job / npix);
            size_t q = (size_t)(job % npix);
            int pix = pixels ? pixels[q] : (int)q;
            orc_ray ray = make_ray(cam, pix % cam->width, pix / cam->width);
            int contig = 1;
            int ne = ray.hit ? brick_stream(&vol, brick_lo + 3 * r, brick_hi + 3 * r, NULL, 0, &ray, tf, entries,
                                            step, e, cap, &contig, a32) : 0;
            int bins[64];
            memset(bins, 0, sizeof bins);
            int m = 0;
            for (int i = 0; i < ne; ++i) {
                if (a32[i] == 0.0f) continue;
                int j = (int)ceilf(64.0f * a32[i]) - 1;
                if (j > 63) j = 63;
                if (j < 0) j = 0;
                bins[j] += 1;
                m += 1;
            }
            size_t o = (size_t)r * npix + q;
            for (int j = 0; j < 64; ++j) hist[o * 64 + j] = bf16_round((float)bins[j] / s_ref);
            nnt[o] = m;
            orc_segrun R = segrun(gmin, 0, 0, ref, 1 << 30, 0.0, NULL, 0);
            seg_run(e, ne, &R);
            cmax[o] = R.count;
        }
        free(e);
        free(a32);
    }
    return 0;
}

/* Supersegment count of each brick-ray at a given per-ray threshold
 * (gamma [nb][npix]) and the smallest |distance - gamma| on its path. */
int orc_count_at(const void *vol_data, int vol_dtype, const int32_t *n,
                 const int32_t *brick_lo, const int32_t *brick_hi, int nb,
                 const orc_camera *cam, const float *tf, int entries, float step, float ref,
                 const float *gamma, int limit, const int32_t *pixels, int npix,
                 int32_t *count, double *margin, int nthreads)
{
    if (!vol_data || !n || nb <= 0 || !cam || !tf || npix < 0) return -1;
    orc_volume vol = { vol_data, vol_dtype, { n[0], n[1], n[2] } };
    int cap = max_samples(step);
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_elem *e = (orc_elem *)malloc(sizeof(orc_elem) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (long long job = 0; job < (long long)nb * npix; ++job) {
            int r = (int)(job / npix);
            size_t q = (size_t)(job % npix);
            int pix = pixels ? pixels[q] : (int)q;
            orc_ray ray = make_ray(cam, pix % cam->width, pix / cam->width);
            int contig = 1;
            int ne = ray.hit ? brick_stream(&vol, brick_lo + 3 * r, brick_hi + 3 * r, NULL, 0, &ray, tf, entries,
                                            step, e, cap, &contig, NULL) : 0;
            size_t o = (size_t)r * npix + q;
            orc_segrun R = segrun(gamma[o], 0, 0, ref, limit, 0.0, NULL, 0);
            seg_run(e, ne, &R);
            count[o] = R.count;
            if (margin) margin[o] = R.margin;
        }
        free(e);
    }
    return 0;
}
