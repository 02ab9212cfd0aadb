/*
 * vdi.h -- C ABI of libvdi: Volumetric Depth Image (VDI) generation and
 * compositing on one AMD Instinct MI355X (gfx950).
 *
 * Method: Gupta et al., "Parallel Compositing of Volumetric Depth Images for
 * Interactive Visualization of Distributed Volumes at High Frame Rates",
 * arXiv 2206.14503.  A VDI holds, for each of the w*h viewport pixels, a list
 * of at most N supersegments (front depth f, back depth b, colour, opacity)
 * cut from the volume-rendering integral along the pixel's ray (Sec. 2.4).
 * Each of k volume bricks yields a sub-VDI on its own (Sec. 5.1); compositing
 * depth-merges the k lists of every pixel and re-segments them into at most
 * N supersegments (Sec. 5.2 and supplementary Algorithm S1).
 *
 * Conventions for every entry point:
 *  - All data pointers are DEVICE pointers unless stated otherwise; the caller
 *    allocates and owns them.  An op that needs device scratch memory (its
 *    workspace, sized by vdi_workspace_size) takes it from the context: either
 *    a caller-owned block set with vdi_ctx_set_workspace (the op then never
 *    allocates, and fails with VDI_E_WORKSPACE if the block is too small), or
 *    the context's own block, grown when a larger problem arrives (growing it
 *    synchronises the device and allocates, so reserve it beforehand with
 *    vdi_ctx_reserve_workspace where a call must not allocate, e.g. under
 *    graph capture).  The workspace is shared by all calls on a context:
 *    calls on different streams of one context must not run concurrently.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Work is enqueued on it and the call returns without synchronising.
 *  - Shape and argument errors are detected on the host before any launch and
 *    returned as a negative vdi_status; vdi_last_error() then describes them
 *    (thread-local, valid until the next call on the same thread).  Nothing
 *    is launched when an error is returned.
 *  - Depths are world-space distances along the unit ray direction, from the
 *    eye (perspective) or from the image plane (orthographic).  The world box
 *    of the volume is [0,1]^3.
 */
#ifndef VDI_H
#define VDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VDI_OK = 0,
    VDI_E_INVALID = -1,     /* bad argument or shape */
    VDI_E_UNSUPPORTED = -2, /* valid but beyond this library's limits (below) */
    VDI_E_HIP = -3,         /* a HIP runtime call failed */
    VDI_E_INPUT = -4,       /* input data violates a precondition (checked on the device; see vdi_ctx_device_status) */
    VDI_E_CAPACITY = -5,    /* a compact output does not fit its capacity */
    VDI_E_WORKSPACE = -6    /* the caller's workspace is smaller than the call needs */
} vdi_status;

typedef enum { VDI_LAYOUT_REGULAR = 0, VDI_LAYOUT_COMPACT = 1 } vdi_layout;
typedef enum { VDI_TAU_FIXED = 0, VDI_TAU_BISECT = 1, VDI_TAU_LEARNED = 2, VDI_TAU_BISECT_SEQ = 3 } vdi_tau_mode;
typedef enum { VDI_F32 = 0, VDI_F16 = 1 } vdi_dtype;

/* Limits of this library. */
#define VDI_MAX_INPUTS 32   /* k in vdi_composite */
#define VDI_MAX_N 64        /* N, supersegments per list */
#define VDI_MAX_TF 1024     /* transfer-function entries */

typedef struct vdi_ctx vdi_ctx;

/* A VDI (Sec. 2.4, Sec. 4).  One list per pixel p = y*width + x (row 0 at the
 * top of the image).
 *
 * Regular layout (Sec. 4, Fig. 2a): slot-major planes.  Supersegment j of
 * pixel p is color[(j*H*W + p)*4 .. +4) and depth[(j*H*W + p)*2 .. +2);
 * slots j >= count[p] hold zeros.  color/depth hold max_n*H*W entries.
 *
 * Compact layout (Sec. 4, Fig. 2b/c): supersegment j of pixel p is entry
 * offset[p] + j of color/depth; offset[p] is the exclusive prefix sum of
 * count and offset[H*W] the total.  color/depth hold `capacity` entries.
 *
 * color: RGB un-premultiplied in [0,1], A = opacity per ref_step of depth
 *        (the total opacity of the supersegment is 1-(1-A)^((b-f)/ref_step)).
 * depth: {f, b}, f < b, lists sorted by f with non-overlapping extents.
 * gamma: per-list threshold the generator or compositor used (optional). */
typedef struct {
    int32_t width, height;
    int32_t max_n;
    int32_t layout;          /* vdi_layout */
    float ref_step;          /* reference step length (world units) of the opacities */
    float *color;            /* float4 per supersegment */
    float *depth;            /* float2 per supersegment */
    int32_t *count;          /* [H*W] */
    uint32_t *offset;        /* [H*W + 1], compact only (else NULL) */
    float *gamma;            /* [H*W] or NULL */
    uint64_t capacity;       /* compact: entries color/depth can hold */
} vdi_t;

/* A brick of the domain decomposition (Sec. 5, Sec. 3): the voxels it owns,
 * [lo, hi) in global voxel indices (x, y, z), and its data with a ghost layer:
 * data covers the global box [data_lo, data_lo + data_dim), x fastest.  The
 * data box must contain [lo-1, hi+1) clipped to the volume, so that samples
 * the brick owns reconstruct exactly as on the whole volume.  A data box must
 * hold less than 4 GiB (else VDI_E_UNSUPPORTED: split into more bricks).
 * Arbitrary, possibly non-convex domains (Sec. 5.3): with `owner` set (a
 * DEVICE array of one byte per voxel of the whole volume, x fastest), the
 * brick owns only the voxels of [lo, hi) where owner == rank, so [lo, hi)
 * is the bounding box of its domain.  A ray may then leave the domain and
 * enter it again; every supersegment ends where the ray leaves.  Owner maps
 * need a bisection threshold mode (FIXED and LEARNED return
 * VDI_E_UNSUPPORTED), and a ray entering a domain more often than N times
 * keeps its first N supersegments (device status flag 4).  owner = NULL:
 * the box alone decides. */
typedef struct {
    const void *data;
    int32_t dtype;           /* vdi_dtype */
    int32_t full_dim[3];     /* global nx, ny, nz */
    int32_t lo[3], hi[3];
    int32_t data_lo[3], data_dim[3];
    const uint8_t *owner;    /* optional rank per voxel [nz][ny][nx] */
    int32_t rank;            /* this brick's rank in owner */
} vdi_brick_t;

/* Shared camera (Sec. 5.1: every brick casts the same rays).  For pixel
 * (x, y): sx = (2x+1)/W - 1, sy = 1 - (2y+1)/H.  Perspective (ortho = 0):
 * origin eye, direction normalize(fwd + sx*right + sy*up).  Orthographic:
 * origin eye + sx*right + sy*up, direction fwd (unit length).  right/up are
 * pre-scaled (tan(fovy/2)*aspect, tan(fovy/2); or the half extents). */
typedef struct {
    int32_t ortho;
    float eye[3], fwd[3], right[3], up[3];
    int32_t width, height;
} vdi_camera_t;

/* 1D transfer function (Sec. 7: VDIs store classified colour): `entries`
 * RGBA rows at scalar s = i/(entries-1), linearly interpolated, A = opacity
 * per ref_step.  rgba is a DEVICE pointer, values in [0,1]. */
typedef struct {
    const float *rgba;
    int32_t entries;
} vdi_tf_t;

/* Threshold selection (Eq. 1 and Sec. 2.4).
 *  FIXED:   gamma = tau; a list saturates at max_n (after max_n-1 closes the
 *           last supersegment absorbs the rest of the ray).
 *  BISECT:  per list, `iters` halvings of [0, gamma_max]; a midpoint is
 *           feasible iff it yields at most max_n supersegments; the result is
 *           the upper bracket.  The search evaluates several midpoints per
 *           sampling pass and replays the halvings from their counts.
 *  BISECT_SEQ: (vdi_generate only) the same halvings with one midpoint per
 *           sampling pass, as Sec. 2.4 describes the search; results are
 *           identical to BISECT.  Kept as the baseline search the learned
 *           threshold is measured against.
 *  LEARNED: (an extension beyond the paper) the bisection of BISECT, its
 *           later scans steered by a regressed threshold; the result is
 *           BISECT's whatever the regressor says.  Per list, y = output of the
 *           MLP `mlp` (a vdi_mlp_t*) on the list's 64-bin opacity histogram
 *           (see vdi_tau_features), or y from the caller's array `y`.  The
 *           feature pass is also the bisection's first scan (states at
 *           gamma_max/2 ... gamma_max/64, as BISECT's); the next scan carries
 *           the midpoints of up to five further levels along the path toward
 *           2^y, its decisions are replayed up to the first one that differs
 *           from the path, and any levels left run as in BISECT.  Lists with
 *           at most N non-transparent samples take the bisection's result
 *           directly (every threshold is feasible there).  Regular layout
 *           only, at most 16 bricks per call (else VDI_E_UNSUPPORTED). */
typedef struct {
    int32_t mode;            /* vdi_tau_mode */
    float tau;
    int32_t iters;           /* B, 1..24 */
    float gamma_max;         /* > sqrt(3), normally 2 */
    const void *mlp;         /* LEARNED: const vdi_mlp_t* */
    float fallback_tol;      /* unused (kept for the layout) */
    float feature_scale;     /* LEARNED: histogram counts are divided by this (s_ref) */
    const float *y;          /* LEARNED: optional device array [k][H*W] of log2 thresholds
                                used instead of the MLP's output (NULL: run the MLP) */
    uint16_t *features;      /* vdi_composite: optional DEVICE output [H*W][64] bf16, the
                                threshold-prediction features of every pixel the general
                                merge re-segmented (others left unwritten; see below) */
} vdi_tau_t;

/* Context: one per device and thread of use.  vdi_ctx_create makes `device`
 * current and keeps it; VDI_E_HIP if the device cannot be used. */
vdi_status vdi_ctx_create(vdi_ctx **out, int device);
vdi_status vdi_ctx_destroy(vdi_ctx *ctx);
const char *vdi_last_error(void);

/* Workspace (device scratch memory) of an op, for the shape it is called
 * with; 0 when the op needs none.  Ops whose workspace is known from this
 * shape: VDI_OP_GENERATE (vdi_generate: width, height = camera size, k
 * bricks, layout of the outputs, tau_mode), VDI_OP_COMPOSITE (vdi_composite:
 * width, height, k inputs, in_max_n_sum = sum of the inputs' max_n),
 * VDI_OP_MLP_BACKWARD (vdi_mlp_backward: rows).  Other ops need none.  The
 * bytes depend on the device (its compute-unit count) but not on the data.
 * For VDI_OP_COMPOSITE the size is the recommended one (the general merge
 * stages up to 1.25 GiB of merged lists per chunk, in up to three buffers, so
 * that the next chunks are staged while one is re-segmented): a smaller
 * caller workspace
 * (vdi_ctx_set_workspace) makes vdi_composite stage in smaller chunks, down
 * to 64 pixels, the queues still fitting beside them; below that it reports
 * VDI_E_WORKSPACE.  Results do not depend on the chunk size. */
typedef enum { VDI_OP_GENERATE = 0, VDI_OP_COMPOSITE = 1, VDI_OP_MLP_BACKWARD = 2 } vdi_op;
typedef struct {
    int32_t op;              /* vdi_op */
    int32_t width, height;
    int32_t k;
    int32_t layout;          /* GENERATE: vdi_layout of the outputs */
    int32_t tau_mode;        /* GENERATE: vdi_tau_mode */
    int32_t in_max_n_sum;    /* COMPOSITE */
    int32_t rows;            /* MLP_BACKWARD */
} vdi_shape_t;
vdi_status vdi_workspace_size(vdi_ctx *ctx, const vdi_shape_t *shape, size_t *bytes);

/* Caller-owned workspace: a DEVICE block of `bytes` (256-byte aligned) that
 * every later op on ctx uses as its scratch memory instead of allocating;
 * it must stay valid until replaced.  The context's own block is freed.
 * workspace = NULL returns to the context's own, growing block.
 * Synchronises the device. */
vdi_status vdi_ctx_set_workspace(vdi_ctx *ctx, void *workspace, size_t bytes);

/* Grows the context's own workspace to at least `bytes` now (allocates and
 * synchronises the device if it grows), so that later ops of that size
 * neither allocate nor synchronise.  VDI_E_INVALID while a caller workspace
 * is set. */
vdi_status vdi_ctx_reserve_workspace(vdi_ctx *ctx, size_t bytes);

/* Sub-VDI generation (Sec. 5.1, Sec. 4, Eq. 1).  For each brick r < k, every
 * pixel's ray is sampled front to back on the global sample grid (sample i
 * covers [t_in + i*step, t_in + (i+1)*step), taken at its midpoint; t_in is
 * the ray's entry into the volume box), samples the brick owns are
 * classified by the transfer function (opacity corrected to the step length)
 * and cut into at most out[r].max_n supersegments by the criterion
 * gamma < |C(S)a(S) - C'a'| on per-step premultiplied RGB, with gamma chosen
 * per `tau`.  A supersegment also ends where the ray leaves the brick.
 * out[r] must match the camera's width/height and share ref_step; regular or
 * compact layout per out[r].layout (compact: capacity must hold the total,
 * else VDI_E_CAPACITY is reported through vdi_ctx_device_status after the
 * stream completes and the entries beyond capacity are not written).
 * step > 0 is the sampling distance in world units. */
vdi_status vdi_generate(vdi_ctx *ctx, const vdi_brick_t *bricks, int k, const vdi_camera_t *cam,
                        const vdi_tf_t *tf, float step, const vdi_tau_t *tau, vdi_t *out, void *stream);

/* Compositing (Sec. 5.2, Algorithm S1).  For every pixel, the k input lists
 * are merged by front depth (equal fronts: lower input index first; each
 * input must already be sorted).  If the merged list has at most out->max_n
 * entries it is written unchanged; otherwise each entry is treated as a
 * sample of its own length with opacity corrected by Eq. 2, empty space
 * between entries as transparent samples, and the list is re-segmented with
 * the Eq. 1 criterion and a threshold chosen per `tau` (FIXED, BISECT or
 * LEARNED).  BISECT and LEARNED give the same result, the bisection's: on
 * pixels whose lists interleave in depth (the general merge), the first scan
 * of the bisection evaluates the midpoints along the path toward a predicted
 * threshold, from a 64-bin histogram of log2 of the distances between
 * consecutive merged elements' per-step premultiplied colours (bins over
 * [-8, 1), counts divided by out->max_n): BISECT predicts the out->max_n-th
 * largest distance, LEARNED the MLP tau->mlp's output (log2 threshold; an
 * extension beyond the paper, trained on such histograms; see vdi_mlp_*).
 * tau->features, if set, receives those histograms (bf16) per pixel.
 * All inputs share width, height and ref_step with out; out must be regular.
 * Inputs may mix layouts.  k in [1, VDI_MAX_INPUTS].
 * Streams: when the general merge's pixels span several staging chunks, the
 * call forks work onto a second stream of the context (the next chunk's merge
 * beside the current chunk's re-segmentation) after an event on `stream`, and
 * joins it back into `stream` with an event before returning; work enqueued
 * on `stream` afterwards runs after all of it (also under graph capture).
 * Calls on different streams of one context must not overlap. */
vdi_status vdi_composite(vdi_ctx *ctx, const vdi_t *in, int k, const vdi_tau_t *tau, vdi_t *out,
                         void *stream);

/* vdi_composite for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same composite, with its scratch (the queue of pixels left to the
 * general merge and the block order) in a fixed device array of the library,
 * 32 MiB per device, held until the process ends, instead of the context's
 * workspace.  It calls no allocator.  The general merge then keeps each
 * pixel's merge sequence in LDS instead of staging merged lists.  The output
 * equals vdi_composite's bit for bit.  Limits: 4*(H*W + 64) + 8*ceil(H*W/64)
 * bytes of scratch must fit in 32 MiB (about 8.1 million pixels), and the
 * merged lists' capacity (sum of the inputs' max_n) must leave the merge
 * sequence room in LDS; beyond either VDI_E_UNSUPPORTED.  Every call on a
 * device shares that device's array (also across contexts): calls that
 * overlap on one device race, so serialise them (one stream, or events). */
vdi_status vdi_composite_noalloc(vdi_ctx *ctx, const vdi_t *in, int k, const vdi_tau_t *tau, vdi_t *out,
                                 void *stream);

/* Rendering from the viewpoint of generation (Sec. 2.3): per pixel, the
 * supersegments are composited front to back with the over operator using
 * their total opacities.  rgba: [H*W][4] premultiplied, fp32. */
vdi_status vdi_render_original_view(vdi_ctx *ctx, const vdi_t *vdi, float *rgba, void *stream);

/* Rendering from another viewpoint (Sec. 7 renders VDIs at viewpoint
 * deviations from the viewpoint of generation and compares them with DVR;
 * the rendering method itself is prior work the paper cites).  The VDI,
 * generated through camera vdi_cam, is read as the piecewise-constant field
 * it encodes: supersegment j of pixel q fills the part of q's view frustum
 * between its front and back depths with its colour and per-ref_step
 * opacity, and nothing lies outside the supersegments.  Each ray of `view`
 * is sampled like a generation ray (midpoints of [tn + k step, tn + (k+1)
 * step) from its entry into [0,1]^3); a sample point belongs to the vdi_cam
 * pixel whose frustum contains it, at the depth the VDI measures (distance
 * from the eye, perspective; along fwd from the image plane, orthographic),
 * both decided in fp64.  A sample inside supersegment (rgb, a) adds colour
 * rgb with opacity 1 - (1 - a)^(step/ref_step) (Eq. 2), front to back.
 *   vdi_cam: the VDI's generation camera (same width and height as the VDI;
 *            fwd, right and up orthogonal).  Lists must be front to back with
 *            disjoint [front, back) intervals, as generated or composited.
 *   view:    the new camera; rgba: [view H*W][4] premultiplied fp32 (device).
 *   step:    sampling distance of the new rays (world units, > 0).
 * A list with a count outside [0, max_n] (or past a compact VDI's capacity)
 * is read as empty and sets device status flag 2. */
vdi_status vdi_render_novel_view(vdi_ctx *ctx, const vdi_t *vdi, const vdi_camera_t *vdi_cam,
                                 const vdi_camera_t *view, float step, float *rgba, void *stream);

/* ---------------------------------------------------------------------------
 * Learned threshold (an extension beyond the paper: a regressor replaces the
 * per-ray bisection of Sec. 2.4).
 *
 * MLP 64 -> 128 -> 128 -> 1, GELU (erf form) after both hidden layers, linear
 * output = log2(gamma).  Parameters are one flat array in this order:
 * W1 [128][64] (out, in), b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]
 * (VDI_MLP_PARAMS values).  The kernels multiply bf16 matrices and bf16
 * activations on the matrix cores with fp32 accumulation; biases are read from
 * the fp32 copy.  Hidden activations are rounded to bf16 between layers.
 * ------------------------------------------------------------------------ */
#define VDI_MLP_PARAMS 24961
#define VDI_MLP_ACT_FLOATS 384   /* per row: z1[128], z2[128] fp32, h1[128], h2[128] bf16 */

typedef struct {
    uint16_t *w_bf16;        /* [VDI_MLP_PARAMS] bf16 bits */
    float *w_f32;            /* [VDI_MLP_PARAMS] fp32 master copy */
} vdi_mlp_t;

/* Per brick-ray features for the regressor.  Over the samples brick r owns
 * along pixel p's ray (same grid and classification as vdi_generate):
 * hist[(r*P + p)*64 + j] = bf16(#{non-transparent samples with opacity a in
 * (j/64, (j+1)/64]} / feature_scale), nnt[r*P + p] = number of non-transparent
 * samples, cmax[r*P + p] = min(count at threshold gamma_max*2^-iters, N+1).
 * tau supplies iters, gamma_max and feature_scale; N = max_n.  The bins count
 * to 65535: step must exceed sqrt(3)/65535 (else VDI_E_UNSUPPORTED; the same
 * holds for vdi_generate in LEARNED mode). */
vdi_status vdi_tau_features(vdi_ctx *ctx, const vdi_brick_t *bricks, int k, const vdi_camera_t *cam,
                            const vdi_tf_t *tf, float step, float ref_step, int max_n, const vdi_tau_t *tau,
                            uint16_t *hist, int32_t *nnt, int32_t *cmax, void *stream);

/* y[i] = MLP(x[i]) for rows i < rows; x is [rows][64] bf16.  If acts is not
 * NULL it receives [rows][VDI_MLP_ACT_FLOATS] activations for the backward. */
vdi_status vdi_mlp_forward(vdi_ctx *ctx, const vdi_mlp_t *mlp, const uint16_t *x, int rows, float *y,
                           float *acts, void *stream);

/* grad[VDI_MLP_PARAMS] = sum over rows of d(y_i)/d(params) * dy[i], from the
 * activations of vdi_mlp_forward on the same x.  Deterministic (fixed
 * reduction order); uses context scratch. */
vdi_status vdi_mlp_backward(vdi_ctx *ctx, const vdi_mlp_t *mlp, const uint16_t *x, const float *acts,
                            const float *dy, int rows, float *grad, void *stream);

/* One Adam step (step >= 1) on w_f32 with moments m, v ([VDI_MLP_PARAMS]);
 * refreshes w_bf16. */
vdi_status vdi_mlp_adam(vdi_ctx *ctx, vdi_mlp_t *mlp, const float *grad, float *m, float *v, int step, float lr,
                        float beta1, float beta2, float eps, void *stream);

/* Training step of the regressor (log2 thresholds): dy[i] = scale * (y[i] -
 * log2(gamma[i])) for i < rows (gamma > 0, e.g. the plain bisection's
 * thresholds), the gradient of 0.5 * sum (y - log2 gamma)^2 times scale; if
 * loss_part is not NULL, loss_part[b] = that loss over rows [256 b, 256 b +
 * 256) in fp64, summed in a fixed order ((rows + 255) / 256 entries). */
vdi_status vdi_mlp_mse(vdi_ctx *ctx, const float *y, const float *gamma, int rows, float scale, float *dy,
                       double *loss_part, void *stream);

/* w_bf16 = bf16(w_f32) (round to nearest even), e.g. after loading the fp32
 * master parameters. */
vdi_status vdi_mlp_pack(vdi_ctx *ctx, vdi_mlp_t *mlp, void *stream);

/* Counts of the learned path since the last call (synchronises `stream`):
 * stats[0] lists whose steered scan settled every remaining level, [1] lists
 * taking the all-feasible shortcut, [2] always 0, [3] empty lists, [4] lists
 * that needed further scans after the steered one.  stats holds 5 entries.
 * Clears them. */
vdi_status vdi_learned_stats(vdi_ctx *ctx, int64_t *stats, void *stream);

/* Diagnostic: D = A B for 16x16 bf16 A, B (row-major) through one matrix-core
 * instruction with the fragment layout the MLP kernels use; D fp32 16x16. */
vdi_status vdi_debug_mfma(vdi_ctx *ctx, const uint16_t *A, const uint16_t *B, float *D, void *stream);

/* ---------------------------------------------------------------------------
 * Batched compositing (an extension beyond the paper): many independent
 * composites of different viewport size, k and N in one persistent launch.
 * Each job is exactly what vdi_composite computes for it (same kernels, bit
 * for bit).
 * ------------------------------------------------------------------------ */
typedef struct {
    const vdi_t *in;         /* HOST array of k input VDIs (their data on the device) */
    int32_t k;               /* 1..VDI_MAX_INPUTS */
    vdi_t out;               /* regular output, same width/height/ref_step as the inputs */
    vdi_tau_t tau;           /* FIXED or BISECT */
} vdi_job_t;

typedef struct vdi_batch vdi_batch;

/* Checks the jobs (as vdi_composite would), then uploads a device job table
 * and a tile queue: jobs ordered by decreasing estimated work (k*N*pixels),
 * each job's image cut into blocks of 64 consecutive pixels (one per
 * wavefront) and the blocks into tiles of tile_pixels/64 blocks, tile_pixels read from
 * `autotune_cache` (a file written by vdi_autotune; NULL or no entry: 256)
 * for the job's (k bucket, N) with k buckets 1-4, 5-8, 9-32.  Jobs with more
 * than 16 inputs, and pixels whose input lists interleave in depth, are
 * composited by a second persistent kernel of the same run.  This is the only
 * batch call that allocates device memory; the job descriptors are copied,
 * the VDIs they point to must stay valid while the batch is used. */
vdi_status vdi_batch_create(vdi_ctx *ctx, const vdi_job_t *jobs, int n_jobs, const char *autotune_cache,
                            vdi_batch **out);

/* One persistent launch (grid sized to fill the device) whose blocks pull
 * tiles from a device counter until none is left, then the persistent
 * general-merge launch; preceded by small fill kernels that reset the
 * counters and t_start_end.  t_start_end: DEVICE [2*n_jobs] or NULL; per job
 * the earliest start and the latest end of its work in ticks of the device's
 * constant-rate clock (see vdi_batch_info).  Neither allocates nor
 * synchronises, so it can be captured in a graph. */
vdi_status vdi_batch_run(vdi_batch *batch, uint64_t *t_start_end, void *stream);

/* Captures vdi_batch_run(batch, t_start_end, stream) into a hipGraph (once;
 * a second call replaces it).  vdi_batch_replay launches the graph on stream. */
vdi_status vdi_batch_capture(vdi_batch *batch, uint64_t *t_start_end, void *stream);
vdi_status vdi_batch_replay(vdi_batch *batch, void *stream);

/* n_tiles, persistent grid (blocks of 64 threads), dynamic LDS bytes per block,
 * and the frequency of the timestamp clock in Hz.  Any pointer may be NULL. */
vdi_status vdi_batch_info(const vdi_batch *batch, int32_t *n_tiles, int32_t *grid, int32_t *lds_bytes,
                          double *clock_hz);
vdi_status vdi_batch_destroy(vdi_batch *batch);

/* Tile-size autotuner: for each (k bucket, N) present in `jobs`, runs those
 * jobs as a batch with each candidate tile size (64, 128, 256, 512, 1024
 * pixels), keeps the fastest (median of 3 timed runs after one warm-up) and
 * writes one line per bucket, "arch kbucket N tile_pixels milliseconds", to
 * cache_path (replacing the file).  The jobs' outputs are overwritten.
 * Synchronises stream. */
vdi_status vdi_autotune(vdi_ctx *ctx, const vdi_job_t *jobs, int n_jobs, const char *cache_path, void *stream);

/* Device-side status of the context since the last call to this function
 * (synchronises `stream` first): bit 0 = a compact output overflowed its
 * capacity, bit 1 = a composite input list was invalid (count outside
 * [0, max_n], f >= b, or fronts not sorted; such pixels are written empty;
 * also a list the novel-view rendering read as empty), bit 2 = a ray entered
 * a brick's owner-map domain more often than N times (its list keeps the
 * first N supersegments).  Clears the flags. */
vdi_status vdi_ctx_device_status(vdi_ctx *ctx, int32_t *flags, void *stream);

/* Diagnostic: the fp32 ray of each pixel as the kernels compute it.
 * o, d: [H*W][3]; tn, tf: [H*W]; nsamples: [H*W] (-1 for a miss). */
vdi_status vdi_debug_rays(vdi_ctx *ctx, const vdi_camera_t *cam, float step, float *o, float *d,
                          float *tn, float *tf, int32_t *nsamples, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VDI_H */
