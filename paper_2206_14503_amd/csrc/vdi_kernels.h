// vdi_kernels.h -- kernel parameter blocks and launchers (host <-> device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vdi_internal.h"

namespace vdi {

// ---------------------------------------------------------------- generation

struct GenParams {
    Cam cam;
    int n[3];            // global volume dims
    float step;          // sampling distance (world units)
    float l_step;        // step / ref_step
    int mode;            // vdi_tau_mode (FIXED or BISECT)
    float tau;
    int iters;
    float gmax;
    int max_n;
    int tf_entries;
    const float4* tf;
    int* status;         // device flags word
};

struct GenBrick {
    const void* data;
    float4* color;
    float2* depth;
    int* count;
    float* gamma;
    const uint32_t* offset;
    const uint8_t* owner;     // optional rank per voxel of the whole volume
    int rank;
    uint64_t capacity;
    int lo[3], hi[3];
    int dlo[3], ddim[3];
};

constexpr int kGenBricksPerLaunch = 16;
struct GenBricks {
    GenBrick b[kGenBricksPerLaunch];
    int first;           // index of b[0] among all bricks of the call
    int total;           // bricks of the call
};

// Outcome of a brick-ray on the learned path (indices into LearnBufs::stats):
// the regressed threshold's scan settled every level left (KEPT) or more
// scans followed (REFINED); at most N non-transparent samples (SHORTCUT); no
// sample (EMPTY).  FALLBACK stays 0 (every ray ends with the bisection's result).
enum { LEARN_KEPT = 0, LEARN_SHORTCUT = 1, LEARN_FALLBACK = 2, LEARN_EMPTY = 3, LEARN_REFINED = 4 };
constexpr int kLearnStats = 5;

// Work lists of the learned path.  A slot numbers a ray in the launch order
// of the 2D generation kernels: slot = (16x16-block index) * 256 + thread.
// Each list holds its rays in slot order (image-tile order), so the waves of
// the list-driven kernels sample neighbouring voxels: per 256-slot block the
// producers count their rays, the counts are scanned, and a compaction kernel
// places each ray at its block's offset plus its rank in the block.
enum { Q_SERVED = 0, Q_SHORT = 1, kQueues = 2 };

// Buffers of the learned-threshold path (per-ray arrays indexed brick * npix + pixel).
struct LearnBufs {
    uint16_t* hist;      // [nb][npix][64] bf16 features; with hist_list: per brick, compacted
    int* nnt;            // [nb][npix] non-transparent samples
    int* cmax;           // [nb][npix] features only: count at the smallest threshold (saturates at N+1)
    int* level;          // [nb][npix] generation: bisection levels the first scan settled
    float2* bracket;     // [nb][npix] generation: the bisection's bracket (lo, hi) after them
    const float* y;      // [nb][npix] log2(gamma) from the regressor (or the caller)
    int2* span;          // [nb][npix] first non-transparent sample, one past the last (listed rays)
    int* hist_list;      // optional [nb][npix]: pixel of each compacted histogram row
    int* hist_count;     // [nb]
    uint8_t* kind;       // [nb][slots] 1 + the list a slot's ray is on (0: none)
    int* qcnt;           // [kQueues][nb * nblk] rays per 256-slot block
    uint32_t* qoff;      // [kQueues][nb * nblk + 1] exclusive scans of qcnt
    int* qlist;          // [kQueues][nb * npix] pixels, per brick in slot order
    int nblk;            // 256-slot blocks per brick
    int* stats;          // [kLearnStats]
    float s_ref;
    int blocks_per_brick;  // grid of the list-driven kernels
};

// kind: 0 = search + regular write, 1 = search only, 2 = compact write
void launch_generate(int kind, int dtype, const GenParams& P, const GenBricks& B, int nb, hipStream_t s);
// phase 0: features and the bisection's first scan (finishes empty lists,
// lists the others), 1: the rest of the bisection steered by the regressed
// threshold, with the write, 4: the all-feasible list
void launch_learned(int phase, int dtype, const GenParams& P, const GenBricks& B, int nb, const LearnBufs& L,
                    hipStream_t s);
// Places the rays of list q (kind == 1 + q) at their offsets, in slot order.
void launch_compact(int q, const GenParams& P, int nb, const LearnBufs& L, hipStream_t s);
void launch_rays(const Cam& cam, float step, float* o, float* d, float* tn, float* tf, int* ns, hipStream_t s);

// ---------------------------------------------------------------- scan

// Exclusive prefix sum of n int32 counts into n+1 uint32 offsets.
// Scratch: scan_scratch_bytes(n) bytes of device memory.
size_t scan_scratch_bytes(size_t n);
void launch_scan(const int* counts, uint32_t* offsets, size_t n, void* scratch, hipStream_t s);

// ---------------------------------------------------------------- compositing

struct CompInput {
    const float4* color;
    const float2* depth;
    const int* count;
    const uint32_t* offset;   // compact only
    uint64_t capacity;        // entries color/depth hold
    int max_n;
    int compact;
};

constexpr int kMaxInputs = VDI_MAX_INPUTS;
struct CompParams {
    CompInput in[kMaxInputs];
    int k;
    uint32_t npix;
    int cache_bound;          // compact inputs: launch at the general merge's occupancy
    float inv_ref;
    int mode;
    float tau;
    int iters;
    float gmax;
    int out_n;
    float4* out_color;
    float2* out_depth;
    int* out_count;
    float* out_gamma;
    int* status;
    int seq_cap;              // merged-list capacity per pixel (sum of input max_n)
    int* q_list;              // [npix] pixels left to the general merge
    int* q_count;             // their number
    // optional ordered general merge, in chunks of `chunk` queue entries
    // (a multiple of 64): each entry's merged list staged for the
    // re-segmentation scans; per group of 64 entries a slab of seq_cap * 64
    // elements, entry t's element i at [i * 64 + t]
    uint32_t chunk;           // 0: no staging (merge sequence in LDS)
    uint16_t* seq;            // [chunk / 8][seq_cap][8]: merged element rows (input base + slot)
    int* qtot;                // [chunk]: merged-list length (-1: rejected)
    float* ghat;              // [chunk]: predicted threshold (speculation only; NULL: none),
                              // as log2 when predicted by the MLP (mlp_wb set)
    uint16_t* feat;           // [chunk][64]: prediction features (bf16), the MLP's input
    uint16_t* feat_out;       // optional [npix][64]: the same per pixel (training pairs)
    const uint16_t* mlp_wb;   // LEARNED: the threshold MLP (bf16 weights, fp32 master)
    const float* mlp_wf;
    int num_cus;              // compute units of the device (grid sizes of the persistent kernels)
    float4* stage_c;
    float2* stage_d;
    // deferral of the staged re-segmentation (NULL: none): a pixel whose
    // first scan left the predicted path before its last level goes on this
    // list with its bracket (lo, hi) and levels done, and a last round of
    // chunks finishes those pixels together
    int* dq_count;            // one word after q_count (cleared with it)
    int* dq_pix;              // [npix]
    float2* dq_br;            // [npix]
    int* dq_lv;               // [npix]
    // resume mode (that last round): entry e0 + le's bracket and levels
    const float2* rs_br;
    const int* rs_lv;
    // optional order of the 64-pixel blocks for the depth-disjoint pass
    // (longest merged list first), and its work space (a bucket per block)
    uint32_t* order;
    uint32_t* bucket;
};
constexpr int kOrderBuckets = 64;

// Inputs up to which the depth-disjoint path runs (4-bit list ids).
constexpr int kCatMaxInputs = 16;

size_t composite_lds_bytes(int k, int seq_cap);   // general merge
// Merged-list capacity up to which the ordered general merge runs.
constexpr int kOrderedMaxCap = 512;
// Blocks per CU of the re-segmentation's persistent grid (one wavefront of
// 64 entries each: two waves per SIMD).
constexpr int kResegBlocksPerCU = 8;
// Staging budget per buffer of the ordered merge.  Within it a chunk is a
// whole number of the re-segmentation's grids (num_cus * kResegBlocksPerCU
// * 64 entries), so that its wavefronts start together and end together:
// the chunk size sets how the two streams' work interleaves, and on the
// 16 x 20 frame (1920 x 1080, N = 20) one grid per chunk (16 chunks of
// 129,600 pixels) took 31.2 ms, 0.93 of one (17 chunks) 32.8 ms, 0.83 of one
// 33.8 ms, 1.13 of one 43 ms.  Each chunk's launches cost about 20 us where
// the queue is empty (frames of depth-disjoint lists).
constexpr size_t kStageBudget = (size_t)5 << 28;
// Queue entries per chunk of the ordered merge for a staging budget of
// `bytes`, in whole multiples of `grid` entries where the budget holds one
// (0 if seq_cap exceeds kOrderedMaxCap); workspace of one chunk.
uint32_t ordered_chunk(int seq_cap, size_t bytes, uint32_t npix, uint32_t grid);
size_t ordered_ws_bytes(int seq_cap, uint32_t chunk);
size_t cat_lds_bytes(int k);                      // depth-disjoint path
// Staging buffers of the ordered general merge when the queue spans several
// chunks: chunk c is staged into buffer c % kStageBufs.
constexpr int kStageBufs = 3;
// The ordered general merge runs the merge-order and staging kernels of
// chunk c + 1 (and, with a third buffer, c + 2) on a second stream while
// the re-segmentation of chunk c runs on the caller's (the buffers' params
// differ only in their staging buffers), joined back by events: ev[0] fork
// and join, ev[1 + b] staging into buffer b done, ev[1 + kStageBufs + b]
// re-segmentation of buffer b done.
struct OrderedSync {
    hipStream_t aux;
    hipEvent_t ev[1 + 2 * kStageBufs];
    const CompParams* B[kStageBufs];   // the buffers (B[0] the call's params)
    int nbuf;                          // buffers in use (2 or 3)
};
// grid_general: blocks of the queue-driven general merge without staging
void launch_composite(const CompParams& P, int grid_general, hipStream_t s, const OrderedSync* sync = nullptr);
// Blocks of 64 consecutive pixels (one per wavefront) covering the image.
__host__ __device__ inline uint32_t composite_blocks(const CompParams& P) { return (P.npix + 63u) / 64u; }

// Persistent batched compositing: tiles[i] = {job | blocks << 16, first block}
// for the depth-disjoint path (jobs with k <= kCatMaxInputs), then the general
// merge over every job's queue (all pixels of jobs with larger k).
void launch_batch(const CompParams* jobs, const uint2* tiles, uint32_t n_tiles, uint32_t* head, int* q_counts,
                  unsigned long long* t_se, int n_jobs, size_t lds_cat, int grid_cat, size_t lds_gen, int grid_gen,
                  hipStream_t s);

// ---------------------------------------------------------------- MLP (learned threshold)

int mlp_params();
int mlp_act_floats();
int mlp_rows_per_block();
// rows: row count (an upper bound when rows_dev holds the count on the
// device); out_idx: optional row -> output index map; max_blocks: grid cap
// rows_dev (optional): a device count; the rows are then min(rows, *rows_dev - row_off).
void launch_mlp_fwd(const uint16_t* wb, const float* wf, const uint16_t* x, int rows, const int* rows_dev,
                    const int* out_idx, int max_blocks, float* y, float* acts, hipStream_t s, int row_off = 0);
void launch_mlp_bwd(const uint16_t* wb, const uint16_t* x, const float* acts, const float* dy, int rows,
                    float* partial, float* grad, hipStream_t s);
void launch_mlp_adam(float* wf, uint16_t* wb, const float* grad, float* m, float* v, float lr, float b1, float b2,
                     float eps, int step, hipStream_t s);
void launch_mfma_probe(const uint16_t* A, const uint16_t* B, float* D, hipStream_t s);
void launch_mlp_mse(const float* y, const float* gamma, int rows, float scale, float* dy, double* loss_part,
                    hipStream_t s);
void launch_mlp_pack(const float* wf, uint16_t* wb, hipStream_t s);

// ---------------------------------------------------------------- rendering

// A VDI rendered from camera `view` (the VDI generated through camera `vcam`).
struct NovelParams {
    Cam view, vcam;
    const float4* color;
    const float2* depth;
    const int* count;
    const uint32_t* offset;   // compact only
    uint64_t capacity;        // entries color/depth hold
    int max_n;
    uint32_t npix;            // VDI pixels
    float step;               // sampling distance of the new rays
    float l;                  // step / ref_step
    float4* rgba;             // [view pixels]
    int* status;
};
void launch_novel(const NovelParams& N, hipStream_t s);

void launch_render(const float4* color, const float2* depth, const int* count, const uint32_t* offset,
                   uint64_t capacity, int max_n, uint32_t npix, float inv_ref, float4* rgba, int* status,
                   hipStream_t s);

}  // namespace vdi
