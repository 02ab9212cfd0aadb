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
    uint64_t capacity;
    int lo[3], hi[3];
    int dlo[3], ddim[3];
};

constexpr int kGenBricksPerLaunch = 16;
struct GenBricks {
    GenBrick b[kGenBricksPerLaunch];
};

// kind: 0 = search + regular write, 1 = search only, 2 = compact write
void launch_generate(int kind, int dtype, const GenParams& P, const GenBricks& B, int nb, hipStream_t s);
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
};

void launch_composite(const CompParams& P, hipStream_t s);

// ---------------------------------------------------------------- rendering

void launch_render(const float4* color, const float2* depth, const int* count, const uint32_t* offset,
                   uint64_t capacity, int max_n, uint32_t npix, float inv_ref, float4* rgba, int* status,
                   hipStream_t s);

}  // namespace vdi
