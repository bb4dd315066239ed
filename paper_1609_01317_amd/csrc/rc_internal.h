// Internal declarations of the raycaster library: the volume handle, error
// reporting, the brick layout and the parameter block of the render kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "../../include/rc.h"

struct rc_volume {
    int nx, ny, nz;
    rc_dtype dtype;
    int elem_bytes;
    double spacing[3];
    float vmin, vmax;
    int nbx, nby, nbz;          // bricks per axis
    long long nbricks;
    void* bricked;              // nbricks * 512 voxels of dtype
    float2* brick_range;        // nbricks (min, max) or null before rc_build_bricks
    // super-bricks: 4x4x4 bricks (32^3 voxels); empty iff all their bricks are
    int nsx, nsy, nsz;
    long long nsuper;
    int device;
};

namespace rc {

// ---------------------------------------------------------------- errors
rc_status fail(rc_status st, const char* fmt, ...);
rc_status hip_fail(hipError_t e, const char* what);

#define RC_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return rc::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- brick layout
// Bricks of 8^3 voxels, bricks in x-fastest order, voxels inside a brick in
// Morton order (bit i of x, y, z -> bits 3i, 3i+1, 3i+2).  The offset of a
// voxel is separable: off(x,y,z) = ox(x) + oy(y) + oz(z), so a stencil
// gathers from 4+4+4 per-axis offsets.
constexpr int kBrick = 8;
constexpr int kBrickVox = 512;

// v < 8: bit 0 stays, bit 1 -> 3, bit 2 -> 6 (v | v << 2 | v << 4 puts each
// bit i at 3i among copies that the mask drops)
__host__ __device__ inline uint32_t spread3(uint32_t v) {
    return (v | (v << 2) | (v << 4)) & 0x49u;
}
__host__ __device__ inline uint32_t compact3(uint32_t m) {
    return (m & 1u) | ((m >> 2) & 2u) | ((m >> 4) & 4u);
}
__host__ __device__ inline int off_x(int x) { return (x >> 3) * kBrickVox + (int)spread3(x & 7); }
__host__ __device__ inline int off_y(int y, int sy) { return (y >> 3) * sy + ((int)spread3(y & 7) << 1); }
__host__ __device__ inline int off_z(int z, int sz) { return (z >> 3) * sz + ((int)spread3(z & 7) << 2); }

// ---------------------------------------------------------------- render parameters
// One image: camera frame (FP64: ray set-up is exact to double), tiling
// and the per-image buffers.
struct ViewParams {
    double eye[3], f[3], r[3], u[3];
    double tan_half, aspect, ortho_half;
    int projection, W, H;
    int tile_w;                 // tile width in pixels (tile height = 64 / tile_w)
    int tiles_x, n_tiles;
    float4* out;
    rc_aux* aux;
    const float4* grad;         // reverse pass: dL/d(rgba)
};

// Flags of a super-brick (4x4x4 bricks): every brick empty; every brick
// detail-poor; no brick detail-poor (the last two for adaptive sampling).
constexpr uint8_t kSuperEmpty = 1, kSuperPoor = 2, kSuperRich = 4;

struct RenderParams {
    ViewParams view;            // the image of a single render / batch item
    // sampling box (world) and lattice
    double lo[3], hi[3];
    double step;
    double inv_s[3];
    double inv_step;            // 1 / step (chunk extents only; the lattice uses step)
    float s[3];
    // volume (bricked)
    const void* vox;
    int nx, ny, nz;
    int sy, sz;                 // brick-row and brick-slab strides in voxels
    int nbx, nby, nbz;
    float vmin, inv_range;
    // transfer function
    const float4* tf;
    int M;
    float Mm1;
    // gradient scale: 1 / (gain * spacing_a * (vmax - vmin))
    float gscale[3];
    // shading
    int shade;
    float ka, kd, ks, shininess;
    int light_is_point;
    float light[3];             // position, or unit direction towards the light
    float grad_eps;
    // options
    float tau;
    int skip;
    int nearest;                // 1: nearest-voxel sampling
    double round_bias;          // 0.5 with nearest sampling (round half up), else 0
    float frac_keep;            // 0 with nearest sampling (cell fraction 0), else 1
    float ocorr;                // opacity-correction exponent step / ref_step, 0 = off
    // adaptive sampling: samples in bricks whose range is <= adapt_range
    // advance by adapt steps; their opacity exponent is adapt_e (else ocorr)
    int adapt;                  // factor, 0 or 1 = off
    float adapt_range;
    float adapt_e;
    const float2* range;        // per-brick (min, max) value ranges
    const uint8_t* empty;       // per-brick flag, 1 = every sample has alpha 0
    const uint8_t* super_empty; // per-super-brick flags (4x4x4 bricks, kSuper*), or null
    int nsx, nsy, nsz;          // super-bricks per axis
    rc_stats* stats;            // kStatSlots consecutive copies, or null
    unsigned int* dbg;          // bounds-checked build: violation counter; else null
    // chunk shape: LDS bytes a chunk's box may take (capped by the wave's
    // allocation) and the first chunk length in lattice samples
    int box_bytes;
    int chunk_init;
};

// Several images of one volume in one launch (kernel-argument block).
constexpr int kMaxViews = 16;
struct ViewSet {
    int n;
    int block_off[kMaxViews + 1];   // first block of each view
    ViewParams v[kMaxViews];
};
static_assert(sizeof(RenderParams) + sizeof(ViewSet) <= 3800,
              "kernel arguments of the multi-view kernels must stay below 4 KiB");

// Host-side preparation shared by the forward, reverse and batch paths.
rc_status check_render_args(const rc_volume* v, const rc_camera* cam, const float* tf, int tf_len,
                            const rc_shading* sh, const rc_options* opt);
void fill_render_params(RenderParams& P, const rc_volume* v, const rc_camera* cam,
                        const float* tf, int tf_len, const rc_shading* sh, const rc_options* opt);
// Launch the prefix + empty-mask kernels into `mask` (nbricks bytes) using
// `prefix` (tf_len + 1 ints) as scratch.
// adapt_range: the detail-poor bound of an adaptive render, NaN otherwise.
rc_status launch_empty_mask(const rc_volume* v, const float* tf, int tf_len, uint8_t* mask,
                            uint8_t* super_mask, int* prefix, float adapt_range, hipStream_t st);
// Super-brick flags (one thread each), kSuperEmpty | kSuperPoor | kSuperRich
// over the bricks of super-brick s.
__global__ void super_mask_kernel(const uint8_t* __restrict__ mask, const float2* __restrict__ range,
                                  float adapt_range, uint8_t* __restrict__ smask, int nbx, int nby,
                                  int nbz, int nsx, int nsy, long long nsuper);
// Bytes of per-render skip scratch: brick mask, super-brick mask, prefix counts.
size_t skip_scratch_bytes(const rc_volume* v, int tf_len, size_t* mask_bytes,
                          size_t* super_bytes);
void set_tiling(ViewParams& V, int tile_w);     // tile_w in {4, 8, 16, 32, 64}
void fill_view(ViewParams& V, const rc_camera* cam);
// the bounds-checked build's violation counter on the current device (null
// in the product build)
unsigned int* debug_counter();
rc_status launch_forward(const RenderParams& P, rc_dtype dt, int op, hipStream_t st);
// Work queues of the persistent batched kernel (persist.h): one per XCD,
// their counters kQueueStride ints apart; kQueueGroup consecutive tiles per
// group dealt to the queues round-robin.
constexpr int kQueues = 8, kQueueGroup = 8, kQueueStride = 256;

// The persistent batched kernel over n items already in device memory
// (queue reset included); total = the items' tiles, kinds/order as in
// rc_batch_create, counter = kQueues * kQueueStride ints of device memory
// for the work queues, kind_mask = the set of the items' kinds (bit per kind).
rc_status launch_batch_items(const RenderParams* items, const int* kinds, const int* tile_off,
                             const int* order, int n, int total, int* counter, int lds_bytes,
                             unsigned kind_mask, hipStream_t s);
// Several views of one volume (rc_render_views and its allocation-free
// variant): argument checks, the scratch the call needs, and the enqueue
// with that scratch supplied by the caller.
size_t views_scratch_bytes(const rc_volume* v, int tf_len, const rc_options* opt);
rc_status check_views_args(const rc_volume* v, const rc_camera* cams, int n_views,
                           const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                           const rc_options* opt, float* const* out_rgba, const char* who);
rc_status render_views_into(const rc_volume* v, const rc_camera* cams, int n_views,
                            const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                            const rc_options* opt, float* const* out_rgba, rc_aux* const* aux,
                            char* scratch, hipStream_t s);
// The batched kernel's instantiation of an item: dtype * 3 + operator
// (shaded), 9 + dtype (unshaded), 12 + dtype * 3 + operator (adaptive).
int item_kind(const rc_volume* v, const rc_shading* sh, const rc_options* opt);
// per-lane adaptive-step march (P.adapt > 1)
rc_status launch_adaptive(const RenderParams& P, rc_dtype dt, int op, hipStream_t st);

}  // namespace rc
