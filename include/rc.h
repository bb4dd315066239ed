/*
 * rc.h -- C ABI of the MI355X (gfx950) volume raycaster.
 *
 * What the library computes follows "Volume Raycasting mit OpenCL"
 * (Kopal): a voxel grid V: N^3 -> R (Section 2.1, eq. 1) is rendered by
 * casting one ray per pixel from a camera (Section 3.3, Section 3.10 step
 * 1), clipping it to a bounding box (Sections 3.3 and 3.6), sampling it at
 * a regular step with trilinear interpolation (Sections 3.3-3.4, eq. 2),
 * colouring each sample through a lookup table (Section 3.7), lighting it
 * with a gradient from the central-difference, Sobel3D or Zucker-Hummel
 * operator (Sections 3.5 and 3.8, eqs. 3-4, Listing 3), and compositing the
 * samples with the transparency formula (Section 3.9, eq. 6) until the ray
 * is opaque.  Empty-space skipping (Section 5.3) uses a grid of 8^3-voxel
 * bricks with per-brick value ranges.
 *
 * Conventions
 *  - World coordinates: voxel (i,j,k) sits at (i*sx, j*sy, k*sz); the
 *    volume box is [0,(nx-1)sx] x [0,(ny-1)sy] x [0,(nz-1)sz].
 *  - Linear voxel arrays are [nz][ny][nx], x fastest.
 *  - Images are [height][width][4] float32, row 0 at the top, RGBA
 *    premultiplied over black; a ray that misses the box gives (0,0,0,0).
 *  - Every device pointer is a HIP device allocation owned by the caller,
 *    except the bricked copy a volume handle owns.  `stream` is a
 *    hipStream_t; NULL means the default stream.  All work is enqueued on
 *    that stream; calls return before it runs.
 *  - Device memory the library allocates itself: a volume handle's bricked
 *    copy and brick ranges (hipMalloc; freed by rc_destroy_volume), a
 *    batch's descriptors, queue and masks (rc_batch_create; freed by
 *    rc_batch_destroy), and the per-call scratch of rc_render and
 *    rc_render_views (skip masks, counters, the views' item descriptors)
 *    and the reverse pass's tile counter (rc_render_backward,
 *    rc_render_backward_views) as stream-ordered allocations on `stream`
 *    (hipMallocAsync, released with hipFreeAsync in the same call).
 *  - Errors: every argument is checked on the host before anything is
 *    enqueued, so a failing call leaves no partial work.  A call returns a
 *    negative rc_status and rc_last_error() describes it.  Nothing aborts
 *    and nothing throws across this interface.
 *  - Threading: calls on distinct volumes may run concurrently; one volume
 *    may be rendered from several threads, but not while it is updated or
 *    destroyed.
 */
#ifndef RC_H
#define RC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RC_OK = 0,
    RC_E_INVALID = -1,      /* a bad argument (null pointer, size, enum, NaN ...) */
    RC_E_OOM = -2,          /* a device allocation failed */
    RC_E_DEVICE = -3,       /* a HIP runtime call failed */
    RC_E_STATE = -4,        /* wrong call order (e.g. skipping before rc_build_bricks) */
    RC_E_UNSUPPORTED = -5   /* a valid request this build does not implement */
} rc_status;

typedef enum { RC_U8 = 0, RC_U16 = 1, RC_F32 = 2 } rc_dtype;

/* Section 3.5: eq. (3), eq. (4), and the Zucker-Hummel operator. */
typedef enum { RC_GRAD_CENTRAL = 0, RC_GRAD_SOBEL3D = 1, RC_GRAD_ZUCKER_HUMMEL = 2 } rc_gradient_op;

/* Section 3.8.  NONE: colour = TF rgb.  BLINN_PHONG: rgb (ka + kd max(0,N.L))
 * + ks max(0,N.H)^shininess with the outward normal N = -G/max(|G|,eps).
 * PAPER_LAMBERT: Listing 3, rgb * dot(normalize(light - p), G/max(|G|,eps)),
 * unclamped, light a point. */
typedef enum { RC_SHADE_NONE = 0, RC_SHADE_BLINN_PHONG = 1, RC_SHADE_PAPER_LAMBERT = 2 } rc_shading_model;

typedef enum { RC_ORTHOGRAPHIC = 0, RC_PERSPECTIVE = 1 } rc_projection;

typedef struct rc_volume rc_volume;   /* opaque: owns the bricked device copy */

/* Camera (Section 3.3: one ray per pixel through the image plane).  Look-at
 * frame f = normalize(target - eye), r = normalize(f x up), u = r x f; pixel
 * centres at x = 2(px+1/2)/W - 1, y = 1 - 2(py+1/2)/H.  Perspective rays
 * start at the eye with d = normalize(f + x tan(fov/2) W/H r + y tan(fov/2) u);
 * orthographic rays have d = f and start at eye + (x W/H r + y u) h/2.
 * Geometry is double so that ray set-up is exact to FP64. */
typedef struct {
    int32_t projection;       /* rc_projection */
    int32_t width, height;    /* image size in pixels, 1..16384 each */
    int32_t reserved;         /* must be 0 */
    double eye[3], target[3], up[3];
    double fov_y_deg;         /* perspective: full vertical field of view, (0, 180) */
    double ortho_height;      /* orthographic: world height of the image, > 0 */
} rc_camera;

typedef struct {
    int32_t model;            /* rc_shading_model */
    int32_t light_is_point;   /* 1: light = world position; 0: direction towards the light */
    float ka, kd, ks, shininess;
    float light[3];
    float grad_eps;           /* > 0: floor of |G| (normalised value per world unit) */
} rc_shading;

/* Section 3.3: coordinates rounded to whole voxels (the simplest scheme,
 * round half up) or trilinear interpolation of the 8 surrounding voxels. */
typedef enum { RC_SAMPLE_TRILINEAR = 0, RC_SAMPLE_NEAREST = 1 } rc_sampling;

typedef struct {
    double step;              /* sample distance in world units, > 0 */
    double clip_lo[3];        /* clip box in world units, intersected with the volume box */
    double clip_hi[3];
    float ert_threshold;      /* 0: off; else stop after the first sample with 1-T >= it, (0,1] */
    int32_t gradient_op;      /* rc_gradient_op */
    int32_t skip_empty;       /* 1: skip bricks whose samples all have alpha 0 (needs rc_build_bricks) */
    int32_t reserved;         /* must be 0 */
    int32_t sampling;         /* rc_sampling; with NEAREST the value and the gradient stencil sit
                                 on the voxel nearest to the sample point */
    float opacity_ref_step;   /* 0: off; > 0: table opacities are per this sample distance and
                                 are corrected to `step`: a = 1 - (1 - a_tf)^(step / ref) */
    int32_t adapt_factor;     /* 0 or 1: fixed step.  2..64: adaptive sampling (Section 5.2):
                                 a sample in an 8^3 brick whose value range (rc_build_bricks)
                                 is at most adapt_range advances the ray by adapt_factor steps,
                                 any other by one; each sample's opacity is corrected to the
                                 distance it stands for, relative to opacity_ref_step or, if
                                 that is 0, to `step`.  Samples are taken while t <= t_out.
                                 Needs rc_build_bricks.  Forward calls only (single, multi-view,
                                 batched); the reverse calls return RC_E_UNSUPPORTED. */
    float adapt_range;        /* raw-value range up to which a brick counts as detail-poor */
} rc_options;

/* Optional per-render counters, accumulated (+=) with device atomics. */
typedef struct {
    unsigned long long lattice_samples;   /* sum over hit rays of (index of last sample + 1) */
    unsigned long long evaluated_samples; /* lattice samples minus those skipped in empty bricks */
    unsigned long long shaded_samples;    /* samples with alpha != 0 */
    unsigned long long rays_hit;          /* rays that met the sampling box */
    /* march diagnostics: a wave marches its rays in chunks of ray parameter */
    unsigned long long chunks_staged;     /* chunks whose voxel box was staged in LDS */
    unsigned long long chunks_empty;      /* chunks skipped: every brick they touch is empty */
    unsigned long long chunks_direct;     /* chunks evaluated from the bricked volume directly */
    unsigned long long samples_direct;    /* evaluated samples that read the bricked volume */
} rc_stats;

/* Per-pixel side output of a forward render, read by the reverse pass. */
typedef struct {
    int32_t k_last;           /* index of the last composited sample, -1 on a miss */
    float t_final;            /* transmittance after that sample */
} rc_aux;

/*
 * Copy a linear voxel grid (Section 2.1, eq. 1; Section 3.1 copies the data
 * to the GPU) into a new handle that owns a brick-tiled device copy: 8^3
 * bricks in x-fastest order, voxels inside a brick in Morton order, edge
 * voxels replicated into the padding.
 *   src_dev   device pointer, [nz][ny][nx] of dtype; read on `stream`, so it
 *             must stay valid until the stream has passed this call
 *   nx,ny,nz  1 .. 4096 each, padded voxel count below 2^31
 *   spacing   world units between neighbouring voxels, finite and > 0
 *   vmin,vmax raw values mapped to transfer-function coordinates 0 and 1,
 *             vmax > vmin
 *   out       receives the handle (NULL on failure)
 * Errors: RC_E_INVALID, RC_E_OOM, RC_E_DEVICE.
 */
rc_status rc_create_volume(const void* src_dev, int nx, int ny, int nz,
                           int32_t dtype /* rc_dtype */, const double spacing[3], float vmin,
                           float vmax, void* stream, rc_volume** out);

/* Overwrite the voxels of `vol` from a grid of the same shape and dtype.
 * If rc_build_bricks ran before, the brick ranges are rebuilt on the same
 * stream.  Errors: RC_E_INVALID, RC_E_DEVICE. */
rc_status rc_update_volume(rc_volume* vol, const void* src_dev, void* stream);

/* Build the per-brick value ranges used by empty-space skipping (Section
 * 5.3): for each 8^3 brick, min and max over the voxels its samples can
 * touch (the brick plus one voxel on its high side).  brick_edge must be 8
 * (RC_E_UNSUPPORTED otherwise).  Errors: RC_E_INVALID, RC_E_OOM,
 * RC_E_DEVICE, RC_E_UNSUPPORTED. */
rc_status rc_build_bricks(rc_volume* vol, int brick_edge, void* stream);

/*
 * Render one image (Section 3.10: raycasting, sampling, shading,
 * compositing).
 *   tf_rgba_dev  device [tf_len][4] float32 lookup table (Section 3.7),
 *                indexed by clamp((v-vmin)/(vmax-vmin),0,1)*(tf_len-1) and
 *                interpolated linearly between entries; 2 <= tf_len <= 65536
 *   out_rgba_dev device [height][width][4] float32
 *   aux_dev      NULL or device [height][width] rc_aux
 *   stats_dev    NULL or a device rc_stats, accumulated
 * Samples: t_k = t_in + k*step, k = 0..floor((t_out-t_in)/step), from the
 * entry to the exit of the ray through the volume box intersected with the
 * clip box.  Each sample: trilinear value, TF colour and opacity a; if a is
 * not 0, a gradient and the shading model; then C += T a c, T *= (1 - a).
 * Output (C, 1 - T).  With skip_empty, samples in bricks whose value range
 * maps to table entries of zero opacity are not evaluated; the image is
 * unchanged because those samples contribute exactly nothing.
 * Errors: RC_E_INVALID, RC_E_STATE (skip_empty before rc_build_bricks),
 * RC_E_OOM, RC_E_DEVICE.
 */
rc_status rc_render(const rc_volume* vol, const rc_camera* cam, const float* tf_rgba_dev,
                    int tf_len, const rc_shading* sh, const rc_options* opt, float* out_rgba_dev,
                    rc_aux* aux_dev, rc_stats* stats_dev, void* stream);

/*
 * Reverse mode of rc_render (the output is differentiable in the voxels and
 * the table almost everywhere; at the kinks -- table breakpoints, max(0, .)
 * in the lighting, the |G| floor -- the derivative of the branch the forward
 * took is used).  With a shading model the chain runs through the lighting,
 * the normalisation and every tap of the gradient operator (up to 64 voxels
 * per sample); where a sample's opacity is 0 its lit colour still enters
 * dL/dalpha.
 *   aux_dev        the rc_aux written by the forward render with the same
 *                  volume contents, camera, table and options
 *   grad_rgba_dev  device [height][width][4] float32, dL/d(output)
 *   grad_volume_dev device [nz][ny][nx] float32, accumulated (+=) with atomics;
 *                  indices follow the clamp-to-edge rule of the sampling
 *   grad_tf_dev    device [tf_len][4] float32, accumulated (+=)
 * The march runs back to front from each ray's last sample and recovers the
 * transmittance from aux.t_final instead of storing per-sample state.
 * Errors: RC_E_INVALID, RC_E_OOM, RC_E_DEVICE.
 */
rc_status rc_render_backward(const rc_volume* vol, const rc_camera* cam, const float* tf_rgba_dev,
                             int tf_len, const rc_shading* sh, const rc_options* opt,
                             const rc_aux* aux_dev, const float* grad_rgba_dev,
                             float* grad_volume_dev, float* grad_tf_dev, void* stream);

/* ------------------------------------------------------------------------
 * Batched rendering: many volumes of uneven size, each with its own camera,
 * image size and table, rendered by ONE persistent kernel launch.  Each
 * item is exactly the argument set of one rc_render call and produces the
 * same image.  Workgroups stay resident and pull (item, tile) work units from
 * a device queue, so small images share the GPU instead of each leaving it
 * mostly idle; the launch can be captured once into a HIP graph and replayed.
 * (Not in the paper: Section 3.10's per-pixel independence is what allows
 * rays of different images to share one launch.)
 * ---------------------------------------------------------------------- */
typedef struct {
    const rc_volume* vol;
    rc_camera cam;
    const float* tf_rgba_dev;   /* device [tf_len][4] */
    int32_t tf_len;
    int32_t reserved;           /* must be 0 */
    rc_shading sh;
    rc_options opt;
    float* out_rgba_dev;        /* device [height][width][4] */
    rc_aux* aux_dev;            /* NULL or device [height][width] */
} rc_batch_item;

/* Launch shape of the persistent kernel and the shape of the voxel boxes
 * its waves stage in LDS.  A wave marches its 64 rays in chunks of ray
 * parameter; each chunk's voxel box (the chunk's cells plus the stencil
 * apron) is staged in LDS.  The box budgets cap a chunk's box in bytes per
 * wave (the chunk length halves until its box fits); every wave of the
 * launch holds the largest budget its items use, so the budgets also set
 * how many waves fit on a compute unit.  The images do not depend on any
 * of these fields (bit-identical to rc_render). */
typedef struct {
    int32_t tile_w;             /* tile width in pixels: 4, 8, 16 or 32 (tiles hold 64 pixels) */
    int32_t waves_per_wg;       /* waves per workgroup: 1, 2 or 4 */
    int32_t wg_per_cu;          /* resident workgroups per compute unit: 1 .. 32 */
    int32_t order;              /* 0: items in the given order; 1: largest images first */
    int32_t box_bytes_grad;     /* LDS box budget per wave of Sobel3D / Zucker-Hummel items
                                   (boxes of FP32 voxels): 0 = 12288, else a multiple of 1024
                                   in 2048 .. 32768 */
    int32_t box_bytes_cd;       /* the same for central-difference items (boxes in the volume's
                                   own type): 0 = 8192, else as above */
    int32_t chunk_len;          /* first chunk length in lattice samples (later chunks adapt):
                                   0 = 16, else 4 .. 64; waves_per_wg times the largest budget
                                   in use must not exceed 65536 */
} rc_batch_config;

typedef struct rc_batch rc_batch;   /* opaque: descriptors, queue, masks, captured graph */

/* Validate every item as rc_render would, upload the descriptors and
 * allocate the queue and mask scratch.  cfg NULL = {8, 1, 8, 1, 0, 0, 0}.  Items
 * that share a volume and a table (the views of an orbit) share one
 * empty-brick mask.  The images are bit-identical to rc_render's.  The
 * items' volumes, tables and outputs must outlive the batch.
 * Errors: RC_E_INVALID (with the failing item index in rc_last_error),
 * RC_E_STATE, RC_E_OOM, RC_E_DEVICE. */
rc_status rc_batch_create(const rc_batch_item* items, int n, const rc_batch_config* cfg,
                          void* stream, rc_batch** out);

/* Render every item with one persistent launch (plus three small mask
 * kernels and a queue reset): resident waves take (item, tile) work from
 * eight work queues, one per XCD (neighbouring tiles stay on one XCD; a
 * wave whose queue is empty takes from the others), which keeps the compute
 * units fuller than one launch per image (an orbit of many views renders
 * faster this way than view by view).  use_graph = 1 captures that sequence into a
 * HIP graph on the first call and replays it afterwards (stream must not be
 * NULL); use_graph = 0 launches eagerly.  Errors: RC_E_INVALID, RC_E_DEVICE. */
rc_status rc_batch_render(rc_batch* b, int use_graph, void* stream);

/* Release a batch (its descriptors, queue, masks and captured graph) after
 * its device has finished all its work, as rc_destroy_volume.  NULL is
 * ignored. */
void rc_batch_destroy(rc_batch* b);

/* create + render (eager) + destroy: one call for one-off batches. */
rc_status rc_render_batch(const rc_batch_item* items, int n, const rc_batch_config* cfg,
                          void* stream);

/* Time candidate configurations on these items and return the fastest in
 * *out.  The search runs in three stages, each keeping the best so far:
 * launch shapes (tile width 8/16/4, 1 or 4 waves per workgroup, 4/8/16
 * resident waves per compute unit, both orders) with the default boxes;
 * then the LDS box budgets of the operator kinds present (8, 12, 16 or 20
 * KiB for Sobel3D / Zucker-Hummel, 4, 8 or 12 KiB for central differences);
 * then the first chunk length (8, 16 or 32).  If cache_path is not NULL,
 * results are kept there as JSON lines keyed by a hash of the items' shapes
 * (volume sizes and types, image sizes, operator, shading, options); a hit
 * returns without timing.  Renders into the items' outputs while timing.
 * Synchronises `stream`.  (This is the autotuner of the batched form; it
 * takes the batch's own items, so it carries the rc_batch_ prefix.)
 * Errors: as rc_batch_create, plus RC_E_INVALID for an unwritable cache. */
rc_status rc_batch_autotune(const rc_batch_item* items, int n, const char* cache_path,
                            void* stream, rc_batch_config* out);

/* ------------------------------------------------------------------------
 * Several views of one volume.  The same volume, table, shading and options
 * rendered from n_views cameras with one launch per 16 views, so small
 * images share the GPU.  Equivalent to n_views rc_render /
 * rc_render_backward calls (Section 3.10: rays are independent).  The
 * forward goes through the persistent kernel of the batch API: its images
 * are bit-identical to rc_render's, adaptive sampling included.
 * ---------------------------------------------------------------------- */
/*   cams      host array [n_views]
 *   out_rgba  host array [n_views] of device pointers, [H_v][W_v][4] each
 *   aux       NULL, or host array [n_views] of device pointers (entries may be NULL)
 * Errors: as rc_render, with the failing view in rc_last_error. */
rc_status rc_render_views(const rc_volume* vol, const rc_camera* cams, int n_views,
                          const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                          const rc_options* opt, float* const* out_rgba, rc_aux* const* aux,
                          void* stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * ---------------------------------------------------------------------- */
/* rc_render_views without any device allocation (no hipMalloc, hipFree or
 * stream-ordered allocation, none by a library it calls).  The per-call
 * scratch -- the views' item descriptors, the work-queue counters, the brick and
 * super-brick skip masks and the table prefix counts -- lives in one fixed
 * device array of RC_NOALLOC_SCRATCH_BYTES inside the library, one copy per
 * device, held from the first call on that device until the process ends.
 * Its size needed by a call is about 17 KiB + (nbricks + nsuper) bytes +
 * 4 (tf_len + 1) bytes with skip_empty, 17 KiB without (a 512^3 volume with
 * skipping and 4096 entries: about 300 KiB).
 * Arguments, images and errors as rc_render_views (the images are
 * bit-identical to it), plus RC_E_INVALID, before anything is enqueued,
 * when a call needs more scratch than the array holds.  Every call on one
 * device shares that device's array and leaves its contents behind; each
 * call rewrites what it reads (masks, descriptors, and the counters, which a
 * kernel clears) before reading it.  Calls that can run at the same time on
 * one device -- on different streams, or enqueued from different threads
 * without ordering -- race on the array: the caller must order them (one
 * stream does). */
#define RC_NOALLOC_SCRATCH_BYTES (4u << 20)
rc_status rc_render_views_noalloc(const rc_volume* vol, const rc_camera* cams, int n_views,
                                  const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                                  const rc_options* opt, float* const* out_rgba,
                                  rc_aux* const* aux, void* stream);

/* Reverse mode of rc_render_views (any shading model): aux[v] and grad_rgba[v] are
 * view v's forward aux and dL/d(rgba); all views accumulate (+=) into one
 * grad_volume_dev and one grad_tf_dev.  Errors: as rc_render_backward. */
rc_status rc_render_backward_views(const rc_volume* vol, const rc_camera* cams, int n_views,
                                   const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                                   const rc_options* opt, const rc_aux* const* aux,
                                   const float* const* grad_rgba, float* grad_volume_dev,
                                   float* grad_tf_dev, void* stream);

/* ------------------------------------------------------------------------
 * First-hit surface mode.  The raycaster of Section 3 draws only the
 * surfaces of the objects in the volume, selected by two thresholds on the
 * data value (Section 3.11), without transparency (Section 3.9).  A coarse
 * march finds the first lattice sample inside the window; hitpoint
 * refinement (Section 5.1, also Section 3.11) then halves the step
 * `refine_steps` times, moving back from a sample inside the window and
 * forward from one outside it, which bisects the last coarse interval
 * (2^n times finer).  A ray whose first sample is already inside (a clip
 * plane through an object) is not refined.  The refined point is coloured
 * with the table's rgb at its value, lit with the gradient and shading
 * model there, and written opaque: (c, 1).  Rays without a surface give
 * (0,0,0,0).
 * ---------------------------------------------------------------------- */
typedef struct {
    double step;              /* coarse sample distance in world units, > 0 */
    double clip_lo[3];        /* clip box in world units, intersected with the volume box */
    double clip_hi[3];
    float iso_lo, iso_hi;     /* raw-value window [iso_lo, iso_hi]; iso_lo <= iso_hi, not NaN */
    int32_t refine_steps;     /* halvings, 0..30 (the paper uses 5 to 6) */
    int32_t gradient_op;      /* rc_gradient_op, for the shading at the hit */
    int32_t skip_empty;       /* 1: skip bricks whose value range misses the window
                                 (needs rc_build_bricks); the image is unchanged */
    int32_t reserved;         /* must be 0 */
} rc_surface_options;

/*   tf_rgba_dev  as rc_render (only rgb is used)
 *   out_rgba_dev device [height][width][4] float32
 *   t_hit_dev    NULL or device [height][width] float32: ray parameter (world
 *                units from the ray origin) of the refined hit, +inf without one
 * Errors: RC_E_INVALID, RC_E_STATE (skip_empty before rc_build_bricks),
 * RC_E_DEVICE. */
rc_status rc_render_surface(const rc_volume* vol, const rc_camera* cam, const float* tf_rgba_dev,
                            int tf_len, const rc_shading* sh, const rc_surface_options* opt,
                            float* out_rgba_dev, float* t_hit_dev, void* stream);

/* Release a handle and its device memory.  Waits until the volume's device
 * has finished all its work first (renders may have read the volume on any
 * stream; the wait is on the volume's device whichever device is current),
 * so destroy handles where stalling that device's other streams is
 * acceptable.  NULL is ignored. */
void rc_destroy_volume(rc_volume* vol);

/* Message for the last non-OK status returned on the calling thread. */
const char* rc_last_error(void);

/* ------------------------------------------------------------------------
 * Bounds-checked build (librc_debug.so, compiled with RC_DEBUG_BOUNDS; for
 * tests).  There every device-side index into a volume, brick mask, table,
 * LDS box, image or gradient buffer is checked against its buffer; an index
 * outside it is counted and replaced by 0, so the access stays inside the
 * buffer and the run goes on.  One counter per device.
 * rc_debug_bounds_violations synchronises the device and writes the count
 * to *out (host pointer); rc_debug_bounds_reset sets it to 0.  In the
 * product build (librc.so) both return RC_E_UNSUPPORTED.
 * ---------------------------------------------------------------------- */
rc_status rc_debug_bounds_violations(unsigned long long* out);
rc_status rc_debug_bounds_reset(void);

#ifdef __cplusplus
}
#endif
#endif
