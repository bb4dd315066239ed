// Forward render: argument checks, the per-render empty-brick mask and the
// raycast kernel (one ray per pixel, Section 3.10).
#include <atomic>
#include <cmath>

#include "march.h"

namespace rc {

// ---------------------------------------------------------------- empty mask
// prefix[i] = number of table entries j < i with alpha != 0 (one workgroup).
__global__ __launch_bounds__(256) void tf_alpha_prefix(const float4* __restrict__ tf, int M,
                                                       int* __restrict__ prefix) {
    __shared__ int part[256];
    int chunk = (M + 255) / 256;
    int lo = threadIdx.x * chunk, hi = min(lo + chunk, M);
    int cnt = 0;
    for (int i = lo; i < hi; ++i) cnt += tf[i].w != 0.0f;
    part[threadIdx.x] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int t = 0; t < 256; ++t) {
            int c = part[t];
            part[t] = acc;
            acc += c;
        }
        prefix[M] = acc;
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        prefix[i] = acc;
        acc += tf[i].w != 0.0f;
    }
}

// empty[b] = 1 iff every table entry a sample in brick b can interpolate has
// alpha 0.  The value of such a sample lies in the brick's [min, max], so its
// table coordinate lies in [u(min), u(max)] (same FP32 mapping as the march,
// which is monotone); one entry of margin on each side absorbs rounding.
__global__ __launch_bounds__(256) void empty_mask(const float2* __restrict__ range,
                                                  const int* __restrict__ prefix, int M,
                                                  float vmin, float inv_range, float Mm1,
                                                  uint8_t* __restrict__ empty, long long nbricks) {
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbricks) return;
    float2 r = range[b];
    float ulo = fminf(fmaxf((r.x - vmin) * inv_range, 0.0f), 1.0f) * Mm1;
    float uhi = fminf(fmaxf((r.y - vmin) * inv_range, 0.0f), 1.0f) * Mm1;
    int ilo = max((int)ulo - 1, 0);
    int ihi = min((int)uhi + 2, M - 1);
    empty[b] = (prefix[ihi + 1] - prefix[ilo]) == 0;
}

rc_status launch_empty_mask(const rc_volume* v, const float* tf, int tf_len, uint8_t* mask,
                            uint8_t* super_mask, int* prefix, float adapt_range, hipStream_t st) {
    float inv_range = (float)(1.0 / ((double)v->vmax - (double)v->vmin));
    hipLaunchKernelGGL(tf_alpha_prefix, dim3(1), dim3(256), 0, st, (const float4*)tf, tf_len,
                       prefix);
    RC_HIP(hipGetLastError());
    unsigned grid = (unsigned)((v->nbricks + 255) / 256);
    hipLaunchKernelGGL(empty_mask, dim3(grid), dim3(256), 0, st, v->brick_range, prefix, tf_len,
                       v->vmin, inv_range, (float)(tf_len - 1), mask, v->nbricks);
    RC_HIP(hipGetLastError());
    grid = (unsigned)((v->nsuper + 255) / 256);
    hipLaunchKernelGGL(super_mask_kernel, dim3(grid), dim3(256), 0, st, mask, v->brick_range,
                       adapt_range, super_mask, v->nbx, v->nby, v->nbz, v->nsx, v->nsy,
                       v->nsuper);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

__global__ __launch_bounds__(256) void super_mask_kernel(const uint8_t* __restrict__ mask,
                                                         const float2* __restrict__ range,
                                                         float adapt_range,
                                                         uint8_t* __restrict__ smask, int nbx,
                                                         int nby, int nbz, int nsx, int nsy,
                                                         long long nsuper) {
    long long sidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= nsuper) return;
    int sx = (int)(sidx % nsx);
    long long rest = sidx / nsx;
    int sy = (int)(rest % nsy), sz = (int)(rest / nsy);
    // a render without adaptive sampling (NaN) reads no brick ranges
    const bool adaptive = !isnan(adapt_range);
    bool all = true, all_poor = adaptive, no_poor = true;
    for (int bz = sz * 4; bz < min(sz * 4 + 4, nbz); ++bz)
        for (int by = sy * 4; by < min(sy * 4 + 4, nby); ++by)
            for (int bx = sx * 4; bx < min(sx * 4 + 4, nbx); ++bx) {
                const long long b = ((long long)bz * nby + by) * nbx + bx;
                all = all && mask[b] != 0;
                const bool poor = adaptive && brick_poor(range[b], adapt_range);
                all_poor = all_poor && poor;
                no_poor = no_poor && !poor;
            }
    smask[sidx] = (all ? kSuperEmpty : 0) | (all_poor ? kSuperPoor : 0) |
                  (no_poor ? kSuperRich : 0);
}

size_t skip_scratch_bytes(const rc_volume* v, int tf_len, size_t* mask_bytes,
                          size_t* super_bytes) {
    *mask_bytes = ((size_t)v->nbricks + 255) & ~(size_t)255;
    *super_bytes = ((size_t)v->nsuper + 255) & ~(size_t)255;
    return *mask_bytes + *super_bytes + sizeof(int) * ((size_t)tf_len + 1);
}

// ---------------------------------------------------------------- the kernel
// Workgroup = one wave = one pixel tile, placed by tile_of_block.
// Shaded renders keep three waves per SIMD (the register allocator holds
// the march within 168 VGPRs); unshaded ones need neither the gradient's
// registers nor the LDS box and ask for eight.
constexpr int waves_for(bool lit) { return lit ? 3 : 6; }
constexpr int lds_for(bool lit) { return lit ? kWaveLdsBytes : 16; }

template <typename VT, int OP, bool LIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_for(LIT)))) void
raycast_fwd(RenderParams P) {
    __shared__ __align__(16) unsigned char lds[lds_for(LIT)];
    const ViewParams& V = P.view;
    int tile = tile_of_block(blockIdx.x, V.tiles_x, V.n_tiles / V.tiles_x);
    if (tile >= 0) render_tile<VT, OP, LIT>(P, V, tile, threadIdx.x, lds, lds_for(LIT));
}

// Several views of one volume go through the persistent batched kernel: one
// item per view, written to device memory by this single-workgroup kernel
// from the views passed as arguments (no host copy, no synchronisation).
__global__ __launch_bounds__(64) void pack_views(RenderParams P, ViewSet S, int kind,
                                                 RenderParams* __restrict__ items,
                                                 int* __restrict__ kinds,
                                                 int* __restrict__ tile_off,
                                                 int* __restrict__ order) {
    const int i = threadIdx.x;
    if (i < S.n) {
        RenderParams q = P;
        q.view = S.v[i];
        items[i] = q;
        kinds[i] = kind;
        order[i] = i;
    }
    if (i == 0) {
        int t = 0;
        for (int j = 0; j < S.n; ++j) {
            tile_off[j] = t;
            t += S.v[j].n_tiles;
        }
        tile_off[S.n] = t;
    }
}

// ---------------------------------------------------------------- counters
// The render kernel spreads its counters over kStatSlots copies; these two
// kernels clear the copies and fold them into the caller's rc_stats.
constexpr int kStatWords = (int)(sizeof(rc_stats) / sizeof(unsigned long long));

__global__ void stats_clear(unsigned long long* slots) {
    for (int i = threadIdx.x; i < kStatSlots * kStatWords; i += blockDim.x) slots[i] = 0ull;
}

__global__ void stats_fold(const unsigned long long* __restrict__ slots,
                           unsigned long long* __restrict__ out) {
    int w = threadIdx.x;
    if (w >= kStatWords) return;
    unsigned long long acc = 0ull;
    for (int s = 0; s < kStatSlots; ++s) acc += slots[s * kStatWords + w];
    out[w] += acc;
}

template <typename VT>
static void launch_fwd_t(const RenderParams& P, int op, hipStream_t st) {
    const ViewParams& V = P.view;
    dim3 grid((unsigned)group_grid_blocks(V.tiles_x, V.n_tiles / V.tiles_x)), block(64);
    if (P.shade == RC_SHADE_NONE)           // no gradient: the operator does not matter
        hipLaunchKernelGGL((raycast_fwd<VT, RC_GRAD_CENTRAL, false>), grid, block, 0, st, P);
    else if (op == RC_GRAD_CENTRAL)
        hipLaunchKernelGGL((raycast_fwd<VT, RC_GRAD_CENTRAL, true>), grid, block, 0, st, P);
    else if (op == RC_GRAD_SOBEL3D)
        hipLaunchKernelGGL((raycast_fwd<VT, RC_GRAD_SOBEL3D, true>), grid, block, 0, st, P);
    else
        hipLaunchKernelGGL((raycast_fwd<VT, RC_GRAD_ZUCKER_HUMMEL, true>), grid, block, 0, st, P);
}

rc_status launch_forward(const RenderParams& P, rc_dtype dt, int op, hipStream_t st) {
    if (dt == RC_U8) launch_fwd_t<uint8_t>(P, op, st);
    else if (dt == RC_U16) launch_fwd_t<uint16_t>(P, op, st);
    else launch_fwd_t<float>(P, op, st);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

// ---------------------------------------------------------------- host side
static bool finite3(const double a[3]) {
    return std::isfinite(a[0]) && std::isfinite(a[1]) && std::isfinite(a[2]);
}
static void normalize3(const double a[3], double out[3]) {
    double n = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double s = n > 0.0 ? 1.0 / n : 0.0;
    out[0] = a[0] * s; out[1] = a[1] * s; out[2] = a[2] * s;
}
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void sampling_box(const rc_volume* v, const rc_options* opt, double lo[3], double hi[3]) {
    const int n[3] = {v->nx, v->ny, v->nz};
    for (int a = 0; a < 3; ++a) {
        double ext = (n[a] - 1) * v->spacing[a];
        lo[a] = opt->clip_lo[a] > 0.0 ? opt->clip_lo[a] : 0.0;
        hi[a] = opt->clip_hi[a] < ext ? opt->clip_hi[a] : ext;
    }
}

rc_status check_render_args(const rc_volume* v, const rc_camera* cam, const float* tf, int tf_len,
                            const rc_shading* sh, const rc_options* opt) {
    if (!v) return fail(RC_E_INVALID, "volume is NULL");
    if (!cam) return fail(RC_E_INVALID, "camera is NULL");
    if (!tf) return fail(RC_E_INVALID, "transfer function is NULL");
    if (!sh) return fail(RC_E_INVALID, "shading is NULL");
    if (!opt) return fail(RC_E_INVALID, "options is NULL");
    if (cam->projection != RC_PERSPECTIVE && cam->projection != RC_ORTHOGRAPHIC)
        return fail(RC_E_INVALID, "camera: unknown projection %d", cam->projection);
    if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
        return fail(RC_E_INVALID, "camera: image %d x %d outside 1..16384", cam->width, cam->height);
    if (cam->reserved != 0) return fail(RC_E_INVALID, "camera: reserved field must be 0");
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up))
        return fail(RC_E_INVALID, "camera: eye/target/up must be finite");
    double f[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1],
                   cam->target[2] - cam->eye[2]}, fr[3];
    normalize3(f, f);
    cross3(f, cam->up, fr);
    if (f[0] == 0.0 && f[1] == 0.0 && f[2] == 0.0)
        return fail(RC_E_INVALID, "camera: eye equals target");
    if (std::sqrt(fr[0] * fr[0] + fr[1] * fr[1] + fr[2] * fr[2]) < 1e-12)
        return fail(RC_E_INVALID, "camera: up is parallel to the view direction");
    if (cam->projection == RC_PERSPECTIVE &&
        !(std::isfinite(cam->fov_y_deg) && cam->fov_y_deg > 0.0 && cam->fov_y_deg < 180.0))
        return fail(RC_E_INVALID, "camera: fov_y_deg must be in (0, 180)");
    if (cam->projection == RC_ORTHOGRAPHIC &&
        !(std::isfinite(cam->ortho_height) && cam->ortho_height > 0.0))
        return fail(RC_E_INVALID, "camera: ortho_height must be finite and > 0");
    if (tf_len < 2 || tf_len > 65536)
        return fail(RC_E_INVALID, "transfer function length %d outside 2..65536", tf_len);
    if (sh->model != RC_SHADE_NONE && sh->model != RC_SHADE_BLINN_PHONG &&
        sh->model != RC_SHADE_PAPER_LAMBERT)
        return fail(RC_E_INVALID, "shading: unknown model %d", sh->model);
    if (sh->model != RC_SHADE_NONE) {
        if (!(std::isfinite(sh->grad_eps) && sh->grad_eps > 0.0f))
            return fail(RC_E_INVALID, "shading: grad_eps must be finite and > 0");
        if (!(std::isfinite(sh->ka) && std::isfinite(sh->kd) && std::isfinite(sh->ks) &&
              std::isfinite(sh->shininess) && sh->shininess >= 0.0f))
            return fail(RC_E_INVALID, "shading: ka/kd/ks/shininess must be finite, shininess >= 0");
        if (!(std::isfinite(sh->light[0]) && std::isfinite(sh->light[1]) &&
              std::isfinite(sh->light[2])))
            return fail(RC_E_INVALID, "shading: light must be finite");
        if (!sh->light_is_point && sh->light[0] == 0.0f && sh->light[1] == 0.0f &&
            sh->light[2] == 0.0f)
            return fail(RC_E_INVALID, "shading: directional light is the zero vector");
        if (sh->light_is_point != 0 && sh->light_is_point != 1)
            return fail(RC_E_INVALID, "shading: light_is_point must be 0 or 1");
    }
    if (!(std::isfinite(opt->step) && opt->step > 0.0))
        return fail(RC_E_INVALID, "options: step must be finite and > 0");
    if (!(opt->ert_threshold >= 0.0f && opt->ert_threshold <= 1.0f))
        return fail(RC_E_INVALID, "options: ert_threshold must be in [0, 1]");
    if (opt->gradient_op != RC_GRAD_CENTRAL && opt->gradient_op != RC_GRAD_SOBEL3D &&
        opt->gradient_op != RC_GRAD_ZUCKER_HUMMEL)
        return fail(RC_E_INVALID, "options: unknown gradient operator %d", opt->gradient_op);
    if (opt->skip_empty != 0 && opt->skip_empty != 1)
        return fail(RC_E_INVALID, "options: skip_empty must be 0 or 1");
    if (opt->reserved != 0) return fail(RC_E_INVALID, "options: reserved field must be 0");
    if (opt->sampling != RC_SAMPLE_TRILINEAR && opt->sampling != RC_SAMPLE_NEAREST)
        return fail(RC_E_INVALID, "options: unknown sampling %d", opt->sampling);
    if (!(std::isfinite(opt->opacity_ref_step) && opt->opacity_ref_step >= 0.0f))
        return fail(RC_E_INVALID, "options: opacity_ref_step must be finite and >= 0");
    if (opt->adapt_factor < 0 || opt->adapt_factor > 64)
        return fail(RC_E_INVALID, "options: adapt_factor %d outside 0..64", opt->adapt_factor);
    if (std::isnan(opt->adapt_range))
        return fail(RC_E_INVALID, "options: adapt_range is NaN");
    for (int a = 0; a < 3; ++a)
        if (std::isnan(opt->clip_lo[a]) || std::isnan(opt->clip_hi[a]))
            return fail(RC_E_INVALID, "options: clip box has NaN");
    double lo[3], hi[3];
    sampling_box(v, opt, lo, hi);
    double diag2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = hi[a] > lo[a] ? hi[a] - lo[a] : 0.0;
        diag2 += e * e;
    }
    if (std::sqrt(diag2) / opt->step > 16777216.0)
        return fail(RC_E_INVALID, "options: more than 2^24 samples per ray (step too small)");
    if (opt->skip_empty && !v->brick_range)
        return fail(RC_E_STATE, "options: skip_empty needs rc_build_bricks first");
    if (opt->adapt_factor > 1 && !v->brick_range)
        return fail(RC_E_STATE, "options: adaptive sampling needs rc_build_bricks first");
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess && dev != v->device)
        return fail(RC_E_INVALID, "volume lives on device %d, current device is %d", v->device, dev);
    return RC_OK;
}

void set_tiling(ViewParams& V, int tile_w) {
    int th = 64 / tile_w;
    V.tile_w = tile_w;
    V.tiles_x = (V.W + tile_w - 1) / tile_w;
    V.n_tiles = V.tiles_x * ((V.H + th - 1) / th);
}

void fill_view(ViewParams& V, const rc_camera* cam) {
    double tmp[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1],
                     cam->target[2] - cam->eye[2]};
    normalize3(tmp, V.f);
    cross3(V.f, cam->up, tmp);
    normalize3(tmp, V.r);
    cross3(V.r, V.f, V.u);
    for (int a = 0; a < 3; ++a) V.eye[a] = cam->eye[a];
    V.tan_half = std::tan(cam->fov_y_deg * 0.5 * M_PI / 180.0);
    V.aspect = (double)cam->width / (double)cam->height;
    V.ortho_half = cam->ortho_height * 0.5;
    V.projection = cam->projection;
    V.W = cam->width;
    V.H = cam->height;
    set_tiling(V, 8);
    V.out = nullptr;
    V.aux = nullptr;
    V.grad = nullptr;
}

static double op_gain(int op) {
    if (op == RC_GRAD_CENTRAL) return 2.0;
    if (op == RC_GRAD_SOBEL3D) {
        int s = 0;
        for (int b = -1; b <= 1; ++b)
            for (int e = -1; e <= 1; ++e) s += sobel_weight(b, e);
        return 2.0 * s;
    }
    double s = 0.0;
    for (int b = -1; b <= 1; ++b)
        for (int e = -1; e <= 1; ++e) s += 1.0 / std::sqrt(1.0 + b * b + e * e);
    return 2.0 * s;
}

// ---------------------------------------------------------------- bounds-checked build
// One violation counter per device: a file-scope device variable (zero at
// load), whose address on each device is looked up once; null in the
// product build.
#ifdef RC_DEBUG_BOUNDS
static __device__ unsigned int g_dbg_count;
static std::atomic<unsigned int*> g_dbg[64];
#endif
unsigned int* debug_counter() {
#ifdef RC_DEBUG_BOUNDS
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    unsigned int* p = g_dbg[dev].load(std::memory_order_acquire);
    if (!p) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(g_dbg_count)) != hipSuccess) return nullptr;
        p = (unsigned int*)q;
        g_dbg[dev].store(p, std::memory_order_release);
    }
    return p;
#else
    return nullptr;
#endif
}

extern "C" rc_status rc_debug_bounds_violations(unsigned long long* out) {
    if (!out) return fail(RC_E_INVALID, "rc_debug_bounds_violations: out is NULL");
#ifdef RC_DEBUG_BOUNDS
    unsigned int* p = debug_counter();
    if (!p) return fail(RC_E_DEVICE, "rc_debug_bounds_violations: no counter on this device");
    unsigned int h = 0;
    RC_HIP(hipDeviceSynchronize());
    RC_HIP(hipMemcpy(&h, p, sizeof h, hipMemcpyDeviceToHost));
    *out = h;
    return RC_OK;
#else
    return fail(RC_E_UNSUPPORTED, "rc_debug_bounds_violations: built without bounds checks");
#endif
}

extern "C" rc_status rc_debug_bounds_reset(void) {
#ifdef RC_DEBUG_BOUNDS
    unsigned int* p = debug_counter();
    if (!p) return fail(RC_E_DEVICE, "rc_debug_bounds_reset: no counter on this device");
    RC_HIP(hipDeviceSynchronize());
    RC_HIP(hipMemset(p, 0, sizeof(unsigned int)));
    RC_HIP(hipDeviceSynchronize());
    return RC_OK;
#else
    return fail(RC_E_UNSUPPORTED, "rc_debug_bounds_reset: built without bounds checks");
#endif
}

void fill_render_params(RenderParams& P, const rc_volume* v, const rc_camera* cam,
                        const float* tf, int tf_len, const rc_shading* sh, const rc_options* opt) {
    fill_view(P.view, cam);
    sampling_box(v, opt, P.lo, P.hi);
    P.step = opt->step;
    P.inv_step = 1.0 / opt->step;
    for (int a = 0; a < 3; ++a) {
        P.inv_s[a] = 1.0 / v->spacing[a];
        P.s[a] = (float)v->spacing[a];
    }
    P.vox = v->bricked;
    P.nx = v->nx; P.ny = v->ny; P.nz = v->nz;
    P.sy = v->nbx * kBrickVox;
    P.sz = v->nbx * v->nby * kBrickVox;
    P.nbx = v->nbx; P.nby = v->nby; P.nbz = v->nbz;
    double range = (double)v->vmax - (double)v->vmin;
    P.vmin = v->vmin;
    P.inv_range = (float)(1.0 / range);
    P.tf = (const float4*)tf;
    P.M = tf_len;
    P.Mm1 = (float)(tf_len - 1);
    double gain = op_gain(opt->gradient_op);
    for (int a = 0; a < 3; ++a) P.gscale[a] = (float)(1.0 / (gain * v->spacing[a] * range));
    P.shade = sh->model;
    P.ka = sh->ka; P.kd = sh->kd; P.ks = sh->ks; P.shininess = sh->shininess;
    P.light_is_point = sh->light_is_point;
    if (sh->light_is_point) {
        for (int a = 0; a < 3; ++a) P.light[a] = sh->light[a];
    } else {
        double l[3] = {sh->light[0], sh->light[1], sh->light[2]}, ln[3];
        normalize3(l, ln);
        for (int a = 0; a < 3; ++a) P.light[a] = (float)ln[a];
    }
    P.grad_eps = sh->grad_eps;
    P.tau = opt->ert_threshold;
    P.skip = opt->skip_empty;
    P.nearest = opt->sampling == RC_SAMPLE_NEAREST;
    P.round_bias = P.nearest ? 0.5 : 0.0;
    P.frac_keep = P.nearest ? 0.0f : 1.0f;
    // exponent 1 is the identity: left off (0) so no kernel meets 0^0
    double e = opt->opacity_ref_step > 0.0f ? opt->step / (double)opt->opacity_ref_step : 0.0;
    P.ocorr = e == 1.0 ? 0.0f : (float)e;
    P.adapt = opt->adapt_factor > 1 ? opt->adapt_factor : 0;
    P.adapt_range = opt->adapt_range;
    {
        // exponent of a sample that stands for adapt_factor steps
        double ref = opt->opacity_ref_step > 0.0f ? (double)opt->opacity_ref_step : opt->step;
        double ea = (double)opt->adapt_factor * opt->step / ref;
        P.adapt_e = ea == 1.0 ? 0.0f : (float)ea;
    }
    P.range = v->brick_range;
    P.empty = nullptr;
    P.super_empty = nullptr;
    P.nsx = v->nsx;
    P.nsy = v->nsy;
    P.nsz = v->nsz;
    P.stats = nullptr;
    P.dbg = debug_counter();
    P.box_bytes = kWaveLdsBytes;
    P.chunk_init = kChunkInit;
}

}  // namespace rc

using namespace rc;

extern "C" rc_status rc_render(const rc_volume* v, const rc_camera* cam, const float* tf_rgba_dev,
                               int tf_len, const rc_shading* sh, const rc_options* opt,
                               float* out_rgba_dev, rc_aux* aux_dev, rc_stats* stats_dev,
                               void* stream) {
    rc_status st = check_render_args(v, cam, tf_rgba_dev, tf_len, sh, opt);
    if (st != RC_OK) return st;
    if (!out_rgba_dev) return fail(RC_E_INVALID, "rc_render: out_rgba_dev is NULL");
    hipStream_t s = (hipStream_t)stream;
    RenderParams P;
    fill_render_params(P, v, cam, tf_rgba_dev, tf_len, sh, opt);
    P.view.out = (float4*)out_rgba_dev;
    P.view.aux = aux_dev;
    // per-render scratch: counter slots, empty mask, table prefix counts
    const size_t stat_bytes = stats_dev ? sizeof(rc_stats) * kStatSlots : 0;
    size_t mask_bytes = 0, super_bytes = 0;
    const size_t skip_bytes =
        opt->skip_empty ? skip_scratch_bytes(v, tf_len, &mask_bytes, &super_bytes) : 0;
    void* scratch = nullptr;
    if (stat_bytes + skip_bytes > 0) RC_HIP(hipMallocAsync(&scratch, stat_bytes + skip_bytes, s));
    char* sp = (char*)scratch;
    if (stats_dev) {
        P.stats = (rc_stats*)sp;
        hipLaunchKernelGGL(stats_clear, dim3(1), dim3(256), 0, s, (unsigned long long*)sp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = hip_fail(e, "stats_clear");
    }
    if (st == RC_OK && opt->skip_empty) {
        uint8_t* mask = (uint8_t*)(sp + stat_bytes);
        uint8_t* smask = mask + mask_bytes;
        int* prefix = (int*)(smask + super_bytes);
        st = launch_empty_mask(v, tf_rgba_dev, tf_len, mask, smask, prefix,
                               P.adapt ? P.adapt_range : NAN, s);
        P.empty = mask;
        P.super_empty = smask;
    }
    if (st == RC_OK)
        st = P.adapt ? launch_adaptive(P, v->dtype, opt->gradient_op, s)
                     : launch_forward(P, v->dtype, opt->gradient_op, s);
    if (st == RC_OK && stats_dev) {
        hipLaunchKernelGGL(stats_fold, dim3(1), dim3(64), 0, s, (const unsigned long long*)sp,
                           (unsigned long long*)stats_dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = hip_fail(e, "stats_fold");
    }
    if (scratch) {
        hipError_t e = hipFreeAsync(scratch, s);
        if (st == RC_OK && e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    }
    return st;
}

namespace rc {

// ---------------------------------------------------------------- several views
// Several views of one volume, table, shading and options in as few launches
// as possible (up to kMaxViews views per launch).  The per-call scratch
// holds the items of one launch, their kinds, tile offsets and order (one
// 256-byte slot each, kViewsMetaBytes in all) and the work-queue counters,
// then the skip masks.
constexpr size_t kViewsMetaBytes = 1024;

size_t views_scratch_bytes(const rc_volume* v, int tf_len, const rc_options* opt) {
    const size_t items_bytes = ((sizeof(RenderParams) * kMaxViews + 255) / 256) * 256;
    const size_t queue_bytes = kViewsMetaBytes + sizeof(int) * kQueues * kQueueStride;
    size_t mask_bytes = 0, super_bytes = 0, skip_bytes = 0;
    if (opt->skip_empty) skip_bytes = skip_scratch_bytes(v, tf_len, &mask_bytes, &super_bytes);
    return items_bytes + queue_bytes + skip_bytes;
}

rc_status check_views_args(const rc_volume* v, const rc_camera* cams, int n_views,
                           const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                           const rc_options* opt, float* const* out_rgba, const char* who) {
    if (!cams || !out_rgba) return fail(RC_E_INVALID, "%s: cams/out_rgba is NULL", who);
    if (n_views < 1) return fail(RC_E_INVALID, "%s: n_views must be >= 1", who);
    for (int i = 0; i < n_views; ++i) {
        rc_status st = check_render_args(v, &cams[i], tf_rgba_dev, tf_len, sh, opt);
        if (st != RC_OK) return fail(st, "view %d: %s", i, rc_last_error());
        if (!out_rgba[i]) return fail(RC_E_INVALID, "view %d: out_rgba is NULL", i);
    }
    return RC_OK;
}

int item_kind(const rc_volume* v, const rc_shading* sh, const rc_options* opt) {
    if (opt->adapt_factor > 1) return 12 + (int)v->dtype * 3 + opt->gradient_op;
    if (sh->model == RC_SHADE_NONE) return 9 + (int)v->dtype;
    return (int)v->dtype * 3 + opt->gradient_op;
}

// The enqueue part of rc_render_views, with `scratch` (device memory of at
// least views_scratch_bytes, 256-byte aligned) supplied by the caller.
// Everything in it is written by this call's kernels before it is read: the
// skip masks by the mask kernels, the items by pack_views, the counter by
// the batch kernel's reset.
rc_status render_views_into(const rc_volume* v, const rc_camera* cams, int n_views,
                            const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                            const rc_options* opt, float* const* out_rgba, rc_aux* const* aux,
                            char* scratch, hipStream_t s) {
    RenderParams P;
    fill_render_params(P, v, &cams[0], tf_rgba_dev, tf_len, sh, opt);
    const bool lit = sh->model != RC_SHADE_NONE;
    const int kind = item_kind(v, sh, opt);
    // unshaded marches stage nothing
    const int lds_bytes = !lit ? 16
                          : opt->gradient_op != RC_GRAD_CENTRAL ? kWaveLdsBytes
                                                                : kBatchWaveLdsBytes;
    P.box_bytes = lds_bytes;
    const size_t items_bytes = ((sizeof(RenderParams) * kMaxViews + 255) / 256) * 256;
    const size_t queue_bytes = kViewsMetaBytes + sizeof(int) * kQueues * kQueueStride;
    size_t mask_bytes = 0, super_bytes = 0;
    if (opt->skip_empty) (void)skip_scratch_bytes(v, tf_len, &mask_bytes, &super_bytes);
    char* base = scratch;
    RenderParams* items = (RenderParams*)base;
    int* kinds = (int*)(base + items_bytes);
    int* tile_off = (int*)(base + items_bytes + 256);
    int* order = (int*)(base + items_bytes + 512);
    int* counter = (int*)(base + items_bytes + kViewsMetaBytes);  // work-queue counters
    rc_status st = RC_OK;
    if (opt->skip_empty) {
        char* sk = base + items_bytes + queue_bytes;
        P.empty = (uint8_t*)sk;
        P.super_empty = P.empty + mask_bytes;
        st = launch_empty_mask(v, tf_rgba_dev, tf_len, (uint8_t*)P.empty,
                               (uint8_t*)P.super_empty, (int*)(sk + mask_bytes + super_bytes),
                               P.adapt ? P.adapt_range : NAN, s);
    }
    for (int first = 0; st == RC_OK && first < n_views; first += kMaxViews) {
        ViewSet S;
        S.n = n_views - first < kMaxViews ? n_views - first : kMaxViews;
        int total = 0;
        for (int j = 0; j < S.n; ++j) {
            ViewParams& V = S.v[j];
            fill_view(V, &cams[first + j]);
            V.out = (float4*)out_rgba[first + j];
            V.aux = aux ? aux[first + j] : nullptr;
            S.block_off[j] = total;
            total += V.n_tiles;
        }
        S.block_off[S.n] = total;
        hipLaunchKernelGGL(pack_views, dim3(1), dim3(64), 0, s, P, S, kind, items, kinds,
                           tile_off, order);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            st = hip_fail(e, "pack_views");
            break;
        }
        st = launch_batch_items(items, kinds, tile_off, order, S.n, total, counter, lds_bytes,
                                1u << kind, s);
    }
    return st;
}

}  // namespace rc

extern "C" rc_status rc_render_views(const rc_volume* v, const rc_camera* cams, int n_views,
                                     const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                                     const rc_options* opt, float* const* out_rgba,
                                     rc_aux* const* aux, void* stream) {
    rc_status st = check_views_args(v, cams, n_views, tf_rgba_dev, tf_len, sh, opt, out_rgba,
                                    "rc_render_views");
    if (st != RC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    void* scratch = nullptr;
    RC_HIP(hipMallocAsync(&scratch, views_scratch_bytes(v, tf_len, opt), s));
    st = render_views_into(v, cams, n_views, tf_rgba_dev, tf_len, sh, opt, out_rgba, aux,
                           (char*)scratch, s);
    hipError_t e = hipFreeAsync(scratch, s);
    if (st == RC_OK && e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return st;
}

// ---------------------------------------------------------------- allocation-free views
// rc_render_views' scratch in a fixed device array instead of a
// stream-ordered allocation.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[RC_NOALLOC_SCRATCH_BYTES];
static std::atomic<char*> g_scratch_dev[64];

static rc_status noalloc_scratch(char** out) {
    int dev = -1;
    RC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        return fail(RC_E_UNSUPPORTED, "rc_render_views_noalloc: device %d (at most 64 devices)", dev);
    char* p = g_scratch_dev[dev].load(std::memory_order_acquire);
    if (!p) {
        void* q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        // threads racing here store the same address
        p = (char*)q;
        g_scratch_dev[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return RC_OK;
}

extern "C" rc_status rc_render_views_noalloc(const rc_volume* v, const rc_camera* cams,
                                             int n_views, const float* tf_rgba_dev, int tf_len,
                                             const rc_shading* sh, const rc_options* opt,
                                             float* const* out_rgba, rc_aux* const* aux,
                                             void* stream) {
    rc_status st = check_views_args(v, cams, n_views, tf_rgba_dev, tf_len, sh, opt, out_rgba,
                                    "rc_render_views_noalloc");
    if (st != RC_OK) return st;
    const size_t need = views_scratch_bytes(v, tf_len, opt);
    if (need > (size_t)RC_NOALLOC_SCRATCH_BYTES)
        return fail(RC_E_INVALID,
                    "rc_render_views_noalloc: this call needs %zu bytes of scratch, more than the "
                    "%u the library holds (fewer bricks or table entries, or rc_render_views)",
                    need, (unsigned)RC_NOALLOC_SCRATCH_BYTES);
    char* sp = nullptr;
    st = noalloc_scratch(&sp);
    if (st != RC_OK) return st;
    return render_views_into(v, cams, n_views, tf_rgba_dev, tf_len, sh, opt, out_rgba, aux, sp,
                             (hipStream_t)stream);
}
