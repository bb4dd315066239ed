// First-hit surface mode: the raycaster of Section 3 shows only the surface
// of the material selected by a window of two value thresholds (Section
// 3.11), opaque (Section 3.9 composites nothing).  Each lane marches its
// own ray over a coarse lattice to the first sample inside the window and
// refines the hit by halving steps (Section 5.1: back while inside, forward
// while outside, i.e. a bisection of the last coarse interval), then lights
// the refined point with the gradient and shading of the volume mode.
//
// The march reads values only (8 voxels per sample), so it gathers straight
// from the bricked volume; with skipping, a sample whose brick value range
// misses the window is not evaluated (its trilinear value lies inside that
// range, so it cannot be in the window).
#include <cmath>

#include "march.h"

namespace rc {

struct SurfaceParams {
    float iso_lo, iso_hi;       // the window
    float skip_lo, skip_hi;     // the window widened by a margin, for the brick test
    const float2* range;        // per-brick (min, max), or null without skipping
    int refine;                 // halving steps
    float* t_hit;               // optional [H][W]
};

__device__ __forceinline__ bool in_window(const SurfaceParams& S, float v) {
    return v >= S.iso_lo && v <= S.iso_hi;
}

template <typename VT>
__device__ __forceinline__ float value_of(const GlobalSrc<VT>& src, const Cell& C) {
    int ox[4], oy[4], oz[4];
    src.offsets(C, ox, oy, oz);
    return sample_value<VT>(src.gbase(), ox, oy, oz, C);
}

template <typename VT, int OP>
__global__ __launch_bounds__(64) void raycast_surface(RenderParams P, SurfaceParams S) {
    const ViewParams& V = P.view;
    int tile = tile_of_block(blockIdx.x, V.tiles_x, V.n_tiles / V.tiles_x);
    if (tile < 0) return;
    const int lane = threadIdx.x, tw = V.tile_w, th = 64 / tw;
    int px = (tile % V.tiles_x) * tw + lane % tw;
    int py = (tile / V.tiles_x) * th + lane / tw;
    if (px >= V.W || py >= V.H) return;
    Ray R;
    setup_ray(P, V, px, py, R);
    const GlobalSrc<VT> src{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz,
                             (long long)P.nbx * P.nby * P.nbz * 512, P.dbg};
    Cell C;
    double pv[3];
    // coarse march: the first lattice sample inside the window
    int first = -1;
    for (int k = 0; k <= R.K; ++k) {
        lattice_point(P, R, k, C, pv);
        if (S.range) {
            int b0 = clampi(C.c[0], 0, P.nx - 1) >> 3, b1 = clampi(C.c[1], 0, P.ny - 1) >> 3,
                b2 = clampi(C.c[2], 0, P.nz - 1) >> 3;
            float2 r = S.range[RC_IDX(P.dbg, (b2 * P.nby + b1) * P.nbx + b0,
                                      (long long)P.nbx * P.nby * P.nbz)];
            if (r.y < S.skip_lo || r.x > S.skip_hi) continue;
        }
        if (in_window(S, value_of<VT>(src, C))) {
            first = k;
            break;
        }
    }
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    float t_hit = INFINITY;
    if (first >= 0) {
        double t = R.t_in + (double)first * P.step;
        if (first > 0) {
            // hitpoint refinement: halve the step, back when inside the window
            double h = P.step;
            bool inside = true;
            for (int i = 0; i < S.refine; ++i) {
                h *= 0.5;
                t = inside ? t - h : t + h;
                if (i + 1 < S.refine) {
                    point_at(P, R, t, C, pv);
                    inside = in_window(S, value_of<VT>(src, C));
                }
            }
        }
        point_at(P, R, t, C, pv);
        int ox[4], oy[4], oz[4];
        src.offsets(C, ox, oy, oz);
        float4 rgba = tf_lookup(P, sample_value<VT>(src.gbase(), ox, oy, oz, C));
        float c[3] = {rgba.x, rgba.y, rgba.z};
        if (P.shade != RC_SHADE_NONE) {
            float g[3];
            gradient<VT, OP>(P, src.gbase(), ox, oy, oz, C, g);
            RayShade rs;
            ray_shade(P, R, rs);
            shade(P, rgba, g, pv, rs, c);
        }
        out = make_float4(c[0], c[1], c[2], 1.0f);
        t_hit = (float)t;
    }
    long long pix = (long long)py * V.W + px;
    V.out[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = out;
    if (S.t_hit) S.t_hit[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = t_hit;
}

template <typename VT>
static void launch_surface_t(const RenderParams& P, const SurfaceParams& S, int op,
                             hipStream_t st) {
    const ViewParams& V = P.view;
    dim3 grid((unsigned)group_grid_blocks(V.tiles_x, V.n_tiles / V.tiles_x)), block(64);
    if (op == RC_GRAD_CENTRAL)
        hipLaunchKernelGGL((raycast_surface<VT, RC_GRAD_CENTRAL>), grid, block, 0, st, P, S);
    else if (op == RC_GRAD_SOBEL3D)
        hipLaunchKernelGGL((raycast_surface<VT, RC_GRAD_SOBEL3D>), grid, block, 0, st, P, S);
    else
        hipLaunchKernelGGL((raycast_surface<VT, RC_GRAD_ZUCKER_HUMMEL>), grid, block, 0, st, P, S);
}

}  // namespace rc

using namespace rc;

extern "C" rc_status rc_render_surface(const rc_volume* v, const rc_camera* cam,
                                       const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                                       const rc_surface_options* so, float* out_rgba_dev,
                                       float* t_hit_dev, void* stream) {
    if (!so) return fail(RC_E_INVALID, "rc_render_surface: options is NULL");
    rc_options opt{};       // every field not set below is 0 (off)
    opt.step = so->step;
    for (int a = 0; a < 3; ++a) {
        opt.clip_lo[a] = so->clip_lo[a];
        opt.clip_hi[a] = so->clip_hi[a];
    }
    opt.ert_threshold = 0.0f;
    opt.gradient_op = so->gradient_op;
    opt.skip_empty = so->skip_empty;
    opt.reserved = so->reserved;
    opt.sampling = RC_SAMPLE_TRILINEAR;
    opt.opacity_ref_step = 0.0f;
    if (std::isnan(so->iso_lo) || std::isnan(so->iso_hi) || !(so->iso_lo <= so->iso_hi))
        return fail(RC_E_INVALID, "rc_render_surface: need iso_lo <= iso_hi, not NaN");
    if (so->refine_steps < 0 || so->refine_steps > 30)
        return fail(RC_E_INVALID, "rc_render_surface: refine_steps %d outside 0..30",
                    so->refine_steps);
    rc_status st = check_render_args(v, cam, tf_rgba_dev, tf_len, sh, &opt);
    if (st != RC_OK) return st;
    if (!out_rgba_dev) return fail(RC_E_INVALID, "rc_render_surface: out_rgba_dev is NULL");
    RenderParams P;
    fill_render_params(P, v, cam, tf_rgba_dev, tf_len, sh, &opt);
    P.view.out = (float4*)out_rgba_dev;
    SurfaceParams S;
    S.iso_lo = so->iso_lo;
    S.iso_hi = so->iso_hi;
    // FP32 trilinear values may leave a brick's exact range by rounding;
    // the brick test uses a window widened by far more than that
    float margin = 1e-5f * (v->vmax - v->vmin);
    S.skip_lo = so->iso_lo - margin;
    S.skip_hi = so->iso_hi + margin;
    S.range = so->skip_empty ? v->brick_range : nullptr;
    S.refine = so->refine_steps;
    S.t_hit = t_hit_dev;
    hipStream_t s = (hipStream_t)stream;
    if (v->dtype == RC_U8) launch_surface_t<uint8_t>(P, S, so->gradient_op, s);
    else if (v->dtype == RC_U16) launch_surface_t<uint16_t>(P, S, so->gradient_op, s);
    else launch_surface_t<float>(P, S, so->gradient_op, s);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
