// Adaptive sampling (Section 5.2: detail-poor regions are sampled at a lower
// rate).  A sample in an 8^3 brick whose value range is at most adapt_range
// advances its ray by adapt steps, any other by one; each sample's opacity
// is corrected to the distance it stands for.  The sample positions depend
// on the bricks met along each ray, so there is no shared lattice for the
// wave to chunk: each lane marches its own ray and gathers straight from the
// bricked volume.  Arithmetic per sample is the volume mode's (march.h).
#include "march.h"

namespace rc {

template <typename VT, int OP>
__global__ __launch_bounds__(64) void raycast_adaptive(RenderParams P) {
    const ViewParams& V = P.view;
    int tile = tile_of_block(blockIdx.x, V.tiles_x, V.n_tiles / V.tiles_x);
    if (tile < 0) return;
    const int lane = threadIdx.x, tw = V.tile_w, th = 64 / tw;
    int px = (tile % V.tiles_x) * tw + lane % tw;
    int py = (tile / V.tiles_x) * th + lane / tw;
    const bool valid = px < V.W && py < V.H;
    Ray R;
    R.K = -1;
    R.t_in = R.t_out = 0.0;
    for (int a = 0; a < 3; ++a) R.o[a] = R.d[a] = R.p0[a] = R.dp[a] = 0.0;
    if (valid) setup_ray(P, V, px, py, R);
    RayShade rs;
    ray_shade(P, R, rs);
    const GlobalSrc<VT> src{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz,
                             (long long)P.nbx * P.nby * P.nbz * 512, P.dbg};
    const double big_step = (double)P.adapt * P.step;
    float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.0f;
    int j = 0, last = -1;
    unsigned evaluated = 0, shaded = 0;
    if (valid && R.K >= 0) {
        double t = R.t_in;
        while (t <= R.t_out) {
            Cell C;
            double pv[3];
            point_at(P, R, t, C, pv);
            const int b = ((clampi(C.c[2], 0, P.nz - 1) >> 3) * P.nby +
                           (clampi(C.c[1], 0, P.ny - 1) >> 3)) * P.nbx +
                          (clampi(C.c[0], 0, P.nx - 1) >> 3);
            const float2 r = P.range[b];
            const bool poor = (double)r.y - (double)r.x <= (double)P.adapt_range;
            const double step = poor ? big_step : P.step;
            last = j;
            if (!(P.skip && P.empty[RC_IDX(P.dbg, b, (long long)P.nbx * P.nby * P.nbz)])) {
                ++evaluated;
                int ox[4], oy[4], oz[4];
                src.offsets(C, ox, oy, oz);
                float corner[8];
                float v = sample_value<VT>(src.base, ox, oy, oz, C, corner);
                float4 rgba = tf_lookup(P, v);
                float a = rgba.w;
                if (a != 0.0f) {
                    const float e = poor ? P.adapt_e : P.ocorr;
                    if (e > 0.0f) a = 1.0f - __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(1.0f - a));
                    ++shaded;
                    float c[3] = {rgba.x, rgba.y, rgba.z};
                    if (P.shade != RC_SHADE_NONE) {
                        float g[3];
                        gradient<VT, OP, true>(P, src.base, ox, oy, oz, C, g, corner);
                        shade(P, rgba, g, pv, rs, c);
                    }
                    float ta = T * a;
                    Cr = fmaf(ta, c[0], Cr);
                    Cg = fmaf(ta, c[1], Cg);
                    Cb = fmaf(ta, c[2], Cb);
                    T *= (1.0f - a);
                    if (P.tau > 0.0f && 1.0f - T >= P.tau) break;
                }
            }
            t += step;
            ++j;
        }
    }
    if (valid) {
        long long pix = (long long)py * V.W + px;
        V.out[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = make_float4(Cr, Cg, Cb, 1.0f - T);
        if (V.aux) V.aux[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = rc_aux{(int)last, T};
    }
    if (P.stats) {
        unsigned lat = wave_sum(valid ? (unsigned)(last + 1) : 0u);
        unsigned ev = wave_sum(evaluated);
        unsigned sh = wave_sum(shaded);
        unsigned hit = wave_sum(valid && R.K >= 0 ? 1u : 0u);
        if (lane == 0) {
            rc_stats* st = P.stats + (tile & (kStatSlots - 1));
            atomicAdd(&st->lattice_samples, (unsigned long long)lat);
            atomicAdd(&st->evaluated_samples, (unsigned long long)ev);
            atomicAdd(&st->shaded_samples, (unsigned long long)sh);
            atomicAdd(&st->rays_hit, (unsigned long long)hit);
        }
    }
}

template <typename VT>
static void launch_adaptive_t(const RenderParams& P, int op, hipStream_t st) {
    const ViewParams& V = P.view;
    dim3 grid((unsigned)group_grid_blocks(V.tiles_x, V.n_tiles / V.tiles_x)), block(64);
    if (op == RC_GRAD_CENTRAL)
        hipLaunchKernelGGL((raycast_adaptive<VT, RC_GRAD_CENTRAL>), grid, block, 0, st, P);
    else if (op == RC_GRAD_SOBEL3D)
        hipLaunchKernelGGL((raycast_adaptive<VT, RC_GRAD_SOBEL3D>), grid, block, 0, st, P);
    else
        hipLaunchKernelGGL((raycast_adaptive<VT, RC_GRAD_ZUCKER_HUMMEL>), grid, block, 0, st, P);
}

rc_status launch_adaptive(const RenderParams& P, rc_dtype dt, int op, hipStream_t st) {
    if (dt == RC_U8) launch_adaptive_t<uint8_t>(P, op, st);
    else if (dt == RC_U16) launch_adaptive_t<uint16_t>(P, op, st);
    else launch_adaptive_t<float>(P, op, st);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

}  // namespace rc
