// Adaptive sampling (Section 5.2), one tile of one image: each lane
// marches its own ray; a sample in an 8^3 brick whose value range is at
// most adapt_range advances the ray by adapt steps, any other by one, and
// its opacity is corrected to the distance it stands for.  Used by the
// single-image adaptive kernel and by the persistent batched kernel.
#pragma once

#include "march.h"

namespace rc {

template <typename VT, int OP>
__device__ inline void adaptive_tile(const RenderParams& P, const ViewParams& V, int tile,
                                     int lane) {
    const int tw = V.tile_w, th = 64 / tw;
    int px = (tile % V.tiles_x) * tw + lane % tw;
    int py = (tile / V.tiles_x) * th + lane / tw;
    const bool valid = px >= 0 && py >= 0 && px < V.W && py < V.H;
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
        // every step is at least P.step, so a ray takes at most K + 1
        // samples (one more allows for the rounding of the accumulated t);
        // the index bound also ends the loop where t + step == t
        while (t <= R.t_out && j <= R.K + 1) {
            Cell C;
            double pv[3];
            point_at(P, R, t, C, pv);
            const int b = ((clampi(C.c[2], 0, P.nz - 1) >> 3) * P.nby +
                           (clampi(C.c[1], 0, P.ny - 1) >> 3)) * P.nbx +
                          (clampi(C.c[0], 0, P.nx - 1) >> 3);
            const float2 r = P.range[RC_IDX(P.dbg, b, (long long)P.nbx * P.nby * P.nbz)];
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

}  // namespace rc
