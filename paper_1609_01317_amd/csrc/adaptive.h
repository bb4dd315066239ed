// Adaptive sampling (Section 5.2), one tile of one image: a sample in an
// 8^3 brick whose value range is at most adapt_range advances its ray by
// adapt steps, any other by one, and its opacity is corrected to the
// distance it stands for.  Used by the single-image adaptive kernel and by
// the persistent batched kernel.
//  * shaded renders: the wave marches its rays together in chunks of ray
//    parameter t with LDS-staged voxel boxes (march_wave_adaptive);
//  * unshaded renders (8 voxel reads per sample, nothing to stage): each
//    lane marches its own ray with gathers (adaptive_lanes).
// Both take the same samples in the same FP64 arithmetic and produce the
// same image.
#pragma once

#include "march.h"

namespace rc {

// This lane's samples with t < t_end, all in empty bricks of one step class:
// nothing to evaluate, only the FP64 accumulation of t that the per-sample
// march does.
__device__ __forceinline__ void advance_empty(const Ray& R, double t_end, double step, double& t,
                                              int& j, int& last) {
    while (t < t_end && t <= R.t_out && j <= R.K + 1) {
        last = j;
        t += step;
        ++j;
    }
}

// Cells of this lane's pending samples with t in [t, min(t_end, t_out)]
// reduced over the wave.  Returns false when no lane has one.
__device__ __forceinline__ bool adaptive_cells(const RenderParams& P, const Ray& R, bool active,
                                               double t, double t_end, int cmin[3], int cmax[3]) {
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    if (active && t < t_end) {
        Cell c0, c1;
        double pv[3];
        point_at(P, R, t, c0, pv);
        point_at(P, R, fmin(t_end, R.t_out), c1, pv);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(c0.c[a], c1.c[a]);
            mx[a] = max(c0.c[a], c1.c[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cmin[a] = wave_min(mn[a]);
        cmax[a] = wave_max(mx[a]);
    }
    return cmin[0] <= cmax[0];
}

// Super-brick test of the chunk [tau, tau + len * step), shrinking len until
// its cells span at most 64 super-bricks (not below kSuperMin).  Returns the
// step of every sample in it when all its super-bricks are empty and of one
// step class (all bricks detail-poor, or none), else 0.
__device__ __forceinline__ double adaptive_super_step(const RenderParams& P, const Ray& R,
                                                      bool active, double t, double tau,
                                                      int& len, int lane) {
    const int n[3] = {P.nx, P.ny, P.nz};
    for (;; len >>= 1) {
        int cmin[3], cmax[3];
        if (!adaptive_cells(P, R, active, t, tau + (double)len * P.step, cmin, cmax)) return 0.0;
        int slo[3], sdim[3], nsr = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            slo[a] = clampi(cmin[a], 0, n[a] - 1) >> 5;
            sdim[a] = (clampi(cmax[a], 0, n[a] - 1) >> 5) - slo[a] + 1;
            nsr *= sdim[a];
        }
        if (nsr > 64) {
            if (len <= kSuperMin) return 0.0;
            continue;
        }
        unsigned f = kSuperEmpty | kSuperPoor | kSuperRich;
        if (lane < nsr) {
            const int r01 = small_quot(lane, small_inv(sdim[0]));
            const int r2 = small_quot(r01, small_inv(sdim[1]));
            const int r0 = lane - r01 * sdim[0], r1 = r01 - r2 * sdim[1];
            f = to_gmem(P.super_empty)[RC_IDX(P.dbg,
                                     ((slo[2] + r2) * P.nsy + slo[1] + r1) * P.nsx + slo[0] + r0,
                                     (long long)P.nsx * P.nsy * P.nsz)];
        }
        if (__ballot((f & kSuperEmpty) == 0) != 0ull) return 0.0;
        if (__ballot((f & kSuperPoor) == 0) == 0ull) return (double)P.adapt * P.step;
        if (__ballot((f & kSuperRich) == 0) == 0ull) return P.step;
        return 0.0;
    }
}

// The wave's rays in chunks [tau, tau + len * step) of ray parameter shared
// by its lanes.  Inside a chunk each lane takes its own samples exactly as a
// lane marching alone would: t accumulates in FP64, the sample's brick
// decides its step and whether it is evaluated.  Positions (o + t d) / s are
// monotone in t, so the cells of a lane's samples in the chunk lie between
// the cells at its first pending t and at min(chunk end, t_out); the wave
// reduces those to one voxel box (plus the stencil apron), stages it in LDS
// and reads every sample's cell and 4x4x4 footprint there.  One ballot per
// chunk over its bricks (at most 64) gives which are empty and which are
// detail-poor; the samples of a chunk whose bricks are all empty only
// advance their rays, nothing is staged.  Empty space: at the start and
// after every empty chunk the wave tries a longer chunk against the 32^3
// super-brick flags; when all its super-bricks are empty and of one step
// class, every lane steps through it with that step and no per-sample test.
template <typename VT, int OP>
__device__ inline void march_wave_adaptive(const RenderParams& P, const Ray& R, bool has_ray,
                                           void* lds_raw, int lds_bytes, int lane,
                                           MarchOut& M, int& last) {
    LaneState S;
    S.Cr = S.Cg = S.Cb = 0.f;
    S.T = 1.0f;
    S.k = 0;
    S.k_term = -1;
    S.done = !has_ray || R.K < 0;
    S.evaluated = S.shaded = S.direct = 0;
    unsigned n_staged = 0, n_empty = 0, n_direct = 0;
    RayShade rs;
    ray_shade(P, R, rs);
    const GlobalSrc<VT> gsrc{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz,
                             (long long)P.nbx * P.nby * P.nbz * 512, P.dbg};
    using LT = typename LdsT<VT, OP>::type;
    LT* lds = (LT*)lds_raw;
    const int cap = min(lds_bytes, P.box_bytes) / (int)sizeof(LT);
    const long long nbricks = (long long)P.nbx * P.nby * P.nbz;
    const double big_step = (double)P.adapt * P.step;
    double t = R.t_in;
    int j = 0;
    last = -1;
    int len = P.chunk_init;
    // Every chunk takes at least one sample of the lane that defines its
    // start, and a lane takes at most K + 2 samples, so 64 (K_max + 2)
    // chunks finish any wave; the cap turns a broken invariant into a wrong
    // image instead of a wave that never ends.
    const long long chunk_cap = 64ll * (wave_max(has_ray ? (int)R.K : -1) + 3);
    long long n_chunks = 0;
    bool try_super = P.skip && P.super_empty != nullptr;
    for (;;) {
        bool active = !S.done && t <= R.t_out && j <= R.K + 1;
        if (!active) S.done = true;
        if (__ballot(active) == 0ull || ++n_chunks > chunk_cap) break;
        // the chunk starts at the earliest pending sample of the wave
        const double tau = wave_min_nonneg(active ? t : INFINITY);
        if (try_super) {
            int slen = max(len * 8, kSuperInit);
            const double st = adaptive_super_step(P, R, active, t, tau, slen, lane);
            if (st > 0.0) {
                ++n_empty;
                if (active) advance_empty(R, tau + (double)slen * P.step, st, t, j, last);
                len = min(len * 2, kChunkMax);
                continue;
            }
            try_super = false;
        }
        Chunk ch;
        double tau_end = tau;
        bool fits = false, mine = false;
        for (;;) {
            tau_end = tau + (double)len * P.step;
            mine = active && t < tau_end;
            int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
            if (mine) {
                Cell c0, c1;
                double pv[3];
                point_at(P, R, t, c0, pv);
                point_at(P, R, fmin(tau_end, R.t_out), c1, pv);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(c0.c[a], c1.c[a]);
                    mx[a] = max(c0.c[a], c1.c[a]);
                }
            }
            int cmin[3], cmax[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cmin[a] = wave_min(mn[a]);
                cmax[a] = wave_max(mx[a]);
            }
            if (cmin[0] > cmax[0]) {            // no lane has a sample in the chunk
                fits = false;
                ch.mask_valid = false;
                for (int a = 0; a < 3; ++a) ch.lo[a] = ch.dim[a] = ch.blo[a] = ch.bdim[a] = 0;
                break;
            }
            const int n[3] = {P.nx, P.ny, P.nz};
            long long vol = 1;
            int nbr = 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ch.lo[a] = (cmin[a] - 1) & ~1;                    // even, one voxel of apron
                ch.dim[a] = (((cmax[a] + 2) | 1) - ch.lo[a]) + 1;  // even, two voxels of apron
                vol *= ch.dim[a];
                ch.blo[a] = clampi(cmin[a], 0, n[a] - 1) >> 3;
                ch.bdim[a] = (clampi(cmax[a], 0, n[a] - 1) >> 3) - ch.blo[a] + 1;
                nbr *= ch.bdim[a];
            }
            fits = vol <= cap;
            ch.mask_valid = nbr <= 64;
            if ((fits && ch.mask_valid) || len <= kChunkMin) break;
            len >>= 1;
        }
        // the chunk's bricks: lane i tests brick i (empty, detail-poor)
        unsigned long long live = ~0ull, poorm = 0ull, all = 0ull;
        bool any_live = true;
        if (ch.mask_valid) {
            const int nbr = ch.bdim[0] * ch.bdim[1] * ch.bdim[2];
            all = nbr == 64 ? ~0ull : (1ull << nbr) - 1ull;
            bool lv = false, pr = false;
            if (lane < nbr) {
                const int r01 = small_quot(lane, small_inv(ch.bdim[0]));
                const int r2 = small_quot(r01, small_inv(ch.bdim[1]));
                const int r0 = lane - r01 * ch.bdim[0], r1 = r01 - r2 * ch.bdim[1];
                const int b = ((ch.blo[2] + r2) * P.nby + ch.blo[1] + r1) * P.nbx + ch.blo[0] + r0;
                pr = brick_poor(gload(P.range + RC_IDX(P.dbg, b, nbricks)), P.adapt_range);
                lv = !P.skip || to_gmem(P.empty)[RC_IDX(P.dbg, b, nbricks)] == 0;
            }
            live = __ballot(lv);
            poorm = __ballot(pr);
            any_live = live != 0ull;
        }
        const bool staged = fits && any_live;
        if (staged) {
            ++n_staged;
            stage_box<VT, LT>(P, lds, ch.lo, ch.dim, lane);
            wave_lds_sync();
        } else if (any_live) {
            ++n_direct;
        } else {
            ++n_empty;
        }
        // one step class over the chunk's bricks
        const bool one_class = ch.mask_valid && (poorm == all || poorm == 0ull);
        if (!any_live) {
            // nothing to evaluate, no per-sample test
            if (one_class) {
                if (mine) advance_empty(R, tau_end, poorm ? big_step : P.step, t, j, last);
                len = min(len * 2, kChunkMax);
                try_super = P.super_empty != nullptr;
                continue;
            }
        }
        // every brick live and of one step class: no per-sample brick test
        const bool uniform = one_class && live == all;
        if (mine) {
            const LdsSrc<LT> lsrc{lds, {ch.lo[0], ch.lo[1], ch.lo[2]}, ch.dim[0],
                                  ch.dim[0] * ch.dim[1], ch.dim[0] * ch.dim[1] * ch.dim[2], P.dbg};
            while (t < tau_end && t <= R.t_out && j <= R.K + 1) {
                Cell C;
                double pv[3];
                point_at(P, R, t, C, pv);
                const int b0 = clampi(C.c[0], 0, P.nx - 1) >> 3,
                          b1 = clampi(C.c[1], 0, P.ny - 1) >> 3,
                          b2 = clampi(C.c[2], 0, P.nz - 1) >> 3;
                const int r0 = b0 - ch.blo[0], r1 = b1 - ch.blo[1], r2 = b2 - ch.blo[2];
                bool poor, empty;
                if (uniform) {
                    poor = poorm != 0ull;
                    empty = false;
                } else if (ch.mask_valid && r0 >= 0 && r1 >= 0 && r2 >= 0 && r0 < ch.bdim[0] &&
                           r1 < ch.bdim[1] && r2 < ch.bdim[2]) {
                    const int bit = (r2 * ch.bdim[1] + r1) * ch.bdim[0] + r0;
                    poor = ((poorm >> bit) & 1ull) != 0;
                    empty = ((live >> bit) & 1ull) == 0;
                } else {
                    const int b = (b2 * P.nby + b1) * P.nbx + b0;
                    poor = brick_poor(gload(P.range + RC_IDX(P.dbg, b, nbricks)), P.adapt_range);
                    empty = P.skip && to_gmem(P.empty)[RC_IDX(P.dbg, b, nbricks)] != 0;
                }
                last = j;
                if (!empty) {
                    ++S.evaluated;
                    const float e = poor ? P.adapt_e : P.ocorr;
                    S.direct += staged ? 0u : 1u;
                    const bool term =
                        staged ? shade_sample<VT, OP, true>(P, lsrc, C, pv, rs, S, e)
                               : shade_sample<VT, OP, true>(P, gsrc, C, pv, rs, S, e);
                    if (term) {
                        S.done = true;
                        break;
                    }
                }
                t += poor ? big_step : P.step;
                ++j;
            }
        }
        if (staged) wave_lds_sync();
        if (!any_live) {
            len = min(len * 2, kChunkMax);
            try_super = P.super_empty != nullptr;
        }
    }
    M.rgba = make_float4(S.Cr, S.Cg, S.Cb, 1.0f - S.T);
    M.k_last = last;
    M.T = S.T;
    M.evaluated = S.evaluated;
    M.shaded = S.shaded;
    M.samples_direct = S.direct;
    M.chunks_staged = n_staged;
    M.chunks_empty = n_empty;
    M.chunks_direct = n_direct;
}

// Each lane marches its own ray and gathers from the bricked volume.
template <typename VT, int OP>
__device__ inline void adaptive_lanes(const RenderParams& P, const ViewParams& V, int tile,
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
            const bool poor =
                brick_poor(gload(P.range + RC_IDX(P.dbg, b, (long long)P.nbx * P.nby * P.nbz)),
                           P.adapt_range);
            const double step = poor ? big_step : P.step;
            last = j;
            if (!(P.skip && to_gmem(P.empty)[RC_IDX(P.dbg, b, (long long)P.nbx * P.nby * P.nbz)])) {
                ++evaluated;
                int ox[4], oy[4], oz[4];
                src.offsets(C, ox, oy, oz);
                float corner[8];
                float v = sample_value<VT>(src.gbase(), ox, oy, oz, C, corner);
                float4 rgba = tf_lookup(P, v);
                float a = rgba.w;
                if (a != 0.0f) {
                    const float e = poor ? P.adapt_e : P.ocorr;
                    if (e > 0.0f) a = 1.0f - __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(1.0f - a));
                    ++shaded;
                    float c[3] = {rgba.x, rgba.y, rgba.z};
                    if (P.shade != RC_SHADE_NONE) {
                        float g[3];
                        gradient<VT, OP, true>(P, src.gbase(), ox, oy, oz, C, g, corner);
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

// One tile: the chunked march for shaded renders, the per-lane march for
// unshaded ones.  `lds` holds lds_bytes for the chunked march's boxes.
template <typename VT, int OP>
__device__ inline void adaptive_tile(const RenderParams& P, const ViewParams& V, int tile,
                                     int lane, void* lds, int lds_bytes) {
    if (P.shade == RC_SHADE_NONE) {
        adaptive_lanes<VT, OP>(P, V, tile, lane);
        return;
    }
    const int tw = V.tile_w, th = 64 / tw;
    const int px = (tile % V.tiles_x) * tw + lane % tw;
    const int py = (tile / V.tiles_x) * th + lane / tw;
    const bool valid = px >= 0 && py >= 0 && px < V.W && py < V.H;
    Ray R;
    R.K = -1;
    R.t_in = R.t_out = 0.0;
    for (int a = 0; a < 3; ++a) R.o[a] = R.d[a] = R.p0[a] = R.dp[a] = 0.0;
    if (valid) setup_ray(P, V, px, py, R);
    MarchOut M;
    int last = -1;
    march_wave_adaptive<VT, OP>(P, R, valid, lds, lds_bytes, lane, M, last);
    if (valid) {
        long long pix = (long long)py * V.W + px;
        V.out[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = M.rgba;
        if (V.aux) V.aux[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = rc_aux{last, M.T};
    }
    if (P.stats) {
        unsigned lat = wave_sum(valid ? (unsigned)(last + 1) : 0u);
        unsigned ev = wave_sum(M.evaluated);
        unsigned sh = wave_sum(M.shaded);
        unsigned hit = wave_sum(valid && R.K >= 0 ? 1u : 0u);
        unsigned dir = wave_sum(M.samples_direct);
        if (lane == 0) {
            rc_stats* st = P.stats + (tile & (kStatSlots - 1));
            atomicAdd(&st->lattice_samples, (unsigned long long)lat);
            atomicAdd(&st->evaluated_samples, (unsigned long long)ev);
            atomicAdd(&st->shaded_samples, (unsigned long long)sh);
            atomicAdd(&st->rays_hit, (unsigned long long)hit);
            atomicAdd(&st->chunks_staged, (unsigned long long)M.chunks_staged);
            atomicAdd(&st->chunks_empty, (unsigned long long)M.chunks_empty);
            atomicAdd(&st->chunks_direct, (unsigned long long)M.chunks_direct);
            atomicAdd(&st->samples_direct, (unsigned long long)dir);
        }
    }
}

}  // namespace rc
