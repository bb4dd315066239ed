// Device side of the per-pixel raycast (Section 3.10): ray set-up, the
// sample lattice, trilinear sampling, the three gradient operators, the
// lookup table, shading and front-to-back compositing with early ray
// termination and brick skipping.  Included by the forward and batched
// kernels so that both run the same arithmetic.
#pragma once

#include "rc_internal.h"

namespace rc {

// Accumulator type of the integer stencils: exact int32 for u8/u16 voxels.
template <typename T> struct Acc { using type = int; };
template <> struct Acc<float> { using type = float; };

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// ---------------------------------------------------------------- ray set-up
// Camera ray through the centre of pixel (px, py) and its span inside the
// sampling box (Section 3.3: no intersection -> black; two -> sample between).
// FP64 throughout so that the lattice matches the FP64 definition.
struct Ray {
    double o[3], d[3];
    double t_in;
    long long K;        // index of the last lattice sample, -1 on a miss
};

__device__ inline void setup_ray(const RenderParams& P, int px, int py, Ray& R) {
    double x = 2.0 * ((double)px + 0.5) / (double)P.W - 1.0;
    double y = 1.0 - 2.0 * ((double)py + 0.5) / (double)P.H;
    if (P.projection == RC_PERSPECTIVE) {
        double th = P.tan_half;
        double t0 = P.f[0] + x * th * P.aspect * P.r[0] + y * th * P.u[0];
        double t1 = P.f[1] + x * th * P.aspect * P.r[1] + y * th * P.u[1];
        double t2 = P.f[2] + x * th * P.aspect * P.r[2] + y * th * P.u[2];
        double n = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
        double s = n > 0.0 ? 1.0 / n : 0.0;
        R.d[0] = t0 * s; R.d[1] = t1 * s; R.d[2] = t2 * s;
        R.o[0] = P.eye[0]; R.o[1] = P.eye[1]; R.o[2] = P.eye[2];
    } else {
        for (int a = 0; a < 3; ++a) {
            R.d[a] = P.f[a];
            R.o[a] = P.eye[a] + (x * P.aspect * P.r[a] + y * P.u[a]) * P.ortho_half;
        }
    }
    // slab method, t >= 0
    double tmin = 0.0, tmax = INFINITY;
    bool hit = true;
    for (int a = 0; a < 3; ++a) {
        if (R.d[a] == 0.0) {
            if (R.o[a] < P.lo[a] || R.o[a] > P.hi[a]) hit = false;
            continue;
        }
        double ta = (P.lo[a] - R.o[a]) / R.d[a], tb = (P.hi[a] - R.o[a]) / R.d[a];
        if (ta > tb) { double q = ta; ta = tb; tb = q; }
        tmin = fmax(tmin, ta);
        tmax = fmin(tmax, tb);
    }
    for (int a = 0; a < 3; ++a)
        if (P.lo[a] > P.hi[a]) hit = false;
    R.t_in = tmin;
    R.K = -1;
    if (hit && tmin <= tmax) R.K = (long long)floor((tmax - tmin) / P.step);
}

// Voxel-space position of lattice sample k: cell index and fraction.
struct Cell {
    int c[3];
    float fr[3];
};

__device__ __forceinline__ void lattice_point(const RenderParams& P, const Ray& R, long long k,
                                              Cell& C, double pv[3]) {
    double t = R.t_in + (double)k * P.step;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = (R.o[a] + t * R.d[a]) * P.inv_s[a];
        pv[a] = p;
        double fl = floor(p);
        fl = fmin(fmax(fl, -2.0), 1.0e7);
        C.c[a] = (int)fl;
        C.fr[a] = (float)(p - fl);
    }
}

// ---------------------------------------------------------------- sampling
// Trilinear interpolation as 7 lerps, x then y then z (Section 3.4, eq. 2),
// voxel indices clamped to the grid.
template <typename VT>
__device__ __forceinline__ float sample_value(const RenderParams& P, const VT* __restrict__ vox,
                                              const Cell& C) {
    int x0 = clampi(C.c[0], 0, P.nx - 1), x1 = clampi(C.c[0] + 1, 0, P.nx - 1);
    int y0 = clampi(C.c[1], 0, P.ny - 1), y1 = clampi(C.c[1] + 1, 0, P.ny - 1);
    int z0 = clampi(C.c[2], 0, P.nz - 1), z1 = clampi(C.c[2] + 1, 0, P.nz - 1);
    int ox0 = off_x(x0), ox1 = off_x(x1);
    int oy0 = off_y(y0, P.sy), oy1 = off_y(y1, P.sy);
    int oz0 = off_z(z0, P.sz), oz1 = off_z(z1, P.sz);
    float v000 = (float)vox[ox0 + oy0 + oz0], v100 = (float)vox[ox1 + oy0 + oz0];
    float v010 = (float)vox[ox0 + oy1 + oz0], v110 = (float)vox[ox1 + oy1 + oz0];
    float v001 = (float)vox[ox0 + oy0 + oz1], v101 = (float)vox[ox1 + oy0 + oz1];
    float v011 = (float)vox[ox0 + oy1 + oz1], v111 = (float)vox[ox1 + oy1 + oz1];
    float i1 = lerpf(v000, v100, C.fr[0]);
    float i2 = lerpf(v010, v110, C.fr[0]);
    float i3 = lerpf(v001, v101, C.fr[0]);
    float i4 = lerpf(v011, v111, C.fr[0]);
    float i5 = lerpf(i1, i2, C.fr[1]);
    float i6 = lerpf(i3, i4, C.fr[1]);
    return lerpf(i5, i6, C.fr[2]);
}

// Lookup table (Section 3.7): u = clamp((v-vmin)/(vmax-vmin),0,1)*(M-1),
// linear between entries floor(u) and floor(u)+1 (clamped to M-1).
__device__ __forceinline__ float4 tf_lookup(const RenderParams& P, float v) {
    float vn = fminf(fmaxf((v - P.vmin) * P.inv_range, 0.0f), 1.0f);
    float uu = vn * P.Mm1;
    int i = min((int)uu, P.M - 1);
    int i1 = min(i + 1, P.M - 1);
    float t = uu - (float)i;
    float4 a = P.tf[i], b = P.tf[i1];
    return make_float4(lerpf(a.x, b.x, t), lerpf(a.y, b.y, t), lerpf(a.z, b.z, t),
                       lerpf(a.w, b.w, t));
}

// ---------------------------------------------------------------- gradients
// Section 3.5.  Each tap of the operator is a trilinear sample at p + o;
// by linearity that equals the trilinear blend of the integer stencil
// evaluated at the 8 corners of the cell, which is what is computed here:
// the 4x4x4 neighbourhood [c-1, c+2]^3 is gathered (each index clamped to
// the grid), the stencil is applied at the 8 corners in exact integer
// arithmetic for u8/u16 (float for f32 voxels and for the irrational
// Zucker-Hummel weights), and the corner results are blended with the
// same 7-lerp cascade as the value.
//   CD      eq. (3): V(+1) - V(-1) along the axis
//   Sobel3D eq. (4): +1 slice minus -1 slice, weights [[1,3,1],[3,6,3],[1,3,1]]
//   ZH      weights 1/sqrt(1 + b^2 + c^2) on the same slices
// Sobel3D smoothing weights of eq. (4): [[1,3,1],[3,6,3],[1,3,1]].
__host__ __device__ constexpr int sobel_weight(int b, int e) {
    return (b == 0 && e == 0) ? 6 : (b == 0 || e == 0) ? 3 : 1;
}

template <typename VT, int OP>
__device__ __forceinline__ void gradient(const RenderParams& P, const VT* __restrict__ vox,
                                         const Cell& C, float g[3]) {
    using A = typename Acc<VT>::type;
    int ox[4], oy[4], oz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ox[i] = off_x(clampi(C.c[0] - 1 + i, 0, P.nx - 1));
        oy[i] = off_y(clampi(C.c[1] - 1 + i, 0, P.ny - 1), P.sy);
        oz[i] = off_z(clampi(C.c[2] - 1 + i, 0, P.nz - 1), P.sz);
    }
    A B[4][4][4];   // [z][y][x]; unused entries are never loaded (CD)
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int x = 0; x < 4; ++x) B[z][y][x] = (A)vox[ox[x] + oy[y] + oz[z]];

    float S[3][2][2][2];   // [component][cz][cy][cx]
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int X = cx + 1, Y = cy + 1, Z = cz + 1;
                if (OP == RC_GRAD_CENTRAL) {
                    S[0][cz][cy][cx] = (float)(B[Z][Y][X + 1] - B[Z][Y][X - 1]);
                    S[1][cz][cy][cx] = (float)(B[Z][Y + 1][X] - B[Z][Y - 1][X]);
                    S[2][cz][cy][cx] = (float)(B[Z + 1][Y][X] - B[Z - 1][Y][X]);
                } else if (OP == RC_GRAD_SOBEL3D) {
                    A sx = 0, sy = 0, sz = 0;
#pragma unroll
                    for (int b = -1; b <= 1; ++b)
#pragma unroll
                        for (int e = -1; e <= 1; ++e) {
                            const A w = (A)sobel_weight(b, e);
                            sx += w * (B[Z + e][Y + b][X + 1] - B[Z + e][Y + b][X - 1]);
                            sy += w * (B[Z + b][Y + 1][X + e] - B[Z + b][Y - 1][X + e]);
                            sz += w * (B[Z + 1][Y + e][X + b] - B[Z - 1][Y + e][X + b]);
                        }
                    S[0][cz][cy][cx] = (float)sx;
                    S[1][cz][cy][cx] = (float)sy;
                    S[2][cz][cy][cx] = (float)sz;
                } else {
                    float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
                    for (int b = -1; b <= 1; ++b)
#pragma unroll
                        for (int e = -1; e <= 1; ++e) {
                            const int n2 = b * b + e * e;
                            const float w = n2 == 0 ? 1.0f : n2 == 1 ? 0.70710678118654752f
                                                                    : 0.57735026918962576f;
                            sx = fmaf(w, (float)(B[Z + e][Y + b][X + 1] - B[Z + e][Y + b][X - 1]), sx);
                            sy = fmaf(w, (float)(B[Z + b][Y + 1][X + e] - B[Z + b][Y - 1][X + e]), sy);
                            sz = fmaf(w, (float)(B[Z + 1][Y + e][X + b] - B[Z - 1][Y + e][X + b]), sz);
                        }
                    S[0][cz][cy][cx] = sx;
                    S[1][cz][cy][cx] = sy;
                    S[2][cz][cy][cx] = sz;
                }
            }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float i1 = lerpf(S[a][0][0][0], S[a][0][0][1], C.fr[0]);
        float i2 = lerpf(S[a][0][1][0], S[a][0][1][1], C.fr[0]);
        float i3 = lerpf(S[a][1][0][0], S[a][1][0][1], C.fr[0]);
        float i4 = lerpf(S[a][1][1][0], S[a][1][1][1], C.fr[0]);
        float i5 = lerpf(i1, i2, C.fr[1]);
        float i6 = lerpf(i3, i4, C.fr[1]);
        g[a] = lerpf(i5, i6, C.fr[2]) * P.gscale[a];
    }
}

// ---------------------------------------------------------------- shading
// Section 3.8.  G points towards larger values; the outward normal is
// N = -G/max(|G|, eps).  Alpha is never shaded.
__device__ __forceinline__ void shade(const RenderParams& P, const float4& rgba, const float g[3],
                                      const double pv[3], const float dneg[3], float c[3]) {
    float gl = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    float inv = 1.0f / fmaxf(gl, P.grad_eps);
    float gh[3] = {g[0] * inv, g[1] * inv, g[2] * inv};
    float L[3];
    if (P.light_is_point) {
        float q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = P.light[a] - (float)pv[a] * P.s[a];
        float ql = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        float qi = ql > 0.0f ? 1.0f / ql : 0.0f;
        L[0] = q[0] * qi; L[1] = q[1] * qi; L[2] = q[2] * qi;
    } else {
        L[0] = P.light[0]; L[1] = P.light[1]; L[2] = P.light[2];
    }
    if (P.shade == RC_SHADE_PAPER_LAMBERT) {
        // Listing 3: illum = dot(normalize(lightPosition - pos), norm), unclamped
        float illum = L[0] * gh[0] + L[1] * gh[1] + L[2] * gh[2];
        c[0] = rgba.x * illum; c[1] = rgba.y * illum; c[2] = rgba.z * illum;
        return;
    }
    float h[3] = {L[0] + dneg[0], L[1] + dneg[1], L[2] + dneg[2]};
    float hl = sqrtf(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    float hi = hl > 0.0f ? 1.0f / hl : 0.0f;
    float nl = -(gh[0] * L[0] + gh[1] * L[1] + gh[2] * L[2]);
    float nh = -(gh[0] * h[0] + gh[1] * h[1] + gh[2] * h[2]) * hi;
    float diff = fmaxf(nl, 0.0f);
    float spec = nh > 0.0f ? exp2f(P.shininess * log2f(nh)) : (P.shininess == 0.0f ? 1.0f : 0.0f);
    float k = P.ka + P.kd * diff;
    c[0] = fmaf(rgba.x, k, P.ks * spec);
    c[1] = fmaf(rgba.y, k, P.ks * spec);
    c[2] = fmaf(rgba.z, k, P.ks * spec);
}

// ---------------------------------------------------------------- skipping
// Brick of a cell: the brick holding the clamped cell index; every voxel a
// sample in that cell reads lies inside the brick's recorded range.
__device__ __forceinline__ int brick_of(const RenderParams& P, const Cell& C, int b[3]) {
    b[0] = clampi(C.c[0], 0, P.nx - 1) >> 3;
    b[1] = clampi(C.c[1], 0, P.ny - 1) >> 3;
    b[2] = clampi(C.c[2], 0, P.nz - 1) >> 3;
    return (b[2] * P.nby + b[1]) * P.nbx + b[0];
}

// First lattice index that may lie outside brick b, rounded down so that no
// sample outside the brick is ever skipped: along each axis the ray leaves
// the brick through the plane 8(b+1) (moving up) or 8b (moving down); the
// last/first brick extends to the end of the clamped range.
__device__ inline long long brick_exit(const RenderParams& P, const Ray& R, const int b[3],
                                       long long k) {
    const int nb[3] = {P.nbx, P.nby, P.nbz};
    double kmin = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double D = P.step * R.d[a] * P.inv_s[a];
        double P0 = (R.o[a] + R.t_in * R.d[a]) * P.inv_s[a];
        double plane;
        if (D > 0.0) {
            if (b[a] == nb[a] - 1) continue;
            plane = 8.0 * (b[a] + 1);
        } else if (D < 0.0) {
            if (b[a] == 0) continue;
            plane = 8.0 * b[a];
        } else {
            continue;
        }
        kmin = fmin(kmin, (plane - P0) / D);
    }
    if (!(kmin < 9.0e15)) return R.K + 1;
    long long kn = (long long)floor(kmin);
    return kn > k + 1 ? kn : k + 1;
}

// ---------------------------------------------------------------- the march
struct MarchOut {
    float4 rgba;
    int k_last;
    float T;
    unsigned evaluated, shaded;
};

// Section 3.10: sampling -> shading -> compositing, front to back.  The
// transparency formula of Section 3.9 (eq. 6, back to front) is evaluated
// in its equivalent front-to-back form C += T a c, T *= (1 - a); the march
// stops after the first sample with 1 - T >= tau (early ray termination).
template <typename VT, int OP>
__device__ inline void march(const RenderParams& P, const Ray& R, MarchOut& M) {
    const VT* __restrict__ vox = (const VT*)P.vox;
    float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.0f;
    const float dneg[3] = {(float)-R.d[0], (float)-R.d[1], (float)-R.d[2]};
    unsigned evaluated = 0, shaded = 0;
    long long k_last = R.K;
    for (long long k = 0; k <= R.K;) {
        Cell C;
        double pv[3];
        lattice_point(P, R, k, C, pv);
        if (P.skip) {
            int b[3];
            int bi = brick_of(P, C, b);
            if (P.empty[bi]) {
                k = brick_exit(P, R, b, k);
                continue;
            }
        }
        ++evaluated;
        float v = sample_value<VT>(P, vox, C);
        float4 rgba = tf_lookup(P, v);
        float a = rgba.w;
        if (a != 0.0f) {
            ++shaded;
            float c[3] = {rgba.x, rgba.y, rgba.z};
            if (P.shade != RC_SHADE_NONE) {
                float g[3];
                gradient<VT, OP>(P, vox, C, g);
                shade(P, rgba, g, pv, dneg, c);
            }
            float ta = T * a;
            Cr = fmaf(ta, c[0], Cr);
            Cg = fmaf(ta, c[1], Cg);
            Cb = fmaf(ta, c[2], Cb);
            T *= (1.0f - a);
            if (P.tau > 0.0f && 1.0f - T >= P.tau) {
                k_last = k;
                break;
            }
        }
        ++k;
    }
    M.rgba = make_float4(Cr, Cg, Cb, 1.0f - T);
    M.k_last = (int)k_last;
    M.T = T;
    M.evaluated = evaluated;
    M.shaded = shaded;
}

// ---------------------------------------------------------------- one tile
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One wave renders one tile of tile_w x (64 / tile_w) pixels; `tile` is the
// tile's row-major index in the image.  Lanes outside the image idle.
template <typename VT, int OP>
__device__ inline void render_tile(const RenderParams& P, int tile, int lane) {
    const int tw = P.tile_w, th = 64 / P.tile_w;
    int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
    int px = tx * tw + (lane % tw), py = ty * th + (lane / tw);
    bool valid = px < P.W && py < P.H;
    MarchOut M;
    M.rgba = make_float4(0.f, 0.f, 0.f, 0.f);
    M.k_last = -1;
    M.T = 1.0f;
    M.evaluated = M.shaded = 0;
    Ray R;
    R.K = -1;
    if (valid) {
        setup_ray(P, px, py, R);
        if (R.K >= 0) march<VT, OP>(P, R, M);
        long long pix = (long long)py * P.W + px;
        P.out[pix] = M.rgba;
        if (P.aux) P.aux[pix] = rc_aux{M.k_last, M.T};
    }
    if (P.stats) {
        unsigned lat = wave_sum(R.K >= 0 ? (unsigned)(M.k_last + 1) : 0u);
        unsigned ev = wave_sum(M.evaluated);
        unsigned sh = wave_sum(M.shaded);
        unsigned hit = wave_sum(R.K >= 0 ? 1u : 0u);
        if (lane == 0) {
            atomicAdd(&P.stats->lattice_samples, (unsigned long long)lat);
            atomicAdd(&P.stats->evaluated_samples, (unsigned long long)ev);
            atomicAdd(&P.stats->shaded_samples, (unsigned long long)sh);
            atomicAdd(&P.stats->rays_hit, (unsigned long long)hit);
        }
    }
}

}  // namespace rc
