// The gradient operators evaluated differences first, for the reverse pass.
//
// Section 3.5.  Each tap of the operator is a trilinear sample at p + o; by
// linearity the gradient at p is the trilinear blend, over the 8 corners c
// of p's cell, of the operator applied at the voxel c:
//   G(p) = sum_c w_c(frac) S(c),
//   S_x(c) = sum_{b,e} W(b,e) [V(c + (1,b,e)) - V(c + (-1,b,e))]   (y, z alike)
// with W = A (x) A + gamma delta (OpTaps).  S is evaluated differences first:
// the +-1 voxel differences come before any weighting, so for integer
// volumes the differences are exact, and with the integer weights of
// central differences and Sobel3D S is an exact integer; otherwise the
// rounding of S is relative to the size of the differences (the gradient)
// rather than of the voxel values.
//
// The forward march evaluates the same operator as separable 4x4x4 filters
// over raw values (march.h: fewer operations per sample); its rounding is
// relative to the values, which is harmless for the image but not for the
// reverse pass, whose normalisation adjoint (I - N N^T)/|G| amplifies the
// error of a small G in a bright region.  The reverse pass recomputes the
// lit colour with this form; it needs the forward's opacities exactly (they
// come from the value path, which both share) but not its colours.
#pragma once

#include "march.h"

namespace rc {

// Arithmetic types of S: differences (DT) and weighted sums (WT).  Integer
// volumes difference in int; sums stay int for the integer weights of
// central differences and Sobel3D and are float for Zucker-Hummel.
template <typename VT, int OP> struct StencilT {
    static constexpr bool kFloatVox = std::is_same<VT, float>::value;
    using DT = typename std::conditional<kFloatVox, float, int>::type;
    using WT = typename std::conditional<kFloatVox || OP == RC_GRAD_ZUCKER_HUMMEL, float,
                                         int>::type;
};

// a1 (p + n) + a0 c: smoothing along one axis
template <int OP, typename WT>
__device__ __forceinline__ WT sm3(WT p, WT c, WT n) {
    if constexpr (std::is_same<WT, int>::value) return (p + n) + 3 * c;
    else if constexpr (OP == RC_GRAD_SOBEL3D) return fmaf(3.0f, c, p + n);
    else return fmaf(OpTaps<OP>::a0, c, OpTaps<OP>::a1 * (p + n));
}
// s + gamma d: the centre term
template <int OP, typename WT>
__device__ __forceinline__ WT centre(WT s, WT d) {
    if constexpr (std::is_same<WT, int>::value) return s - 3 * d;
    else return fmaf(OpTaps<OP>::gamma, d, s);
}

// What one z plane contributes to S at a voxel of the plane below, on or
// above it: v[b][a] = V(x + a - 1, y + b - 1) on that plane.
template <typename WT> struct PlaneP {
    WT ax, ay;          // sum_b A_b dx(b), sum_a A_a dy(a)
    WT dx0, dy0;        // the centre row / column differences
};

template <typename VT, int OP>
__device__ __forceinline__ PlaneP<typename StencilT<VT, OP>::WT> plane_partials(
    const typename StencilT<VT, OP>::DT v[3][3]) {
    using WT = typename StencilT<VT, OP>::WT;
    PlaneP<WT> r;
    r.dx0 = (WT)(v[1][2] - v[1][0]);
    r.dy0 = (WT)(v[2][1] - v[0][1]);
    if constexpr (OpTaps<OP>::kSep) {
        r.ax = sm3<OP, WT>((WT)(v[0][2] - v[0][0]), r.dx0, (WT)(v[2][2] - v[2][0]));
        r.ay = sm3<OP, WT>((WT)(v[2][0] - v[0][0]), r.dy0, (WT)(v[2][2] - v[0][2]));
    } else {
        r.ax = r.ay = (WT)0;
    }
    return r;
}

// S_z at a voxel from the planes below (lo) and above (hi) it.
template <typename VT, int OP>
__device__ __forceinline__ typename StencilT<VT, OP>::WT z_part(
    const typename StencilT<VT, OP>::DT lo[3][3], const typename StencilT<VT, OP>::DT hi[3][3]) {
    using WT = typename StencilT<VT, OP>::WT;
    const WT d11 = (WT)(hi[1][1] - lo[1][1]);
    if constexpr (!OpTaps<OP>::kSep) {
        return d11;
    } else {
        WT r[3];
#pragma unroll
        for (int b = 0; b < 3; ++b)
            r[b] = sm3<OP, WT>((WT)(hi[b][0] - lo[b][0]),
                               b == 1 ? d11 : (WT)(hi[b][1] - lo[b][1]),
                               (WT)(hi[b][2] - lo[b][2]));
        return centre<OP, WT>(sm3<OP, WT>(r[0], r[1], r[2]), d11);
    }
}

// S at a voxel from its three planes' partials and its z part.
template <typename VT, int OP>
__device__ __forceinline__ void voxel_stencil(const PlaneP<typename StencilT<VT, OP>::WT>& lo,
                                              const PlaneP<typename StencilT<VT, OP>::WT>& mid,
                                              const PlaneP<typename StencilT<VT, OP>::WT>& hi,
                                              typename StencilT<VT, OP>::WT sz, float S[3]) {
    using WT = typename StencilT<VT, OP>::WT;
    if constexpr (OpTaps<OP>::kSep) {
        S[0] = (float)centre<OP, WT>(sm3<OP, WT>(lo.ax, mid.ax, hi.ax), mid.dx0);
        S[1] = (float)centre<OP, WT>(sm3<OP, WT>(lo.ay, mid.ay, hi.ay), mid.dy0);
    } else {
        S[0] = (float)mid.dx0;
        S[1] = (float)mid.dy0;
    }
    S[2] = (float)sz;
}

// Gradient at the point of cell C from the 4x4x4 footprint of ox/oy/oz in
// the bricked volume: the operator at each of the cell's 8 corners, then
// their trilinear blend (x, then y, then z), scaled to normalised value per
// world unit like the forward.  corner: the cell's own 8 voxels as the
// value path read them (x + 2y + 4z), exact in FP32 for every volume type.
template <typename VT, int OP>
__device__ __forceinline__ void gradient_exact(const RenderParams& P, const VT* base,
                                               const int ox[4], const int oy[4], const int oz[4],
                                               const Cell& C, const float corner[8], float g[3]) {
    using DT = typename StencilT<VT, OP>::DT;
    using WT = typename StencilT<VT, OP>::WT;
    DT f[4][4][4];              // [z][y][x] of the footprint
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                // central differences never read the footprint's edges
                const bool used = OpTaps<OP>::kSep || (x == 1 || x == 2) + (y == 1 || y == 2) +
                                                          (z == 1 || z == 2) >= 2;
                const bool inner = (x == 1 || x == 2) && (y == 1 || y == 2) && (z == 1 || z == 2);
                f[z][y][x] = inner  ? (DT)corner[(z - 1) * 4 + (y - 1) * 2 + (x - 1)]
                             : used ? (DT)base[ox[x] + oy[y] + oz[z]]
                                    : (DT)0;
            }
    // plane partials of the 4 corner columns on the 4 planes
    PlaneP<WT> pp[4][2][2];
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                DT w[3][3];
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int a = 0; a < 3; ++a) w[b][a] = f[z][cy + b][cx + a];
                pp[z][cy][cx] = plane_partials<VT, OP>(w);
            }
    float sx[8], sy[8], sz[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int cx = q & 1, cy = (q >> 1) & 1, cz = q >> 2;
        DT lo[3][3], hi[3][3];
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[b][a] = f[cz][cy + b][cx + a];
                hi[b][a] = f[cz + 2][cy + b][cx + a];
            }
        float S[3];
        voxel_stencil<VT, OP>(pp[cz][cy][cx], pp[cz + 1][cy][cx], pp[cz + 2][cy][cx],
                              z_part<VT, OP>(lo, hi), S);
        sx[q] = S[0];
        sy[q] = S[1];
        sz[q] = S[2];
    }
    g[0] = trilinear(sx, C) * P.gscale[0];
    g[1] = trilinear(sy, C) * P.gscale[1];
    g[2] = trilinear(sz, C) * P.gscale[2];
}

}  // namespace rc
