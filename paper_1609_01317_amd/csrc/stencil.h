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
    // S at the 8 corners (i, j, k) = footprint voxel (i + 1, j + 1, k + 1),
    // separably and differences first: the +-1 differences along each axis
    // at the corner positions, then the smoothing along the other two axes,
    // then the centre term.  S_x: x differences, smoothed along y, then z.
    WT s3[3][2][2][2];              // [component][k][j][i]
    if constexpr (OpTaps<OP>::kSep) {
        WT dx[4][4][2], dy[4][2][4], dz[2][4][4];
#pragma unroll
        for (int z = 0; z < 4; ++z)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    if (x < 2) dx[z][y][x] = (WT)(f[z][y][x + 2] - f[z][y][x]);
                    if (y < 2) dy[z][y][x] = (WT)(f[z][y + 2][x] - f[z][y][x]);
                    if (z < 2) dz[z][y][x] = (WT)(f[z + 2][y][x] - f[z][y][x]);
                }
        WT tx[4][2][2], ty[4][2][2], tz[2][4][2];
#pragma unroll
        for (int z = 0; z < 4; ++z)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    tx[z][j][i] = sm3<OP, WT>(dx[z][j][i], dx[z][j + 1][i], dx[z][j + 2][i]);
                    ty[z][j][i] = sm3<OP, WT>(dy[z][j][i], dy[z][j][i + 1], dy[z][j][i + 2]);
                }
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    tz[k][y][i] = sm3<OP, WT>(dz[k][y][i], dz[k][y][i + 1], dz[k][y][i + 2]);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    s3[0][k][j][i] = centre<OP, WT>(
                        sm3<OP, WT>(tx[k][j][i], tx[k + 1][j][i], tx[k + 2][j][i]),
                        dx[k + 1][j + 1][i]);
                    s3[1][k][j][i] = centre<OP, WT>(
                        sm3<OP, WT>(ty[k][j][i], ty[k + 1][j][i], ty[k + 2][j][i]),
                        dy[k + 1][j][i + 1]);
                    s3[2][k][j][i] = centre<OP, WT>(
                        sm3<OP, WT>(tz[k][j][i], tz[k][j + 1][i], tz[k][j + 2][i]),
                        dz[k][j + 1][i + 1]);
                }
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    s3[0][k][j][i] = (WT)(f[k + 1][j + 1][i + 2] - f[k + 1][j + 1][i]);
                    s3[1][k][j][i] = (WT)(f[k + 1][j + 2][i + 1] - f[k + 1][j][i + 1]);
                    s3[2][k][j][i] = (WT)(f[k + 2][j + 1][i + 1] - f[k][j + 1][i + 1]);
                }
    }
    float sx[8], sy[8], sz[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int i = q & 1, j = (q >> 1) & 1, k = q >> 2;
        sx[q] = (float)s3[0][k][j][i];
        sy[q] = (float)s3[1][k][j][i];
        sz[q] = (float)s3[2][k][j][i];
    }
    g[0] = trilinear(sx, C) * P.gscale[0];
    g[1] = trilinear(sy, C) * P.gscale[1];
    g[2] = trilinear(sz, C) * P.gscale[2];
}

}  // namespace rc
