// Device side of the per-pixel raycast (Section 3.10): ray set-up, the
// sample lattice, trilinear sampling, the three gradient operators, the
// lookup table, shading and front-to-back compositing with early ray
// termination and brick skipping.  Included by the forward and batched
// kernels so that both run the same arithmetic.
//
// Execution model: one wave (64 lanes) renders one pixel tile, one ray per
// lane.  The wave marches in chunks of ray parameter t shared by all its
// lanes.  For each chunk it reduces the lanes' sample cells to one
// axis-aligned voxel box, asks the brick grid (one brick per lane, a wave
// ballot) whether any sample in the chunk can have non-zero opacity, and
// if so stages the box -- the chunk's cells plus the one-voxel-low /
// two-voxel-high apron the 3x3x3 stencils and the trilinear corners need --
// in LDS with 16-byte Morton-group loads.  The samples then read their
// 8-voxel cell and 64-voxel stencil neighbourhood from LDS.  A chunk whose
// box does not fit falls back to per-lane gathers from the bricked volume;
// both sources hold the same voxel values, so the arithmetic and the
// result are identical.
#pragma once

#include <climits>
#include <type_traits>

#include "rc_internal.h"

namespace rc {

constexpr int kWaveLdsBytes = 12288;    // LDS box budget per wave (single-image kernels)
constexpr int kBatchWaveLdsBytes = 8192; // per wave in the batched kernel (measured better there)
constexpr int kStatSlots = 64;          // per-render counter copies (see render_tile)

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// n / d for 0 <= n, 1 <= d, n + d < 2^20 without an integer division:
// (n + 1/2) / d lies at least 1 / (2d) from an integer, and the FP32 product
// with the reciprocal (hardware rcp, within 1 ulp) is within 2^-21 of it
// relatively, so truncation gives the exact quotient.
__device__ __forceinline__ float small_inv(int d) { return __builtin_amdgcn_rcpf((float)d); }
__device__ __forceinline__ int small_quot(int n, float inv_d) {
    return (int)(((float)n + 0.5f) * inv_d);
}

// Device memory read through global (not flat) loads: a wait for them does
// not also wait for the wave's LDS traffic, nor a wait for LDS for them.
template <typename T>
using gmem = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gmem<T> to_gmem(const T* p) {
    return (gmem<T>)p;
}
// The same for the HIP vector structs (their constructors take generic
// references): loaded as a builtin vector of 32-bit words.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
    typedef unsigned words __attribute__((ext_vector_type(sizeof(T) / 4)));
    return __builtin_bit_cast(T, *(gmem<words>)p);
}

// Adaptive sampling (Section 5.2): a brick is detail-poor when its value
// range is at most adapt_range (NaN: no brick is).
__device__ __forceinline__ bool brick_poor(float2 r, float adapt_range) {
    return (double)r.y - (double)r.x <= (double)adapt_range;
}

// ---------------------------------------------------------------- wave helpers
// Wave-wide min / max through DPP lane moves (quad permutes, row mirrors,
// row broadcasts 15 and 31): the total lands in lane 63 and is read back as
// a wave-uniform scalar.
template <typename Op>
__device__ __forceinline__ int wave_reduce_dpp(int v, int ident, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
struct MinOp { __device__ int operator()(int a, int b) const { return min(a, b); } };
struct MaxOp { __device__ int operator()(int a, int b) const { return max(a, b); } };
__device__ __forceinline__ int wave_min(int v) { return wave_reduce_dpp(v, INT_MAX, MinOp()); }
__device__ __forceinline__ int wave_max(int v) { return wave_reduce_dpp(v, INT_MIN, MaxOp()); }
// Minimum of non-negative doubles (+inf allowed), exact: their bit patterns
// order like unsigned 64-bit integers, so the same DPP steps run on both
// halves with a 64-bit compare (no LDS permutes).
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const int ones = -1;    // identity of the minimum in lanes the move does not write
    unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(ones, (int)(unsigned)v, CTRL, ROWS, 0xF, false);
    unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(ones, (int)(unsigned)(v >> 32), CTRL, ROWS, 0xF, false);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double wave_min_nonneg(double x) {
    unsigned long long v = (unsigned long long)__double_as_longlong(x);
    v = min(v, dpp_u64<0xB1, 0xF>(v));     // quad_perm 1,0,3,2
    v = min(v, dpp_u64<0x4E, 0xF>(v));     // quad_perm 2,3,0,1
    v = min(v, dpp_u64<0x141, 0xF>(v));    // row_half_mirror
    v = min(v, dpp_u64<0x140, 0xF>(v));    // row_mirror
    v = min(v, dpp_u64<0x142, 0xA>(v));    // row_bcast:15
    v = min(v, dpp_u64<0x143, 0xC>(v));    // row_bcast:31
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// Orders this wave's LDS writes before its later LDS reads (all lanes of a
// wave run in lockstep, so waiting for the wave's own LDS traffic suffices).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---------------------------------------------------------------- tile placement
// Workgroup = one wave = one pixel tile.  Workgroups are dealt to the 8 XCDs
// round-robin by block index.  Tiles are grouped 4x4 (32x32 pixels) and the
// groups are dealt round-robin to the XCDs: neighbouring tiles of a group
// share one XCD's L2, and every XCD gets groups from all over the image, so
// the dense middle of a volume is not left to one or two XCDs.
constexpr int kGroupTiles = 4;

__host__ __device__ inline int group_grid_blocks(int tiles_x, int tiles_y) {
    int gx = (tiles_x + kGroupTiles - 1) / kGroupTiles;
    int gy = (tiles_y + kGroupTiles - 1) / kGroupTiles;
    return ((gx * gy + 7) / 8) * 8 * kGroupTiles * kGroupTiles;
}

__host__ __device__ __forceinline__ int tile_of_block(int b, int tiles_x, int tiles_y) {
    const int per = kGroupTiles * kGroupTiles;
    int gx = (tiles_x + kGroupTiles - 1) / kGroupTiles;
    int xcd = b & 7, q = b >> 3;
    int g = (q / per) * 8 + xcd, pos = q % per;
    int tx = (g % gx) * kGroupTiles + pos % kGroupTiles;
    int ty = (g / gx) * kGroupTiles + pos / kGroupTiles;
    return (tx < tiles_x && ty < tiles_y) ? ty * tiles_x + tx : -1;
}

// Work order of the multi-view reverse pass, whose rays are long serial
// chains (every sample of a ray, one after the other): the long rays
// through the middle of the volume must not be left to the end.
//  * Position k of 0 .. n-1 taken centre-out: n/2, n/2 - 1, n/2 + 1, ...
//    (tile rows from the middle row outwards, each row from its middle).
//  * view_of_unit: unit j of the grid -> its view and its rank among that
//    view's units.  Views take turns, one unit each while they have units
//    left, so every view's first (centre) tiles run before the last tiles
//    of any view.  View v owns (block_off[v+1] - block_off[v]) / unit
//    units.  Returns the view, or -1 for j outside the grid.
// (The forward march keeps its row-major groups: measured faster there.)
__host__ __device__ inline int centre_out(int k, int n) {
    const int m = n / 2;
    return (k & 1) ? m - (k + 1) / 2 : m + k / 2;
}

__host__ __device__ inline int view_of_unit(const ViewSet& S, int unit, int j, int& rank) {
    int umax = 0;
    for (int v = 0; v < S.n; ++v) umax = max(umax, (S.block_off[v + 1] - S.block_off[v]) / unit);
    auto below = [&](int r) {               // units of rank < r
        int c = 0;
        for (int v = 0; v < S.n; ++v) c += min((S.block_off[v + 1] - S.block_off[v]) / unit, r);
        return c;
    };
    if (j < 0 || j >= below(umax)) return -1;
    int lo = 0, hi = umax;                  // below(lo) <= j < below(hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (below(mid) <= j) lo = mid;
        else hi = mid;
    }
    int o = j - below(lo);
    rank = lo;
    for (int v = 0; v < S.n; ++v)
        if ((S.block_off[v + 1] - S.block_off[v]) / unit > lo && o-- == 0) return v;
    return -1;
}

// ---------------------------------------------------------------- index checks
// In the bounds-checked build (RC_DEBUG_BOUNDS) an index outside [0, n) is
// counted in P.dbg and replaced by 0, so the access stays inside its buffer
// and the run continues; in the product build the index passes unchanged.
#ifdef RC_DEBUG_BOUNDS
__device__ __forceinline__ long long rc_checked(unsigned int* dbg, long long i, long long n) {
    if (i >= 0 && i < n) return i;
    if (dbg) atomicAdd(dbg, 1u);
    return 0;
}
#define RC_IDX(dbg, i, n) rc_checked((dbg), (i), (n))
#else
#define RC_IDX(dbg, i, n) (i)
#endif

// ---------------------------------------------------------------- ray set-up
// Camera ray through the centre of pixel (px, py) and its span inside the
// sampling box (Section 3.3: no intersection -> black; two -> sample between).
// FP64 throughout so that the lattice matches the FP64 definition.
struct Ray {
    double o[3], d[3];
    double t_in, t_out;
    int K;              // index of the last lattice sample, -1 on a miss (< 2^24)
    double p0[3], dp[3];    // voxel-space position of sample 0 and step between samples
};

__device__ inline void setup_ray(const RenderParams& P, const ViewParams& V, int px, int py,
                                 Ray& R) {
    double x = 2.0 * ((double)px + 0.5) / (double)V.W - 1.0;
    double y = 1.0 - 2.0 * ((double)py + 0.5) / (double)V.H;
    if (V.projection == RC_PERSPECTIVE) {
        double th = V.tan_half;
        double t0 = V.f[0] + x * th * V.aspect * V.r[0] + y * th * V.u[0];
        double t1 = V.f[1] + x * th * V.aspect * V.r[1] + y * th * V.u[1];
        double t2 = V.f[2] + x * th * V.aspect * V.r[2] + y * th * V.u[2];
        double n = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
        double s = n > 0.0 ? 1.0 / n : 0.0;
        R.d[0] = t0 * s; R.d[1] = t1 * s; R.d[2] = t2 * s;
        R.o[0] = V.eye[0]; R.o[1] = V.eye[1]; R.o[2] = V.eye[2];
    } else {
        for (int a = 0; a < 3; ++a) {
            R.d[a] = V.f[a];
            R.o[a] = V.eye[a] + (x * V.aspect * V.r[a] + y * V.u[a]) * V.ortho_half;
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
    R.t_out = tmax;
    R.K = -1;
    if (hit && tmin <= tmax) R.K = (int)floor((tmax - tmin) / P.step);
    for (int a = 0; a < 3; ++a) {
        R.p0[a] = (R.o[a] + tmin * R.d[a]) * P.inv_s[a];
        R.dp[a] = P.step * R.d[a] * P.inv_s[a];
    }
}

// A voxel-space point split into cell index and fraction (cell_of), for the
// point at ray parameter t (point_at) or lattice sample k (lattice_point).
struct Cell {
    int c[3];
    float fr[3];
};

__device__ __forceinline__ void cell_of(const RenderParams& P, const double p3[3], Cell& C,
                                        double pv[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = p3[a];
        pv[a] = p;
        // nearest sampling (Section 3.3, round half up): the cell of the
        // rounded point with fraction 0, so the trilinear and stencil code
        // reduce exactly to that voxel
        // (round_bias is 0.5 for nearest sampling, else 0; frac_keep 0 or 1).
        // Sample points lie in the sampling box, [0, n - 1] in voxel units
        // up to rounding, so the cell index fits an int without a clamp.
        const double fl = floor(p + P.round_bias);
        C.c[a] = (int)fl;
        C.fr[a] = (float)(p - fl) * P.frac_keep;
    }
}

__device__ __forceinline__ void point_at(const RenderParams& P, const Ray& R, double t, Cell& C,
                                         double pv[3]) {
    double p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = (R.o[a] + t * R.d[a]) * P.inv_s[a];
    cell_of(P, p, C, pv);
}

// Lattice sample k: p0 + k dp, one FP64 FMA per axis.  Monotone in k, so
// the cells of samples between two lattice indices lie between theirs.
__device__ __forceinline__ void lattice_point(const RenderParams& P, const Ray& R, int k,
                                              Cell& C, double pv[3]) {
    double p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = fma((double)k, R.dp[a], R.p0[a]);
    cell_of(P, p, C, pv);
}

// ---------------------------------------------------------------- voxel sources
// A source turns the footprint [c-1, c+2] of a cell, per axis, into element
// offsets; the voxel at footprint position (i, j, k) is base[ox[i]+oy[j]+oz[k]].
//  * GlobalSrc: the bricked volume, indices clamped to the grid.
//  * LdsSrc: the chunk box staged in LDS, which already holds the clamped
//    values, so offsets are plain strides (constant x steps -> immediate
//    LDS offsets).
template <typename VT>
struct GlobalSrc {
    using elem = VT;
    const VT* __restrict__ base;
    int nx, ny, nz, sy, sz;
    long long n;            // elements of the bricked volume
    unsigned int* dbg;
    __device__ __forceinline__ gmem<VT> gbase() const { return to_gmem(base); }
    __device__ __forceinline__ void offsets(const Cell& C, int ox[4], int oy[4], int oz[4]) const {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ox[i] = off_x(clampi(C.c[0] - 1 + i, 0, nx - 1));
            oy[i] = off_y(clampi(C.c[1] - 1 + i, 0, ny - 1), sy);
            oz[i] = off_z(clampi(C.c[2] - 1 + i, 0, nz - 1), sz);
        }
#ifdef RC_DEBUG_BOUNDS
        // the separable terms are non-negative: the footprint's largest
        // offset is the sum of the per-axis largest
        int mx = 0, my = 0, mz = 0, lx = ox[0], ly = oy[0], lz = oz[0];
        for (int i = 0; i < 4; ++i) {
            mx = max(mx, ox[i]); my = max(my, oy[i]); mz = max(mz, oz[i]);
            lx = min(lx, ox[i]); ly = min(ly, oy[i]); lz = min(lz, oz[i]);
        }
        if (RC_IDX(dbg, (long long)lx + ly + lz, n) != (long long)lx + ly + lz ||
            RC_IDX(dbg, (long long)mx + my + mz, n) != (long long)mx + my + mz)
            for (int i = 0; i < 4; ++i) ox[i] = oy[i] = oz[i] = 0;
#endif
    }
};

template <typename VT>
struct LdsSrc {
    using elem = VT;        // the staged element type (see LdsT)
    const VT* base;
    int lo[3];          // box origin (voxel index, may be negative)
    int bx, bxy;        // row and slab strides in elements
    int n;              // elements of the staged box
    unsigned int* dbg;
    __device__ __forceinline__ void offsets(const Cell& C, int ox[4], int oy[4], int oz[4]) const {
        int x0 = C.c[0] - 1 - lo[0], y0 = C.c[1] - 1 - lo[1], z0 = C.c[2] - 1 - lo[2];
        // box coordinates and strides are far below 2^23: 24-bit multiplies
        const int yb = __mul24(y0, bx), zb = __mul24(z0, bxy);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ox[i] = x0 + i;
            oy[i] = yb + i * bx;
            oz[i] = zb + i * bxy;
        }
#ifdef RC_DEBUG_BOUNDS
        // offsets grow with i on every axis: check the two extreme corners
        // and every per-axis coordinate against the box
        const int zd = n / bxy, yd = bxy / bx;
        const bool bad = x0 < 0 || x0 + 3 >= bx || y0 < 0 || y0 + 3 >= yd || z0 < 0 ||
                         z0 + 3 >= zd;
        if (bad || RC_IDX(dbg, (long long)ox[0] + oy[0] + oz[0], n) != ox[0] + oy[0] + oz[0] ||
            RC_IDX(dbg, (long long)ox[3] + oy[3] + oz[3], n) != ox[3] + oy[3] + oz[3]) {
            if (bad && dbg) atomicAdd(dbg, 1u);
            for (int i = 0; i < 4; ++i) ox[i] = oy[i] = oz[i] = 0;
        }
#endif
    }
    // The same footprint as a per-lane base (the footprint's first voxel)
    // plus offsets that are the same for every lane: x steps 0..3 and the
    // chunk's row and slab strides.  A footprint voxel's address is then one
    // add of a wave-uniform row offset, with the x step in the instruction's
    // immediate offset.
    __device__ __forceinline__ const VT* lane_offsets(const Cell& C, int ox[4], int oy[4],
                                                      int oz[4]) const {
        offsets(C, ox, oy, oz);
        const int first = ox[0] + oy[0] + oz[0];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ox[i] = i;
            oy[i] = i * bx;
            oz[i] = i * bxy;
        }
        return base + first;
    }
};

template <typename VT>
__device__ __forceinline__ gmem<VT> footprint(const GlobalSrc<VT>& s, const Cell& C, int ox[4],
                                              int oy[4], int oz[4]) {
    s.offsets(C, ox, oy, oz);
    return s.gbase();
}
template <typename VT>
__device__ __forceinline__ const VT* footprint(const LdsSrc<VT>& s, const Cell& C, int ox[4],
                                               int oy[4], int oz[4]) {
    return s.lane_offsets(C, ox, oy, oz);
}

// ---------------------------------------------------------------- sampling
// Trilinear interpolation as 7 lerps, x then y then z (Section 3.4, eq. 2).
template <typename VT, typename Ptr = const VT*>
__device__ __forceinline__ void load_corners(Ptr base, const int ox[4], const int oy[4],
                                             const int oz[4], float corner[8]) {
    // corner[(z-1)*4 + (y-1)*2 + (x-1)] = voxel (x, y, z) of the 4x4x4 footprint
#pragma unroll
    for (int q = 0; q < 8; ++q)
        corner[q] = (float)base[ox[1 + (q & 1)] + oy[1 + ((q >> 1) & 1)] + oz[1 + (q >> 2)]];
}

// Section 3.4: 7 lerps, x then y then z, of the cell's 8 voxels.
__device__ __forceinline__ float trilinear(const float corner[8], const Cell& C) {
    const float v000 = corner[0], v100 = corner[1], v010 = corner[2], v110 = corner[3];
    const float v001 = corner[4], v101 = corner[5], v011 = corner[6], v111 = corner[7];
    float i1 = lerpf(v000, v100, C.fr[0]);
    float i2 = lerpf(v010, v110, C.fr[0]);
    float i3 = lerpf(v001, v101, C.fr[0]);
    float i4 = lerpf(v011, v111, C.fr[0]);
    float i5 = lerpf(i1, i2, C.fr[1]);
    float i6 = lerpf(i3, i4, C.fr[1]);
    return lerpf(i5, i6, C.fr[2]);
}

template <typename VT, typename Ptr = const VT*>
__device__ __forceinline__ float sample_value(Ptr base, const int ox[4], const int oy[4],
                                              const int oz[4], const Cell& C, float corner[8]) {
    load_corners<VT>(base, ox, oy, oz, corner);
    return trilinear(corner, C);
}

template <typename VT, typename Ptr = const VT*>
__device__ __forceinline__ float sample_value(Ptr base, const int ox[4], const int oy[4],
                                              const int oz[4], const Cell& C) {
    float corner[8];
    return sample_value<VT>(base, ox, oy, oz, C, corner);
}

// Lookup table (Section 3.7): u = clamp((v-vmin)/(vmax-vmin),0,1)*(M-1),
// linear between entries floor(u) and floor(u)+1 (clamped to M-1).
__device__ __forceinline__ float4 tf_lookup(const RenderParams& P, float v) {
    float vn = fminf(fmaxf((v - P.vmin) * P.inv_range, 0.0f), 1.0f);
    float uu = vn * P.Mm1;
    int i = min((int)uu, P.M - 1);
    int i1 = min(i + 1, P.M - 1);
    float t = uu - (float)i;
    const float4 a = gload(P.tf + RC_IDX(P.dbg, i, P.M)), b = gload(P.tf + RC_IDX(P.dbg, i1, P.M));
    return make_float4(lerpf(a.x, b.x, t), lerpf(a.y, b.y, t), lerpf(a.z, b.z, t),
                       lerpf(a.w, b.w, t));
}

// ---------------------------------------------------------------- gradients
// Sobel3D smoothing weights of eq. (4): [[1,3,1],[3,6,3],[1,3,1]].
__host__ __device__ constexpr int sobel_weight(int b, int e) {
    return (b == 0 && e == 0) ? 6 : (b == 0 || e == 0) ? 3 : 1;
}

// Section 3.5.  Each tap of the operator is a trilinear sample at p + o;
// by linearity that equals the trilinear blend of the stencil evaluated at
// the 8 corners of the cell:
//   G_x = sum_c w_c sum_{b,e} W(b,e) [V(c + (1,b,e)) - V(c - (1,-b,-e))]
// over the 4x4x4 neighbourhood [c-1, c+2]^3.  The 3x3 smoothing mask of
// each operator is a separable product plus a centre correction,
//   Sobel3D (eq. 4)  W = A (x) A - 3 delta,  A = [1, 3, 1]
//   Zucker-Hummel    W = A (x) A + (1 - q^2/r) delta,  A = [sqrt r, q/sqrt r, sqrt r],
//                    r = 1/sqrt 3 (corners), q = 1/sqrt 2 (edges), centre 1
//   central diff.    W = delta (eq. 3)
// and the corner weights w_c are separable too, so G is a sum of separable
// 4x4x4 filters.  Their per-axis taps (corner weights folded in, t = the
// cell fraction):
//   L  = [0, 1-t, t, 0]                       (lerp)
//   D' = [-(1-t), -t, 1-t, t]                 (lerp (x) the +-1 difference)
//   A' = [a1(1-t), a0(1-t)+a1 t, a1(1-t)+a0 t, a1 t]   (lerp (x) A = [a1,a0,a1])
// G_x = sum V D'x A'y A'z + gamma sum V D'x Ly Lz, cyclically for y and z.
// The neighbourhood is streamed one z-slice (4x4 voxels) at a time.
template <int OP> struct OpTaps;
template <> struct OpTaps<RC_GRAD_CENTRAL> {
    static constexpr bool kSep = false;
    static constexpr float a0 = 0.f, a1 = 0.f, gamma = 1.0f;
};
template <> struct OpTaps<RC_GRAD_SOBEL3D> {
    static constexpr bool kSep = true;
    static constexpr float a0 = 3.0f, a1 = 1.0f, gamma = -3.0f;
};
template <> struct OpTaps<RC_GRAD_ZUCKER_HUMMEL> {
    // a1 = sqrt(1/sqrt 3), a0 = (1/sqrt 2) / a1, gamma = 1 - a0^2
    static constexpr bool kSep = true;
    static constexpr float a1 = 0.75983568565159271f, a0 = 0.93060485910209953f,
                           gamma = 0.13397459621556135f;
};

__device__ __forceinline__ float dot4(const float a[4], const float b[4]) {
    return fmaf(a[3], b[3], fmaf(a[2], b[2], fmaf(a[1], b[1], a[0] * b[0])));
}

struct AxisTaps {
    float L[4], D[4], A[4];
};

template <int OP>
__device__ __forceinline__ void axis_taps(float t, AxisTaps& k) {
    const float w0 = 1.0f - t, w1 = t;
    k.L[0] = 0.f; k.L[1] = w0; k.L[2] = w1; k.L[3] = 0.f;
    k.D[0] = -w0; k.D[1] = -w1; k.D[2] = w0; k.D[3] = w1;
    const float a0 = OpTaps<OP>::a0, a1 = OpTaps<OP>::a1;
    k.A[0] = a1 * w0;
    k.A[1] = fmaf(a0, w0, a1 * w1);
    k.A[2] = fmaf(a1, w0, a0 * w1);
    k.A[3] = a1 * w1;
}

template <typename VT, int OP, bool HAVE_CORNERS = false, typename Ptr = const VT*>
__device__ __forceinline__ void gradient(const RenderParams& P, Ptr base, const int ox[4],
                                         const int oy[4], const int oz[4], const Cell& C,
                                         float g[3], const float* corner = nullptr) {
    constexpr bool SEP = OpTaps<OP>::kSep;
    AxisTaps kx, ky, kz;
    axis_taps<OP>(C.fr[0], kx);
    axis_taps<OP>(C.fr[1], ky);
    axis_taps<OP>(C.fr[2], kz);
    float gxA = 0.f, gyA = 0.f, gzA = 0.f, gxL = 0.f, gyL = 0.f, gzL = 0.f;
#pragma unroll
    for (int z = 0; z < 4; ++z) {
        float rowD[4], rowA[4], rowL[4];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            float v[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                // the cell's own 8 voxels were read for the value already
                const bool inner = (x == 1 || x == 2) && (y == 1 || y == 2) && (z == 1 || z == 2);
                v[x] = (HAVE_CORNERS && inner) ? corner[(z - 1) * 4 + (y - 1) * 2 + (x - 1)]
                                               : (float)base[ox[x] + oy[y] + oz[z]];
            }
            rowD[y] = dot4(kx.D, v);
            rowL[y] = fmaf(kx.L[2], v[2], kx.L[1] * v[1]);
            rowA[y] = SEP ? dot4(kx.A, v) : 0.f;
        }
        const float xL = fmaf(ky.L[2], rowD[2], ky.L[1] * rowD[1]);
        const float yL = dot4(ky.D, rowL);
        const float zL = fmaf(ky.L[2], rowL[2], ky.L[1] * rowL[1]);
        if (z == 1 || z == 2) {             // L vanishes on the outer slices
            gxL = fmaf(kz.L[z], xL, gxL);
            gyL = fmaf(kz.L[z], yL, gyL);
        }
        gzL = fmaf(kz.D[z], zL, gzL);
        if (SEP) {
            const float xA = dot4(ky.A, rowD);
            const float yA = dot4(ky.D, rowA);
            const float zA = dot4(ky.A, rowA);
            gxA = fmaf(kz.A[z], xA, gxA);
            gyA = fmaf(kz.A[z], yA, gyA);
            gzA = fmaf(kz.D[z], zA, gzA);
        }
    }
    const float gm = OpTaps<OP>::gamma;
    g[0] = fmaf(gm, gxL, gxA) * P.gscale[0];
    g[1] = fmaf(gm, gyL, gyA) * P.gscale[1];
    g[2] = fmaf(gm, gzL, gzA) * P.gscale[2];
}

// ---------------------------------------------------------------- shading
// Per-ray shading constants: the view vector V = -d and, for a directional
// light, the Blinn-Phong half vector H = normalize(L + V), which is the same
// for every sample of the ray.
struct RayShade {
    float v[3];
    float h[3];
};

__device__ __forceinline__ float rsq_or_zero(float x) {
    return x > 0.0f ? __builtin_amdgcn_rsqf(x) : 0.0f;
}

__device__ __forceinline__ void ray_shade(const RenderParams& P, const Ray& R, RayShade& rs) {
    rs.v[0] = (float)-R.d[0];
    rs.v[1] = (float)-R.d[1];
    rs.v[2] = (float)-R.d[2];
    float h[3] = {P.light[0] + rs.v[0], P.light[1] + rs.v[1], P.light[2] + rs.v[2]};
    float hi = rsq_or_zero(fmaf(h[2], h[2], fmaf(h[1], h[1], h[0] * h[0])));
    rs.h[0] = h[0] * hi; rs.h[1] = h[1] * hi; rs.h[2] = h[2] * hi;
}

// Section 3.8.  G points towards larger values; the outward normal is
// N = -G/max(|G|, eps).  Alpha is never shaded.  Hardware rsq / log2 / exp2
// (about 1 ulp) stand in for the library normalise and pow.
__device__ __forceinline__ void shade(const RenderParams& P, const float4& rgba, const float g[3],
                                      const double pv[3], const RayShade& rs, float c[3]) {
    float g2 = fmaf(g[2], g[2], fmaf(g[1], g[1], g[0] * g[0]));
    // 1 / max(|G|, eps) = min(1/|G|, 1/eps); rsq(0) = +inf
    float inv = fminf(__builtin_amdgcn_rsqf(g2), 1.0f / P.grad_eps);
    float gh[3] = {g[0] * inv, g[1] * inv, g[2] * inv};
    float L[3], H[3];
    if (P.light_is_point) {
        float q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = P.light[a] - (float)pv[a] * P.s[a];
        float qi = rsq_or_zero(fmaf(q[2], q[2], fmaf(q[1], q[1], q[0] * q[0])));
        L[0] = q[0] * qi; L[1] = q[1] * qi; L[2] = q[2] * qi;
        if (P.shade == RC_SHADE_BLINN_PHONG) {
            float h[3] = {L[0] + rs.v[0], L[1] + rs.v[1], L[2] + rs.v[2]};
            float hi = rsq_or_zero(fmaf(h[2], h[2], fmaf(h[1], h[1], h[0] * h[0])));
            H[0] = h[0] * hi; H[1] = h[1] * hi; H[2] = h[2] * hi;
        }
    } else {
        L[0] = P.light[0]; L[1] = P.light[1]; L[2] = P.light[2];
        H[0] = rs.h[0]; H[1] = rs.h[1]; H[2] = rs.h[2];
    }
    if (P.shade == RC_SHADE_PAPER_LAMBERT) {
        // Listing 3: illum = dot(normalize(lightPosition - pos), norm), unclamped
        float illum = fmaf(L[2], gh[2], fmaf(L[1], gh[1], L[0] * gh[0]));
        c[0] = rgba.x * illum; c[1] = rgba.y * illum; c[2] = rgba.z * illum;
        return;
    }
    float nl = -fmaf(gh[2], L[2], fmaf(gh[1], L[1], gh[0] * L[0]));
    float nh = -fmaf(gh[2], H[2], fmaf(gh[1], H[1], gh[0] * H[0]));
    float diff = fmaxf(nl, 0.0f);
    float spec = nh > 0.0f ? __builtin_amdgcn_exp2f(P.shininess * __builtin_amdgcn_logf(nh))
                           : (P.shininess == 0.0f ? 1.0f : 0.0f);
    float k = fmaf(P.kd, diff, P.ka);
    float ks = P.ks * spec;
    c[0] = fmaf(rgba.x, k, ks);
    c[1] = fmaf(rgba.y, k, ks);
    c[2] = fmaf(rgba.z, k, ks);
}

// ---------------------------------------------------------------- LDS staging
// Stage the voxel box [lo, lo + dim) (dims even, lo even) into LDS as
// [z][y][x] elements of type LT.  The Sobel3D and Zucker-Hummel samples
// read 64 voxels each, so their boxes hold FP32 (each voxel converted once
// here, not at every read); central differences read 32 and keep the
// volume's own type (half the LDS bytes per voxel: longer chunks).  Work
// unit: a 2x2x2 Morton group, which is 8 contiguous voxels in the bricked
// layout (one 16-byte load for u16) and 4 x-pairs of the LDS box.  Groups
// that reach outside the padded brick grid (volume edges) are read voxel by
// voxel with clamped indices.
template <typename VT, int OP> struct LdsT { using type = float; };
template <typename VT> struct LdsT<VT, RC_GRAD_CENTRAL> { using type = VT; };

template <typename VT> struct PairT;
template <> struct PairT<uint8_t> { using type = uint16_t; };
template <> struct PairT<uint16_t> { using type = uint32_t; };
template <> struct PairT<float> { using type = uint2; };

template <typename VT> struct GroupT;
template <> struct GroupT<uint8_t> { using type = uint2; };
template <> struct GroupT<uint16_t> { using type = uint4; };
template <> struct GroupT<float> { struct type { uint4 a, b; }; };

// A group's 4 x-pairs as they lie in memory (Morton order x + 2y + 4z).
template <typename VT>
__device__ __forceinline__ void group_pairs(const typename GroupT<VT>::type& g,
                                            typename PairT<VT>::type p[4]);
template <>
__device__ __forceinline__ void group_pairs<uint8_t>(const uint2& g, uint16_t p[4]) {
    p[0] = (uint16_t)(g.x & 0xffffu); p[1] = (uint16_t)(g.x >> 16);
    p[2] = (uint16_t)(g.y & 0xffffu); p[3] = (uint16_t)(g.y >> 16);
}
template <>
__device__ __forceinline__ void group_pairs<uint16_t>(const uint4& g, uint32_t p[4]) {
    p[0] = g.x; p[1] = g.y; p[2] = g.z; p[3] = g.w;
}
template <>
__device__ __forceinline__ void group_pairs<float>(const GroupT<float>::type& g, uint2 p[4]) {
    p[0] = make_uint2(g.a.x, g.a.y); p[1] = make_uint2(g.a.z, g.a.w);
    p[2] = make_uint2(g.b.x, g.b.y); p[3] = make_uint2(g.b.z, g.b.w);
}

// The 8 voxels of a group in Morton order (x + 2y + 4z), as floats.
template <typename VT>
__device__ __forceinline__ void group_values(const typename GroupT<VT>::type& g, float f[8]);
template <>
__device__ __forceinline__ void group_values<uint8_t>(const uint2& g, float f[8]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[q] = (float)((g.x >> (8 * q)) & 0xffu);
        f[4 + q] = (float)((g.y >> (8 * q)) & 0xffu);
    }
}
template <>
__device__ __forceinline__ void group_values<uint16_t>(const uint4& g, float f[8]) {
    const unsigned w[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[2 * q] = (float)(w[q] & 0xffffu);
        f[2 * q + 1] = (float)(w[q] >> 16);
    }
}
template <>
__device__ __forceinline__ void group_values<float>(const GroupT<float>::type& g, float f[8]) {
    const unsigned w[8] = {g.a.x, g.a.y, g.a.z, g.a.w, g.b.x, g.b.y, g.b.z, g.b.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = __uint_as_float(w[q]);
}

template <typename VT, typename LT>
__device__ inline void stage_box(const RenderParams& P, LT* lds, const int lo[3], const int dim[3],
                                 int lane) {
    using G = typename GroupT<VT>::type;
    using PT = typename PairT<VT>::type;
    const VT* vox = (const VT*)P.vox;
    const int gx = dim[0] >> 1, gy = dim[1] >> 1, gz = dim[2] >> 1;
    const int ncol = gx * gy;
    const float inv_gx = small_inv(gx);
    const int xmax = P.nbx * 8, ymax = P.nby * 8, zmax = P.nbz * 8;
    const int bx = dim[0], bxy = dim[0] * dim[1];
    // each lane owns (x, y) columns of groups and walks them along z
    for (int col = lane; col < ncol; col += 64) {
        const int iy = small_quot(col, inv_gx), ix = col - iy * gx;
        int x0 = lo[0] + 2 * ix, y0 = lo[1] + 2 * iy;
        bool xy_in = x0 >= 0 && y0 >= 0 && x0 + 1 < xmax && y0 + 1 < ymax;
        int oxy = xy_in ? off_x(x0) + off_y(y0, P.sy) : 0;
        int l0 = 2 * iy * bx + 2 * ix;
        for (int iz = 0; iz < gz; ++iz, l0 += 2 * bxy) {
            int z0 = lo[2] + 2 * iz;
            if (xy_in && z0 >= 0 && z0 + 1 < zmax) {
#ifdef RC_DEBUG_BOUNDS
                // the group's 8 voxels and its 4 pair stores
                if (RC_IDX(P.dbg, (long long)oxy + off_z(z0, P.sz) + 7,
                           (long long)P.nbx * P.nby * P.nbz * 512) == 0 ||
                    RC_IDX(P.dbg, l0 + bxy + bx + 1, bxy * dim[2]) == 0)
                    continue;
#endif
                const G grp = gload((const G*)(vox + oxy + off_z(z0, P.sz)));
                // l0 and the strides are even: pair-aligned stores
                if constexpr (std::is_same<LT, float>::value) {
                    float f[8];
                    group_values<VT>(grp, f);
                    *(float2*)(lds + l0) = make_float2(f[0], f[1]);
                    *(float2*)(lds + l0 + bx) = make_float2(f[2], f[3]);
                    *(float2*)(lds + l0 + bxy) = make_float2(f[4], f[5]);
                    *(float2*)(lds + l0 + bxy + bx) = make_float2(f[6], f[7]);
                } else {
                    PT p[4];
                    group_pairs<VT>(grp, p);
                    *(PT*)(lds + l0) = p[0];
                    *(PT*)(lds + l0 + bx) = p[1];
                    *(PT*)(lds + l0 + bxy) = p[2];
                    *(PT*)(lds + l0 + bxy + bx) = p[3];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
                    int x = clampi(x0 + dx, 0, P.nx - 1), y = clampi(y0 + dy, 0, P.ny - 1),
                        z = clampi(z0 + dz, 0, P.nz - 1);
                    lds[RC_IDX(P.dbg, l0 + dz * bxy + dy * bx + dx, bxy * dim[2])] =
                        (LT)to_gmem(vox)[RC_IDX(P.dbg, off_x(x) + off_y(y, P.sy) + off_z(z, P.sz),
                                                (long long)P.nbx * P.nby * P.nbz * 512)];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- the march
struct MarchOut {
    float4 rgba;
    int k_last;
    float T;
    unsigned evaluated, shaded;
    unsigned samples_direct;                        // per lane
    unsigned chunks_staged, chunks_empty, chunks_direct;  // per wave (uniform)
};

// Opacity correction for the sample distance: a = 1 - (1 - a_tf)^e with
// e = step / ref, through hardware log2 / exp2 (0 stays 0, 1 stays 1).
__device__ __forceinline__ float correct_opacity(float e, float a) {
    return 1.0f - __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(1.0f - a));
}

// Per-lane compositing state (Section 3.9, eq. 6 evaluated front to back:
// C += T a c, T *= 1 - a; early termination after the first sample with
// 1 - T >= tau).
struct LaneState {
    float Cr, Cg, Cb, T;
    int k;                  // next lattice index
    int k_term;             // index where early termination fired, -1 if not
    bool done;
    unsigned evaluated, shaded, direct;
};

// Chunk geometry shared by the wave.
struct Chunk {
    int lo[3], dim[3];          // LDS box
    int blo[3], bdim[3];        // brick range of the samples' cells
    unsigned long long live;    // bit set = brick may hold a non-zero-opacity sample
    bool mask_valid;            // live covers every brick of the chunk
    bool mixed;                 // some sample may sit in an empty brick: test per sample
};

// One evaluated sample: value, table, and for non-zero opacity the
// gradient, shading and compositing.  Returns true when the ray terminates.
// LIT: a shading model is on (the unshaded instantiations carry none of the
// gradient's registers, so they keep more waves resident).  e: the opacity
// correction exponent of the distance the sample stands for (0 = none).
template <typename VT, int OP, bool LIT, typename Src>
__device__ __forceinline__ bool shade_sample(const RenderParams& P, const Src& src, const Cell& C,
                                             const double pv[3], const RayShade& rs,
                                             LaneState& S, float e) {
    int ox[4], oy[4], oz[4];
    using ET = typename Src::elem;          // element type of the source
    const auto base = footprint(src, C, ox, oy, oz);
    float corner[8];
    float v = sample_value<ET>(base, ox, oy, oz, C, corner);
    float4 rgba = tf_lookup(P, v);
    float a = rgba.w;
    if (a == 0.0f) return false;
    if (e > 0.0f) a = correct_opacity(e, a);
    ++S.shaded;
    float c[3] = {rgba.x, rgba.y, rgba.z};
    if (LIT) {
        float g[3];
        gradient<ET, OP, true>(P, base, ox, oy, oz, C, g, corner);
        shade(P, rgba, g, pv, rs, c);
    }
    float ta = S.T * a;
    S.Cr = fmaf(ta, c[0], S.Cr);
    S.Cg = fmaf(ta, c[1], S.Cg);
    S.Cb = fmaf(ta, c[2], S.Cb);
    S.T *= (1.0f - a);
    return P.tau > 0.0f && 1.0f - S.T >= P.tau;
}

// A sample whose brick is known to be empty (its opacity is exactly 0).
__device__ __forceinline__ bool in_empty_brick(const RenderParams& P, const Chunk& ch,
                                               const Cell& C) {
    int b0 = clampi(C.c[0], 0, P.nx - 1) >> 3, b1 = clampi(C.c[1], 0, P.ny - 1) >> 3,
        b2 = clampi(C.c[2], 0, P.nz - 1) >> 3;
    int r0 = b0 - ch.blo[0], r1 = b1 - ch.blo[1], r2 = b2 - ch.blo[2];
    if (ch.mask_valid && r0 >= 0 && r1 >= 0 && r2 >= 0 && r0 < ch.bdim[0] && r1 < ch.bdim[1] &&
        r2 < ch.bdim[2])
        return ((ch.live >> ((r2 * ch.bdim[1] + r1) * ch.bdim[0] + r0)) & 1ull) == 0;
    return to_gmem(P.empty)[RC_IDX(P.dbg, (b2 * P.nby + b1) * P.nbx + b0,
                          (long long)P.nbx * P.nby * P.nbz)] != 0;
}

// Evaluate lattice samples S.k .. kstop of this lane's ray.  Samples in
// bricks known to be empty are not evaluated (their opacity is exactly 0,
// so they change nothing).  A sample reads the LDS box when `staged` and its
// 4x4x4 footprint lies inside the box, else the bricked volume.
template <typename VT, int OP, bool LIT>
__device__ __forceinline__ void run_samples(const RenderParams& P, const Ray& R,
                                            const LdsSrc<typename LdsT<VT, OP>::type>& lsrc,
                                            const GlobalSrc<VT>& gsrc,
                                            bool staged, const Chunk& ch, int kstop,
                                            const RayShade& rs, LaneState& S) {
    for (int k = S.k; k <= kstop; ++k) {
        Cell C;
        double pv[3];
        lattice_point(P, R, k, C, pv);
        if (ch.mixed && in_empty_brick(P, ch, C)) continue;
        ++S.evaluated;
        // A lane's cells are monotone along its straight ray (each step of
        // lattice_point is a monotone rounding), so its samples S.k..kstop lie
        // between the two end cells that chunk_cells reduced into the box:
        // a staged chunk's samples always read the box.
        const bool in = staged;
        S.direct += in ? 0u : 1u;
        bool term = in ? shade_sample<VT, OP, LIT>(P, lsrc, C, pv, rs, S, P.ocorr)
                       : shade_sample<VT, OP, LIT>(P, gsrc, C, pv, rs, S, P.ocorr);
        if (term) {
            S.k_term = k;
            S.done = true;
            return;
        }
    }
}

// Chunk lengths in lattice steps; super-chunks test 32^3 super-bricks.
constexpr int kChunkMin = 2, kChunkInit = 16, kChunkMax = 128;
constexpr int kSuperMin = 64, kSuperInit = 256;

// This lane's lattice samples in [tau, tau + len * step): indices S.k ..
// kstop (kstop < S.k when it has none), and the wave-wide bounds of their
// cells.  Returns false when no lane of the wave has a sample there.
__device__ __forceinline__ bool chunk_cells(const RenderParams& P, const Ray& R, bool active,
                                            int k, double tau, int len, int& kstop,
                                            int cmin[3], int cmax[3]) {
    double tau_end = tau + (double)len * P.step;
    kstop = -1;
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    if (active) {
        // which samples fall in a chunk only groups the work: any rounding here is harmless
        double q = ceil((tau_end - R.t_in) * P.inv_step) - 1.0;
        kstop = q < (double)R.K ? (int)fmax(q, -1.0) : R.K;
        // the lane(s) defining tau always own at least their next sample
        if (R.t_in + (double)k * P.step < tau_end && kstop < k) kstop = k;
        if (kstop >= k) {
            // cells are monotone along a straight ray: the end points bound them
            Cell c0, c1;
            double pv[3];
            lattice_point(P, R, k, c0, pv);
            lattice_point(P, R, kstop, c1, pv);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = min(c0.c[a], c1.c[a]);
                mx[a] = max(c0.c[a], c1.c[a]);
            }
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
// its cells span at most 64 super-bricks.  Returns true when every one of
// them is empty; kstop is then this lane's last sample in the chunk.
__device__ __forceinline__ bool super_chunk_empty(const RenderParams& P, const Ray& R, bool active,
                                                  int k, double tau, int& len,
                                                  int& kstop, int lane) {
    const int n[3] = {P.nx, P.ny, P.nz};
    for (;; len >>= 1) {
        int cmin[3], cmax[3];
        if (!chunk_cells(P, R, active, k, tau, len, kstop, cmin, cmax)) return false;
        int slo[3], sdim[3], nsr = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            slo[a] = clampi(cmin[a], 0, n[a] - 1) >> 5;
            sdim[a] = (clampi(cmax[a], 0, n[a] - 1) >> 5) - slo[a] + 1;
            nsr *= sdim[a];
        }
        if (nsr > 64) {
            if (len <= kSuperMin) return false;
            continue;
        }
        bool live = false;
        if (lane < nsr) {
            const int r01 = small_quot(lane, small_inv(sdim[0]));
            const int r2 = small_quot(r01, small_inv(sdim[1]));
            const int r0 = lane - r01 * sdim[0], r1 = r01 - r2 * sdim[1];
            live = (to_gmem(P.super_empty)[RC_IDX(P.dbg,
                                         ((slo[2] + r2) * P.nsy + slo[1] + r1) * P.nsx + slo[0] + r0,
                                         (long long)P.nsx * P.nsy * P.nsz)] & kSuperEmpty) == 0;
        }
        return __ballot(live) == 0ull;
    }
}

// First lattice index of this lane's ray that may lie in a non-empty
// super-brick: a 3D DDA over the 32^3 super-brick grid along the ray in
// voxel space (p = p0 + k dp, k in lattice units), stopping at the first
// super-brick whose flag is clear.  The start cell comes from the FP64
// position; the crossings are stepped in FP32 (relative error ~1e-7 of k,
// k < 2^24), and every sample before the returned index lies at least two
// lattice steps before the crossing, so no rounding puts it into a
// non-empty super-brick.  Those samples have opacity 0 and are skipped.
// Returns K + 1 when the whole ray is empty.
__device__ __forceinline__ int entry_index(const RenderParams& P, const Ray& R) {
    const int n[3] = {P.nx, P.ny, P.nz}, ns[3] = {P.nsx, P.nsy, P.nsz};
    int cell[3], dir[3];
    float kb[3], dk[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cell[a] = clampi((int)floor(R.p0[a]), 0, n[a] - 1) >> 5;
        const float d = (float)R.dp[a];
        dir[a] = d > 0.0f ? 1 : (d < 0.0f ? -1 : 0);
        const float bound = (float)(cell[a] + (d > 0.0f ? 1 : 0)) * 32.0f;
        dk[a] = dir[a] != 0 ? 32.0f / fabsf(d) : INFINITY;
        kb[a] = dir[a] != 0 ? (bound - (float)R.p0[a]) / d : INFINITY;
    }
    float k_enter = 0.0f;
    const float kmax = (float)R.K;
#pragma unroll 1
    for (int it = 0; it < ns[0] + ns[1] + ns[2]; ++it) {
        if ((to_gmem(P.super_empty)[RC_IDX(P.dbg, (cell[2] * P.nsy + cell[1]) * P.nsx + cell[0],
                                  (long long)P.nsx * P.nsy * P.nsz)] & kSuperEmpty) == 0)
            break;
        int a = kb[0] <= kb[1] ? (kb[0] <= kb[2] ? 0 : 2) : (kb[1] <= kb[2] ? 1 : 2);
        k_enter = kb[a];
        cell[a] += dir[a];
        if (!(k_enter <= kmax) || cell[a] < 0 || cell[a] >= ns[a]) return R.K + 1;
        kb[a] += dk[a];
    }
    return max(0, (int)floorf(k_enter) - 2);
}

// March the 64 rays of this wave together.  `has_ray` is false for lanes
// outside the image; they still take part in the wave-wide steps.  LIT must
// equal (P.shade != RC_SHADE_NONE).
template <typename VT, int OP, bool LIT>
__device__ inline void march_wave(const RenderParams& P, const Ray& R, bool has_ray, void* lds_raw,
                                  int lds_bytes, int lane, MarchOut& M) {
    LaneState S;
    S.Cr = S.Cg = S.Cb = 0.f;
    S.T = 1.0f;
    S.k = 0;
    S.k_term = -1;
    S.done = !has_ray || R.K < 0;
    S.evaluated = S.shaded = S.direct = 0;
    // leading empty space: each lane jumps over its empty super-bricks
    if (!S.done && P.skip && P.super_empty != nullptr) S.k = entry_index(P, R);
    unsigned n_staged = 0, n_empty = 0, n_direct = 0;
    // Staging pays off when samples need the stencil neighbourhood; an
    // unshaded march reads 8 voxels per sample and gathers them directly.
    const bool stage = LIT;
    RayShade rs;
    ray_shade(P, R, rs);
    const GlobalSrc<VT> gsrc{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz,
                             (long long)P.nbx * P.nby * P.nbz * 512, P.dbg};
    using LT = typename LdsT<VT, OP>::type;
    LT* lds = (LT*)lds_raw;
    const int cap = min(lds_bytes, P.box_bytes) / (int)sizeof(LT);
    int len = P.chunk_init;
    // a super-chunk is tried at the start and after every empty chunk
    bool try_super = P.skip && P.super_empty != nullptr;
    // Every chunk advances at least the lane that owns the earliest pending
    // sample, so 64 (K_max + 1) chunks finish any wave; the cap only turns a
    // broken invariant into a wrong image instead of a wave that never ends.
    const long long chunk_cap = 64ll * (wave_max(has_ray ? (int)R.K : -1) + 2);
    long long n_chunks = 0;
    for (;;) {
        bool active = !S.done && S.k <= R.K;
        if (!active) S.done = true;
        if (__ballot(active) == 0ull || ++n_chunks > chunk_cap) break;
        // the chunk starts at the earliest pending sample of the wave
        double tau = wave_min_nonneg(active ? R.t_in + (double)S.k * P.step : INFINITY);
        Chunk ch;
        int kstop = -1;
        if (try_super) {
            // grows with the brick chunk length (up to 1024 after empty chunks)
            int slen = max(len * 8, kSuperInit);
            if (super_chunk_empty(P, R, active, S.k, tau, slen, kstop, lane)) {
                ++n_empty;
                if (active && kstop >= S.k) S.k = kstop + 1;
                len = min(len * 2, kChunkMax);
                continue;
            }
            try_super = false;
        }
        bool fits = false;
        for (;;) {
            int cmin[3], cmax[3];
            if (!chunk_cells(P, R, active, S.k, tau, len, kstop, cmin, cmax)) {
                fits = false;                   // no lane has a sample in the chunk
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
            fits = stage && vol <= cap;
            ch.mask_valid = nbr <= 64;
            if (((fits || !stage) && ch.mask_valid) || len <= kChunkMin) break;
            len >>= 1;
        }
        // brick occupancy of the chunk: one brick per lane, one ballot
        ch.live = ~0ull;
        ch.mixed = P.skip && !ch.mask_valid;
        if (P.skip && ch.mask_valid) {
            int nbr = ch.bdim[0] * ch.bdim[1] * ch.bdim[2];
            bool live = false;
            if (lane < nbr) {
                const int r01 = small_quot(lane, small_inv(ch.bdim[0]));
                const int r2 = small_quot(r01, small_inv(ch.bdim[1]));
                const int r0 = lane - r01 * ch.bdim[0], r1 = r01 - r2 * ch.bdim[1];
                int b = ((ch.blo[2] + r2) * P.nby + ch.blo[1] + r1) * P.nbx + ch.blo[0] + r0;
                live = to_gmem(P.empty)[RC_IDX(P.dbg, b, (long long)P.nbx * P.nby * P.nbz)] == 0;
            }
            ch.live = __ballot(live);
            ch.mixed = ch.live != (nbr == 64 ? ~0ull : ((1ull << nbr) - 1ull));
            if (ch.live == 0ull) {              // every sample of the chunk has alpha 0
                ++n_empty;
                if (active && kstop >= S.k) S.k = kstop + 1;
                len = min(len * 2, kChunkMax);
                try_super = P.super_empty != nullptr;
                continue;
            }
        }
        if (fits) {
            ++n_staged;
            stage_box<VT, LT>(P, lds, ch.lo, ch.dim, lane);
            wave_lds_sync();
        } else {
            ++n_direct;
        }
        LdsSrc<LT> lsrc{lds, {ch.lo[0], ch.lo[1], ch.lo[2]}, ch.dim[0], ch.dim[0] * ch.dim[1],
                        ch.dim[0] * ch.dim[1] * ch.dim[2], P.dbg};
        if (active && kstop >= S.k)
            run_samples<VT, OP, LIT>(P, R, lsrc, gsrc, fits, ch, kstop, rs, S);
        if (fits) wave_lds_sync();
        if (active && !S.done && kstop >= S.k) S.k = kstop + 1;
    }
    M.rgba = make_float4(S.Cr, S.Cg, S.Cb, 1.0f - S.T);
    M.k_last = (int)(S.k_term >= 0 ? S.k_term : R.K);
    M.T = S.T;
    M.evaluated = S.evaluated;
    M.shaded = S.shaded;
    M.samples_direct = S.direct;
    M.chunks_staged = n_staged;
    M.chunks_empty = n_empty;
    M.chunks_direct = n_direct;
}

// ---------------------------------------------------------------- one tile
// One wave renders one tile of tile_w x (64 / tile_w) pixels; `tile` is the
// tile's row-major index in the image.  Lanes outside the image take part
// in the wave-wide steps without a ray.
template <typename VT, int OP, bool LIT>
__device__ inline void render_tile(const RenderParams& P, const ViewParams& V, int tile, int lane,
                                   void* lds, int lds_bytes) {
    const int tw = V.tile_w, th = 64 / V.tile_w;
    int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    int px = tx * tw + (lane % tw), py = ty * th + (lane / tw);
    bool valid = px >= 0 && py >= 0 && px < V.W && py < V.H;
    Ray R;
    R.K = -1;
    R.t_in = R.t_out = 0.0;
    for (int a = 0; a < 3; ++a) R.o[a] = R.d[a] = R.p0[a] = R.dp[a] = 0.0;
    if (valid) setup_ray(P, V, px, py, R);
    MarchOut M;
    march_wave<VT, OP, LIT>(P, R, valid, lds, lds_bytes, lane, M);
    if (valid) {
        long long pix = (long long)py * V.W + px;
        V.out[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = M.rgba;
        if (V.aux) V.aux[RC_IDX(P.dbg, pix, (long long)V.W * V.H)] = rc_aux{M.k_last, M.T};
    }
    if (P.stats) {
        unsigned lat = wave_sum(R.K >= 0 ? (unsigned)(M.k_last + 1) : 0u);
        unsigned ev = wave_sum(M.evaluated);
        unsigned sh = wave_sum(M.shaded);
        unsigned hit = wave_sum(R.K >= 0 ? 1u : 0u);
        unsigned dir = wave_sum(M.samples_direct);
        if (lane == 0) {
            // one of kStatSlots copies, so waves do not all hit one address
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
