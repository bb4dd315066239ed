// Reverse mode of the render: one ray per lane marches back to front
// from its last composited sample and accumulates dL/dvolume and
// dL/dtable, through the lighting and the gradient operator's taps when a
// shading model is on.  No per-sample state is stored by the forward pass; the
// transmittance in front of each sample is recovered from the final
// transmittance written to rc_aux.
#include <algorithm>
#include <cmath>

#include "stencil.h"

namespace rc {

struct BackwardParams {
    float* dvol;            // [nz][ny][nx]
    float* dtf;             // [M][4]
    int lds_tf;             // 1: accumulate the table gradient in LDS first
    int lds_table;          // 1: read the table from an LDS copy
    int M4;                 // table entries * 4 (the dTF length)
    unsigned int* dbg;      // bounds-checked build: violation counter; else null
    int box_bytes;          // LDS per wave of the chunked kernel (dV box + voxel box)
    int chunk_len;          // first chunk length, lattice steps
    int* next_unit;         // the chunked kernel's tile counter, zero at launch
};

constexpr int kBwdTile = 8;               // 8x8 pixels, one wave per tile
constexpr int kBwdLdsTable = 1024;        // tables up to this are read from an LDS copy
constexpr float kTinyT = 1e-30f;
// The reverse kernel: resident blocks of kBwdBoxWaves waves (each wave
// taking tiles one at a time from a counter) share
// the table gradient in LDS -- tables up to kBwdBoxTfEntries entries, so a
// whole block's samples, which mostly read a few hot entries, meet in LDS
// instead of at a few device addresses -- and each wave has up to
// kBwdBoxBytes of what the 160 KiB of LDS leave for its chunk's dV box and
// staged voxel box.
constexpr int kBwdBoxWaves = 8;
constexpr int kBwdBoxTfEntries = 4096;
constexpr int kBwdBoxBytes = 20480;
constexpr int kBwdLdsBytes = 160 * 1024;
constexpr int kBwdChunk = 16;             // first chunk length in lattice steps

__device__ __forceinline__ void add_dtf(const BackwardParams& B, float* lds, int i, int ch, float v) {
    if (v == 0.0f) return;
    if (B.lds_tf) atomicAdd(&lds[RC_IDX(B.dbg, i * 4 + ch, B.M4)], v);
    else unsafeAtomicAdd(&B.dtf[RC_IDX(B.dbg, i * 4 + ch, B.M4)], v);
}

// A ray's table-gradient contributions, summed in registers while its
// samples stay between the same two entries (i, i+1) and added to the
// shared sum when the entry pair changes or the ray ends.  Neighbouring
// samples mostly share the pair (all of a transparent background reads
// entry 0), so this replaces most of the same-address atomics that
// serialise when every lane of a wave adds to one entry.
struct DtfRun {
    int i = -1;                 // lower entry, -1 = empty
    float a0[4], a1[4];         // contributions to entries i and min(i + 1, M - 1)
};

__device__ __forceinline__ void dtf_flush(const RenderParams& P, const BackwardParams& B, float* lds,
                                          DtfRun& r) {
    if (r.i < 0) return;
    const int i1 = min(r.i + 1, P.M - 1);
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        add_dtf(B, lds, r.i, ch, r.a0[ch]);
        add_dtf(B, lds, i1, ch, r.a1[ch]);
    }
    r.i = -1;
}

__device__ __forceinline__ void dtf_add(const RenderParams& P, const BackwardParams& B, float* lds,
                                        DtfRun& r, int i, float w0, float w1, const float d[4]) {
    if (i != r.i) {
        dtf_flush(P, B, lds, r);
        r.i = i;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) r.a0[ch] = r.a1[ch] = 0.0f;
    }
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        r.a0[ch] = fmaf(w0, d[ch], r.a0[ch]);
        r.a1[ch] = fmaf(w1, d[ch], r.a1[ch]);
    }
}

// Value, table entry pair, opacity and colour of lattice sample k.  With a
// shading model the colour is the lit one, also where the opacity is 0:
// the forward skips the lighting there only because the colour is
// multiplied by 0, and dC/da needs it.
struct BwdSample {
    Cell C;
    int ox[4], oy[4], oz[4];    // footprint offsets in the bricked volume
    double pv[3];
    float vn;                   // normalised value before clamping
    int i, i1;
    float t;                    // position between entries i and i1
    float4 e0, e1;              // table entries
    float4 rgba;                // table rgb and opacity before correction
    float a;                    // opacity after correction
    float da_dtf;               // d a / d (table opacity)
    float g[3];                 // gradient (shaded renders)
    float c[3];                 // colour
};

// Sample k's position, footprint offsets and its cell's 8 voxels (the loads
// are issued here and consumed by bwd_finish, so a caller can overlap them
// with other work).
// The source is the bricked volume (GlobalSrc) or a chunk's voxel box
// staged in LDS (LdsSrc, which holds the same values).
template <typename VT, typename Src>
__device__ __forceinline__ void bwd_fetch_from(const RenderParams& P, const Ray& R, int k,
                                               const Src& src, BwdSample& S, float corner[8]) {
    lattice_point(P, R, k, S.C, S.pv);
    src.offsets(S.C, S.ox, S.oy, S.oz);
    load_corners<VT>(src.base, S.ox, S.oy, S.oz, corner);
}

template <typename VT>
__device__ __forceinline__ void bwd_fetch(const RenderParams& P, const Ray& R, int k,
                                          BwdSample& S, float corner[8]) {
    const GlobalSrc<VT> src{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz,
                             (long long)P.nbx * P.nby * P.nbz * 512, P.dbg};
    bwd_fetch_from<VT>(P, R, k, src, S, corner);
}

// base: the voxel source the sample was fetched from (its offsets S.ox ..),
// null for the bricked volume.
template <typename VT, int OP, bool LIT>
__device__ __forceinline__ void bwd_finish(const RenderParams& P, const float4* tab,
                                           const RayShade& rs, bool lit, const float corner[8],
                                           BwdSample& S, const VT* base = nullptr) {
    if (!base) base = (const VT*)P.vox;
    float v = trilinear(corner, S.C);
    S.vn = (v - P.vmin) * P.inv_range;
    float uu = fminf(fmaxf(S.vn, 0.0f), 1.0f) * P.Mm1;
    S.i = min((int)uu, P.M - 1);
    S.i1 = min(S.i + 1, P.M - 1);
    S.t = uu - (float)S.i;
    S.e0 = tab[RC_IDX(P.dbg, S.i, P.M)];
    S.e1 = tab[RC_IDX(P.dbg, S.i1, P.M)];
    S.rgba = make_float4(lerpf(S.e0.x, S.e1.x, S.t), lerpf(S.e0.y, S.e1.y, S.t),
                         lerpf(S.e0.z, S.e1.z, S.t), lerpf(S.e0.w, S.e1.w, S.t));
    S.a = S.rgba.w;
    S.da_dtf = 1.0f;
    if (P.ocorr > 0.0f) {
        // a = 1 - (1 - a_tf)^e: da/da_tf = e (1 - a_tf)^(e - 1) (e at a_tf = 0),
        // taken as 0 at a_tf = 1 when e < 1
        float om = 1.0f - S.a;
        S.da_dtf = (om > 0.0f || P.ocorr >= 1.0f)
                       ? P.ocorr * __builtin_amdgcn_exp2f((P.ocorr - 1.0f) * __builtin_amdgcn_logf(om))
                       : 0.0f;
        if (S.a != 0.0f) S.a = correct_opacity(P.ocorr, S.a);
    }
    S.c[0] = S.rgba.x; S.c[1] = S.rgba.y; S.c[2] = S.rgba.z;
    if (LIT && lit) {
        gradient_exact<VT, OP>(P, base, S.ox, S.oy, S.oz, S.C, corner, S.g);
        shade(P, S.rgba, S.g, S.pv, rs, S.c);
    }
}

template <typename VT, int OP, bool LIT>
__device__ __forceinline__ void bwd_sample(const RenderParams& P, const float4* tab, const Ray& R,
                                           const RayShade& rs, int k, bool lit,
                                           BwdSample& S) {
    float corner[8];
    bwd_fetch<VT>(P, R, k, S, corner);
    bwd_finish<VT, OP, LIT>(P, tab, rs, lit, corner, S);
}

// Where volume-gradient contributions go: straight to dV in device memory
// (lds == null), or to a chunk's voxel box in LDS (the box covers every
// voxel the chunk's samples reach, clamped indices included), which is
// added to dV once per chunk (dv_box_flush).
struct DvSink {
    float* lds;             // box [dim2][dim1][dim0] or null
    int lo[3];              // voxel index of box voxel (0, 0, 0)
    int bx, bxy, n;         // row and slab strides, voxels in the box
};

__device__ __forceinline__ void dv_atomic(const RenderParams& P, const BackwardParams& B,
                                          const DvSink& sk, int x, int y, int z, float w) {
    if (sk.lds) {
        atomicAdd(&sk.lds[RC_IDX(P.dbg, (z - sk.lo[2]) * sk.bxy + (y - sk.lo[1]) * sk.bx +
                                             (x - sk.lo[0]),
                                 sk.n)],
                  w);
    } else {
        unsafeAtomicAdd(&B.dvol[RC_IDX(P.dbg, ((long long)z * P.ny + y) * P.nx + x,
                                       (long long)P.nx * P.ny * P.nz)],
                        w);
    }
}

// A ray's volume-gradient contributions to the 8 corners of one cell,
// summed while its samples stay in that cell (at half-voxel steps most
// cells hold two or more consecutive samples) and added to dV when the ray
// moves to another cell or ends.
struct DvRun {
    int c[3] = {INT_MIN, 0, 0};     // cell, c[0] = INT_MIN when empty
    float w[8];                     // corner (x + 2y + 4z) contributions
};

__device__ __forceinline__ void dv_flush(const RenderParams& P, const BackwardParams& B,
                                         const DvSink& sk, DvRun& r) {
    if (r.c[0] == INT_MIN) return;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (r.w[q] == 0.0f) continue;
        int x = clampi(r.c[0] + (q & 1), 0, P.nx - 1);
        int y = clampi(r.c[1] + ((q >> 1) & 1), 0, P.ny - 1);
        int z = clampi(r.c[2] + (q >> 2), 0, P.nz - 1);
        dv_atomic(P, B, sk, x, y, z, r.w[q]);
    }
    r.c[0] = INT_MIN;
}

__device__ __forceinline__ void dv_add(const RenderParams& P, const BackwardParams& B,
                                       const DvSink& sk, DvRun& r, const Cell& C, float dv) {
    if (C.c[0] != r.c[0] || C.c[1] != r.c[1] || C.c[2] != r.c[2]) {
        dv_flush(P, B, sk, r);
        r.c[0] = C.c[0]; r.c[1] = C.c[1]; r.c[2] = C.c[2];
#pragma unroll
        for (int q = 0; q < 8; ++q) r.w[q] = 0.0f;
    }
    const float fx = C.fr[0], fy = C.fr[1], fz = C.fr[2];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float w = ((q & 1) ? fx : 1.0f - fx) * (((q >> 1) & 1) ? fy : 1.0f - fy) *
                  ((q >> 2) ? fz : 1.0f - fz);
        r.w[q] = fmaf(w, dv, r.w[q]);
    }
}

// Reverse of shade(): dL/dc -> dL/d(table rgb) and dL/dG, through the same
// branches the forward took (max(0, .), the |G| floor).
__device__ __forceinline__ void shade_adjoint(const RenderParams& P, const BwdSample& S,
                                              const RayShade& rs, const float dc[3],
                                              float drgb[3], float dg[3]) {
    const float* g = S.g;
    float g2 = fmaf(g[2], g[2], fmaf(g[1], g[1], g[0] * g[0]));
    float rq = __builtin_amdgcn_rsqf(g2), cap = 1.0f / P.grad_eps;
    bool floored = !(rq < cap);
    float inv = floored ? cap : rq;
    float gh[3] = {g[0] * inv, g[1] * inv, g[2] * inv};
    float L[3], H[3];
    if (P.light_is_point) {
        float q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = P.light[a] - (float)S.pv[a] * P.s[a];
        float qi = rsq_or_zero(fmaf(q[2], q[2], fmaf(q[1], q[1], q[0] * q[0])));
        L[0] = q[0] * qi; L[1] = q[1] * qi; L[2] = q[2] * qi;
        float h[3] = {L[0] + rs.v[0], L[1] + rs.v[1], L[2] + rs.v[2]};
        float hi = rsq_or_zero(fmaf(h[2], h[2], fmaf(h[1], h[1], h[0] * h[0])));
        H[0] = h[0] * hi; H[1] = h[1] * hi; H[2] = h[2] * hi;
    } else {
        L[0] = P.light[0]; L[1] = P.light[1]; L[2] = P.light[2];
        H[0] = rs.h[0]; H[1] = rs.h[1]; H[2] = rs.h[2];
    }
    const float dc_rgb = fmaf(dc[2], S.rgba.z, fmaf(dc[1], S.rgba.y, dc[0] * S.rgba.x));
    float dgh[3];
    if (P.shade == RC_SHADE_PAPER_LAMBERT) {
        float illum = fmaf(L[2], gh[2], fmaf(L[1], gh[1], L[0] * gh[0]));
        drgb[0] = dc[0] * illum; drgb[1] = dc[1] * illum; drgb[2] = dc[2] * illum;
        dgh[0] = dc_rgb * L[0]; dgh[1] = dc_rgb * L[1]; dgh[2] = dc_rgb * L[2];
    } else {
        float nl = -fmaf(gh[2], L[2], fmaf(gh[1], L[1], gh[0] * L[0]));
        float nh = -fmaf(gh[2], H[2], fmaf(gh[1], H[1], gh[0] * H[0]));
        float k = fmaf(P.kd, fmaxf(nl, 0.0f), P.ka);
        drgb[0] = dc[0] * k; drgb[1] = dc[1] * k; drgb[2] = dc[2] * k;
        float wl = nl > 0.0f ? P.kd * dc_rgb : 0.0f;
        // d/dnh of nh^s = s nh^(s-1) = s spec / nh
        float wh = 0.0f;
        if (nh > 0.0f && P.shininess != 0.0f) {
            float spec = __builtin_amdgcn_exp2f(P.shininess * __builtin_amdgcn_logf(nh));
            wh = P.ks * (dc[0] + dc[1] + dc[2]) * P.shininess * spec / nh;
        }
        // N = -gh
#pragma unroll
        for (int a = 0; a < 3; ++a) dgh[a] = -fmaf(wl, L[a], wh * H[a]);
    }
    if (floored) {
        dg[0] = dgh[0] * inv; dg[1] = dgh[1] * inv; dg[2] = dgh[2] * inv;
    } else {
        float proj = fmaf(gh[2], dgh[2], fmaf(gh[1], dgh[1], gh[0] * dgh[0]));
#pragma unroll
        for (int a = 0; a < 3; ++a) dg[a] = (dgh[a] - gh[a] * proj) * inv;
    }
}

// Reverse of the gradient operator (gradient, gradient_exact: the same
// linear map of the footprint's voxels), as its separable 4x4x4 filters
// transposed.  A footprint voxel (x, y, z) carries, for dL/dG = (gx, gy, gz)
// in scaled units,
//   gx (D'x A'y A'z + gamma D'x Ly Lz) + gy (A'x D'y A'z + gamma Lx D'y Lz)
//   + gz (A'x A'y D'z + gamma Lx Ly D'z),
// added to the clamped voxel of the linear gradient array.
template <int OP>
__device__ __forceinline__ void gradient_adjoint(const RenderParams& P, const BackwardParams& Bp,
                                                 const DvSink& sk, const Cell& C,
                                                 const float dg[3]) {
    constexpr bool SEP = OpTaps<OP>::kSep;
    const float gm = OpTaps<OP>::gamma;
    const float gx = dg[0] * P.gscale[0], gy = dg[1] * P.gscale[1], gz = dg[2] * P.gscale[2];
    if (gx == 0.0f && gy == 0.0f && gz == 0.0f) return;
    AxisTaps kx, ky, kz;
    axis_taps<OP>(C.fr[0], kx);
    axis_taps<OP>(C.fr[1], ky);
    axis_taps<OP>(C.fr[2], kz);
    int xi[4], yi[4], zi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        xi[i] = clampi(C.c[0] - 1 + i, 0, P.nx - 1);
        yi[i] = clampi(C.c[1] - 1 + i, 0, P.ny - 1);
        zi[i] = clampi(C.c[2] - 1 + i, 0, P.nz - 1);
    }
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            // per-(y, z) factors of the three components
            const float fxA = SEP ? ky.A[y] * kz.A[z] : 0.0f, fxL = gm * ky.L[y] * kz.L[z];
            const float fyA = SEP ? ky.D[y] * kz.A[z] : 0.0f, fyL = gm * ky.D[y] * kz.L[z];
            const float fzA = SEP ? ky.A[y] * kz.D[z] : 0.0f, fzL = gm * ky.L[y] * kz.D[z];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                float w = gx * kx.D[x] * (fxA + fxL);
                w = fmaf(gy, fmaf(kx.A[x], fyA, kx.L[x] * fyL), w);
                w = fmaf(gz, fmaf(kx.A[x], fzA, kx.L[x] * fzL), w);
                if (w != 0.0f) dv_atomic(P, Bp, sk, xi[x], yi[y], zi[z], w);
            }
        }
}

// Chain rule for one sample (see the forward: C = sum T_k a_k c_k,
// A = 1 - prod(1 - a_k)):
//   dL/dc_k = g_rgb T_k a_k
//   dL/da_k = T_k [ g_rgb . (c_k - Bk1) + g_A Pk1 ]
// with Bk1 the colour composited behind k (eq. 6 run back to front) and
// Pk1 the transmittance of the samples behind k.  Then through the
// lighting to the table rgb and the gradient, through the opacity
// correction, the table interpolation to u, the clamp to the value, and the
// trilinear weights; the gradient goes back through the operator's taps.
template <typename VT, int OP, bool LIT>
__device__ __forceinline__ void bwd_accumulate(const RenderParams& P, const BackwardParams& Bp,
                                               float* lds, DtfRun& run, DvRun& vrun,
                                               const DvSink& sk, const BwdSample& S,
                                               const RayShade& rs,
                                               float Tk, const float4& g, const float Bk1[3],
                                               float Pk1) {
    float ta = Tk * S.a;
    float dc[3] = {g.x * ta, g.y * ta, g.z * ta};
    float da = Tk * (g.x * (S.c[0] - Bk1[0]) + g.y * (S.c[1] - Bk1[1]) +
                     g.z * (S.c[2] - Bk1[2]) + g.w * Pk1) * S.da_dtf;
    float drgb[3] = {dc[0], dc[1], dc[2]}, dg[3] = {0.f, 0.f, 0.f};
    if (LIT && S.a != 0.0f) shade_adjoint(P, S, rs, dc, drgb, dg);
    float w0 = 1.0f - S.t, w1 = S.t;
    const float d4[4] = {drgb[0], drgb[1], drgb[2], da};
    dtf_add(P, Bp, lds, run, S.i, w0, w1, d4);
    if (LIT) gradient_adjoint<OP>(P, Bp, sk, S.C, dg);
    if (!(S.vn > 0.0f && S.vn < 1.0f)) return;      // clamped: no dependence on the value
    float du = drgb[0] * (S.e1.x - S.e0.x) + drgb[1] * (S.e1.y - S.e0.y) +
               drgb[2] * (S.e1.z - S.e0.z) + da * (S.e1.w - S.e0.w);
    float dv = du * P.Mm1 * P.inv_range;
    if (dv == 0.0f) return;
    // nearest sampling has fraction 0: only corner 0 gets a non-zero weight
    dv_add(P, Bp, sk, vrun, S.C, dv);
}

// Maximum of non-negative doubles over the wave, exact: their bit patterns
// order like unsigned 64-bit integers (0 is the identity for lanes a DPP
// move does not write).
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64_or0(unsigned long long v) {
    unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, ROWS, 0xF, false);
    unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, ROWS, 0xF, false);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double wave_max_nonneg(double x) {
    unsigned long long v = (unsigned long long)__double_as_longlong(x);
    v = max(v, dpp_u64_or0<0xB1, 0xF>(v));     // quad_perm 1,0,3,2
    v = max(v, dpp_u64_or0<0x4E, 0xF>(v));     // quad_perm 2,3,0,1
    v = max(v, dpp_u64_or0<0x141, 0xF>(v));    // row_half_mirror
    v = max(v, dpp_u64_or0<0x140, 0xF>(v));    // row_mirror
    v = max(v, dpp_u64_or0<0x142, 0xA>(v));    // row_bcast:15
    v = max(v, dpp_u64_or0<0x143, 0xC>(v));    // row_bcast:31
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Add a chunk's dV box to dV and clear it.  Lane i reads box entries i,
// i + 64, ...; box coordinates advance incrementally (no divisions).
__device__ __forceinline__ void dv_box_flush(const RenderParams& P, const BackwardParams& B,
                                             const DvSink& sk, int lane) {
    const int bx = sk.bx, by = sk.bxy / sk.bx;
    int x = lane % bx, y = (lane / bx) % by, z = lane / sk.bxy;
    const int step_x = 64 % bx, step_y = 64 / bx;
    for (int i = lane; i < sk.n; i += 64) {
        const float w = sk.lds[i];
        if (w != 0.0f) {
            const int gx = sk.lo[0] + x, gy = sk.lo[1] + y, gz = sk.lo[2] + z;
            // taps are clamped into the grid: entries outside it stay 0
            if (gx >= 0 && gy >= 0 && gz >= 0 && gx < P.nx && gy < P.ny && gz < P.nz)
                unsafeAtomicAdd(&B.dvol[RC_IDX(P.dbg, ((long long)gz * P.ny + gy) * P.nx + gx,
                                               (long long)P.nx * P.ny * P.nz)],
                                w);
            sk.lds[i] = 0.0f;
        }
        x += step_x;
        y += step_y;
        if (x >= bx) { x -= bx; ++y; }
        while (y >= by) { y -= by; ++z; }
    }
}

// Issue priority of a wave for its current tile, from the tile's longest ray
// (last composited index, as a share of the most lattice steps a ray
// through the volume can take): the long rays are serial chains that set
// the pass's length, so the SIMD's arbiter serves their waves first and
// the other waves fill the remaining issue slots.  Scheduling only.
__device__ __forceinline__ void prioritise_long_rays(const RenderParams& P, int wave_last) {
    const float dx = (float)(P.nx - 1) * P.s[0], dy = (float)(P.ny - 1) * P.s[1],
                dz = (float)(P.nz - 1) * P.s[2];
    const float kmax = sqrtf(dx * dx + dy * dy + dz * dz) * (float)P.inv_step + 2.0f;
    const float r = (float)(wave_last + 1) / kmax;
    if (r >= 0.75f) __builtin_amdgcn_s_setprio(3);
    else if (r >= 0.5f) __builtin_amdgcn_s_setprio(2);
    else if (r >= 0.25f) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// The reverse march in chunks shared by the wave.  A wave renders one 8x8
// pixel tile at a time; each lane runs its own ray back to front, and the
// wave only agrees on a window of ray parameter (thi - len step, thi],
// thi = the latest pending sample of any lane, in which every lane
// processes its samples.  Their contributions to dV go to an LDS box over
// the window's voxels (LDS atomics), which is added to dV once per chunk:
// one device atomic per touched voxel instead of one per tap (up to 64 per
// shaded sample) or corner and sample.  A window whose box does not fit even
// at 2 steps sends its contributions straight to dV.  Shaded renders also
// stage the window's voxels in LDS (the operator reads 64 per sample).
// Work order (view_of_unit, centre_out): views take turns, each view's
// tiles centre-out, so the long rays through the middle start first.
template <typename VT, int OP, bool LIT>
__global__ __launch_bounds__(64 * kBwdBoxWaves) void raycast_bwd_box(RenderParams P, ViewSet S,
                                                                    BackwardParams Bp) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float4* tab = P.tf;
    // LDS: the block's table gradient (shared by its waves), the table copy,
    // then one dV box per wave
    const int tf_floats = (Bp.lds_tf ? P.M * 4 : 0) + (Bp.lds_table ? P.M * 4 : 0);
    float* dvb = lds + tf_floats + wave * (Bp.box_bytes / 4);
    if (Bp.lds_tf)
        for (int i = threadIdx.x; i < P.M * 4; i += blockDim.x) lds[i] = 0.0f;
    if (Bp.lds_table) {
        float4* t = (float4*)(lds + (Bp.lds_tf ? P.M * 4 : 0));
        for (int i = threadIdx.x; i < P.M; i += blockDim.x) t[i] = P.tf[i];
        tab = t;
    }
    for (int i = lane; i < Bp.box_bytes / 4; i += 64) dvb[i] = 0.0f;
    __syncthreads();
    // This wave's LDS: the dV box grows from the start, the chunk's voxel box
    // sits at the end.  [0, zero_end) is known to be all zero; the dV box
    // must start zeroed, so where it grows into bytes a voxel box used it is
    // cleared first.
    unsigned char* wl = (unsigned char*)dvb;
    const int wave_bytes = Bp.box_bytes;
    int zero_end = wave_bytes;
    // Resident waves take the tiles in that work order from a counter, one
    // atomic add per tile: a wave whose rays end early takes the next tile
    // instead of holding its slot until the block's slowest ray ends, and
    // the block's table gradient is flushed once.  The counter only grows,
    // so each wave leaves at its first index past the tiles (compared
    // unsigned: a bad start also ends the loop).
    const unsigned n_units = (unsigned)S.block_off[S.n];
    for (;;) {
        int fetched = 0;
        if (lane == 0) fetched = atomicAdd(Bp.next_unit, 1);
        const unsigned unit = (unsigned)__builtin_amdgcn_readfirstlane(__shfl(fetched, 0));
        if (unit >= n_units) break;
        int b = 0, v = view_of_unit(S, 1, (int)unit, b);
        const ViewParams& V = S.v[v < 0 ? 0 : v];
        int tiles_x = (V.W + kBwdTile - 1) / kBwdTile, tiles_y = (V.H + kBwdTile - 1) / kBwdTile;
        int tx = centre_out(b % tiles_x, tiles_x), ty = centre_out(b / tiles_x, tiles_y);
        int px = tx * kBwdTile + (lane % kBwdTile);
        int py = ty * kBwdTile + (lane / kBwdTile);
        const bool valid = v >= 0 && b < tiles_x * tiles_y && px < V.W && py < V.H;
        Ray R;
        R.K = -1;
        R.t_in = R.t_out = 0.0;
        for (int a = 0; a < 3; ++a) R.o[a] = R.d[a] = R.p0[a] = R.dp[a] = 0.0;
        if (valid) setup_ray(P, V, px, py, R);
        RayShade rs;
        ray_shade(P, R, rs);
        rc_aux ax{-1, 0.0f};
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) {
            long long pix = (long long)py * V.W + px;
            ax = V.aux[RC_IDX(P.dbg, pix, (long long)V.W * V.H)];
            g = V.grad[RC_IDX(P.dbg, pix, (long long)V.W * V.H)];
        }
        const int last = ax.k_last;
        const bool has = valid && R.K >= 0 && last >= 0 && last <= R.K;
        prioritise_long_rays(P, wave_max(has ? last : -1));
        // Anchor: the last index a whose front transmittance T_a is at least
        // kTinyT.  Normally a = last + 1 with T_a = t_final; if the ray went
        // (nearly) opaque, a forward pass finds a instead.  Samples from a on
        // are composited but get no gradient (their T is below kTinyT).
        int anchor = last + 1;
        float Ta = ax.t_final;
        if (has && !(Ta >= kTinyT)) {
            float T = 1.0f;
            anchor = 0;
            for (int k = 0; k <= last; ++k) {
                BwdSample Sx;
                bwd_sample<VT, OP, LIT>(P, tab, R, rs, k, false, Sx);
                float Tn = T * (1.0f - Sx.a);
                if (!(Tn >= kTinyT)) break;
                T = Tn;
                anchor = k + 1;
            }
            Ta = T;
        }
        float Bk1[3] = {0.f, 0.f, 0.f};
        float Pk1 = 1.0f, Q = 1.0f;
        DtfRun run;
        DvRun vrun;
        int k = has ? last : -1;
        const GlobalSrc<VT> gsrc{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz,
                                 (long long)P.nbx * P.nby * P.nbz * 512, P.dbg};
        const DvSink glob{nullptr, {0, 0, 0}, 0, 0, 0};
        // Every chunk moves at least the lane that defines thi one sample on,
        // so 64 (K_max + 1) chunks finish any wave; the cap only turns a broken
        // invariant into a wrong gradient instead of a wave that never ends.
        const long long chunk_cap = 64ll * (wave_max(has ? last : -1) + 2);
        long long n_chunks = 0;
        for (;;) {
            const bool active = k >= 0;
            if (__ballot(active) == 0ull || ++n_chunks > chunk_cap) break;
            const double thi = wave_max_nonneg(active ? R.t_in + (double)k * P.step : 0.0);
            int len = Bp.chunk_len, kstop = k + 1;
            DvSink sk = glob;
            int vlo[3] = {0, 0, 0}, vdim[3] = {0, 0, 0}, vbytes = 0;
            for (;;) {
                const double tlo = thi - (double)len * P.step;
                int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
                kstop = k + 1;
                if (active) {
                    // first index past tlo (rounding here only groups the work)
                    const double q = floor((tlo - R.t_in) * P.inv_step) + 1.0;
                    kstop = q <= 0.0 ? 0 : (q > (double)k ? k + 1 : (int)q);
                    // the lane(s) that define thi always own their next sample
                    if (R.t_in + (double)k * P.step >= thi) kstop = min(kstop, k);
                    if (kstop <= k) {
                        Cell c0, c1;
                        double pv[3];
                        lattice_point(P, R, kstop, c0, pv);
                        lattice_point(P, R, k, c1, pv);
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            mn[a] = min(c0.c[a], c1.c[a]);
                            mx[a] = max(c0.c[a], c1.c[a]);
                        }
                    }
                }
                int lo[3], dim[3];
                long long nvox = 1, vvox = 1;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int cmin = wave_min(mn[a]), cmax = wave_max(mx[a]);
                    lo[a] = cmin - 1;                   // the taps reach one voxel below
                    dim[a] = cmax - cmin + 4;           // and two above the cells
                    nvox *= dim[a];
                    // the voxel box: the same span, widened to even bounds for
                    // the 2x2x2 group loads of stage_box
                    vlo[a] = lo[a] & ~1;
                    vdim[a] = ((cmax + 2) | 1) - vlo[a] + 1;
                    vvox *= vdim[a];
                }
                const long long dvb16 = (nvox * 4 + 15) & ~15ll;
                // unshaded samples read 8 voxels each: staging does not pay
                // (measured); shaded ones read the operator's 64
                const long long vb16 = LIT ? (vvox * (long long)sizeof(VT) + 15) & ~15ll : 0;
                if (dvb16 + vb16 <= wave_bytes) {
                    sk = DvSink{dvb, {lo[0], lo[1], lo[2]}, dim[0], dim[0] * dim[1], (int)nvox};
                    vbytes = (int)vb16;
                    break;
                }
                if (len <= 2) break;                    // read and scatter in device memory
                len >>= 1;
            }
            const VT* vbox = nullptr;
            if (sk.lds && !LIT) {
                if (zero_end < sk.n * 4) {
                    for (int i = zero_end / 4 + lane; i < sk.n; i += 64) dvb[i] = 0.0f;
                    zero_end = sk.n * 4;
                }
                wave_lds_sync();
            } else if (sk.lds) {
                if (zero_end < sk.n * 4) {
                    for (int i = zero_end / 4 + lane; i < sk.n; i += 64) dvb[i] = 0.0f;
                    zero_end = sk.n * 4;
                }
                VT* vb = (VT*)(wl + wave_bytes - vbytes);
                stage_box<VT, VT>(P, vb, vlo, vdim, lane);
                zero_end = min(zero_end, wave_bytes - vbytes);
                wave_lds_sync();
                vbox = vb;
            }
            const LdsSrc<VT> lsrc{vbox, {vlo[0], vlo[1], vlo[2]}, vdim[0], vdim[0] * vdim[1],
                                  vdim[0] * vdim[1] * vdim[2], P.dbg};
            // this lane's samples k .. kstop, back to front, read from the box
            // (every one of them lies in it: their cells lie between the end
            // cells the box was built from) or from the bricked volume
            while (k >= kstop) {
                BwdSample Sm;
                float cn[8];
                if (vbox) {
                    bwd_fetch_from<VT>(P, R, k, lsrc, Sm, cn);
                    bwd_finish<VT, OP, LIT>(P, tab, rs, true, cn, Sm, vbox);
                } else {
                    bwd_fetch_from<VT>(P, R, k, gsrc, Sm, cn);
                    bwd_finish<VT, OP, LIT>(P, tab, rs, true, cn, Sm);
                }
                const float om = 1.0f - Sm.a;
                if (k < anchor) {
                    Q *= om;
                    const float Tk = Q > 0.0f ? Ta / Q : 0.0f;
                    bwd_accumulate<VT, OP, LIT>(P, Bp, lds, run, vrun, sk, Sm, rs, Tk, g, Bk1, Pk1);
                }
                Bk1[0] = fmaf(Sm.a, Sm.c[0], om * Bk1[0]);
                Bk1[1] = fmaf(Sm.a, Sm.c[1], om * Bk1[1]);
                Bk1[2] = fmaf(Sm.a, Sm.c[2], om * Bk1[2]);
                Pk1 *= om;
                --k;
            }
            dv_flush(P, Bp, sk, vrun);              // a cell run does not outlive its chunk
            if (sk.lds) {
                wave_lds_sync();
                dv_box_flush(P, Bp, sk, lane);
                wave_lds_sync();
            }
        }
        dtf_flush(P, Bp, lds, run);
    }
    if (Bp.lds_tf) {
        __syncthreads();
        for (int i = threadIdx.x; i < P.M * 4; i += blockDim.x) {
            float w = lds[i];
            if (w != 0.0f) unsafeAtomicAdd(&Bp.dtf[i], w);
        }
    }
}

__global__ void bwd_reset(int* next_unit) {
    if (threadIdx.x == 0) *next_unit = 0;
}

template <typename VT>
static rc_status launch_bwd_t(const RenderParams& P, const ViewSet& S, const BackwardParams& Bp,
                              int op, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    using BwdFn = void (*)(RenderParams, ViewSet, BackwardParams);
    BwdFn fn;
    if (P.shade == RC_SHADE_NONE) {
        fn = raycast_bwd_box<VT, RC_GRAD_CENTRAL, false>;
    } else if (op == RC_GRAD_CENTRAL) {
        fn = raycast_bwd_box<VT, RC_GRAD_CENTRAL, true>;
    } else if (op == RC_GRAD_SOBEL3D) {
        fn = raycast_bwd_box<VT, RC_GRAD_SOBEL3D, true>;
    } else {
        fn = raycast_bwd_box<VT, RC_GRAD_ZUCKER_HUMMEL, true>;
    }
    // the waves take tiles from the counter: launch what stays resident
    int dev = 0, n_cu = 0, per_cu = 0;
    RC_HIP(hipGetDevice(&dev));
    RC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    RC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn,
                                                        (int)block.x, lds));
    const unsigned resident = (unsigned)(std::max(1, n_cu) * std::max(1, per_cu));
    grid.x = std::min(grid.x, resident);
    hipLaunchKernelGGL(bwd_reset, dim3(1), dim3(64), 0, s, Bp.next_unit);
    hipLaunchKernelGGL(fn, grid, block, lds, s, P, S, Bp);
    return RC_OK;
}

}  // namespace rc

using namespace rc;

static rc_status backward_views(const rc_volume* v, const rc_camera* cams, int n_views,
                                const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                                const rc_options* opt, const rc_aux* const* aux,
                                const float* const* grad_rgba, float* grad_volume_dev,
                                float* grad_tf_dev, hipStream_t s) {
    for (int i = 0; i < n_views; ++i) {
        rc_status st = check_render_args(v, &cams[i], tf_rgba_dev, tf_len, sh, opt);
        if (st != RC_OK) return n_views > 1 ? fail(st, "view %d: %s", i, rc_last_error()) : st;
    }
    if (opt->adapt_factor > 1)
        return fail(RC_E_UNSUPPORTED, "rc_render_backward: adaptive sampling is not differentiated");
    for (int i = 0; i < n_views; ++i)
        if (!aux[i] || !grad_rgba[i])
            return fail(RC_E_INVALID, "rc_render_backward: aux/grad pointers must not be NULL");
    if (!grad_volume_dev || !grad_tf_dev)
        return fail(RC_E_INVALID, "rc_render_backward: aux/grad pointers must not be NULL");
    RenderParams P;
    fill_render_params(P, v, &cams[0], tf_rgba_dev, tf_len, sh, opt);
    BackwardParams Bp;
    Bp.dvol = grad_volume_dev;
    Bp.dtf = grad_tf_dev;
    Bp.M4 = tf_len * 4;
    Bp.dbg = P.dbg;
    // LDS a block may take on this device (160 KiB on gfx950): the table
    // gradient shared by the block's waves (tables up to kBwdBoxTfEntries),
    // the table itself for small tables, and per wave its dV and voxel boxes
    int dev = 0, lds_max = 0;
    RC_HIP(hipGetDevice(&dev));
    RC_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t budget = (size_t)std::min(lds_max, kBwdLdsBytes);
    const int waves = kBwdBoxWaves;
    Bp.lds_tf = tf_len <= kBwdBoxTfEntries && (size_t)tf_len * 16 + 4096 <= budget;
    Bp.lds_table = tf_len <= kBwdLdsTable;
    size_t tf_bytes = ((Bp.lds_tf ? 1 : 0) + (Bp.lds_table ? 1 : 0)) * (size_t)tf_len * 16;
    if (tf_bytes + 4096 > budget) {     // no room for the table copy: read it from memory
        Bp.lds_table = 0;
        tf_bytes = (Bp.lds_tf ? 1 : 0) * (size_t)tf_len * 16;
    }
    Bp.box_bytes = (int)(std::min<size_t>(kBwdBoxBytes, (budget - tf_bytes) / kBwdBoxWaves) &
                         ~(size_t)15);
    Bp.chunk_len = kBwdChunk;
    const size_t lds = tf_bytes + (size_t)Bp.box_bytes * kBwdBoxWaves;
    // the tile counter: a stream-ordered allocation, zeroed by a small kernel
    // before each launch
    Bp.next_unit = nullptr;
    RC_HIP(hipMallocAsync((void**)&Bp.next_unit, 256, s));
    rc_status st = RC_OK;
    for (int first = 0; st == RC_OK && first < n_views; first += kMaxViews) {
        ViewSet S;
        S.n = n_views - first < kMaxViews ? n_views - first : kMaxViews;
        int off = 0;
        for (int j = 0; j < S.n; ++j) {
            ViewParams& V = S.v[j];
            fill_view(V, &cams[first + j]);
            V.aux = (rc_aux*)aux[first + j];
            V.grad = (const float4*)grad_rgba[first + j];
            S.block_off[j] = off;
            off += ((V.W + kBwdTile - 1) / kBwdTile) * ((V.H + kBwdTile - 1) / kBwdTile);
        }
        S.block_off[S.n] = off;
        dim3 grid((unsigned)((off + waves - 1) / waves)), block(kBwdTile * kBwdTile * waves);
        int op = opt->gradient_op;
        if (v->dtype == RC_U8) st = launch_bwd_t<uint8_t>(P, S, Bp, op, grid, block, lds, s);
        else if (v->dtype == RC_U16) st = launch_bwd_t<uint16_t>(P, S, Bp, op, grid, block, lds, s);
        else st = launch_bwd_t<float>(P, S, Bp, op, grid, block, lds, s);
        if (st == RC_OK) {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) st = hip_fail(e, "reverse-pass launch");
        }
    }
    if (Bp.next_unit) {
        hipError_t e = hipFreeAsync(Bp.next_unit, s);
        if (st == RC_OK && e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    }
    return st;
}

extern "C" rc_status rc_render_backward(const rc_volume* v, const rc_camera* cam,
                                        const float* tf_rgba_dev, int tf_len, const rc_shading* sh,
                                        const rc_options* opt, const rc_aux* aux_dev,
                                        const float* grad_rgba_dev, float* grad_volume_dev,
                                        float* grad_tf_dev, void* stream) {
    if (!cam) return check_render_args(v, cam, tf_rgba_dev, tf_len, sh, opt);
    const rc_aux* aux[1] = {aux_dev};
    const float* grad[1] = {grad_rgba_dev};
    return backward_views(v, cam, 1, tf_rgba_dev, tf_len, sh, opt, aux, grad, grad_volume_dev,
                          grad_tf_dev, (hipStream_t)stream);
}

extern "C" rc_status rc_render_backward_views(const rc_volume* v, const rc_camera* cams,
                                              int n_views, const float* tf_rgba_dev, int tf_len,
                                              const rc_shading* sh, const rc_options* opt,
                                              const rc_aux* const* aux,
                                              const float* const* grad_rgba,
                                              float* grad_volume_dev, float* grad_tf_dev,
                                              void* stream) {
    if (!cams || !aux || !grad_rgba || n_views < 1)
        return fail(RC_E_INVALID, "rc_render_backward_views: need n_views >= 1 and non-NULL arrays");
    return backward_views(v, cams, n_views, tf_rgba_dev, tf_len, sh, opt, aux, grad_rgba,
                          grad_volume_dev, grad_tf_dev, (hipStream_t)stream);
}
