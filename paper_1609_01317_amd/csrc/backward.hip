// Reverse mode of the unshaded render: one ray per thread marches back to
// front from its last composited sample and accumulates dL/dvolume and
// dL/dtable.  No per-sample state is stored by the forward pass; the
// transmittance in front of each sample is recovered from the final
// transmittance written to rc_aux.
#include <cmath>

#include "march.h"

namespace rc {

struct BackwardParams {
    float* dvol;            // [nz][ny][nx]
    float* dtf;             // [M][4]
    int lds_tf;             // 1: accumulate the table gradient in LDS first
};

constexpr int kBwdTile = 16;              // 16x16 pixels, 4 waves per workgroup
constexpr int kBwdLdsEntries = 2048;      // table sizes up to this are privatised in LDS
constexpr float kTinyT = 1e-30f;

__device__ __forceinline__ void add_dtf(const BackwardParams& B, float* lds, int i, int ch, float v) {
    if (v == 0.0f) return;
    if (B.lds_tf) atomicAdd(&lds[i * 4 + ch], v);
    else unsafeAtomicAdd(&B.dtf[i * 4 + ch], v);
}

// Value, table entry pair and colour of lattice sample k (shading NONE).
struct BwdSample {
    Cell C;
    float vn;                   // normalised value before clamping
    int i, i1;
    float t;                    // position between entries i and i1
    float4 e0, e1;              // table entries
    float a;
    float c[3];
};

template <typename VT>
__device__ __forceinline__ void bwd_sample(const RenderParams& P, const Ray& R, long long k,
                                           BwdSample& S) {
    double pv[3];
    lattice_point(P, R, k, S.C, pv);
    const GlobalSrc<VT> src{(const VT*)P.vox, P.nx, P.ny, P.nz, P.sy, P.sz};
    int ox[4], oy[4], oz[4];
    src.offsets(S.C, ox, oy, oz);
    float v = sample_value<VT>(src.base, ox, oy, oz, S.C);
    S.vn = (v - P.vmin) * P.inv_range;
    float uu = fminf(fmaxf(S.vn, 0.0f), 1.0f) * P.Mm1;
    S.i = min((int)uu, P.M - 1);
    S.i1 = min(S.i + 1, P.M - 1);
    S.t = uu - (float)S.i;
    S.e0 = P.tf[S.i];
    S.e1 = P.tf[S.i1];
    S.a = lerpf(S.e0.w, S.e1.w, S.t);
    S.c[0] = lerpf(S.e0.x, S.e1.x, S.t);
    S.c[1] = lerpf(S.e0.y, S.e1.y, S.t);
    S.c[2] = lerpf(S.e0.z, S.e1.z, S.t);
}

// Chain rule for one sample (see the forward: C = sum T_k a_k c_k,
// A = 1 - prod(1 - a_k)):
//   dL/dc_k = g_rgb T_k a_k
//   dL/da_k = T_k [ g_rgb . (c_k - Bk1) + g_A Pk1 ]
// with Bk1 the colour composited behind k (eq. 6 run back to front) and
// Pk1 the transmittance of the samples behind k.  Then through the table
// interpolation to u, the clamp to the value, and the trilinear weights.
template <typename VT>
__device__ __forceinline__ void bwd_accumulate(const RenderParams& P, const BackwardParams& Bp,
                                               float* lds, const BwdSample& S, float Tk,
                                               const float4& g, const float Bk1[3], float Pk1) {
    float ta = Tk * S.a;
    float dc[3] = {g.x * ta, g.y * ta, g.z * ta};
    float da = Tk * (g.x * (S.c[0] - Bk1[0]) + g.y * (S.c[1] - Bk1[1]) +
                     g.z * (S.c[2] - Bk1[2]) + g.w * Pk1);
    float w0 = 1.0f - S.t, w1 = S.t;
    const float d4[4] = {dc[0], dc[1], dc[2], da};
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        add_dtf(Bp, lds, S.i, ch, w0 * d4[ch]);
        add_dtf(Bp, lds, S.i1, ch, w1 * d4[ch]);
    }
    if (!(S.vn > 0.0f && S.vn < 1.0f)) return;      // clamped: no dependence on the value
    float du = dc[0] * (S.e1.x - S.e0.x) + dc[1] * (S.e1.y - S.e0.y) +
               dc[2] * (S.e1.z - S.e0.z) + da * (S.e1.w - S.e0.w);
    float dv = du * P.Mm1 * P.inv_range;
    if (dv == 0.0f) return;
    const float fx = S.C.fr[0], fy = S.C.fr[1], fz = S.C.fr[2];
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                float w = (cx ? fx : 1.0f - fx) * (cy ? fy : 1.0f - fy) * (cz ? fz : 1.0f - fz);
                int x = clampi(S.C.c[0] + cx, 0, P.nx - 1);
                int y = clampi(S.C.c[1] + cy, 0, P.ny - 1);
                int z = clampi(S.C.c[2] + cz, 0, P.nz - 1);
                unsafeAtomicAdd(&Bp.dvol[((long long)z * P.ny + y) * P.nx + x], w * dv);
            }
}

// One workgroup = one 16x16 pixel tile of one view; views own consecutive
// runs of workgroups (ViewSet::block_off).
template <typename VT>
__global__ __launch_bounds__(256) void raycast_bwd(RenderParams P, ViewSet S, BackwardParams Bp) {
    extern __shared__ float lds[];
    if (Bp.lds_tf) {
        for (int i = threadIdx.x; i < P.M * 4; i += blockDim.x) lds[i] = 0.0f;
        __syncthreads();
    }
    int b = blockIdx.x, v = 0;
    while (v + 1 < S.n && S.block_off[v + 1] <= b) ++v;
    const ViewParams& V = S.v[v];
    b -= S.block_off[v];
    int tiles_x = (V.W + kBwdTile - 1) / kBwdTile;
    int tx = b % tiles_x, ty = b / tiles_x;
    int px = tx * kBwdTile + (threadIdx.x % kBwdTile);
    int py = ty * kBwdTile + (threadIdx.x / kBwdTile);
    if (px < V.W && py < V.H) {
        Ray R;
        setup_ray(P, V, px, py, R);
        long long pix = (long long)py * V.W + px;
        rc_aux ax = V.aux[pix];
        float4 g = V.grad[pix];
        long long last = ax.k_last;
        if (R.K >= 0 && last >= 0 && last <= R.K) {
            // Anchor: the last index a whose front transmittance T_a is at
            // least kTinyT.  Normally a = last + 1 with T_a = t_final; if the
            // ray went (nearly) opaque, a forward pass finds a instead.
            long long anchor = last + 1;
            float Ta = ax.t_final;
            if (!(Ta >= kTinyT)) {
                float T = 1.0f;
                anchor = 0;
                for (long long k = 0; k <= last; ++k) {
                    BwdSample S;
                    bwd_sample<VT>(P, R, k, S);
                    float Tn = T * (1.0f - S.a);
                    if (!(Tn >= kTinyT)) break;
                    T = Tn;
                    anchor = k + 1;
                }
                Ta = T;
            }
            float Bk1[3] = {0.f, 0.f, 0.f};
            float Pk1 = 1.0f;       // prod over samples behind k of (1 - a)
            float Q = 1.0f;         // prod over samples k .. anchor-1 of (1 - a)
            for (long long k = last; k >= 0; --k) {
                BwdSample S;
                bwd_sample<VT>(P, R, k, S);
                float om = 1.0f - S.a;
                if (k < anchor) {
                    Q *= om;
                    float Tk = Q > 0.0f ? Ta / Q : 0.0f;
                    bwd_accumulate<VT>(P, Bp, lds, S, Tk, g, Bk1, Pk1);
                }
                Bk1[0] = fmaf(S.a, S.c[0], om * Bk1[0]);
                Bk1[1] = fmaf(S.a, S.c[1], om * Bk1[1]);
                Bk1[2] = fmaf(S.a, S.c[2], om * Bk1[2]);
                Pk1 *= om;
            }
        }
    }
    if (Bp.lds_tf) {
        __syncthreads();
        for (int i = threadIdx.x; i < P.M * 4; i += blockDim.x) {
            float v = lds[i];
            if (v != 0.0f) unsafeAtomicAdd(&Bp.dtf[i], v);
        }
    }
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
    if (sh->model != RC_SHADE_NONE)
        return fail(RC_E_UNSUPPORTED, "rc_render_backward: only shading NONE is differentiated");
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
    Bp.lds_tf = tf_len <= kBwdLdsEntries;
    size_t lds = Bp.lds_tf ? (size_t)tf_len * 4 * sizeof(float) : 0;
    for (int first = 0; first < n_views; first += kMaxViews) {
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
        dim3 grid((unsigned)off), block(kBwdTile * kBwdTile);
        if (v->dtype == RC_U8)
            hipLaunchKernelGGL(raycast_bwd<uint8_t>, grid, block, lds, s, P, S, Bp);
        else if (v->dtype == RC_U16)
            hipLaunchKernelGGL(raycast_bwd<uint16_t>, grid, block, lds, s, P, S, Bp);
        else
            hipLaunchKernelGGL(raycast_bwd<float>, grid, block, lds, s, P, S, Bp);
        RC_HIP(hipGetLastError());
    }
    return RC_OK;
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
