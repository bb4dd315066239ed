/*
 * oracle.c -- plain FP64 CPU volume raycaster (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares nothing with the GPU library.
 * Each function follows one passage of "Volume Raycasting mit OpenCL"
 * (Kopal); where the paper is silent the reading taken is stated inline.
 * No blocking, no skipping, no reordering: one ray per pixel, one sample
 * after the other, exactly in the pipeline order of Section 3.10.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
/* x / |x|; a zero vector stays zero */
static void normalize3(const double a[3], double out[3]) {
    double n = sqrt(dot3(a, a));
    double s = n > 0.0 ? 1.0 / n : 0.0;
    out[0] = a[0] * s; out[1] = a[1] * s; out[2] = a[2] * s;
}

/* ------------------------------------------------------------------ */
/* Section 2.1, eq. (1): V maps an integer triple to a value.  Indices   */
/* outside the grid take the nearest edge voxel (reading: clamp to edge, */
/* the paper does not say what lies outside the data).                   */
/* ------------------------------------------------------------------ */
static long clampl(long i, long n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

static double voxel(const orc_volume* v, long i, long j, long k) {
    i = clampl(i, v->nx);
    j = clampl(j, v->ny);
    k = clampl(k, v->nz);
    return v->data[(k * (long)v->ny + j) * (long)v->nx + i];
}

/* Section 3.4, eq. (2): the line through f(x0) and f(x1), x1 - x0 = 1,
 * evaluated at x0 + t. */
static double lerp(double f0, double f1, double t) { return f0 + (f1 - f0) * t; }

/* Section 3.4: trilinear interpolation of the 8 surrounding voxels as 7
 * linear interpolations -- four along x, two along y, one along z.  The
 * paper's pairing figure is missing; the axis order is x, y, z (every
 * order agrees in exact arithmetic). */
double orc_sample(const orc_volume* v, const double p[3]) {
    double fx0 = floor(p[0]), fy0 = floor(p[1]), fz0 = floor(p[2]);
    long i = (long)fx0, j = (long)fy0, k = (long)fz0;
    double tx = p[0] - fx0, ty = p[1] - fy0, tz = p[2] - fz0;
    double I1 = lerp(voxel(v, i, j, k), voxel(v, i + 1, j, k), tx);
    double I2 = lerp(voxel(v, i, j + 1, k), voxel(v, i + 1, j + 1, k), tx);
    double I3 = lerp(voxel(v, i, j, k + 1), voxel(v, i + 1, j, k + 1), tx);
    double I4 = lerp(voxel(v, i, j + 1, k + 1), voxel(v, i + 1, j + 1, k + 1), tx);
    double I5 = lerp(I1, I2, ty);
    double I6 = lerp(I3, I4, ty);
    return lerp(I5, I6, tz);
}

/* Section 3.3: the simplest sampling rounds the coordinates to whole
 * voxels.  Reading: round half up, floor(p + 1/2), then the edge clamp. */
double orc_sample_nearest(const orc_volume* v, const double p[3]) {
    return voxel(v, (long)floor(p[0] + 0.5), (long)floor(p[1] + 0.5), (long)floor(p[2] + 0.5));
}

/* ------------------------------------------------------------------ */
/* Section 3.5: gradient operators.                                    */
/*                                                                     */
/* The mask is laid one voxel before, on and after the sample point    */
/* along each axis; values between voxels are interpolated (Section    */
/* 2.1), so every tap is a trilinear sample at p + offset.             */
/*  - central difference, eq. (3): d_a = V(p+e_a) - V(p-e_a); the       */
/*    equation is taken over the prose, which words the difference the  */
/*    other way round.                                                 */
/*  - Sobel3D, eq. (4): the x+1 slice carries +w, the x-1 slice -w,     */
/*    w = [[1,3,1],[3,6,3],[1,3,1]] exactly as printed.  The y and z    */
/*    masks in the equation are garbled; they are read as the same      */
/*    operator turned onto the y and z axes ("+1 side minus -1 side").  */
/*  - Zucker-Hummel: named, never printed.  Read from the operator's     */
/*    own definition (the x/|r| basis on the 3x3x3 neighbourhood):       */
/*    w(b,c) = 1/sqrt(1+b^2+c^2); 18 taps per component, 54 in all as   */
/*    the paper counts.                                                 */
/* Scale (the paper normalises, Section 3.5, so the scale is free):    */
/* raw sum / gain / spacing_a / (vmax - vmin), where gain is the raw    */
/* response to a unit-slope field, so the result estimates the          */
/* gradient of the normalised value per world unit.                     */
/* ------------------------------------------------------------------ */
static double mask_weight(int op, int b, int c) {
    if (op == ORC_OP_SOBEL3D) {
        static const double w[3][3] = {{1, 3, 1}, {3, 6, 3}, {1, 3, 1}};
        return w[b + 1][c + 1];
    }
    return 1.0 / sqrt(1.0 + (double)(b * b) + (double)(c * c));   /* Zucker-Hummel */
}

static double op_gain(int op) {
    if (op == ORC_OP_CENTRAL) return 2.0;
    double s = 0.0;
    for (int b = -1; b <= 1; ++b)
        for (int c = -1; c <= 1; ++c) s += mask_weight(op, b, c);
    return 2.0 * s;
}

void orc_gradient(const orc_volume* v, int op, const double p[3], double g[3], double raw[3]) {
    for (int a = 0; a < 3; ++a) {
        int beta = (a + 1) % 3, gamma = (a + 2) % 3;
        double sum = 0.0;
        if (op == ORC_OP_CENTRAL) {
            double q1[3] = {p[0], p[1], p[2]}, q0[3] = {p[0], p[1], p[2]};
            q1[a] += 1.0;
            q0[a] -= 1.0;
            sum = orc_sample(v, q1) - orc_sample(v, q0);
        } else {
            for (int b = -1; b <= 1; ++b)
                for (int c = -1; c <= 1; ++c) {
                    double q1[3] = {p[0], p[1], p[2]}, q0[3];
                    q1[beta] += b;
                    q1[gamma] += c;
                    memcpy(q0, q1, sizeof q0);
                    q1[a] += 1.0;
                    q0[a] -= 1.0;
                    sum += mask_weight(op, b, c) * (orc_sample(v, q1) - orc_sample(v, q0));
                }
        }
        if (raw) raw[a] = sum;
        g[a] = sum / op_gain(op) / v->spacing[a] / (v->vmax - v->vmin);
    }
}

/* ------------------------------------------------------------------ */
/* Section 3.7: the value -> colour lookup table.  Reading: the table    */
/* is indexed by the normalised value u = clamp((v-vmin)/(vmax-vmin))   */
/* * (M-1) and interpolated linearly (eq. 2) between neighbouring       */
/* entries; the upper neighbour is clamped to the last entry.           */
/* ------------------------------------------------------------------ */
void orc_tf(const double* tf, int M, double u, double rgba[4]) {
    double fi = floor(u);
    long i = (long)fi;
    if (i < 0) i = 0;
    if (i > M - 1) i = M - 1;
    long i1 = i + 1 < M ? i + 1 : M - 1;
    double t = u - (double)i;
    for (int ch = 0; ch < 4; ++ch) rgba[ch] = lerp(tf[i * 4 + ch], tf[i1 * 4 + ch], t);
}

static double value_to_u(const orc_volume* v, double val, int M, int* interior) {
    double vn = (val - v->vmin) / (v->vmax - v->vmin);
    if (interior) *interior = (vn > 0.0 && vn < 1.0);
    if (vn < 0.0) vn = 0.0;
    if (vn > 1.0) vn = 1.0;
    return vn * (double)(M - 1);
}

/* ------------------------------------------------------------------ */
/* Camera (Section 3.3: a ray from the eye through every pixel; the      */
/* paper gives no camera model).  Reading: right-handed look-at frame    */
/* f = normalize(target-eye), r = normalize(f x up), u = r x f; pixel    */
/* centres at NDC x = 2(px+1/2)/W - 1, y = 1 - 2(py+1/2)/H, row 0 at the */
/* top.  Perspective: o = eye, d = normalize(f + x tan(fov/2) W/H r +    */
/* y tan(fov/2) u).  Orthographic: d = f, o = eye + (x W/H r + y u) h/2. */
/* ------------------------------------------------------------------ */
void orc_camera_ray(const orc_camera* cam, int px, int py, double o[3], double d[3]) {
    double f[3], r[3], u[3], tmp[3];
    for (int a = 0; a < 3; ++a) tmp[a] = cam->target[a] - cam->eye[a];
    normalize3(tmp, f);
    cross3(f, cam->up, tmp);
    normalize3(tmp, r);
    cross3(r, f, u);
    double aspect = (double)cam->width / (double)cam->height;
    double x = 2.0 * ((double)px + 0.5) / (double)cam->width - 1.0;
    double y = 1.0 - 2.0 * ((double)py + 0.5) / (double)cam->height;
    if (cam->projection == ORC_PERSPECTIVE) {
        double th = tan(cam->fov_y_deg * 0.5 * M_PI / 180.0);
        for (int a = 0; a < 3; ++a) tmp[a] = f[a] + x * th * aspect * r[a] + y * th * u[a];
        normalize3(tmp, d);
        for (int a = 0; a < 3; ++a) o[a] = cam->eye[a];
    } else {
        double hh = cam->ortho_height * 0.5;
        for (int a = 0; a < 3; ++a) {
            d[a] = f[a];
            o[a] = cam->eye[a] + (x * aspect * r[a] + y * u[a]) * hh;
        }
    }
}

/* Section 3.3 / 3.6: entry and exit of the ray through the bounding box
 * (slab method).  A ray parallel to a slab misses if its origin is outside
 * it; only t >= 0 (in front of the eye) counts. */
int orc_ray_box(const double o[3], const double d[3], const double lo[3], const double hi[3],
                double* t_in, double* t_out) {
    double tmin = 0.0, tmax = INFINITY;
    *t_in = INFINITY;
    *t_out = -INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            continue;
        }
        double t0 = (lo[a] - o[a]) / d[a], t1 = (hi[a] - o[a]) / d[a];
        if (t0 > t1) { double s = t0; t0 = t1; t1 = s; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
    }
    *t_in = tmin;
    *t_out = tmax;
    return tmin <= tmax;
}

/* ------------------------------------------------------------------ */
/* Section 3.8: shading.                                               */
/*  NONE          c = rgb.                                              */
/*  PAPER_LAMBERT Listing 3 literally: a white point light, the cosine   */
/*                between normalize(light - p) and the normalised        */
/*                gradient, unclamped; c = rgb * illum.                  */
/*  BLINN_PHONG   c = rgb (ka + kd max(0, N.L)) + ks max(0, N.H)^s, with  */
/*                N = -G/max(|G|,eps) the outward normal (G points to     */
/*                higher values), L towards the light, V = -d,           */
/*                H = normalize(L+V).  Constants are the caller's.       */
/* The soft floor eps keeps N defined where G vanishes inside material   */
/* (Section 3.6 notes G = 0 there).  Alpha is never shaded: the light's  */
/* colour has alpha 0 in Listing 3.                                      */
/* ------------------------------------------------------------------ */
void orc_shade(const orc_shading* sh, const double rgb[3], const double g[3],
               const double p_world[3], const double d[3], double c[3]) {
    if (sh->model == ORC_SHADE_NONE) {
        c[0] = rgb[0]; c[1] = rgb[1]; c[2] = rgb[2];
        return;
    }
    double gn = sqrt(dot3(g, g));
    double den = gn > sh->grad_eps ? gn : sh->grad_eps;
    double ghat[3] = {g[0] / den, g[1] / den, g[2] / den};
    double L[3], tmp[3];
    if (sh->light_is_point) {
        for (int a = 0; a < 3; ++a) tmp[a] = sh->light[a] - p_world[a];
        normalize3(tmp, L);
    } else {
        normalize3(sh->light, L);
    }
    if (sh->model == ORC_SHADE_PAPER_LAMBERT) {
        double illum = dot3(L, ghat);
        for (int ch = 0; ch < 3; ++ch) c[ch] = rgb[ch] * illum;
        return;
    }
    double N[3] = {-ghat[0], -ghat[1], -ghat[2]};
    double H[3];
    for (int a = 0; a < 3; ++a) tmp[a] = L[a] - d[a];
    normalize3(tmp, H);
    double nl = dot3(N, L), nh = dot3(N, H);
    double diff = nl > 0.0 ? nl : 0.0;
    double spec = pow(nh > 0.0 ? nh : 0.0, sh->shininess);
    for (int ch = 0; ch < 3; ++ch) c[ch] = rgb[ch] * (sh->ka + sh->kd * diff) + sh->ks * spec;
}

/* ------------------------------------------------------------------ */
/* ray set-up shared by the forward and reverse passes                 */
/* ------------------------------------------------------------------ */
typedef struct {
    double o[3], d[3];
    double t_in, t_out;
    int hit;
    long K, K_alt;   /* primary / alternative index of the last lattice sample (-1 = miss) */
    int tie;
} ray_setup;

/* Sampling box = volume box [0,(n-1)s] (voxel centres at i*s, reading:
 * the box encloses the data, Section 3.3) intersected with the clip box
 * (Section 3.6).  Lattice (Section 3.3: regular distances between entry
 * and exit): t_k = t_in + k*step, k = 0..K, K = floor((t_out-t_in)/step).
 * When the ratio is within ORC_TIE_EPS of an integer R, both R-1 and R
 * are admissible last indices (-1 = miss). */
static void setup_ray(const orc_volume* v, const orc_camera* cam, const orc_options* opt,
                      int px, int py, ray_setup* rs) {
    double lo[3], hi[3];
    const double ext[3] = {(v->nx - 1) * v->spacing[0], (v->ny - 1) * v->spacing[1],
                           (v->nz - 1) * v->spacing[2]};
    for (int a = 0; a < 3; ++a) {
        lo[a] = opt->clip_lo[a] > 0.0 ? opt->clip_lo[a] : 0.0;
        hi[a] = opt->clip_hi[a] < ext[a] ? opt->clip_hi[a] : ext[a];
    }
    orc_camera_ray(cam, px, py, rs->o, rs->d);
    rs->tie = 0;
    rs->K = rs->K_alt = -1;
    rs->hit = 0;
    for (int a = 0; a < 3; ++a)
        if (lo[a] > hi[a]) return;
    double t_in, t_out;
    int hit = orc_ray_box(rs->o, rs->d, lo, hi, &t_in, &t_out);
    rs->t_in = t_in;
    rs->t_out = t_out;
    if (!isfinite(t_in) || !isfinite(t_out)) return;   /* parallel-slab miss */
    double r = (t_out - t_in) / opt->step;
    double R = nearbyint(r);
    long K = hit ? (long)floor(r) : -1;
    if (K < -1) K = -1;
    rs->K = K;
    rs->hit = K >= 0;
    if (fabs(r - R) < ORC_TIE_EPS && R >= 0.0) {
        rs->tie = 1;
        rs->K_alt = (K == (long)R) ? (long)R - 1 : (long)R;
    }
}

/* one lattice sample: value, TF colour, gradient and shaded colour */
typedef struct {
    double pw[3];       /* world position */
    double pv[3];       /* voxel-space position */
    double val, u;
    int interior;       /* 0 < normalised value < 1 */
    double rgba[4];     /* TF output (alpha after opacity correction) */
    double alpha_tf;    /* TF alpha before opacity correction */
    double c[3];        /* shaded colour */
} sample_state;

static void eval_sample(const orc_volume* v, const double* tf, int M, const orc_shading* sh,
                        const orc_options* opt, const ray_setup* rs, long k, sample_state* s) {
    double t = rs->t_in + (double)k * opt->step;
    double* pw = s->pw;
    for (int a = 0; a < 3; ++a) {
        pw[a] = rs->o[a] + t * rs->d[a];
        s->pv[a] = pw[a] / v->spacing[a];
    }
    /* nearest sampling: the value and the gradient taps are taken at the
     * rounded point, so the operator's stencil sits on one voxel */
    double pr[3];
    for (int a = 0; a < 3; ++a) pr[a] = opt->nearest ? floor(s->pv[a] + 0.5) : s->pv[a];
    s->val = opt->nearest ? orc_sample_nearest(v, s->pv) : orc_sample(v, s->pv);
    s->u = value_to_u(v, s->val, M, &s->interior);
    orc_tf(tf, M, s->u, s->rgba);
    s->alpha_tf = s->rgba[3];
    if (opt->ref_step > 0.0)
        s->rgba[3] = 1.0 - pow(1.0 - s->rgba[3], opt->step / opt->ref_step);
    if (sh->model == ORC_SHADE_NONE || s->rgba[3] == 0.0) {
        /* no light needed: empty samples get no colour (Section 3.5) */
        s->c[0] = s->rgba[0]; s->c[1] = s->rgba[1]; s->c[2] = s->rgba[2];
        return;
    }
    double g[3];
    orc_gradient(v, opt->gradient_op, pr, g, NULL);
    orc_shade(sh, s->rgba, g, pw, rs->d, s->c);
}

/* Opacity correction (not in the paper, which is silent on the step
 * dependence of a): with ref_step > 0 the table opacity is taken as
 * defined for a sample distance ref_step and converted to the step in use,
 * a = 1 - (1 - a_tf)^(step/ref_step), so that a slab of constant a_tf has
 * the same opacity at every step.  Off (ref_step = 0) by default. */

/* Section 3.9, eq. (6) composites back to front: C_out = C_in (1 - a) + C a.
 * Evaluated front to back with the transmittance T = prod (1 - a_j) of the
 * samples in front, which gives the same sum: C = sum_k T_k a_k c_k,
 * opacity 1 - T.  Early termination (Section 3.9: the recursion runs until
 * an opaque sample is met): stop after the first sample with 1-T >= tau. */
static void march(const orc_volume* v, const double* tf, int M, const orc_shading* sh,
                  const orc_options* opt, const ray_setup* rs, long K, double out[4],
                  int* k_last, double* t_final, int* ert_near) {
    double C[3] = {0, 0, 0}, T = 1.0;
    long last = -1;
    double tau = opt->ert_threshold;
    for (long k = 0; k <= K; ++k) {
        sample_state s;
        eval_sample(v, tf, M, sh, opt, rs, k, &s);
        double a = s.rgba[3];
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * a * s.c[ch];
        T *= (1.0 - a);
        last = k;
        if (tau > 0.0) {
            if (fabs((1.0 - T) - tau) < ORC_ERT_EPS) *ert_near = 1;
            if (1.0 - T >= tau) break;
        }
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    *k_last = (int)last;
    *t_final = T;
}

/* ------------------------------------------------------------------ */
/* Adaptive sampling (Section 5.2: detail-poor regions are sampled at a */
/* lower rate, detail-rich ones at the full rate).  Reading: the regions */
/* are the 8^3 bricks of the empty-space grid; a brick is detail-poor    */
/* when the range of the voxels its samples can touch (the brick plus    */
/* its one-voxel high apron) is at most adapt_range.  A sample in a poor */
/* brick advances the ray by adapt_factor steps, any other by one; each  */
/* sample's opacity is corrected to the distance it stands for           */
/* (a = 1 - (1 - a_tf)^(d / ref), ref = ref_step or the base step), so a */
/* homogeneous region keeps its opacity.  Samples are taken while        */
/* t <= t_out; t accumulates in FP64.                                    */
/* ------------------------------------------------------------------ */
static unsigned char* poor_bricks(const orc_volume* v, double range) {
    long nbx = (v->nx + 7) / 8, nby = (v->ny + 7) / 8, nbz = (v->nz + 7) / 8;
    unsigned char* poor = (unsigned char*)malloc((size_t)(nbx * nby * nbz));
    if (!poor) return NULL;
    for (long bz = 0; bz < nbz; ++bz)
        for (long by = 0; by < nby; ++by)
            for (long bx = 0; bx < nbx; ++bx) {
                double lo = INFINITY, hi = -INFINITY;
                for (long z = 8 * bz; z <= 8 * bz + 8; ++z)
                    for (long y = 8 * by; y <= 8 * by + 8; ++y)
                        for (long x = 8 * bx; x <= 8 * bx + 8; ++x) {
                            double val = voxel(v, x, y, z);
                            if (val < lo) lo = val;
                            if (val > hi) hi = val;
                        }
                poor[(bz * nby + by) * nbx + bx] = (hi - lo) <= range;
            }
    return poor;
}

static void march_adaptive(const orc_volume* v, const double* tf, int M, const orc_shading* sh,
                           const orc_options* opt, const ray_setup* rs, const unsigned char* poor,
                           double t_end, double out[4], int* k_last, double* t_final,
                           int* ert_near, int* adapt_near, double* t_tie) {
    const long nbx = (v->nx + 7) / 8, nby = (v->ny + 7) / 8;
    const long n[3] = {v->nx, v->ny, v->nz};
    const double ref = opt->ref_step > 0.0 ? opt->ref_step : opt->step;
    double C[3] = {0, 0, 0}, T = 1.0, t = rs->t_in;
    long j = 0, last = -1;
    *t_tie = NAN;
    while (t <= t_end) {
        if (fabs(t - rs->t_out) < ORC_TIE_EPS * opt->step) *t_tie = t;
        double pv[3], pw[3];
        long b[3];
        for (int a = 0; a < 3; ++a) {
            pw[a] = rs->o[a] + t * rs->d[a];
            pv[a] = pw[a] / v->spacing[a];
            long c = (long)floor(pv[a]);
            b[a] = clampl(c, n[a]) / 8;
            double r = pv[a] - 8.0 * floor(pv[a] / 8.0 + 0.5);   /* distance to a brick plane */
            if (fabs(r) < ORC_ADAPT_EPS && pv[a] > 0.5 && pv[a] < (double)n[a] - 1.5) *adapt_near = 1;
        }
        int is_poor = poor[(b[2] * nby + b[1]) * nbx + b[0]];
        double step = is_poor ? (double)opt->adapt_factor * opt->step : opt->step;
        /* one sample, as in eval_sample, with the opacity corrected to `step` */
        double pr[3];
        for (int a = 0; a < 3; ++a) pr[a] = opt->nearest ? floor(pv[a] + 0.5) : pv[a];
        double val = opt->nearest ? orc_sample_nearest(v, pv) : orc_sample(v, pv);
        int interior;
        double u = value_to_u(v, val, M, &interior), rgba[4], c[3];
        orc_tf(tf, M, u, rgba);
        double a = rgba[3];
        if (a != 0.0 && step != ref) a = 1.0 - pow(1.0 - a, step / ref);
        if (sh->model == ORC_SHADE_NONE || a == 0.0) {
            c[0] = rgba[0]; c[1] = rgba[1]; c[2] = rgba[2];
        } else {
            double g[3];
            orc_gradient(v, opt->gradient_op, pr, g, NULL);
            orc_shade(sh, rgba, g, pw, rs->d, c);
        }
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * a * c[ch];
        T *= (1.0 - a);
        last = j;
        if (opt->ert_threshold > 0.0) {
            if (fabs((1.0 - T) - opt->ert_threshold) < ORC_ERT_EPS) *ert_near = 1;
            if (1.0 - T >= opt->ert_threshold) break;
        }
        t += step;
        ++j;
    }
    if (fabs(t - rs->t_out) < ORC_TIE_EPS * opt->step && last + 1 == j) *t_tie = t;
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    *k_last = (int)last;
    *t_final = T;
}

static int check_args(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
                      const orc_options* opt) {
    if (!v || !v->data || !cam || !tf || !opt) return -1;
    if (v->nx < 1 || v->ny < 1 || v->nz < 1 || M < 2) return -1;
    if (!(opt->step > 0.0) || !(v->vmax > v->vmin)) return -1;
    if (!(opt->ref_step >= 0.0) || isinf(opt->ref_step)) return -1;
    if (opt->adapt_factor < 0 || opt->adapt_factor > 64 || isnan(opt->adapt_range)) return -1;
    if (cam->width < 1 || cam->height < 1) return -1;
    return 0;
}

int orc_render(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
               const orc_shading* sh, const orc_options* opt, const long* pix, long n,
               double* rgba, double* rgba_alt, int* flags, int* k_last, double* t_final,
               int threads) {
    if (check_args(v, cam, tf, M, opt) || !sh || !rgba) return -1;
    long total = (long)cam->width * cam->height;
    if (!pix) n = total;
    const int adaptive = opt->adapt_factor > 1;
    unsigned char* poor = adaptive ? poor_bricks(v, opt->adapt_range) : NULL;
    if (adaptive && !poor) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    #pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < n; ++q) {
        long id = pix ? pix[q] : q;
        int px = (int)(id % cam->width), py = (int)(id / cam->width);
        ray_setup rs;
        setup_ray(v, cam, opt, px, py, &rs);
        double out[4] = {0, 0, 0, 0}, alt[4] = {0, 0, 0, 0};
        int kl = -1, kl_alt = -1, near = 0, near_alt = 0, anear = 0, tie = rs.tie;
        double tf_ = 1.0, tf_alt = 1.0;
        if (adaptive) {
            /* the adaptive march has its own end rule: a sample within
             * ORC_TIE_EPS steps of t_out may or may not be taken */
            double t_tie = NAN, t_tie2;
            if (rs.hit) {
                march_adaptive(v, tf, M, sh, opt, &rs, poor, rs.t_out, out, &kl, &tf_, &near,
                               &anear, &t_tie);
                memcpy(alt, out, sizeof out);
            }
            tie = !isnan(t_tie);
            if (tie) {
                double end = t_tie <= rs.t_out ? nextafter(t_tie, -INFINITY) : t_tie;
                march_adaptive(v, tf, M, sh, opt, &rs, poor, end, alt, &kl_alt, &tf_alt,
                               &near_alt, &anear, &t_tie2);
            }
        } else {
            if (rs.K >= 0) march(v, tf, M, sh, opt, &rs, rs.K, out, &kl, &tf_, &near);
            if (rs.tie && rs.K_alt >= 0)
                march(v, tf, M, sh, opt, &rs, rs.K_alt, alt, &kl_alt, &tf_alt, &near_alt);
        }
        memcpy(rgba + q * 4, out, sizeof out);
        if (rgba_alt) memcpy(rgba_alt + q * 4, tie ? alt : out, sizeof out);
        if (flags)
            flags[q] = (rs.hit ? ORC_FLAG_HIT : 0) | (tie ? ORC_FLAG_LATTICE_TIE : 0) |
                       ((near || near_alt) ? ORC_FLAG_ERT_NEAR : 0) |
                       (anear ? ORC_FLAG_ADAPT_NEAR : 0);
        if (k_last) k_last[q] = kl;
        if (t_final) t_final[q] = tf_;
    }
    free(poor);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Reverse mode (shading NONE).  With c_k = rgb_k and T_k the           */
/* transmittance in front of sample k:                                   */
/*   C = sum_k T_k a_k c_k,  A = 1 - prod_k (1 - a_k)                    */
/*   dC/dc_k = T_k a_k                                                   */
/*   dC/da_k = T_k (c_k - B_{k+1}),  B_k = a_k c_k + (1-a_k) B_{k+1}     */
/*             (B = colour composited behind k, eq. (6) run back to front)*/
/*   dA/da_k = T_k P_{k+1},          P_k = (1-a_k) P_{k+1}               */
/* T_k comes from a forward FP64 pass (stored per sample).  The chain    */
/* continues through the TF interpolation to u, through the clamp to    */
/* the value, and through the trilinear weights to the 8 voxels.        */
/* ------------------------------------------------------------------ */
/* Trilinear weights of p (Section 3.4) scattered: dvol[corner] += w * s.
 * With dabs, |w * s| is summed there as well: the magnitude of the terms
 * whose sum is dvol, i.e. how much cancellation each entry carries. */
static void scatter_trilinear(const orc_volume* v, const double p[3], double s, double* dvol,
                              double* dabs) {
    double fx0 = floor(p[0]), fy0 = floor(p[1]), fz0 = floor(p[2]);
    double tx = p[0] - fx0, ty = p[1] - fy0, tz = p[2] - fz0;
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        double w = (cx ? tx : 1 - tx) * (cy ? ty : 1 - ty) * (cz ? tz : 1 - tz);
        long ii = clampl((long)fx0 + cx, v->nx), jj = clampl((long)fy0 + cy, v->ny),
             kk = clampl((long)fz0 + cz, v->nz);
        long at = (kk * (long)v->ny + jj) * (long)v->nx + ii;
        dvol[at] += w * s;
        if (dabs) dabs[at] += fabs(w * s);
    }
}

/* Reverse of orc_gradient: every tap is a trilinear sample at p + offset,
 * so dL/dG_a scatters through each tap's trilinear weights, scaled like
 * the forward (mask weight / gain / spacing / value range). */
static void gradient_adjoint(const orc_volume* v, int op, const double p[3], const double dg[3],
                             double* dvol, double* dabs) {
    for (int a = 0; a < 3; ++a) {
        if (dg[a] == 0.0) continue;
        double s = dg[a] / op_gain(op) / v->spacing[a] / (v->vmax - v->vmin);
        int beta = (a + 1) % 3, gamma = (a + 2) % 3;
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                if (op == ORC_OP_CENTRAL && (b != 0 || c != 0)) continue;
                double w = op == ORC_OP_CENTRAL ? 1.0 : mask_weight(op, b, c);
                double q1[3] = {p[0], p[1], p[2]}, q0[3];
                q1[beta] += b;
                q1[gamma] += c;
                memcpy(q0, q1, sizeof q0);
                q1[a] += 1.0;
                q0[a] -= 1.0;
                scatter_trilinear(v, q1, w * s, dvol, dabs);
                scatter_trilinear(v, q0, -w * s, dvol, dabs);
            }
    }
}

/* Reverse of orc_shade: given dL/dc, dL/drgb and dL/dG.  At the kinks
 * (max(0, .), the |G| floor) the derivative of the branch the forward took
 * is used. */
static void shade_adjoint(const orc_shading* sh, const double rgb[3], const double g[3],
                          const double p_world[3], const double d[3], const double dc[3],
                          double drgb[3], double dg[3]) {
    dg[0] = dg[1] = dg[2] = 0.0;
    if (sh->model == ORC_SHADE_NONE) {
        for (int ch = 0; ch < 3; ++ch) drgb[ch] = dc[ch];
        return;
    }
    double gn = sqrt(dot3(g, g));
    double den = gn > sh->grad_eps ? gn : sh->grad_eps;
    double ghat[3] = {g[0] / den, g[1] / den, g[2] / den};
    double L[3], tmp[3], dghat[3];
    if (sh->light_is_point) {
        for (int a = 0; a < 3; ++a) tmp[a] = sh->light[a] - p_world[a];
        normalize3(tmp, L);
    } else {
        normalize3(sh->light, L);
    }
    double dc_rgb = dc[0] * rgb[0] + dc[1] * rgb[1] + dc[2] * rgb[2];
    if (sh->model == ORC_SHADE_PAPER_LAMBERT) {
        /* c = rgb (L . ghat) */
        double illum = dot3(L, ghat);
        for (int ch = 0; ch < 3; ++ch) drgb[ch] = dc[ch] * illum;
        for (int a = 0; a < 3; ++a) dghat[a] = dc_rgb * L[a];
    } else {
        /* c = rgb (ka + kd max(0, N.L)) + ks max(0, N.H)^s, N = -ghat */
        double N[3] = {-ghat[0], -ghat[1], -ghat[2]}, Hh[3];
        for (int a = 0; a < 3; ++a) tmp[a] = L[a] - d[a];
        normalize3(tmp, Hh);
        double nl = dot3(N, L), nh = dot3(N, Hh);
        double K = sh->ka + sh->kd * (nl > 0.0 ? nl : 0.0);
        for (int ch = 0; ch < 3; ++ch) drgb[ch] = dc[ch] * K;
        double dN[3] = {0.0, 0.0, 0.0};
        if (nl > 0.0)
            for (int a = 0; a < 3; ++a) dN[a] += sh->kd * dc_rgb * L[a];
        if (nh > 0.0 && sh->shininess != 0.0) {
            double ds = sh->ks * (dc[0] + dc[1] + dc[2]) * sh->shininess *
                        pow(nh, sh->shininess - 1.0);
            for (int a = 0; a < 3; ++a) dN[a] += ds * Hh[a];
        }
        for (int a = 0; a < 3; ++a) dghat[a] = -dN[a];
    }
    /* ghat = g / max(|g|, eps) */
    if (gn > sh->grad_eps) {
        double proj = dot3(ghat, dghat);
        for (int a = 0; a < 3; ++a) dg[a] = (dghat[a] - ghat[a] * proj) / gn;
    } else {
        for (int a = 0; a < 3; ++a) dg[a] = dghat[a] / sh->grad_eps;
    }
}

int orc_render_grad(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
                    const orc_shading* sh_in, const orc_options* opt, const long* pix, long n,
                    const double* g_rgba, double* dvol, double* dtf, double* dvol_abs) {
    if (check_args(v, cam, tf, M, opt) || !g_rgba || !dvol || !dtf) return -1;
    if (opt->adapt_factor > 1) return -1;      /* the reverse mode follows the fixed lattice */
    orc_shading none;
    memset(&none, 0, sizeof none);
    none.model = ORC_SHADE_NONE;
    const orc_shading* sh = sh_in ? sh_in : &none;
    long total = (long)cam->width * cam->height;
    if (!pix) n = total;
    for (long q = 0; q < n; ++q) {
        long id = pix ? pix[q] : q;
        int px = (int)(id % cam->width), py = (int)(id / cam->width);
        ray_setup rs;
        setup_ray(v, cam, opt, px, py, &rs);
        if (rs.K < 0) continue;
        /* forward pass, keeping per-sample state */
        long cap = rs.K + 1;
        sample_state* S = (sample_state*)malloc(sizeof(sample_state) * (size_t)cap);
        double* Tk = (double*)malloc(sizeof(double) * (size_t)cap);
        if (!S || !Tk) { free(S); free(Tk); return -1; }
        double T = 1.0;
        long last = -1;
        for (long k = 0; k <= rs.K; ++k) {
            eval_sample(v, tf, M, sh, opt, &rs, k, &S[k]);
            Tk[k] = T;
            T *= (1.0 - S[k].rgba[3]);
            last = k;
            if (opt->ert_threshold > 0.0 && 1.0 - T >= opt->ert_threshold) break;
        }
        const double* g = g_rgba + q * 4;
        double B[3] = {0, 0, 0}, P = 1.0;
        for (long k = last; k >= 0; --k) {
            const sample_state* s = &S[k];
            double a = s->rgba[3];
            double pr[3];
            for (int ax = 0; ax < 3; ++ax)
                pr[ax] = opt->nearest ? floor(s->pv[ax] + 0.5) : s->pv[ax];
            /* the lit colour; the forward skips the lighting where a = 0 (the
             * colour is multiplied by 0 there), but dC/da needs it at a = 0 too */
            double G[3] = {0.0, 0.0, 0.0}, c_lit[3];
            if (sh->model != ORC_SHADE_NONE) {
                orc_gradient(v, opt->gradient_op, pr, G, NULL);
                orc_shade(sh, s->rgba, G, s->pw, rs.d, c_lit);
            } else {
                c_lit[0] = s->c[0]; c_lit[1] = s->c[1]; c_lit[2] = s->c[2];
            }
            double dc[3], da = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                dc[ch] = g[ch] * Tk[k] * a;
                da += g[ch] * (c_lit[ch] - B[ch]);
            }
            da = Tk[k] * (da + g[3] * P);
            /* opacity correction a = 1 - (1 - a_tf)^e: da/da_tf = e (1 - a_tf)^(e-1),
             * taken as 0 at a_tf = 1 when e < 1 (not differentiable there) */
            if (opt->ref_step > 0.0) {
                double e = opt->step / opt->ref_step;
                double om = 1.0 - s->alpha_tf;
                da *= (om > 0.0 || e >= 1.0) ? e * pow(om, e - 1.0) : 0.0;
            }
            /* TF entries i, i1 with weights (1-t, t) -- orc_tf's lerp */
            double fi = floor(s->u);
            long i = (long)fi;
            if (i < 0) i = 0;
            if (i > M - 1) i = M - 1;
            long i1 = i + 1 < M ? i + 1 : M - 1;
            double t = s->u - (double)i;
            /* lighting (Section 3.8): dL/dc -> dL/d(table rgb) and dL/dG */
            double drgb[3] = {dc[0], dc[1], dc[2]}, dG[3] = {0.0, 0.0, 0.0};
            if (sh->model != ORC_SHADE_NONE && a != 0.0)
                shade_adjoint(sh, s->rgba, G, s->pw, rs.d, dc, drgb, dG);
            double dgrad[4] = {drgb[0], drgb[1], drgb[2], da};
            double du = 0.0;
            for (int ch = 0; ch < 4; ++ch) {
                dtf[i * 4 + ch] += (1.0 - t) * dgrad[ch];
                dtf[i1 * 4 + ch] += t * dgrad[ch];
                du += dgrad[ch] * (tf[i1 * 4 + ch] - tf[i * 4 + ch]);
            }
            /* the value: through the clamp to the trilinear (or nearest) weights */
            if (s->interior)
                scatter_trilinear(v, pr, du * (double)(M - 1) / (v->vmax - v->vmin), dvol,
                                  dvol_abs);
            /* the gradient operator's taps */
            gradient_adjoint(v, opt->gradient_op, pr, dG, dvol, dvol_abs);
            for (int ch = 0; ch < 3; ++ch) B[ch] = a * s->c[ch] + (1.0 - a) * B[ch];
            P *= (1.0 - a);
        }
        free(S);
        free(Tk);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* First-hit surface mode.  The raycaster of Section 3 draws only the   */
/* surfaces of the objects in the volume and does not look into the     */
/* material; Section 3.11 selects the drawn voxels by two thresholds on  */
/* the data value (a window), and Section 3.9 states that it composites  */
/* nothing, so a surface pixel is opaque.  Sections 3.11 and 5.1: a      */
/* coarse forward march finds the first sample inside the window, then   */
/* hitpoint refinement halves the step again and again, moving back from */
/* a sample inside the window and forward from one outside it.           */
/* Reading: getting closer to the target value is taken as being on the  */
/* window side of the boundary; the refinement is then a bisection of    */
/* the last coarse interval, 2^n times finer after n steps (the 64-fold  */
/* gain Section 5.1 credits to 6 steps).  A ray whose first sample is    */
/* already inside (a clip plane through the object) is not refined.  The */
/* refined point is shaded with the gradient there and coloured by the  */
/* TF's rgb at its value.                                                */
/* ------------------------------------------------------------------ */
static int in_window(double val, const orc_surface_options* o) {
    return val >= o->iso_lo && val <= o->iso_hi;
}

static int near_bound(double val, const orc_surface_options* o, double eps) {
    return fabs(val - o->iso_lo) <= eps || fabs(val - o->iso_hi) <= eps;
}

static double value_at(const orc_volume* v, const ray_setup* rs, double t, double pv[3],
                       double pw[3]) {
    for (int a = 0; a < 3; ++a) {
        pw[a] = rs->o[a] + t * rs->d[a];
        pv[a] = pw[a] / v->spacing[a];
    }
    return orc_sample(v, pv);
}

int orc_render_surface(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
                       const orc_shading* sh, const orc_surface_options* opt, const long* pix,
                       long n, double* rgba, double* t_hit, int* k_hit, int* flags, int threads) {
    if (!opt || !sh || !rgba) return -1;
    if (!(opt->iso_lo <= opt->iso_hi) || opt->refine < 0 || opt->refine > 60) return -1;
    orc_options base;
    memset(&base, 0, sizeof base);
    base.step = opt->step;
    base.gradient_op = opt->gradient_op;
    for (int a = 0; a < 3; ++a) {
        base.clip_lo[a] = opt->clip_lo[a];
        base.clip_hi[a] = opt->clip_hi[a];
    }
    if (check_args(v, cam, tf, M, &base)) return -1;
    const double eps = ORC_ISO_EPS * (v->vmax - v->vmin);
    long total = (long)cam->width * cam->height;
    if (!pix) n = total;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    #pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < n; ++q) {
        long id = pix ? pix[q] : q;
        int px = (int)(id % cam->width), py = (int)(id / cam->width);
        ray_setup rs;
        setup_ray(v, cam, &base, px, py, &rs);
        double out[4] = {0, 0, 0, 0};
        double th = INFINITY;
        int kh = -1, fl = rs.K >= 0 ? ORC_FLAG_HIT : 0, near = 0;
        long kmax = rs.tie && rs.K_alt > rs.K ? rs.K_alt : rs.K;
        double pv[3], pw[3];
        /* coarse march: first lattice sample inside the window */
        long first = -1;
        for (long k = 0; k <= kmax; ++k) {
            double val = value_at(v, &rs, rs.t_in + (double)k * opt->step, pv, pw);
            if (near_bound(val, opt, eps)) near = 1;
            if (in_window(val, opt)) {
                first = k;
                break;
            }
        }
        if (rs.tie && first >= 0 && first == kmax) fl |= ORC_FLAG_LATTICE_TIE;
        if (first >= 0 && first <= rs.K) {
            kh = (int)first;
            double t = rs.t_in + (double)first * opt->step;
            if (first > 0) {
                /* hitpoint refinement: halve the step, back when inside */
                double h = opt->step;
                int inside = 1;
                for (int i = 0; i < opt->refine; ++i) {
                    h *= 0.5;
                    t = inside ? t - h : t + h;
                    if (i + 1 < opt->refine) {
                        double val = value_at(v, &rs, t, pv, pw);
                        if (near_bound(val, opt, eps)) near = 1;
                        inside = in_window(val, opt);
                    }
                }
            }
            th = t;
            double val = value_at(v, &rs, t, pv, pw);
            int interior;
            double u = value_to_u(v, val, M, &interior);
            double col[4], c[3];
            orc_tf(tf, M, u, col);
            if (sh->model == ORC_SHADE_NONE) {
                c[0] = col[0]; c[1] = col[1]; c[2] = col[2];
            } else {
                double g[3];
                orc_gradient(v, opt->gradient_op, pv, g, NULL);
                orc_shade(sh, col, g, pw, rs.d, c);
            }
            out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = 1.0;
        }
        if (near) fl |= ORC_FLAG_ISO_NEAR;
        memcpy(rgba + q * 4, out, sizeof out);
        if (t_hit) t_hit[q] = th;
        if (k_hit) k_hit[q] = kh;
        if (flags) flags[q] = fl;
    }
    return 0;
}
