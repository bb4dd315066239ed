/*
 * oracle.h -- plain FP64 CPU volume raycaster.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for
 * the GPU raycaster.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * It computes, slowly and literally, what "Volume Raycasting mit OpenCL"
 * (Kopal) describes:
 *   Section 2.1  eq. (1)      the voxel grid V: N^3 -> R
 *   Section 3.3               ray / bounding-box intersection, regular sampling
 *   Section 3.4  eq. (2)      linear and trilinear (7 lerps) interpolation
 *   Section 3.5  eq. (3),(4)  central-difference, Sobel3D, Zucker-Hummel gradients
 *   Section 3.6               bounding box used as a clip ("cut") box
 *   Section 3.7               value -> colour lookup table
 *   Section 3.8  Listing 3    point-light Lambert shading ("Shade")
 *   Section 3.9  eq. (6)      the transparency (compositing) formula
 *   Section 3.10              the four-step pipeline
 *   Sections 3, 3.11, 5.1     first-hit surface mode: a value window, a
 *                             coarse march, hitpoint refinement
 * Readings where the paper is silent (coordinate frame, camera model,
 * lattice anchoring, TF interpolation, gradient scale, Blinn-Phong
 * constants, the Zucker-Hummel mask) are listed with the functions.
 *
 * All arithmetic is IEEE double, no fast-math.  Every function is
 * re-entrant; orc_render parallelises over pixels with OpenMP.
 */
#ifndef RC_ORACLE_H
#define RC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OP_CENTRAL = 0, ORC_OP_SOBEL3D = 1, ORC_OP_ZUCKER_HUMMEL = 2 };
enum { ORC_SHADE_NONE = 0, ORC_SHADE_BLINN_PHONG = 1, ORC_SHADE_PAPER_LAMBERT = 2 };
enum { ORC_PERSPECTIVE = 1, ORC_ORTHOGRAPHIC = 0 };

/* per-pixel result flags */
enum {
    ORC_FLAG_HIT = 1,        /* the ray met the sampling box */
    ORC_FLAG_LATTICE_TIE = 2,/* (t_out-t_in)/step within ORC_TIE_EPS of an integer:
                                rgba_alt holds the result with the other sample count */
    ORC_FLAG_ERT_NEAR = 4,   /* 1-T came within ORC_ERT_EPS of the ERT threshold */
    ORC_FLAG_ISO_NEAR = 8,   /* surface mode: a window test that decided the result had a
                                value within ORC_ISO_EPS*(vmax-vmin) of a window bound */
    ORC_FLAG_ADAPT_NEAR = 16 /* adaptive sampling: a sample lay within ORC_ADAPT_EPS voxels
                                of a brick boundary, where the brick (and so the step) taken
                                depends on rounding */
};
#define ORC_TIE_EPS 1e-6
#define ORC_ERT_EPS 1e-4
#define ORC_ISO_EPS 1e-6
#define ORC_ADAPT_EPS 1e-7

typedef struct {
    const double* data;      /* [nz][ny][nx] voxel values, x fastest */
    int nx, ny, nz;
    double spacing[3];       /* world units between neighbouring voxels */
    double vmin, vmax;       /* raw values mapped to TF coordinates 0 and 1 */
} orc_volume;

typedef struct {
    int projection;          /* ORC_PERSPECTIVE or ORC_ORTHOGRAPHIC */
    double eye[3], target[3], up[3];
    double fov_y_deg;        /* perspective: full vertical field of view */
    double ortho_height;     /* orthographic: world height of the image */
    int width, height;
} orc_camera;

typedef struct {
    int model;               /* ORC_SHADE_* */
    double ka, kd, ks, shininess;
    int light_is_point;      /* 1: light = position, 0: light = direction towards the light */
    double light[3];
    double grad_eps;         /* floor of |G| in the normalisation */
} orc_shading;

typedef struct {
    double step;             /* sample distance in world units */
    int gradient_op;         /* ORC_OP_* */
    double ert_threshold;    /* 0: off, else stop once 1-T >= threshold */
    double clip_lo[3], clip_hi[3]; /* clip box in world units, intersected with the volume box */
    int nearest;             /* 1: nearest-voxel sampling (Section 3.3's rounding) */
    double ref_step;         /* > 0: opacity correction to this reference step; 0: off */
    int adapt_factor;        /* > 1: adaptive sampling (Section 5.2): samples in 8^3 bricks
                                whose value range is at most adapt_range advance by
                                adapt_factor * step; 0 or 1: off */
    double adapt_range;      /* raw-value range up to which a brick counts as detail-poor */
} orc_options;

/* trilinear sample at a voxel-space point (Section 3.4) */
double orc_sample(const orc_volume* v, const double p[3]);
/* nearest-voxel sample: the voxel at floor(p + 1/2) per axis (Section 3.3) */
double orc_sample_nearest(const orc_volume* v, const double p[3]);
/* gradient estimate at a voxel-space point (Section 3.5), scaled to
 * normalised value per world unit; raw = stencil sum before scaling */
void orc_gradient(const orc_volume* v, int op, const double p[3], double g[3], double raw[3]);
/* transfer-function lookup at table coordinate u in [0, M-1] (Section 3.7) */
void orc_tf(const double* tf, int M, double u, double rgba[4]);
/* camera ray through the centre of pixel (px, py); row 0 at the top */
void orc_camera_ray(const orc_camera* cam, int px, int py, double o[3], double d[3]);
/* slab intersection, t >= 0; returns 1 on a hit (Section 3.3) */
int orc_ray_box(const double o[3], const double d[3], const double lo[3], const double hi[3],
                double* t_in, double* t_out);
/* shading of one sample; nrm = outward unit normal -G/max(|G|,eps) */
void orc_shade(const orc_shading* sh, const double rgb[3], const double g[3],
               const double p_world[3], const double d[3], double c[3]);

/*
 * Render pixels.  pix = linear pixel indices (py*W+px) or NULL for all
 * W*H pixels in order; n = number of outputs.
 * rgba[n*4]    premultiplied colour and opacity over black
 * rgba_alt     NULL or [n*4]: result with the other admissible sample count
 * flags        NULL or [n]: ORC_FLAG_* bits
 * k_last       NULL or [n]: index of the last composited sample, -1 on a miss
 * t_final      NULL or [n]: transmittance after the last sample
 * n_lattice    NULL or [n]: number of lattice samples taken (k_last+1)
 * threads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad arguments.
 */
int orc_render(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
               const orc_shading* sh, const orc_options* opt, const long* pix, long n,
               double* rgba, double* rgba_alt, int* flags, int* k_last, double* t_final,
               int threads);

/*
 * Reverse mode of orc_render.  sh = NULL means shading NONE; with a shading
 * model the chain also runs through the lighting, the normalisation and the
 * gradient operator's taps.  g_rgba[n*4] = dL/d(rgba) of the listed pixels.
 * dvol[nz*ny*nx] and dtf[M*4] are accumulated (+=).  dvol_abs (NULL or
 * [nz*ny*nx], accumulated) receives the sum of the magnitudes of the terms
 * added into each dvol entry: an entry whose terms cancel has
 * dvol_abs >> |dvol|, and a finite-precision sum of those terms can only be
 * trusted to a few units of rounding times dvol_abs.  Uses the same lattice
 * (primary sample count) and the same early ray termination as orc_render.
 * Returns 0, or -1 on bad arguments.
 */
int orc_render_grad(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
                    const orc_shading* sh, const orc_options* opt, const long* pix, long n,
                    const double* g_rgba, double* dvol, double* dtf, double* dvol_abs);

/* First-hit surface mode (Sections 3, 3.11 and 5.1). */
typedef struct {
    double step;             /* coarse sample distance in world units */
    int gradient_op;         /* ORC_OP_* */
    double iso_lo, iso_hi;   /* raw-value window drawn as the surface */
    int refine;              /* hitpoint-refinement steps (Section 5.1: 5 to 6) */
    double clip_lo[3], clip_hi[3];
} orc_surface_options;

/*
 * Render the first surface along each ray: the first coarse lattice sample
 * whose value lies in [iso_lo, iso_hi], refined towards the window boundary
 * by `refine` halving steps, then shaded opaquely.  pix/n as orc_render.
 * rgba[n*4]   (c, 1) on a surface hit, 0 otherwise
 * t_hit       NULL or [n]: ray parameter of the refined hit, +inf without one
 * k_hit       NULL or [n]: coarse index of the first sample in the window, -1
 * flags       NULL or [n]: ORC_FLAG_HIT | ORC_FLAG_LATTICE_TIE (the hit is the
 *             last lattice sample of a tie) | ORC_FLAG_ISO_NEAR
 * Returns 0, or -1 on bad arguments.
 */
int orc_render_surface(const orc_volume* v, const orc_camera* cam, const double* tf, int M,
                       const orc_shading* sh, const orc_surface_options* opt, const long* pix,
                       long n, double* rgba, double* t_hit, int* k_hit, int* flags, int threads);

#ifdef __cplusplus
}
#endif
#endif
