/*
 * Test infrastructure: a standalone driver that runs every oracle entry
 * point (forward, reverse, first-hit surface) over small scenes with every
 * gradient operator, shading model and option, for a build with the
 * address and undefined-behaviour sanitizers.  It exits 0 when every call
 * succeeds and every output is finite; the sanitizers abort on any
 * out-of-bounds access, use of freed memory or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int finite_all(const double* a, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int main(void) {
    enum { NX = 11, NY = 9, NZ = 7, M = 64, W = 13, H = 10 };
    double* data = malloc(sizeof(double) * NX * NY * NZ);
    double* tf = malloc(sizeof(double) * M * 4);
    if (!data || !tf) return 2;
    for (int z = 0; z < NZ; ++z)
        for (int y = 0; y < NY; ++y)
            for (int x = 0; x < NX; ++x) {
                double dx = x - 5.0, dy = y - 4.0, dz = z - 3.0;
                data[(z * NY + y) * NX + x] = 200.0 * exp(-(dx * dx + dy * dy + dz * dz) / 9.0);
            }
    for (int i = 0; i < M; ++i) {
        double u = (double)i / (M - 1);
        tf[4 * i + 0] = u;
        tf[4 * i + 1] = 1.0 - u;
        tf[4 * i + 2] = 0.5;
        tf[4 * i + 3] = u > 0.1 ? 0.2 * u : 0.0;
    }
    orc_volume v = {data, NX, NY, NZ, {1.0, 1.2, 0.9}, 0.0, 200.0};
    orc_camera cams[2] = {
        {ORC_PERSPECTIVE, {-8.0, -6.0, 12.0}, {5.0, 4.8, 2.7}, {0.0, 0.0, 1.0}, 50.0, 0.0, W, H},
        {ORC_ORTHOGRAPHIC, {5.0, -20.0, 2.7}, {5.0, 4.8, 2.7}, {0.0, 0.0, 1.0}, 0.0, 14.0, W, H}};
    const long n = (long)W * H;
    double* rgba = malloc(sizeof(double) * n * 4);
    double* alt = malloc(sizeof(double) * n * 4);
    double* tfin = malloc(sizeof(double) * n);
    double* thit = malloc(sizeof(double) * n);
    double* g = malloc(sizeof(double) * n * 4);
    double* dvol = calloc((size_t)NX * NY * NZ, sizeof(double));
    double* dabs = calloc((size_t)NX * NY * NZ, sizeof(double));
    double* dtf = calloc((size_t)M * 4, sizeof(double));
    int* flags = malloc(sizeof(int) * n);
    int* kl = malloc(sizeof(int) * n);
    long pix[5] = {0, 7, 64, 65, n - 1};
    if (!rgba || !alt || !tfin || !thit || !g || !dvol || !dabs || !dtf || !flags || !kl) return 2;
    for (long i = 0; i < n * 4; ++i) g[i] = sin(0.37 * (double)i);
    int calls = 0;
    for (int c = 0; c < 2; ++c)
        for (int op = 0; op < 3; ++op)
            for (int model = 0; model < 3; ++model)
                for (int variant = 0; variant < 4; ++variant) {
                    orc_shading sh = {model, 0.1, 0.7, 0.2, 16.0, model == ORC_SHADE_PAPER_LAMBERT,
                                      {-0.4, -0.5, 0.75}, 1e-3};
                    if (sh.light_is_point) {
                        sh.light[0] = -5.0; sh.light[1] = -5.0; sh.light[2] = 15.0;
                    }
                    orc_options o = {0.5, op, variant == 1 ? 0.9 : 0.0,
                                     {-1e30, -1e30, -1e30}, {1e30, 1e30, 1e30},
                                     variant == 2, variant == 3 ? 0.7 : 0.0,
                                     variant == 3 ? 2 : 0, 30.0};
                    if (orc_render(&v, &cams[c], tf, M, &sh, &o, NULL, n, rgba, alt, flags, kl,
                                   tfin, 2) != 0)
                        return 3;
                    if (!finite_all(rgba, n * 4) || !finite_all(tfin, n)) return 4;
                    if (orc_render(&v, &cams[c], tf, M, &sh, &o, pix, 5, rgba, NULL, NULL, NULL,
                                   NULL, 1) != 0)
                        return 5;
                    if (variant != 3) {     /* the reverse mode has no adaptive sampling */
                        if (orc_render_grad(&v, &cams[c], tf, M,
                                            model == ORC_SHADE_NONE ? NULL : &sh, &o, NULL, n, g,
                                            dvol, dtf, (c & 1) ? dabs : NULL) != 0)
                            return 6;
                        if (!finite_all(dvol, (long)NX * NY * NZ) || !finite_all(dtf, M * 4) ||
                            !finite_all(dabs, (long)NX * NY * NZ))
                            return 7;
                    }
                    orc_surface_options so = {1.0, op, 60.0, 200.0, 6,
                                              {-1e30, -1e30, -1e30}, {1e30, 1e30, 1e30}};
                    if (orc_render_surface(&v, &cams[c], tf, M, &sh, &so, NULL, n, rgba, thit,
                                           kl, flags, 2) != 0)
                        return 8;
                    if (!finite_all(rgba, n * 4)) return 9;
                    calls += 4;
                }
    /* arguments the oracle must reject without touching memory */
    orc_shading sh0 = {ORC_SHADE_NONE, 0, 0, 0, 1, 0, {0, 0, 1}, 1e-3};
    orc_options bad = {0.0, 0, 0.0, {-1e30, -1e30, -1e30}, {1e30, 1e30, 1e30}, 0, 0.0, 0, 0.0};
    if (orc_render(&v, &cams[0], tf, M, &sh0, &bad, NULL, n, rgba, NULL, NULL, NULL, NULL, 1) != -1)
        return 10;
    printf("sanitize_check: %d oracle calls ok\n", calls);
    free(data); free(tf); free(rgba); free(alt); free(tfin); free(thit); free(g);
    free(dvol); free(dabs); free(dtf); free(flags); free(kl);
    return 0;
}
