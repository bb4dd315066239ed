// Host-side checks of the library under AddressSanitizer / UBSan (built
// host-only: no GPU code is run).  Calls every entry point with arguments
// it must reject on the host, and runs the host logic that needs no device
// -- argument validation against a handle built here, camera frames, tiling,
// scratch sizes, the tile and work-order maps, the persistent kernel choice
// -- so that any out-of-bounds access, leak, use after free or undefined
// operation in that code stops the run.  Exit status 0 means every check
// passed.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <set>
#include <vector>

#include "../paper_1609_01317_amd/csrc/march.h"
#include "../paper_1609_01317_amd/csrc/persist.h"

using namespace rc;

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                    \
        }                                                               \
    } while (0)

static rc_camera camera(int w, int h) {
    rc_camera c;
    std::memset(&c, 0, sizeof c);
    c.projection = RC_PERSPECTIVE;
    c.width = w;
    c.height = h;
    c.eye[0] = 100; c.eye[1] = -80; c.eye[2] = 60;
    c.target[0] = 20; c.target[1] = 18; c.target[2] = 16;
    c.up[2] = 1;
    c.fov_y_deg = 60;
    c.ortho_height = 40;
    return c;
}

int main() {
    // ---- entry points, rejected on the host
    rc_volume* out = nullptr;
    const double sp[3] = {1, 1, 1};
    CHECK(rc_create_volume(nullptr, 4, 4, 4, RC_U8, sp, 0, 1, nullptr, &out) == RC_E_INVALID);
    CHECK(std::strlen(rc_last_error()) > 0);
    int dummy = 0;
    CHECK(rc_create_volume(&dummy, 0, 4, 4, RC_U8, sp, 0, 1, nullptr, &out) == RC_E_INVALID);
    CHECK(rc_create_volume(&dummy, 4, 4, 5000, RC_U8, sp, 0, 1, nullptr, &out) == RC_E_INVALID);
    CHECK(rc_create_volume(&dummy, 4, 4, 4, 7, sp, 0, 1, nullptr, &out) == RC_E_INVALID);
    const double bad_sp[3] = {1, NAN, 1};
    CHECK(rc_create_volume(&dummy, 4, 4, 4, RC_U8, bad_sp, 0, 1, nullptr, &out) == RC_E_INVALID);
    CHECK(rc_create_volume(&dummy, 4, 4, 4, RC_U8, sp, 1, 1, nullptr, &out) == RC_E_INVALID);
    CHECK(rc_create_volume(&dummy, 4, 4, 4, RC_U8, sp, 0, 1, nullptr, nullptr) == RC_E_INVALID);
    CHECK(rc_update_volume(nullptr, &dummy, nullptr) != RC_OK);
    CHECK(rc_build_bricks(nullptr, 8, nullptr) != RC_OK);
    rc_camera cam = camera(37, 29);
    rc_shading sh;
    std::memset(&sh, 0, sizeof sh);
    sh.model = RC_SHADE_BLINN_PHONG;
    sh.ka = 0.1f; sh.kd = 0.7f; sh.ks = 0.2f; sh.shininess = 32;
    sh.light[2] = 1; sh.grad_eps = 1e-3f;
    rc_options opt;
    std::memset(&opt, 0, sizeof opt);
    opt.step = 0.5;
    for (int a = 0; a < 3; ++a) { opt.clip_lo[a] = -1e30; opt.clip_hi[a] = 1e30; }
    float tf[8] = {0};
    float img[4] = {0};
    CHECK(rc_render(nullptr, &cam, tf, 2, &sh, &opt, img, nullptr, nullptr, nullptr) ==
          RC_E_INVALID);
    CHECK(rc_render_backward(nullptr, &cam, tf, 2, &sh, &opt, nullptr, img, img, img, nullptr) ==
          RC_E_INVALID);
    float* outs[1] = {img};
    CHECK(rc_render_views(nullptr, &cam, 1, tf, 2, &sh, &opt, outs, nullptr, nullptr) ==
          RC_E_INVALID);
    CHECK(rc_render_views_noalloc(nullptr, &cam, 1, tf, 2, &sh, &opt, outs, nullptr, nullptr) ==
          RC_E_INVALID);
    CHECK(rc_render_views(nullptr, &cam, 0, tf, 2, &sh, &opt, outs, nullptr, nullptr) ==
          RC_E_INVALID);
    CHECK(rc_render_backward_views(nullptr, nullptr, 1, tf, 2, &sh, &opt, nullptr, nullptr, img,
                                   img, nullptr) == RC_E_INVALID);
    rc_surface_options so;
    std::memset(&so, 0, sizeof so);
    so.step = 1;
    CHECK(rc_render_surface(nullptr, &cam, tf, 2, &sh, &so, img, nullptr, nullptr) ==
          RC_E_INVALID);
    rc_batch* b = nullptr;
    CHECK(rc_batch_create(nullptr, 1, nullptr, nullptr, &b) == RC_E_INVALID);
    CHECK(rc_batch_render(nullptr, 0, nullptr) == RC_E_INVALID);
    CHECK(rc_render_batch(nullptr, 0, nullptr, nullptr) == RC_E_INVALID);
    rc_batch_config cfg;
    CHECK(rc_batch_autotune(nullptr, 1, nullptr, nullptr, &cfg) == RC_E_INVALID);
    rc_batch_destroy(nullptr);
    rc_destroy_volume(nullptr);
    CHECK(rc_debug_bounds_violations(nullptr) == RC_E_INVALID);

    // ---- host logic against a handle built here (device pointers are fake
    // and never dereferenced on the host)
    rc_volume v;
    std::memset(&v, 0, sizeof v);
    v.nx = 40; v.ny = 37; v.nz = 33;
    v.dtype = RC_U16;
    v.elem_bytes = 2;
    for (int a = 0; a < 3; ++a) v.spacing[a] = 1.0 + 0.25 * a;
    v.vmin = 0; v.vmax = 4095;
    v.nbx = 5; v.nby = 5; v.nbz = 5;
    v.nbricks = 125;
    v.nsx = v.nsy = v.nsz = 2;
    v.nsuper = 8;
    v.bricked = (void*)0x1000;
    v.brick_range = (float2*)0x2000;
    v.device = 0;
    CHECK(check_render_args(&v, &cam, tf, 2, &sh, &opt) == RC_OK);
    rc_camera bad = cam;
    bad.width = 0;
    CHECK(check_render_args(&v, &bad, tf, 2, &sh, &opt) == RC_E_INVALID);
    bad = cam;
    bad.fov_y_deg = 180;
    CHECK(check_render_args(&v, &bad, tf, 2, &sh, &opt) == RC_E_INVALID);
    bad = cam;
    for (int a = 0; a < 3; ++a) bad.target[a] = bad.eye[a];
    CHECK(check_render_args(&v, &bad, tf, 2, &sh, &opt) == RC_E_INVALID);
    rc_options bo = opt;
    bo.step = 1e-9;
    CHECK(check_render_args(&v, &cam, tf, 2, &sh, &bo) == RC_E_INVALID);
    bo = opt;
    bo.gradient_op = 9;
    CHECK(check_render_args(&v, &cam, tf, 2, &sh, &bo) == RC_E_INVALID);
    bo = opt;
    bo.adapt_factor = 65;
    CHECK(check_render_args(&v, &cam, tf, 2, &sh, &bo) == RC_E_INVALID);
    CHECK(check_render_args(&v, &cam, tf, 70000, &sh, &opt) == RC_E_INVALID);
    rc_shading bs = sh;
    bs.grad_eps = 0;
    CHECK(check_render_args(&v, &cam, tf, 2, &bs, &opt) == RC_E_INVALID);
    rc_volume nb = v;
    nb.brick_range = nullptr;
    bo = opt;
    bo.skip_empty = 1;
    CHECK(check_render_args(&nb, &cam, tf, 2, &sh, &bo) == RC_E_STATE);

    RenderParams P;
    fill_render_params(P, &v, &cam, tf, 256, &sh, &opt);
    CHECK(P.nx == 40 && P.M == 256 && std::fabs(P.view.f[0] * P.view.f[0] + P.view.f[1] * P.view.f[1] +
                                                 P.view.f[2] * P.view.f[2] - 1.0) < 1e-12);
    for (int tw : {4, 8, 16, 32, 64}) {
        ViewParams V = P.view;
        set_tiling(V, tw);
        CHECK(V.tiles_x * tw >= V.W && (V.n_tiles / V.tiles_x) * (64 / tw) >= V.H);
    }
    size_t mb = 0, sb = 0;
    const size_t skip = skip_scratch_bytes(&v, 256, &mb, &sb);
    CHECK(mb >= 125 && sb >= 8 && skip == mb + sb + 4 * 257);
    bo = opt;
    bo.skip_empty = 1;
    CHECK(views_scratch_bytes(&v, 256, &bo) > views_scratch_bytes(&v, 256, &opt));
    CHECK(item_kind(&v, &sh, &opt) == 1 * 3 + 0);

    // every tile of a grid is placed exactly once by tile_of_block
    for (int tx : {1, 5, 16, 33}) for (int ty : {1, 3, 16, 21}) {
        std::set<int> seen;
        const int blocks = group_grid_blocks(tx, ty);
        for (int blk = 0; blk < blocks; ++blk) {
            int t = tile_of_block(blk, tx, ty);
            if (t >= 0) CHECK(seen.insert(t).second);
        }
        CHECK((int)seen.size() == tx * ty);
    }
    // centre_out is a permutation; view_of_unit covers every unit once
    for (int n : {1, 2, 7, 64}) {
        std::set<int> s;
        for (int k = 0; k < n; ++k) s.insert(centre_out(k, n));
        CHECK((int)s.size() == n && *s.begin() == 0 && *s.rbegin() == n - 1);
    }
    ViewSet S;
    S.n = 3;
    const int units[3] = {5, 1, 9};
    S.block_off[0] = 0;
    for (int i = 0; i < 3; ++i) S.block_off[i + 1] = S.block_off[i] + units[i];
    std::set<std::pair<int, int>> cover;
    for (int j = 0; j < S.block_off[3] + 4; ++j) {
        int rank = -1, vw = view_of_unit(S, 1, j, rank);
        if (j >= S.block_off[3]) { CHECK(vw == -1); continue; }
        CHECK(vw >= 0 && rank >= 0 && rank < units[vw]);
        CHECK(cover.insert({vw, rank}).second);
    }
    CHECK((int)cover.size() == S.block_off[3]);
    // the persistent kernel chosen for a set of kinds renders all of them
    for (unsigned mask : {1u, 8u, 0x7u, 0x38u, 0x49u, 0x200u, 0x1000u, 0x1FFu, 0x101u, 0x1FFFFFu}) {
        const PersistKernel& k = persist_kernel(mask);
        CHECK((k.mask & mask) == mask && k.fn != nullptr);
    }
    std::printf("host checks: %d failed\n", fails);
    return fails == 0 ? 0 : 1;
}
