"""GPU forward render vs the FP64 oracle (bar: max-abs 2e-4 per channel;
lattice-end ties may match either admissible sample count; with early
termination, pixels whose opacity came within 1e-4 of the threshold may
differ by up to 1 - tau)."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import TOL, compare, gpu_render, gpu_volume, oracle_render, to_dev

pytestmark = pytest.mark.gpu

import paper_1609_01317_amd as rc  # noqa: E402


def _check(sc, min_content=20, **kw):
    g = gpu_render(sc, **kw)
    r = oracle_render(sc, **{k: v for k, v in kw.items() if k in ("cam", "options", "shading")})
    # a scene that shows nothing would pass trivially
    assert (r["rgba"][..., 3] > 1e-6).sum() >= min_content
    tau = (kw.get("options") or sc.options)["ert_threshold"]
    err, bad = compare(g["rgba"], r, tau)
    print(f"{sc.name}: max err {err:.3e}, failing pixels {int(bad.sum())}", flush=True)
    assert not bad.any(), f"{int(bad.sum())} pixels over tolerance, max err {err:.3e}"
    return g, r


def test_c1_full_frame():
    """64^3 u8 blobs -> 128^2 orthographic, CD, Blinn-Phong, no ERT/skip."""
    sc = W.config_c1()
    g, r = _check(sc)
    hit = r["k_last"] >= 0
    assert hit.sum() > 4000
    tie = (r["flags"] & 2) != 0
    np.testing.assert_array_equal(g["k_last"][~tie], r["k_last"][~tie])


SMALL = [
    dict(seed=1, dtype=np.uint8, op="central", shading="blinn_phong", projection="persp"),
    dict(seed=2, dtype=np.uint8, op="sobel3d", shading="blinn_phong", projection="ortho"),
    dict(seed=3, dtype=np.uint16, op="zucker_hummel", shading="blinn_phong", projection="persp"),
    dict(seed=4, dtype=np.uint16, op="sobel3d", shading="paper_lambert", projection="persp"),
    dict(seed=5, dtype=np.float32, op="central", shading="blinn_phong", projection="persp"),
    dict(seed=6, dtype=np.float32, op="zucker_hummel", shading="none", projection="ortho"),
    dict(seed=7, dtype=np.uint8, op="sobel3d", shading="blinn_phong", projection="persp",
         ert=0.9),
    dict(seed=8, dtype=np.uint16, op="central", shading="blinn_phong", projection="persp",
         ert=0.95, skip=True),
    dict(seed=9, dtype=np.uint8, op="zucker_hummel", shading="paper_lambert", projection="ortho",
         skip=True, step=0.37),
    dict(seed=10, dtype=np.float32, op="sobel3d", shading="blinn_phong", projection="persp",
         spacing=(1.0, 0.7, 1.6), step=0.41),
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"s{c['seed']}")
def test_small_scenes(case):
    """Several tiles plus a ragged tail (image 37x29 is not a multiple of 8)."""
    sc = W.config_small(dims=(26, 21, 19), image=(37, 29), **case)
    if case["shading"] == "paper_lambert":
        sc.shading["light_is_point"] = True
        sc.shading["light"] = (60.0, -40.0, 50.0)
    _check(sc)


VARIANTS = [
    dict(seed=17, dtype=np.uint8, op="sobel3d", nearest=True, ref=0.0, skip=False),
    dict(seed=18, dtype=np.uint16, op="central", nearest=False, ref=1.0, skip=True),
    dict(seed=19, dtype=np.float32, op="zucker_hummel", nearest=True, ref=0.3, skip=False),
    dict(seed=20, dtype=np.uint16, op="sobel3d", nearest=True, ref=2.0, skip=True),
]


@pytest.mark.parametrize("case", VARIANTS, ids=lambda c: f"s{c['seed']}")
def test_sampling_variants(case):
    """Nearest-voxel sampling and opacity correction vs the oracle."""
    sc = W.config_small(seed=case["seed"], dims=(26, 21, 19), dtype=case["dtype"], image=(37, 29),
                        op=case["op"], skip=case["skip"], ert=0.97, step=0.45)
    sc.options.update(nearest=case["nearest"], ref_step=case["ref"])
    _check(sc)


def test_clip_box_and_anisotropic_spacing():
    sc = W.config_small(seed=12, dims=(30, 24, 20), image=(41, 33), op="sobel3d",
                        spacing=(0.8, 1.25, 1.1))
    opt = dict(sc.options, clip_lo=(4.0, 2.5, -5.0), clip_hi=(18.0, 40.0, 15.0))
    _check(sc, options=opt)


@pytest.mark.parametrize("dtype,dims", [(np.uint8, (77, 37, 29)), (np.uint16, (77, 37, 29)),
                                        (np.float32, (77, 37, 29)), (np.uint16, (68, 30, 21)),
                                        (np.uint8, (132, 12, 9))])
def test_update_volume_rebuilds_brick_ranges(dtype, dims):
    """rc_update_volume on a handle whose brick ranges exist rebuilds them in
    the ingest pass (the staged run of bricks plus its one-voxel apron): renders
    with skipping from the updated handle equal, bit for bit and in their skip
    counters, those of a fresh handle built from the same voxels.  Ragged
    dimensions, so runs of fewer than 8 bricks and clamped aprons occur;
    rows of a multiple of 4 voxels take the 4-voxel loads."""
    sc = W.config_small(seed=71, dims=dims, dtype=dtype, image=(48, 40), op="sobel3d",
                        ert=0.95, skip=True)
    old = np.ascontiguousarray(np.roll(sc.volume, (5, -7, 11), axis=(0, 1, 2)))
    upd = rc.rc_create_volume(to_dev(old), sc.spacing, sc.vmin, sc.vmax)
    rc.rc_build_bricks(upd, 8)
    rc.rc_update_volume(upd, to_dev(sc.volume))
    fresh = gpu_volume(sc, bricks=True)
    cams = [W.orbit_camera(dims, sc.spacing, 40.0 * i, 25.0 - 10 * i, 48, 40) for i in range(3)]
    for cam in cams:
        a = gpu_render(sc, cam=cam, vol=upd, stats=True)
        b = gpu_render(sc, cam=cam, vol=fresh, stats=True)
        assert np.array_equal(a["rgba"], b["rgba"]) and np.array_equal(a["k_last"], b["k_last"])
        np.testing.assert_array_equal(a["stats"], b["stats"])
        assert b["stats"][5] > 0            # some chunks were skipped as empty


def test_skip_is_lossless_bitwise():
    """Skipped samples have alpha exactly 0, so skip on == skip off bit for bit."""
    sc = W.config_small(seed=13, dims=(40, 36, 33), dtype=np.uint16, image=(48, 40),
                        op="sobel3d", ert=0.99)
    vol = gpu_volume(sc, bricks=True)
    on = gpu_render(sc, vol=vol, options=dict(sc.options, skip_empty=True), stats=True)
    off = gpu_render(sc, vol=vol, options=dict(sc.options, skip_empty=False), stats=True)
    np.testing.assert_array_equal(on["rgba"], off["rgba"])
    np.testing.assert_array_equal(on["k_last"], off["k_last"])
    assert on["stats"][0] == off["stats"][0]            # same lattice samples
    assert on["stats"][1] < off["stats"][1]             # fewer evaluated
    assert on["stats"][2] == off["stats"][2]            # same non-empty samples


@pytest.mark.parametrize("dtype,projection", [(np.uint16, "persp"), (np.uint8, "ortho"),
                                              (np.float32, "persp")])
def test_sparse_volume_super_bricks(dtype, projection):
    """150x130x120 volume (a ragged 5x5x4 grid of 32^3 super-bricks) that is
    empty except for a few blobs in one corner: long stretches of every ray
    are cleared by the super-brick test.  Skip on == skip off bit for bit,
    and the oracle agrees on a pixel sample."""
    sc = W.config_small(seed=16, dims=(150, 130, 120), dtype=dtype, image=(72, 60),
                        op="sobel3d", ert=0.99, projection=projection)
    sc.volume = W.blob_volume((120, 130, 150), 4, seed=16, dtype=dtype, sigma=(3.0, 6.0),
                              amp=(0.5, 1.0) if dtype == np.float32 else (1500.0, 4000.0)
                              if dtype == np.uint16 else (120.0, 255.0),
                              centre_lo=0.65, centre_hi=0.85, normalise=dtype == np.float32)
    vol = gpu_volume(sc, bricks=True)
    on = gpu_render(sc, vol=vol, options=dict(sc.options, skip_empty=True), stats=True)
    off = gpu_render(sc, vol=vol, options=dict(sc.options, skip_empty=False), stats=True)
    np.testing.assert_array_equal(on["rgba"], off["rgba"])
    np.testing.assert_array_equal(on["k_last"], off["k_last"])
    assert on["stats"][0] == off["stats"][0]
    assert on["stats"][2] == off["stats"][2] > 0
    assert on["stats"][1] < 0.25 * off["stats"][1]      # most of the lattice skipped
    H, Wd = 60, 72
    pix = np.random.default_rng(16).choice(H * Wd, size=600, replace=False)
    ref = oracle_render(sc, options=dict(sc.options, skip_empty=True), pixels=pix)
    err, bad = compare(on["rgba"].reshape(-1, 4)[pix], ref, tau=0.99)
    assert not bad.any(), err


def test_ert_bound():
    sc = W.config_small(seed=14, dims=(24, 24, 24), image=(32, 32), op="central")
    tau = 0.7
    full = gpu_render(sc)
    ert = gpu_render(sc, options=dict(sc.options, ert_threshold=tau))
    assert np.abs(full["rgba"] - ert["rgba"]).max() <= 1 - tau + 1e-5
    stopped = ert["k_last"] < full["k_last"]
    assert stopped.any() and np.all(ert["rgba"][..., 3][stopped] >= tau - 1e-6)


def test_stats_count_the_lattice():
    sc = W.config_c1()
    g = gpu_render(sc, stats=True)
    r = oracle_render(sc)
    tie = (r["flags"] & 2) != 0
    lat_oracle = int((r["k_last"] + 1)[~tie].sum())
    lat_gpu_notie = int((g["k_last"] + 1)[~tie].sum())
    assert lat_gpu_notie == lat_oracle
    assert g["stats"][0] == int((g["k_last"] + 1).sum())
    assert g["stats"][3] == int((g["k_last"] >= 0).sum())


def test_c2_full_frame():
    """256^3 u16 phantom -> 512^2 perspective, Sobel3D, ERT 0.99, skip on."""
    sc = W.config_c2()
    g, r = _check(sc)
    assert (r["k_last"] >= 0).sum() > 100000


@pytest.mark.parametrize("op", ["central", "sobel3d", "zucker_hummel"])
def test_c3_full_size_sampled(op, c3_scene):
    """512^3 u16 -> 1024^2 through rc_render (the single-image kernel), one
    view per operator, 20000 seeded pixels checked against the oracle."""
    sc = c3_scene
    vol = c3_scene.extra["gpu_volume"]
    cam = sc.cameras[7]
    opt = dict(sc.options, gradient_op=op)
    g = gpu_render(sc, cam=cam, vol=vol, options=opt)
    rng = np.random.default_rng(303)
    pix = rng.choice(1024 * 1024, size=20000, replace=False)
    r = oracle_render(sc, cam=cam, options=opt, pixels=pix)
    err, bad = compare(g["rgba"].reshape(-1, 4)[pix], r, opt["ert_threshold"])
    print(f"c3 {op}: max err {err:.3e}", flush=True)
    assert not bad.any()


def _candidate_configs():
    """The configurations the batch autotuner chooses among (its launch
    shapes with default boxes; box budgets and first chunk lengths on two of
    the shapes), plus the library's default: the images must not depend on
    which one the benchmark picks."""
    cfgs = [{"tile_w": 8, "waves_per_wg": 1, "wg_per_cu": 8, "order": 1}]
    for tw in (4, 8, 16):
        for w in (1, 4):
            for pc in (4, 8, 16):
                for od in (0, 1):
                    cfgs.append({"tile_w": tw, "waves_per_wg": w, "wg_per_cu": max(1, pc // w),
                                 "order": od})
    for shape in ({"tile_w": 8, "waves_per_wg": 1, "wg_per_cu": 16, "order": 1},
                  {"tile_w": 16, "waves_per_wg": 4, "wg_per_cu": 2, "order": 0}):
        for g in (8192, 12288, 16384, 20480):
            for d in (4096, 8192, 12288):
                if max(g, d) * shape["waves_per_wg"] <= 65536:
                    cfgs.append(dict(shape, box_bytes_grad=g, box_bytes_cd=d))
        for n in (8, 32):
            cfgs.append(dict(shape, chunk_len=n))
    return cfgs


def test_c3_benchmarked_launch_matches_oracle(c3_scene):
    """The headline launch exactly as bench.py builds and times it: the
    108-item render list (36 orbit views x central difference, Sobel3D,
    Zucker-Hummel) in one persistent rc_batch with the autotuned launch
    configuration.  4096 seeded pixels of every one of the 108 views are
    checked against the FP64 oracle; then the same list rendered with every
    candidate launch configuration gives bit-identical sampled pixels."""
    import bench
    import oracle

    sc = c3_scene
    vol = c3_scene.extra["gpu_volume"]
    tf = to_dev(sc.tf)
    _, all_items = bench.c3_render_list(sc, vol, tf)
    cfg, batch = bench.c3_batch(all_items)
    print(f"c3 batch: autotuned config {cfg}", flush=True)
    rc.rc_batch_render(batch)
    torch.cuda.synchronize()
    rng = np.random.default_rng(404)
    n_pix = 1024 * 1024
    pix = [rng.choice(n_pix, size=4096, replace=False) for _ in all_items]
    idx = [torch.from_numpy(p).cuda() for p in pix]

    def gather():
        return [it["out"].view(-1, 4).index_select(0, i).cpu().numpy()
                for it, i in zip(all_items, idx)]

    got = gather()
    ov = oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    worst = 0.0
    content = 0
    for v, it in enumerate(all_items):
        r = oracle.render(ov, it["camera"], sc.tf, sc.shading, it["options"], pixels=pix[v])
        err, bad = compare(got[v], r, it["options"]["ert_threshold"])
        worst = max(worst, err)
        content += int((r["rgba"][:, 3] > 1e-6).sum())
        assert not bad.any(), (v, it["options"]["gradient_op"], int(bad.sum()), err)
    print(f"c3 batch: 108 views x 4096 pixels, max err {worst:.3e}", flush=True)
    # the comparison is not over empty pixels only: about 16 % of the sampled
    # rays pass through phantom material with non-zero table opacity
    assert content > 108 * 4096 // 10
    rc.rc_batch_destroy(batch)
    for c in _candidate_configs():
        b = rc.rc_batch_create(all_items, c)
        rc.rc_batch_render(b)
        torch.cuda.synchronize()
        other = gather()
        rc.rc_batch_destroy(b)
        for v in range(len(all_items)):
            assert np.array_equal(other[v], got[v]), (c, v)


@pytest.fixture(scope="module")
def c3_scene():
    sc = W.config_c3(n_views=36)
    sc.extra["gpu_volume"] = gpu_volume(sc, bricks=True)
    yield sc
    rc.rc_destroy_volume(sc.extra["gpu_volume"])


# ---------------------------------------------------------------- edge cases
def test_all_rays_miss_and_tiny_images():
    sc = W.config_small(seed=15, dims=(10, 10, 10), image=(1, 1))
    cam = dict(sc.cameras[0], target=(100.0, 100.0, 100.0))
    g = gpu_render(sc, cam=cam)
    assert np.all(g["rgba"] == 0) and np.all(g["k_last"] == -1)
    _check(sc, min_content=0)  # 1x1 image through the centre
    sc2 = W.config_small(seed=16, dims=(10, 10, 10), image=(3, 130))
    _check(sc2, min_content=0)


def test_degenerate_volumes_and_short_tables():
    for dims in [(1, 1, 1), (2, 2, 2), (1, 9, 5), (9, 1, 1)]:
        sc = W.config_small(seed=17, dims=dims, image=(11, 9), dtype=np.float32)
        _check(sc, min_content=0)
    sc = W.config_small(seed=18, dims=(9, 9, 9), image=(12, 12))
    sc.tf = np.array([[0.2, 0.4, 0.6, 0.0], [0.9, 0.5, 0.1, 0.5]], dtype=np.float32)
    _check(sc)


def test_maximum_extents():
    """The edges of the accepted sizes: a 4096-voxel volume axis (the largest
    edge) marched end to end, a 16384-pixel-wide image (the largest image
    edge), and a 65536-entry table; against the oracle (sampled pixels for
    the wide image)."""
    sc = W.config_small(seed=30, dims=(4096, 9, 10), dtype=np.uint8, image=(4, 4),
                        op="sobel3d", ert=0.0, skip=True)
    sc.volume = W.blob_volume((10, 9, 4096), 300, seed=30, dtype=np.uint8, sigma=(2.0, 5.0),
                              centre_lo=0.0, centre_hi=1.0)
    sc.tf = W.tf_ramps(65536, seed=31, alpha_min=0.002, alpha_max=0.01, lo=0.08, hi=0.9)
    # rays along the long axis: about 8190 samples each
    along = {"projection": "ortho", "eye": (-50.0, 4.0, 4.5), "target": (0.0, 4.0, 4.5),
             "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 7.0, "width": 5,
             "height": 4}
    g = gpu_render(sc, cam=along)
    r = oracle_render(sc, cam=along)
    err, bad = compare(g["rgba"], r, 0.0)
    assert not bad.any(), err
    assert r["k_last"].max() > 8000 and (r["rgba"][..., 3] > 1e-6).sum() >= 10
    # a 16384 x 2 image across the long axis
    across = {"projection": "ortho", "eye": (2047.5, -60.0, 4.5), "target": (2047.5, 0.0, 4.5),
              "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 2.5, "width": 16384,
              "height": 2}
    g = gpu_render(sc, cam=across)
    pix = np.random.default_rng(30).choice(16384 * 2, 2000, replace=False)
    r = oracle_render(sc, cam=across, pixels=pix)
    err, bad = compare(g["rgba"].reshape(-1, 4)[pix], r, 0.0)
    assert not bad.any(), err
    assert (r["rgba"][:, 3] > 1e-6).sum() >= 100


def test_empty_clip_box_gives_black():
    sc = W.config_small(seed=19, dims=(12, 12, 12), image=(16, 16))
    opt = dict(sc.options, clip_lo=(8.0, 0.0, 0.0), clip_hi=(4.0, 20.0, 20.0))
    g = gpu_render(sc, options=opt)
    assert np.all(g["rgba"] == 0)


def test_allocation_failure_is_rc_e_oom():
    """A host-forcible failure: with the device memory taken by other
    allocations, rc_create_volume's bricked copy cannot be allocated and the
    call returns RC_E_OOM without creating a volume (the largest accepted
    volume, 2^31 voxels, is far smaller than the device, so only memory
    pressure reaches this status)."""
    src = torch.zeros((128, 512, 512), dtype=torch.float32, device="cuda")   # 128 MiB
    hold = []
    try:
        for chunk in (16 << 30, 1 << 30, 64 << 20):
            while True:
                try:
                    hold.append(torch.empty(chunk, dtype=torch.uint8, device="cuda"))
                except torch.OutOfMemoryError:
                    break
        with pytest.raises(rc.RCError) as e:
            rc.rc_create_volume(src, (1.0, 1.0, 1.0), 0.0, 1.0)
        assert e.value.status == rc.RC_E_OOM, str(e.value)
    finally:
        del hold
        torch.cuda.empty_cache()
    # and the library works again once memory is free
    vol = rc.rc_create_volume(src, (1.0, 1.0, 1.0), 0.0, 1.0)
    del vol


def test_error_statuses():
    sc = W.config_small(seed=20, dims=(12, 12, 12), image=(8, 8))
    vol = gpu_volume(sc, bricks=False)
    tf = to_dev(sc.tf)
    with pytest.raises(rc.RCError) as e:
        rc.rc_render(vol, sc.cameras[0], tf, sc.shading, dict(sc.options, skip_empty=True))
    assert e.value.status == rc.RC_E_STATE
    with pytest.raises(rc.RCError) as e:
        rc.rc_build_bricks(vol, 4)
    assert e.value.status == rc.RC_E_UNSUPPORTED
    with pytest.raises(rc.RCError) as e:
        rc.rc_render(vol, sc.cameras[0], tf, sc.shading, dict(sc.options, step=1e-9))
    assert e.value.status == rc.RC_E_INVALID
    with pytest.raises(rc.RCError) as e:
        rc.rc_render(vol, dict(sc.cameras[0], fov_y_deg=180.0), tf, sc.shading, sc.options)
    assert e.value.status == rc.RC_E_INVALID
    with pytest.raises(rc.RCError) as e:
        rc.rc_render(vol, sc.cameras[0], tf, dict(sc.shading, grad_eps=0.0), sc.options)
    assert e.value.status == rc.RC_E_INVALID
    with pytest.raises(rc.RCError) as e:
        rc.rc_render(vol, sc.cameras[0], tf, sc.shading, dict(sc.options, ref_step=-1.0))
    assert e.value.status == rc.RC_E_INVALID
    aux = rc.new_aux(sc.cameras[0])
    g = torch.zeros((8, 8, 4), device="cuda")
    with pytest.raises(rc.RCError) as e:
        rc.rc_render_backward(vol, sc.cameras[0], tf, sc.shading, sc.options, None, g)
    assert e.value.status == rc.RC_E_INVALID
    # every shading model is differentiated
    rc.rc_render(vol, sc.cameras[0], tf, sc.shading, sc.options, aux=aux)
    rc.rc_render_backward(vol, sc.cameras[0], tf, sc.shading, sc.options, aux, g)
