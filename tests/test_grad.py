"""Reverse mode on the GPU vs the FP64 oracle adjoint and vs central finite
differences of the oracle's forward (bar: relative error 1e-3 per element,
|gpu - ref| <= 1e-3 |ref| + 1e-5 max|ref|)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1609_01317_amd as rc
import workloads as W
from tests.gpu_util import grad_excess, to_dev

pytestmark = pytest.mark.gpu

REL = 1e-3


def _gpu_grads(sc, cam, g, vol=None, tf=None):
    vol_t = to_dev(sc.volume if vol is None else vol)
    h = rc.rc_create_volume(vol_t, sc.spacing, sc.vmin, sc.vmax)
    tf_t = to_dev(sc.tf if tf is None else tf)
    aux = rc.new_aux(cam)
    rc.rc_render(h, cam, tf_t, sc.shading, sc.options, aux=aux)
    gv, gt = rc.rc_render_backward(h, cam, tf_t, sc.shading, sc.options, aux,
                                   to_dev(g.astype(np.float32)))
    torch.cuda.synchronize()
    return gv.cpu().numpy().astype(np.float64), gt.cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def _ok(gv, dv, gt, dt, label):
    """Per-element bar on both gradients; prints the worst ratios."""
    xv, rv = grad_excess(gv, dv)
    xt, rt = grad_excess(gt, dt)
    print(f"{label}: volume worst per-element ratio {xv:.3f} (max-normalised {rv:.2e}), "
          f"tf {xt:.3f} ({rt:.2e})", flush=True)
    return xv <= 1.0 and xt <= 1.0


@pytest.mark.parametrize("seed,dtype,ert,nearest,ref",
                         [(31, np.float32, 0.0, False, 0.0), (32, np.float32, 0.9, False, 0.0),
                          (33, np.uint8, 0.0, False, 0.0), (34, np.uint16, 0.99, False, 0.0),
                          (35, np.float32, 0.0, True, 0.0), (36, np.float32, 0.8, False, 0.35),
                          (37, np.uint16, 0.0, True, 1.7)])
def test_adjoint_matches_oracle_small(seed, dtype, ert, nearest, ref):
    """Also with nearest sampling and with opacity correction."""
    sc = W.config_small(seed=seed, dims=(23, 19, 17), dtype=dtype, image=(35, 27),
                        shading="none", ert=ert)
    sc.options.update(nearest=nearest, ref_step=ref)
    cam = sc.cameras[0]
    g = np.random.default_rng(seed).normal(size=(cam["height"], cam["width"], 4))
    gv, gt = _gpu_grads(sc, cam, g)
    dv, dt = oracle.render_grad(oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax), cam,
                                sc.tf, sc.options, g)
    assert np.abs(dv).max() > 0 and np.abs(dt).max() > 0      # not a blank scene
    assert _ok(gv, dv, gt, dt, f"seed {seed}")


@pytest.mark.parametrize("tf_len", [1024, 1025, 4096, 4097])
def test_adjoint_table_sizes(tf_len):
    """Table lengths on both sides of the two shared-memory limits of the
    adjoint kernel: the table is read from an LDS copy up to 1024 entries and
    its gradient summed in LDS (shared by a block's waves) up to 4096, in
    global memory beyond."""
    sc = W.config_small(seed=38, dims=(23, 19, 17), dtype=np.float32, image=(35, 27),
                        shading="none")
    tf = W.tf_ramps(tf_len, seed=38, alpha_max=0.3)
    cam = sc.cameras[0]
    g = np.random.default_rng(38).normal(size=(cam["height"], cam["width"], 4))
    gv, gt = _gpu_grads(sc, cam, g, tf=tf)
    dv, dt = oracle.render_grad(oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax), cam,
                                tf, sc.options, g)
    assert np.abs(dv).max() > 0 and np.count_nonzero(dt) > 100
    assert _ok(gv, dv, gt, dt, f"M {tf_len}")


SHADED = [
    dict(seed=51, dtype=np.float32, op="central", shading="blinn_phong", nearest=False, ert=0.0),
    dict(seed=52, dtype=np.uint16, op="sobel3d", shading="blinn_phong", nearest=False, ert=0.95),
    dict(seed=53, dtype=np.uint8, op="zucker_hummel", shading="paper_lambert", nearest=False,
         ert=0.0),
    dict(seed=54, dtype=np.float32, op="sobel3d", shading="paper_lambert", nearest=True, ert=0.0),
]


@pytest.mark.parametrize("case", SHADED, ids=lambda c: f"s{c['seed']}")
def test_shaded_adjoint_matches_oracle(case):
    """Reverse mode through Blinn-Phong / the paper's Lambert term, the |G|
    normalisation and the operator's taps, vs the FP64 adjoint."""
    sc = W.config_small(seed=case["seed"], dims=(21, 18, 16), dtype=case["dtype"], image=(31, 25),
                        op=case["op"], shading=case["shading"], ert=case["ert"])
    if case["shading"] == "paper_lambert":
        sc.shading["light_is_point"] = True
        sc.shading["light"] = (40.0, -30.0, 35.0)
    sc.options.update(nearest=case["nearest"])
    cam = sc.cameras[0]
    g = np.random.default_rng(case["seed"]).normal(size=(cam["height"], cam["width"], 4))
    vol_t = to_dev(sc.volume)
    h = rc.rc_create_volume(vol_t, sc.spacing, sc.vmin, sc.vmax)
    tf_t = to_dev(sc.tf)
    aux = rc.new_aux(cam)
    rc.rc_render(h, cam, tf_t, sc.shading, sc.options, aux=aux)
    gv, gt = rc.rc_render_backward(h, cam, tf_t, sc.shading, sc.options, aux,
                                   to_dev(g.astype(np.float32)))
    torch.cuda.synchronize()
    gv, gt = gv.cpu().numpy().astype(np.float64), gt.cpu().numpy().astype(np.float64)
    dv, dt = oracle.render_grad(oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax), cam,
                                sc.tf, sc.options, g, shading=sc.shading)
    assert np.abs(dv).max() > 0 and np.abs(dt).max() > 0
    assert _ok(gv, dv, gt, dt, f"seed {case['seed']}")


def test_autograd_function_matches_direct_calls():
    sc = W.config_small(seed=35, dims=(16, 16, 16), dtype=np.float32, image=(24, 24),
                        shading="none")
    cam = sc.cameras[0]
    v = to_dev(sc.volume)
    h = rc.rc_create_volume(v, sc.spacing, sc.vmin, sc.vmax)
    vp = v.clone().requires_grad_(True)
    tp = to_dev(sc.tf).requires_grad_(True)
    out = rc.RenderFn.apply(vp, tp, h, cam, sc.shading, sc.options)
    g = torch.randn_like(out)
    (out * g).sum().backward()
    gv, gt = _gpu_grads(sc, cam, g.cpu().numpy())
    np.testing.assert_allclose(vp.grad.cpu().numpy(), gv, rtol=0, atol=1e-5 * np.abs(gv).max())
    np.testing.assert_allclose(tp.grad.cpu().numpy(), gt, rtol=0, atol=1e-5 * np.abs(gt).max())


@pytest.fixture(scope="module")
def c5():
    return W.config_c5()


def test_c5_views_match_oracle_adjoint(c5):
    """128^3 f32 density, 256^2 views, L2 loss against a target rendered from
    the seed-55 volume: GPU adjoint vs FP64 adjoint on two views."""
    sc = c5
    for vi in (0, 5):
        cam = sc.cameras[vi]
        target = oracle.render(oracle.Volume(sc.extra["target_volume"], sc.spacing, 0, 1), cam,
                               sc.tf, sc.shading, sc.options)["rgba"]
        cur = oracle.render(oracle.Volume(sc.volume, sc.spacing, 0, 1), cam, sc.tf, sc.shading,
                            sc.options)["rgba"]
        g = 2.0 * (cur - target)                       # dL/drgba of sum (rgba - target)^2
        gv, gt = _gpu_grads(sc, cam, g)
        dv, dt = oracle.render_grad(oracle.Volume(sc.volume, sc.spacing, 0, 1), cam, sc.tf,
                                    sc.options, g)
        assert _ok(gv, dv, gt, dt, f"c5 view {vi}")


def _project(cam, p):
    """Pixel coordinates of world point p for a perspective camera."""
    eye = np.array(cam["eye"])
    f = np.array(cam["target"]) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, cam["up"])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    q = p - eye
    z = q @ f
    th = math.tan(math.radians(cam["fov_y_deg"]) / 2)
    x = (q @ r) / z / (th * cam["width"] / cam["height"])
    y = (q @ u) / z / th
    return (x + 1) / 2 * cam["width"] - 0.5, (1 - y) / 2 * cam["height"] - 0.5


def test_c5_crop_matches_finite_differences(c5):
    """Central differences (FP64 oracle forward, h = 1e-4) for voxels of the
    central 24^3 crop, over the pixels whose rays pass near the voxel;
    voxels whose FD is one-sided (a TF breakpoint inside [v-h, v+h]) are
    skipped."""
    sc = c5
    cam = sc.cameras[0]
    H, Wd = cam["height"], cam["width"]
    rng = np.random.default_rng(505)
    g = rng.normal(size=(H, Wd, 4))
    gv, _ = _gpu_grads(sc, cam, g)
    lo = 64 - 12
    crop = gv[lo:lo + 24, lo:lo + 24, lo:lo + 24]
    cand = np.argwhere(np.abs(crop) > 1e-3 * np.abs(crop).max())
    assert len(cand) > 100
    vol = sc.volume.astype(np.float64)
    h = 1e-4
    checked = 0
    for idx in cand[rng.choice(len(cand), size=40, replace=False)]:
        k, j, i = idx + lo
        px, py = _project(cam, np.array([i, j, k], dtype=float))
        xs = np.arange(max(0, int(px) - 4), min(Wd, int(px) + 6))
        ys = np.arange(max(0, int(py) - 4), min(H, int(py) + 6))
        pix = (ys[:, None] * Wd + xs[None, :]).ravel()
        gp = g.reshape(-1, 4)[pix]

        def loss(delta):
            v2 = vol.copy()
            v2[k, j, i] += delta
            r = oracle.render(oracle.Volume(v2, sc.spacing, 0, 1), cam, sc.tf, sc.shading,
                              sc.options, pixels=pix)
            return float((r["rgba"] * gp).sum())

        l0, lp, lm = loss(0.0), loss(h), loss(-h)
        fd, fl, fr = (lp - lm) / (2 * h), (l0 - lm) / h, (lp - l0) / h
        if abs(fl - fr) > 1e-3 * max(abs(fd), 1e-8):
            continue
        checked += 1
        assert abs(fd - gv[k, j, i]) <= REL * max(abs(fd), np.abs(crop).max() * 1e-2), \
            (idx, fd, gv[k, j, i])
    print(f"c5 FD: {checked} voxels checked", flush=True)
    assert checked >= 20


# ---------------------------------------------------------------- several views, one launch
def _views_scene(n_views, seed=61, image=(40, 36), dtype=np.float32, shading="none",
                 op="central"):
    sc = W.config_small(seed=seed, dims=(21, 19, 17), dtype=dtype, image=image,
                        shading=shading, op=op)
    cams = [W.orbit_camera((21, 19, 17), sc.spacing, 17.0 * i, 25.0 - 3 * i, image[0], image[1])
            for i in range(n_views)]
    return sc, cams


@pytest.mark.parametrize("seed,dtype,op,shading,n_views,skip",
                         [(62, np.uint16, "sobel3d", "blinn_phong", 20, True),
                          (64, np.uint8, "central", "paper_lambert", 33, False),
                          (65, np.float32, "zucker_hummel", "none", 17, True),
                          (66, np.float32, "central", "blinn_phong", 1, True)])
def test_render_views_equals_single_renders(seed, dtype, op, shading, n_views, skip):
    """Views in launches of at most 16 (the item scratch reused across
    launches), mixed image sizes, every box budget and the unshaded kinds:
    bit-identical to one rc_render per view, aux included."""
    sc = W.config_small(seed=seed, dims=(30, 26, 22), dtype=dtype, image=(37, 29), op=op,
                        shading=shading, ert=0.95, skip=skip)
    cams = [W.orbit_camera((30, 26, 22), sc.spacing, 18.0 * i, 30.0 - 4 * (i % 15), 24 + 8 * (i % 3),
                           16 + 8 * (i % 4)) for i in range(n_views)]
    vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
    rc.rc_build_bricks(vol, 8)
    tf = to_dev(sc.tf)
    auxes = [rc.new_aux(c) for c in cams]
    outs = rc.rc_render_views(vol, cams, tf, sc.shading, sc.options, auxes=auxes)
    for c, o, a in zip(cams, outs, auxes):
        a1 = rc.new_aux(c)
        ref = rc.rc_render(vol, c, tf, sc.shading, sc.options, aux=a1)
        torch.cuda.synchronize()
        assert torch.equal(o, ref) and torch.equal(a, a1)


@pytest.mark.parametrize("dtype,shading,op", [(np.float32, "none", "central"),
                                              (np.uint16, "none", "central"),
                                              (np.uint8, "blinn_phong", "sobel3d")])
def test_backward_views_equals_sum_of_single_views(dtype, shading, op):
    """18 views: two reverse launches of at most 16 views each (the tile
    counter zeroed before each), against one rc_render_backward per view:
    unshaded with a 256-entry table (its LDS copy) and with the 4096-entry
    table of u16 volumes (read from memory), and shaded."""
    sc, cams = _views_scene(18, dtype=dtype, shading=shading, op=op)
    vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
    tf = to_dev(sc.tf)
    auxes = [rc.new_aux(c) for c in cams]
    rc.rc_render_views(vol, cams, tf, sc.shading, sc.options, auxes=auxes)
    gen = torch.Generator(device="cuda").manual_seed(7)
    grads = [torch.randn((c["height"], c["width"], 4), device="cuda", generator=gen) for c in cams]
    gv, gt = rc.rc_render_backward_views(vol, cams, tf, sc.shading, sc.options, auxes, grads)
    gv1 = torch.zeros_like(gv)
    gt1 = torch.zeros_like(gt)
    for c, a, g in zip(cams, auxes, grads):
        rc.rc_render_backward(vol, c, tf, sc.shading, sc.options, a, g, gv1, gt1)
    torch.cuda.synchronize()
    a, b = gv.cpu().numpy().astype(np.float64), gv1.cpu().numpy().astype(np.float64)
    c, d = gt.cpu().numpy().astype(np.float64), gt1.cpu().numpy().astype(np.float64)
    assert np.abs(b).max() > 0 and np.abs(d).max() > 0
    assert _rel(a, b) <= 1e-5 and _rel(c, d) <= 1e-5
    assert _ok(a, b, c, d, "views vs single")


def test_backward_views_of_mixed_sizes():
    """Five shaded views of different image sizes (tile counts 1 .. 30, ragged
    edges) in one reverse launch: the tiles of all views come from one counter
    and map back to their view; equal to one rc_render_backward per view."""
    sc = W.config_small(seed=67, dims=(26, 22, 19), dtype=np.uint16, image=(40, 36),
                        op="zucker_hummel", shading="blinn_phong", ert=0.9, skip=True)
    sizes = [(8, 8), (41, 37), (17, 50), (64, 24), (3, 5)]
    cams = [W.orbit_camera((26, 22, 19), sc.spacing, 23.0 * i + 5.0, 20.0 - 6 * i, w, h)
            for i, (w, h) in enumerate(sizes)]
    vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
    rc.rc_build_bricks(vol, 8)
    tf = to_dev(sc.tf)
    auxes = [rc.new_aux(c) for c in cams]
    rc.rc_render_views(vol, cams, tf, sc.shading, sc.options, auxes=auxes)
    gen = torch.Generator(device="cuda").manual_seed(11)
    grads = [torch.randn((c["height"], c["width"], 4), device="cuda", generator=gen) for c in cams]
    gv, gt = rc.rc_render_backward_views(vol, cams, tf, sc.shading, sc.options, auxes, grads)
    gv1 = torch.zeros_like(gv)
    gt1 = torch.zeros_like(gt)
    for c, a, g in zip(cams, auxes, grads):
        rc.rc_render_backward(vol, c, tf, sc.shading, sc.options, a, g, gv1, gt1)
    torch.cuda.synchronize()
    a, b = gv.cpu().numpy().astype(np.float64), gv1.cpu().numpy().astype(np.float64)
    c, d = gt.cpu().numpy().astype(np.float64), gt1.cpu().numpy().astype(np.float64)
    assert np.abs(b).max() > 0 and np.abs(d).max() > 0
    assert _ok(a, b, c, d, "mixed sizes")


def test_render_views_fn_matches_oracle():
    """Two views through the multi-view autograd function vs the FP64 adjoint."""
    sc, cams = _views_scene(2, seed=63)
    v = to_dev(sc.volume)
    h = rc.rc_create_volume(v, sc.spacing, sc.vmin, sc.vmax)
    vp = v.clone().requires_grad_(True)
    tp = to_dev(sc.tf).requires_grad_(True)
    out = rc.RenderViewsFn.apply(vp, tp, h, cams, sc.shading, sc.options)
    rng = np.random.default_rng(63)
    g = rng.normal(size=tuple(out.shape))
    (out * torch.from_numpy(g).float().cuda()).sum().backward()
    ov = oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    dv = np.zeros(sc.volume.shape)
    dt = np.zeros(sc.tf.shape)
    for i, c in enumerate(cams):
        r = oracle.render(ov, c, sc.tf, sc.shading, sc.options)
        err = np.abs(out[i].detach().cpu().numpy() - r["rgba"]).max()
        assert err <= 2e-4, err
        a, b = oracle.render_grad(ov, c, sc.tf, sc.options, g[i])
        dv += a
        dt += b
    assert _ok(vp.grad.cpu().numpy(), dv, tp.grad.cpu().numpy(), dt, "views fn")


def test_c3_full_size_shaded_adjoint_sampled():
    """Forward + backward at the benchmark's size: the 512^3 u16 phantom at
    1024^2 with Sobel3D and Blinn-Phong (step 0.5, ERT 0.99), two orbit
    views in one reverse launch.  dL/d(rgba) is seeded on 1500 pixels per
    view and zero elsewhere, so dL/dvolume and dL/dtable come from those rays
    only; both are compared per element with the FP64 oracle adjoint of the
    same pixels."""
    sc = W.config_c3(n_views=36)
    opt = dict(sc.options, gradient_op="sobel3d")
    vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
    rc.rc_build_bricks(vol, 8)
    tf = to_dev(sc.tf)
    cams = [sc.cameras[4], sc.cameras[22]]
    rng = np.random.default_rng(606)
    n_pix = 1024 * 1024
    auxes = [rc.new_aux(c) for c in cams]
    rc.rc_render_views(vol, cams, tf, sc.shading, opt, auxes=auxes)
    grads, pix, gsub = [], [], []
    for _ in cams:
        p = rng.choice(n_pix, size=1500, replace=False)
        g = np.zeros((n_pix, 4), dtype=np.float32)
        g[p] = rng.normal(size=(1500, 4)).astype(np.float32)
        grads.append(torch.from_numpy(g.reshape(1024, 1024, 4)).cuda())
        pix.append(p)
        gsub.append(g[p].astype(np.float64))
    gv, gt = rc.rc_render_backward_views(vol, cams, tf, sc.shading, opt, auxes, grads)
    torch.cuda.synchronize()
    gv = gv.cpu().numpy()
    gt = gt.cpu().numpy()
    del vol
    ov = oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    dv = np.zeros(sc.volume.shape)
    dt = np.zeros(sc.tf.shape)
    for c, p, g in zip(cams, pix, gsub):
        a, b = oracle.render_grad(ov, c, sc.tf, opt, g, pixels=p, shading=sc.shading)
        dv += a
        dt += b
    del ov
    nz = int((dv != 0).sum())
    print(f"c3 shaded adjoint: {nz} voxels with a gradient", flush=True)
    assert nz > 10000 and np.count_nonzero(dt) > 50
    assert _ok(gv, dv, gt, dt, "c3 shaded adjoint")
