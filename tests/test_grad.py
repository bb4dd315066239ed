"""Reverse mode on the GPU vs the FP64 oracle adjoint and vs central finite
differences of the oracle's forward (bar: relative error 1e-3)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1609_01317_amd as rc
import workloads as W
from tests.gpu_util import to_dev

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


@pytest.mark.parametrize("seed,dtype,ert", [(31, np.float32, 0.0), (32, np.float32, 0.9),
                                             (33, np.uint8, 0.0), (34, np.uint16, 0.99)])
def test_adjoint_matches_oracle_small(seed, dtype, ert):
    sc = W.config_small(seed=seed, dims=(23, 19, 17), dtype=dtype, image=(35, 27),
                        shading="none", ert=ert)
    cam = sc.cameras[0]
    g = np.random.default_rng(seed).normal(size=(cam["height"], cam["width"], 4))
    gv, gt = _gpu_grads(sc, cam, g)
    dv, dt = oracle.render_grad(oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax), cam,
                                sc.tf, sc.options, g)
    print(f"seed {seed}: rel err volume {_rel(gv, dv):.2e} tf {_rel(gt, dt):.2e}", flush=True)
    assert _rel(gv, dv) <= REL and _rel(gt, dt) <= REL


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
        print(f"c5 view {vi}: rel err volume {_rel(gv, dv):.2e} tf {_rel(gt, dt):.2e}", flush=True)
        assert _rel(gv, dv) <= REL and _rel(gt, dt) <= REL


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
