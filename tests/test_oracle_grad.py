"""Pins of the oracle's reverse mode (shading NONE) against central finite
differences of the oracle's forward render, which the other pin files tie
to the paper.  Loss: L = sum(g * rgba) with a fixed random g."""
import numpy as np
import pytest

import workloads as W


def _scene(seed, ert=0.0, nearest=False, ref_step=0.0):
    sc = W.config_small(seed=seed, dims=(7, 6, 8), dtype=np.float32, image=(9, 8),
                        shading="none", ert=ert)
    sc.options.update(nearest=nearest, ref_step=ref_step)
    return sc


def _loss(orc, vol_arr, sc, tf, g):
    v = orc.Volume(vol_arr, sc.spacing, sc.vmin, sc.vmax)
    r = orc.render(v, sc.cameras[0], tf, sc.shading, sc.options)
    return float((r["rgba"] * g).sum())


VARIANTS = [dict(), dict(nearest=True), dict(ref_step=0.8), dict(nearest=True, ref_step=0.3)]


@pytest.mark.parametrize("seed,ert,var", [(21, 0.0, 0), (22, 0.0, 0), (23, 0.8, 0), (26, 0.0, 1),
                                          (27, 0.0, 2), (28, 0.7, 3)])
def test_grad_tf_matches_fd(orc, seed, ert, var):
    """dL/dTF: C is linear in the rgb entries, so their FD is exact up to
    rounding; the alpha entries are smooth away from ERT decisions.  Also
    with nearest sampling and with opacity correction."""
    sc = _scene(seed, ert, **VARIANTS[var])
    rng = np.random.default_rng(seed)
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    g = rng.normal(size=(H, Wd, 4))
    v = orc.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    _, dtf = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g)
    tf = sc.tf.astype(np.float64)
    used = np.argwhere(np.abs(dtf).sum(1) > 0)[:, 0]
    assert used.size > 5
    h = 1e-6
    for i in rng.choice(used, size=min(12, used.size), replace=False):
        for ch in range(4):
            tp, tm = tf.copy(), tf.copy()
            tp[i, ch] += h
            tm[i, ch] -= h
            fd = (_loss(orc, sc.volume, sc, tp, g) - _loss(orc, sc.volume, sc, tm, g)) / (2 * h)
            assert abs(fd - dtf[i, ch]) <= 1e-6 * max(1.0, abs(fd)), (i, ch, fd, dtf[i, ch])


@pytest.mark.parametrize("seed,var", [(24, 0), (25, 0), (29, 1), (30, 2), (31, 3)])
def test_grad_volume_matches_fd(orc, seed, var):
    sc = _scene(seed, **VARIANTS[var])
    rng = np.random.default_rng(seed)
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    g = rng.normal(size=(H, Wd, 4))
    vol = sc.volume.astype(np.float64)
    v = orc.Volume(vol, sc.spacing, sc.vmin, sc.vmax)
    dvol, _ = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g)
    cand = np.argwhere(np.abs(dvol) > 1e-6)
    assert len(cand) > 10
    h = 1e-6
    checked = 0
    for idx in cand[rng.choice(len(cand), size=min(25, len(cand)), replace=False)]:
        k, j, i = idx
        vp, vm = vol.copy(), vol.copy()
        vp[k, j, i] += h
        vm[k, j, i] -= h
        fd = (_loss(orc, vp, sc, sc.tf, g) - _loss(orc, vm, sc, sc.tf, g)) / (2 * h)
        # a TF breakpoint inside [v-h, v+h] makes the FD one-sided: skip those
        fd_l = (_loss(orc, vol, sc, sc.tf, g) - _loss(orc, vm, sc, sc.tf, g)) / h
        fd_r = (_loss(orc, vp, sc, sc.tf, g) - _loss(orc, vol, sc, sc.tf, g)) / h
        if abs(fd_l - fd_r) > 1e-4 * max(1.0, abs(fd)):
            continue
        checked += 1
        assert abs(fd - dvol[k, j, i]) <= 1e-5 * max(1.0, abs(fd)), (idx, fd, dvol[k, j, i])
    assert checked >= 10


SHADED = [("blinn_phong", "central", False), ("blinn_phong", "sobel3d", False),
          ("paper_lambert", "zucker_hummel", False), ("blinn_phong", "zucker_hummel", True),
          ("paper_lambert", "central", True)]


def _shaded_scene(seed, model, op, nearest):
    sc = W.config_small(seed=seed, dims=(7, 6, 8), dtype=np.float32, image=(9, 8), op=op,
                        shading=model, ert=0.0)
    if model == "paper_lambert":
        sc.shading["light_is_point"] = True
        sc.shading["light"] = (14.0, -9.0, 11.0)
    sc.options.update(nearest=nearest)
    return sc


def _loss_sh(orc, vol_arr, sc, tf, g):
    v = orc.Volume(vol_arr, sc.spacing, sc.vmin, sc.vmax)
    r = orc.render(v, sc.cameras[0], tf, sc.shading, sc.options)
    return float((r["rgba"] * g).sum())


@pytest.mark.parametrize("model,op,nearest", SHADED)
def test_shaded_grad_volume_matches_fd(orc, model, op, nearest):
    """Reverse mode through the lighting, the |G| normalisation and the
    gradient operator's taps vs central differences of the forward."""
    seed = 40 + SHADED.index((model, op, nearest))
    sc = _shaded_scene(seed, model, op, nearest)
    rng = np.random.default_rng(seed)
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    g = rng.normal(size=(H, Wd, 4))
    vol = sc.volume.astype(np.float64)
    v = orc.Volume(vol, sc.spacing, sc.vmin, sc.vmax)
    dvol, _ = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g, shading=sc.shading)
    cand = np.argwhere(np.abs(dvol) > 1e-6)
    assert len(cand) > 10
    h = 1e-6
    checked = 0
    for idx in cand[rng.choice(len(cand), size=min(30, len(cand)), replace=False)]:
        k, j, i = idx
        vp, vm = vol.copy(), vol.copy()
        vp[k, j, i] += h
        vm[k, j, i] -= h
        l0 = _loss_sh(orc, vol, sc, sc.tf, g)
        lp, lm = _loss_sh(orc, vp, sc, sc.tf, g), _loss_sh(orc, vm, sc, sc.tf, g)
        fd, fl, fr = (lp - lm) / (2 * h), (l0 - lm) / h, (lp - l0) / h
        if abs(fl - fr) > 1e-4 * max(1.0, abs(fd)):
            continue                      # a kink (TF breakpoint, max(0,.)) inside [v-h, v+h]
        checked += 1
        assert abs(fd - dvol[k, j, i]) <= 1e-5 * max(1.0, abs(fd)), (idx, fd, dvol[k, j, i])
    assert checked >= 10


@pytest.mark.parametrize("model,op,nearest", SHADED[:3])
def test_shaded_grad_tf_matches_fd(orc, model, op, nearest):
    seed = 50 + SHADED.index((model, op, nearest))
    sc = _shaded_scene(seed, model, op, nearest)
    rng = np.random.default_rng(seed)
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    g = rng.normal(size=(H, Wd, 4))
    v = orc.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    _, dtf = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g, shading=sc.shading)
    tf = sc.tf.astype(np.float64)
    used = np.argwhere(np.abs(dtf).sum(1) > 0)[:, 0]
    assert used.size > 5
    h = 1e-6
    for i in rng.choice(used, size=min(10, used.size), replace=False):
        for ch in range(4):
            tp, tm = tf.copy(), tf.copy()
            tp[i, ch] += h
            tm[i, ch] -= h
            fd = (_loss_sh(orc, sc.volume, sc, tp, g) - _loss_sh(orc, sc.volume, sc, tm, g)) / (2 * h)
            assert abs(fd - dtf[i, ch]) <= 1e-6 * max(1.0, abs(fd)), (i, ch, fd, dtf[i, ch])


def test_abs_sum_is_the_sum_of_term_magnitudes(orc):
    """The oracle's optional cancellation measure: per voxel, the sum of the
    magnitudes of the terms added into dL/dvolume.  It leaves dL/dvolume
    unchanged, bounds |dL/dvolume|, adds up over pixels (a sum of
    magnitudes, not the magnitude of a sum: some voxels cancel), is even in
    g and scales with |g|."""
    sc = W.config_small(seed=32, dims=(9, 8, 7), dtype=np.uint8, image=(6, 5), op="sobel3d")
    rng = np.random.default_rng(32)
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    g = rng.normal(size=(H * Wd, 4))
    v = orc.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    dv0, dt0 = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g, shading=sc.shading)
    dv, dt, ab = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g, shading=sc.shading,
                                 abs_sum=True)
    assert np.array_equal(dv, dv0) and np.array_equal(dt, dt0)
    assert (ab >= np.abs(dv) * (1 - 1e-12)).all()
    assert (ab[dv != 0] > 0).all() and (ab > 2 * np.abs(dv) + 1e-12).any()
    per_pixel = np.zeros_like(ab)
    for p in range(H * Wd):
        _, _, a = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, g[p:p + 1], pixels=[p],
                                  shading=sc.shading, abs_sum=True)
        per_pixel += a
    assert np.allclose(per_pixel, ab, rtol=1e-12, atol=0)
    _, _, a_neg = orc.render_grad(v, sc.cameras[0], sc.tf, sc.options, -2.0 * g,
                                  shading=sc.shading, abs_sum=True)
    assert np.allclose(a_neg, 2.0 * ab, rtol=1e-12, atol=0)
