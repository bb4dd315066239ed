"""Pins of the oracle's sampling variants: nearest-voxel sampling (the
simplest scheme of Section 3.3, coordinates rounded to whole voxels) and
opacity correction for the sample distance (off by default; the paper is
silent on it).

Closed forms on a constant slab, the step invariance that defines opacity
correction, nearest sampling reducing to the voxel at the rounded index,
and the independent brute-force formulation on tiny grids."""
import math

import numpy as np
import pytest

import workloads as W
from tests import bruteforce as BF


def _slab_cam(width=6, height=5):
    """Orthographic rays along +x through a 13x6x6 box (x extent 12 voxels)."""
    return {"projection": "ortho", "eye": (-40.0, 2.5, 2.5), "target": (0.0, 2.5, 2.5),
            "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 4.0, "width": width,
            "height": height}


def _flat_tf(a, rgb=(0.2, 0.5, 0.9)):
    tf = np.zeros((256, 4))
    tf[:, :3] = rgb
    tf[:, 3] = a
    return tf


@pytest.mark.parametrize("step,ref", [(0.5, 1.0), (0.25, 1.0), (1.0, 0.4), (0.3, 0.3)])
def test_opacity_correction_constant_slab(orc, step, ref):
    """Constant table alpha a over a 12-voxel slab: n = floor(12/step) + 1
    samples each of alpha 1 - (1-a)^(step/ref), so A = 1 - (1-a)^(n step/ref)
    and C = rgb A (shading NONE)."""
    a = 0.07
    vol = orc.Volume(np.full((6, 6, 13), 100.0), (1, 1, 1), 0.0, 255.0)
    opt = W.default_options(step, "central", ref_step=ref)
    res = orc.render(vol, _slab_cam(), _flat_tf(a), W.default_shading("none"), opt)
    n = math.floor(12.0 / step + 1e-9) + 1
    want = 1.0 - (1.0 - a) ** (n * step / ref)
    ok = (res["flags"] & 2) == 0
    np.testing.assert_allclose(res["rgba"][..., 3][ok], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(res["rgba"][..., 0][ok], 0.2 * want, rtol=0, atol=1e-12)


def test_opacity_correction_makes_opacity_step_invariant(orc):
    """Halving the step doubles the sample count; with correction the opacity
    of the same slab length stays the same (to the lattice's end sample),
    without it the opacity grows."""
    a = 0.05
    vol = orc.Volume(np.full((6, 6, 13), 100.0), (1, 1, 1), 0.0, 255.0)
    cam, sh = _slab_cam(), W.default_shading("none")
    A = {}
    for step in (0.5, 0.25, 0.125):
        for ref in (0.0, 1.0):
            r = orc.render(vol, cam, _flat_tf(a), sh, W.default_options(step, ref_step=ref))
            A[step, ref] = float(np.median(r["rgba"][..., 3]))
    phys = 1.0 - (1.0 - a) ** 12.0                       # 12 voxels at one sample per voxel
    for step in (0.5, 0.25, 0.125):
        # n steps cover 12 + step: the extra end sample adds step/ref of absorption
        assert abs(A[step, 1.0] - (1.0 - (1.0 - a) ** (12.0 + step))) < 1e-12
        assert abs(A[step, 1.0] - phys) < 0.05 * step
    assert A[0.125, 0.0] > A[0.25, 0.0] > A[0.5, 0.0] > A[0.5, 1.0]


def test_opacity_correction_keeps_zero_and_one(orc):
    """alpha 0 stays exactly 0 (so skipping stays lossless), alpha 1 stays 1."""
    vol = orc.Volume(np.full((6, 6, 13), 100.0), (1, 1, 1), 0.0, 255.0)
    sh = W.default_shading("none")
    for a, want in ((0.0, 0.0), (1.0, 1.0)):
        r = orc.render(vol, _slab_cam(), _flat_tf(a), sh, W.default_options(0.37, ref_step=0.9))
        assert np.all(r["rgba"][..., 3] == want)


def test_nearest_sample_is_the_rounded_voxel(orc):
    rng = np.random.default_rng(3)
    arr = rng.integers(0, 4096, (5, 6, 7)).astype(np.float64)
    vol = orc.Volume(arr, (1, 1, 1), 0.0, 4095.0)
    for _ in range(300):
        p = rng.uniform(-1.0, 8.0, 3)
        i, j, k = (min(max(int(math.floor(c + 0.5)), 0), n - 1) for c, n in zip(p, (7, 6, 5)))
        assert orc.sample_nearest(vol, p) == arr[k, j, i]
    # exactly halfway rounds up
    assert orc.sample_nearest(vol, np.array([1.5, 2.0, 3.0])) == arr[3, 2, 2]


def test_nearest_column_closed_form(orc):
    """Axis-aligned orthographic ray along a voxel row, step 0.5 from x = 0:
    sample k lands on x = k/2 and reads voxel floor(k/2 + 1/2).  With a table
    alpha proportional to the value, shading NONE and rgb = 1, the opacity is
    1 - prod_k (1 - a(V[round(k/2)]))."""
    rng = np.random.default_rng(8)
    row = rng.integers(0, 256, 9).astype(np.float64)
    arr = np.zeros((3, 3, 9))
    arr[:, :, :] = row
    vol = orc.Volume(arr, (1, 1, 1), 0.0, 255.0)
    tf = np.zeros((256, 4))
    tf[:, :3] = 1.0
    tf[:, 3] = np.arange(256) / 255.0 * 0.2
    cam = {"projection": "ortho", "eye": (-10.0, 1.0, 1.0), "target": (0.0, 1.0, 1.0),
           "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 0.5, "width": 1,
           "height": 1}
    r = orc.render(vol, cam, tf, W.default_shading("none"), W.default_options(0.5, nearest=True))
    T = 1.0
    for k in range(17):                      # x = 0, 0.5, ..., 8
        T *= 1.0 - 0.2 * row[min(int(math.floor(k / 2 + 0.5)), 8)] / 255.0
    assert abs(r["rgba"].reshape(4)[3] - (1.0 - T)) < 1e-12


CASES = [
    dict(op="central", shading="blinn_phong", projection="persp", nearest=True, ref=0.0),
    dict(op="sobel3d", shading="paper_lambert", projection="ortho", nearest=True, ref=0.6),
    dict(op="zucker_hummel", shading="blinn_phong", projection="persp", nearest=False, ref=0.25),
    dict(op="sobel3d", shading="none", projection="persp", nearest=True, ref=1.3),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [31, 32])
def test_variants_match_bruteforce_on_4cubed(orc, case, seed):
    rng = np.random.default_rng(seed)
    arr = rng.integers(0, 256, (4, 4, 4)).astype(np.uint8)
    tf = W.tf_ramps(256, seed=seed, alpha_max=0.6)
    cam = W.orbit_camera((4, 4, 4), (1, 1, 1), rng.uniform(0, 360), rng.uniform(-60, 60), 9, 7,
                         projection=case["projection"])
    sh = W.default_shading(case["shading"], light=(0.3, -0.7, 0.5),
                           light_is_point=case["shading"] == "paper_lambert")
    if sh["light_is_point"]:
        sh["light"] = (10.0, -6.0, 8.0)
    opt = W.default_options(0.37, case["op"], 0.0, nearest=case["nearest"], ref_step=case["ref"])
    res = orc.render(orc.Volume(arr, (1, 1, 1), 0, 255), cam, tf, sh, opt)
    bf = BF.render(arr, (1, 1, 1), 0, 255, tf, cam, sh, opt)
    got, alt = res["rgba"].reshape(-1, 4), res["rgba_alt"].reshape(-1, 4)
    ok = np.all(np.abs(got - bf) < 1e-9, axis=1) | np.all(np.abs(alt - bf) < 1e-9, axis=1)
    assert ok.all(), np.abs(got - bf).max()
    assert (res["flags"] & 1).sum() > 10
