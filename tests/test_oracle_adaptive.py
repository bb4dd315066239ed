"""Pins of the oracle's adaptive sampling (Section 5.2: detail-poor regions
sampled at a lower rate): reduction to the fixed-step march, the constant
slab's closed form at every factor, and an independent formulation on
small grids with homogeneous and detailed bricks."""
import math

import numpy as np
import pytest

import workloads as W
from tests import bruteforce as BF


def _flat_tf(a, rgb=(0.2, 0.5, 0.9)):
    tf = np.zeros((256, 4))
    tf[:, :3] = rgb
    tf[:, 3] = a
    return tf


def _cam_x(width=6, height=5):
    """Orthographic rays along +x through a 33x6x6 box (x extent 32 voxels)."""
    return {"projection": "ortho", "eye": (-40.0, 2.5, 2.5), "target": (0.0, 2.5, 2.5),
            "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 4.0, "width": width,
            "height": height}


@pytest.mark.parametrize("m", [2, 3, 4])
def test_constant_slab_closed_form(orc, m):
    """Every brick of a constant volume is detail-poor: samples at t_in + j m
    step, each standing for m steps, so A = 1 - (1-a)^(m n) with
    n = floor(32 / (m step)) + 1, and C = rgb A."""
    a, step = 0.03, 0.5
    vol = orc.Volume(np.full((6, 6, 33), 100.0), (1, 1, 1), 0.0, 255.0)
    opt = W.default_options(step, adapt_factor=m, adapt_range=0.0)
    r = orc.render(vol, _cam_x(), _flat_tf(a), W.default_shading("none"), opt)
    # the slab length is a multiple of m step: the last sample sits on the exit
    # plane (a tie, flagged); the primary result takes it
    n = math.floor(32.0 / (m * step) + 1e-9) + 1
    want = 1.0 - (1.0 - a) ** (m * n)
    np.testing.assert_allclose(r["rgba"][..., 3], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["rgba"][..., 2], 0.9 * want, rtol=0, atol=1e-12)
    assert np.all(r["k_last"] == n - 1)
    tie = (r["flags"] & 2) != 0
    assert tie.all() == (32.0 / (m * step) == n - 1)
    np.testing.assert_allclose(r["rgba_alt"][..., 3][tie], 1.0 - (1.0 - a) ** (m * (n - 1)),
                               atol=1e-12)


def test_no_poor_brick_is_the_fixed_step_march(orc):
    sc = W.config_small(seed=71, dims=(20, 18, 17), image=(21, 17), op="sobel3d")
    v = orc.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    plain = orc.render(v, sc.cameras[0], sc.tf, sc.shading, sc.options)
    ad = orc.render(v, sc.cameras[0], sc.tf, sc.shading,
                    dict(sc.options, adapt_factor=4, adapt_range=-1.0))
    ok = (plain["flags"] & 2) == 0
    np.testing.assert_allclose(ad["rgba"][ok], plain["rgba"][ok], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(ad["k_last"][ok], plain["k_last"][ok])


def test_homogeneous_region_keeps_its_opacity(orc):
    """Doubling the factor halves the samples in a homogeneous volume but
    leaves the opacity of the same length unchanged up to the end sample."""
    a = 0.02
    vol = orc.Volume(np.full((6, 6, 33), 100.0), (1, 1, 1), 0.0, 255.0)
    A = {}
    for m in (1, 2, 4, 8):
        opt = W.default_options(0.25, adapt_factor=m, adapt_range=0.0)
        r = orc.render(vol, _cam_x(), _flat_tf(a), W.default_shading("none"), opt)
        A[m] = float(np.median(r["rgba"][..., 3]))
    phys = 1.0 - (1.0 - a) ** (32.0 / 0.25)
    for m, val in A.items():
        assert abs(val - phys) <= (1.0 - a) ** (32.0 / 0.25) * (1.0 - (1.0 - a) ** m) + 1e-12


def _mixed_volume(rng, dims_zyx):
    """Random voxels with a few 8^3 blocks made constant (detail-poor)."""
    v = rng.integers(0, 256, dims_zyx).astype(np.float64)
    v[0:9, 0:9, 0:9] = 40.0
    v[8:17, 0:9, 8:17] = 200.0
    v[0:9, 8:17, 8:17] = rng.integers(120, 125)
    return v


CASES = [
    dict(op="central", shading="blinn_phong", projection="persp", m=2, rng=4.0, ert=0.0),
    dict(op="sobel3d", shading="none", projection="ortho", m=4, rng=0.0, ert=0.0),
    dict(op="zucker_hummel", shading="paper_lambert", projection="persp", m=3, rng=10.0,
         ert=0.9),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [81, 82])
def test_adaptive_matches_bruteforce(orc, case, seed):
    rng = np.random.default_rng(seed)
    arr = _mixed_volume(rng, (17, 17, 17))
    tf = W.tf_ramps(256, seed=seed, alpha_max=0.4)
    cam = W.orbit_camera((17, 17, 17), (1, 1, 1), rng.uniform(0, 360), rng.uniform(-50, 50), 13,
                         11, projection=case["projection"])
    sh = W.default_shading(case["shading"], light=(0.3, -0.7, 0.5),
                           light_is_point=case["shading"] == "paper_lambert")
    if sh["light_is_point"]:
        sh["light"] = (30.0, -16.0, 28.0)
    opt = W.default_options(0.45, case["op"], case["ert"], adapt_factor=case["m"],
                            adapt_range=case["rng"])
    res = orc.render(orc.Volume(arr, (1, 1, 1), 0, 255), cam, tf, sh, opt)
    bf = BF.render_adaptive(arr, (1, 1, 1), 0, 255, tf, cam, sh, opt)
    got, alt = res["rgba"].reshape(-1, 4), res["rgba_alt"].reshape(-1, 4)
    skip = (res["flags"].reshape(-1) & (4 | 16)) != 0
    ok = np.all(np.abs(got - bf) < 1e-9, axis=1) | np.all(np.abs(alt - bf) < 1e-9, axis=1) | skip
    assert ok.all(), np.abs(got - bf).max()
    assert (res["flags"] & 1).sum() > 40
    assert BF.poor_brick_flags(arr, case["rng"]).sum() >= 2
