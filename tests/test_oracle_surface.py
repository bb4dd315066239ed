"""Pins of the oracle's first-hit surface mode (coarse march to the first
sample inside the value window, then hitpoint refinement by halving steps).

Closed forms on affine fields (where trilinear interpolation is exact, so
the window boundary crossing is known exactly), the 2^-n error bound of the
refinement, the special cases (start inside, thin features between coarse
samples, misses), the shaded colour of a known normal, and an independent
interval-bisection formulation (``tests/bruteforce.py``) on tiny grids.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import bruteforce as BF

NX, NY, NZ = 40, 8, 8


def _ramp(orc, c0, slope):
    """V(i, j, k) = c0 + slope * i on a 40x8x8 grid."""
    k, j, i = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    return orc.Volume(c0 + slope * i.astype(float), (1.0, 1.0, 1.0), 0.0, 255.0)


def _cam_x(width=8, height=8, reverse=False):
    """Orthographic camera looking along +x (or -x) through the 8x8 cross-section."""
    eye = (120.0, 3.5, 3.5) if reverse else (-50.0, 3.5, 3.5)
    tgt = (0.0, 3.5, 3.5) if reverse else (10.0, 3.5, 3.5)
    return {"projection": "ortho", "eye": eye, "target": tgt, "up": (0.0, 0.0, 1.0),
            "fov_y_deg": 60.0, "ortho_height": 7.0, "width": width, "height": height}


def _tf_grey():
    tf = np.zeros((256, 4))
    tf[:, 0] = tf[:, 1] = tf[:, 2] = np.linspace(0.0, 1.0, 256)
    tf[:, 3] = 0.5
    return tf


def _x_of(orc, cam, res):
    """World x of each pixel's refined hit."""
    xs = []
    for q, t in enumerate(res["t_hit"].reshape(-1)):
        o, d = orc.camera_ray(cam, q % cam["width"], q // cam["width"])
        xs.append(o[0] + t * d[0])
    return np.array(xs)


NONE = W.default_shading("none")


@pytest.mark.parametrize("refine", [0, 1, 2, 3])
def test_dyadic_crossing_is_found_exactly(orc, refine):
    """V = 10 + 3x, window [V(13.375), inf), coarse step 1 from x = 0: the
    first coarse sample inside is x = 14, and n halvings land on
    14 - 1/2 (n=1), 13.25 (n=2), and the exact crossing 13.375 (n=3)."""
    vol = _ramp(orc, 10.0, 3.0)
    cam = _cam_x()
    opt = W.default_surface_options(step=1.0, iso_lo=10.0 + 3.0 * 13.375, refine=refine)
    res = orc.render_surface(vol, cam, _tf_grey(), NONE, opt)
    expect = {0: 14.0, 1: 13.5, 2: 13.25, 3: 13.375}[refine]
    assert np.all(res["k_hit"] == 14)
    assert np.abs(_x_of(orc, cam, res) - expect).max() < 1e-9
    assert np.all(res["rgba"][..., 3] == 1.0)
    assert np.all(res["flags"] & 1)


@pytest.mark.parametrize("refine", [4, 5, 6, 9])
@pytest.mark.parametrize("xstar", [13.1, 20.77, 7.5001])
def test_refinement_error_bound(orc, refine, xstar):
    """After n halvings the hit is within step/2^n of the crossing and never
    leaves the last coarse interval (Section 5.1: 64 times finer for 6)."""
    step = 1.7
    vol = _ramp(orc, 5.0, 4.0)
    cam = _cam_x()
    opt = W.default_surface_options(step=step, iso_lo=5.0 + 4.0 * xstar, refine=refine)
    res = orc.render_surface(vol, cam, _tf_grey(), NONE, opt)
    x = _x_of(orc, cam, res)
    k = math.ceil(xstar / step)
    assert np.all(res["k_hit"] == k)
    assert np.abs(x - xstar).max() <= step / 2 ** refine + 1e-9
    assert np.all((x >= (k - 1) * step - 1e-9) & (x <= k * step + 1e-9))


def test_crossing_from_above_uses_the_upper_bound(orc):
    """V = 200 - 3x with window (-inf, V(13.375)]: values fall into the window."""
    vol = _ramp(orc, 200.0, -3.0)
    cam = _cam_x()
    opt = W.default_surface_options(step=1.0, iso_lo=-1e30, iso_hi=200.0 - 3.0 * 13.375, refine=3)
    res = orc.render_surface(vol, cam, _tf_grey(), NONE, opt)
    assert np.abs(_x_of(orc, cam, res) - 13.375).max() < 1e-9


def test_reverse_ray_direction(orc):
    """Looking along -x at V = 10 + 3x with window (-inf, V(25.625)]: the first
    sample inside (from x = 39 downwards, step 1) is x = 25; three halvings
    land on the crossing 25.625 exactly."""
    vol = _ramp(orc, 10.0, 3.0)
    cam = _cam_x(reverse=True)
    opt = W.default_surface_options(step=1.0, iso_lo=-1e30, iso_hi=10.0 + 3.0 * 25.625, refine=3)
    res = orc.render_surface(vol, cam, _tf_grey(), NONE, opt)
    assert np.all(res["k_hit"] == 14)
    assert np.abs(_x_of(orc, cam, res) - 25.625).max() < 1e-9


def test_thin_band_between_coarse_samples_is_missed(orc):
    """The window [V(13.5), V(13.8)] lies between the coarse samples x = 13
    and 14: the coarse march never sees it."""
    vol = _ramp(orc, 10.0, 3.0)
    opt = W.default_surface_options(step=1.0, iso_lo=10.0 + 3 * 13.5, iso_hi=10.0 + 3 * 13.8)
    res = orc.render_surface(vol, _cam_x(), _tf_grey(), NONE, opt)
    assert np.all(res["k_hit"] == -1) and np.all(np.isinf(res["t_hit"]))
    assert np.all(res["rgba"] == 0.0)
    assert np.all(res["flags"] == 1)          # the box is hit, the surface is not


def test_start_inside_is_not_refined(orc):
    """A clip plane at x = 20.3 cuts the object (window from V(13.375)): the
    first sample is inside, so the hit is the entry point itself."""
    vol = _ramp(orc, 10.0, 3.0)
    cam = _cam_x()
    opt = W.default_surface_options(step=1.0, iso_lo=10.0 + 3.0 * 13.375, refine=6,
                                    clip_lo=(20.3, -1e30, -1e30))
    res = orc.render_surface(vol, cam, _tf_grey(), NONE, opt)
    assert np.all(res["k_hit"] == 0)
    assert np.abs(_x_of(orc, cam, res) - 20.3).max() < 1e-9


def test_miss_and_empty_window(orc):
    vol = _ramp(orc, 10.0, 3.0)
    away = dict(_cam_x(), eye=(-50.0, 30.0, 3.5), target=(10.0, 30.0, 3.5))
    res = orc.render_surface(vol, away, _tf_grey(), NONE, W.default_surface_options(iso_lo=50.0))
    assert np.all(res["flags"] == 0) and np.all(res["k_hit"] == -1)
    assert np.all(np.isinf(res["t_hit"])) and np.all(res["rgba"] == 0.0)
    none = W.default_surface_options(iso_lo=1000.0, iso_hi=2000.0)
    res = orc.render_surface(vol, _cam_x(), _tf_grey(), NONE, none)
    assert np.all(res["rgba"] == 0.0) and np.all(res["k_hit"] == -1)


def test_colour_is_table_rgb_at_the_refined_value(orc):
    """Shading NONE: rgb = grey ramp at V(x*) / 255 * 255 entries, opaque."""
    vol = _ramp(orc, 10.0, 3.0)
    iso = 10.0 + 3.0 * 13.375
    opt = W.default_surface_options(step=1.0, iso_lo=iso, refine=3)
    res = orc.render_surface(vol, _cam_x(), _tf_grey(), NONE, opt)
    rgba = res["rgba"].reshape(-1, 4)
    np.testing.assert_allclose(rgba[:, :3], iso / 255.0, atol=1e-12)
    assert np.all(rgba[:, 3] == 1.0)


@pytest.mark.parametrize("op", ["central", "sobel3d", "zucker_hummel"])
def test_blinn_phong_of_the_ramp_normal(orc, op):
    """V = 10 + 3x has outward normal N = -x (towards smaller values).  A
    directional light L and view V = -d = -x give the closed-form
    Blinn-Phong colour rgb (ka + kd max(0, N.L)) + ks max(0, N.H)^s."""
    vol = _ramp(orc, 10.0, 3.0)
    iso = 10.0 + 3.0 * 13.375
    L = np.array([-0.6, 0.0, 0.8])
    sh = W.default_shading("blinn_phong", light=tuple(L))
    opt = W.default_surface_options(step=1.0, iso_lo=iso, refine=3, gradient_op=op)
    res = orc.render_surface(vol, _cam_x(), _tf_grey(), sh, opt)
    N = np.array([-1.0, 0.0, 0.0])
    H = (L + np.array([-1.0, 0.0, 0.0]))
    H /= np.linalg.norm(H)
    rgb = iso / 255.0
    want = rgb * (sh["ka"] + sh["kd"] * max(0.0, N @ L)) + sh["ks"] * max(0.0, N @ H) ** sh["shininess"]
    # pixels whose stencil reaches the clamped y/z faces see the same ramp: exact everywhere
    np.testing.assert_allclose(res["rgba"].reshape(-1, 4)[:, :3], want, atol=1e-12)


CASES = [
    dict(op="central", shading="blinn_phong", projection="persp", refine=6, step=0.8),
    dict(op="sobel3d", shading="none", projection="ortho", refine=0, step=0.6),
    dict(op="zucker_hummel", shading="paper_lambert", projection="persp", refine=3, step=1.1),
    dict(op="sobel3d", shading="blinn_phong", projection="persp", refine=5, step=0.45),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [21, 22])
def test_surface_matches_bisection_bruteforce(orc, case, seed):
    rng = np.random.default_rng(seed)
    arr = rng.integers(0, 256, (5, 4, 6)).astype(np.uint8)
    tf = W.tf_ramps(256, seed=seed, alpha_max=0.6)
    cam = W.orbit_camera((6, 4, 5), (1, 1, 1), rng.uniform(0, 360), rng.uniform(-60, 60), 15, 12,
                         projection=case["projection"])
    sh = W.default_shading(case["shading"], light=(0.3, -0.7, 0.5),
                           light_is_point=case["shading"] == "paper_lambert")
    if sh["light_is_point"]:
        sh["light"] = (10.0, -6.0, 8.0)
    opt = W.default_surface_options(step=case["step"], gradient_op=case["op"], iso_lo=150.0,
                                    iso_hi=230.0 if seed == 22 else 1e30, refine=case["refine"])
    if seed == 22:
        opt["clip_lo"], opt["clip_hi"] = (0.5, 0.0, 0.2), (4.6, 2.6, 3.5)
    vol = orc.Volume(arr, (1, 1, 1), 0, 255)
    res = orc.render_surface(vol, cam, tf, sh, opt)
    rgba, th = BF.render_surface(arr, (1, 1, 1), 0, 255, tf, cam, sh, opt)
    ok = (res["flags"].reshape(-1) & 2) == 0           # lattice-end ties: either answer
    got = res["rgba"].reshape(-1, 4)
    assert np.abs(got[ok] - rgba[ok]).max() < 1e-9
    t = res["t_hit"].reshape(-1)[ok]
    fin = np.isfinite(th[ok])
    assert np.array_equal(np.isfinite(t), fin)
    assert np.abs(t[fin] - th[ok][fin]).max(initial=0.0) < 1e-9
    assert (res["k_hit"] >= 0).sum() >= 8 and (res["k_hit"] > 0).sum() >= 3


def test_iso_near_flag(orc):
    """A window bound equal to a coarse sample's value is flagged."""
    vol = _ramp(orc, 10.0, 3.0)
    opt = W.default_surface_options(step=1.0, iso_lo=10.0 + 3.0 * 14, refine=4)
    res = orc.render_surface(vol, _cam_x(), _tf_grey(), NONE, opt)
    assert np.all(res["flags"] & 8)
    opt["iso_lo"] = 10.0 + 3.0 * 13.4
    res = orc.render_surface(vol, _cam_x(), _tf_grey(), NONE, opt)
    assert not np.any(res["flags"] & 8)
