"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these re-types the oracle's own formulas: each checks a closed
form, an invariant, a special case that reduces to a textbook result, the
masks printed in the paper (via impulse responses), or an independent
second formulation (``tests/bruteforce.py``) on tiny grids.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from tests import bruteforce as BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OPS = ["central", "sobel3d", "zucker_hummel"]


def _vol(orc, arr, spacing=(1.0, 1.0, 1.0), vmin=0.0, vmax=1.0):
    return orc.Volume(arr, spacing, vmin, vmax)


def _field(shape_zyx, fn):
    nz, ny, nx = shape_zyx
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return fn(i.astype(float), j.astype(float), k.astype(float))


# ------------------------------------------------------------ trilinear (Section 3.4)
def test_trilinear_exact_on_affine_fields(orc):
    rng = np.random.default_rng(0)
    c0, g = 3.0, np.array([0.7, -1.3, 2.1])
    vol = _vol(orc, _field((7, 6, 5), lambda i, j, k: c0 + g[0] * i + g[1] * j + g[2] * k))
    for _ in range(200):
        p = rng.uniform([0, 0, 0], [4, 5, 6])
        assert abs(orc.sample(vol, p) - (c0 + g @ p)) < 1e-12


def test_trilinear_hits_voxels_at_integer_points(orc):
    rng = np.random.default_rng(1)
    arr = rng.uniform(0, 100, (5, 6, 7))
    vol = _vol(orc, arr)
    for k in range(5):
        for j in range(6):
            for i in range(7):
                assert orc.sample(vol, [i, j, k]) == arr[k, j, i]


def test_trilinear_reduces_to_eq2_on_axis_lines(orc):
    """On a line x in [x0, x0+1] at integer y, z the sample is eq. (2)."""
    rng = np.random.default_rng(2)
    arr = rng.uniform(0, 50, (4, 4, 4))
    vol = _vol(orc, arr)
    for _ in range(50):
        x0, y, z = rng.integers(0, 3), rng.integers(0, 4), rng.integers(0, 4)
        x = x0 + rng.uniform()
        f0, f1 = arr[z, y, x0], arr[z, y, x0 + 1]
        g = f0 + (f1 - f0) / ((x0 + 1) - x0) * (x - x0)
        assert abs(orc.sample(vol, [x, y, z]) - g) < 1e-12


def test_trilinear_clamps_to_edge(orc):
    arr = np.arange(27, dtype=float).reshape(3, 3, 3)
    vol = _vol(orc, arr)
    assert orc.sample(vol, [-5.0, 0.0, 0.0]) == arr[0, 0, 0]
    assert orc.sample(vol, [9.0, 2.0, 2.0]) == arr[2, 2, 2]
    assert orc.sample(vol, [1.0, -0.25, 7.5]) == arr[2, 0, 1]


def test_trilinear_matches_bruteforce_sum(orc):
    rng = np.random.default_rng(3)
    arr = rng.uniform(0, 255, (4, 4, 4))
    vol, grid = _vol(orc, arr), BF.Grid(arr, (1, 1, 1), 0, 255)
    for _ in range(300):
        p = rng.uniform(-0.5, 3.5, 3)
        assert abs(orc.sample(vol, p) - grid.sample(p)) < 1e-10


# ------------------------------------------------------------ gradients (Section 3.5)
def _golden_masks():
    out, name, rows = {}, None, []
    for line in open(os.path.join(GOLDEN, "gradient_masks.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            name, rows = line[1:-1], []
            out[name] = rows
            continue
        rows.append([[float(x) for x in grp.split()] for grp in line.split("|")])
    masks = {}
    for name, rows in out.items():
        m = np.zeros((3, 3, 3))          # [dx][dy][dz]
        for dy in range(3):
            for dx in range(3):
                m[dx, dy, :] = rows[dy][dx]
        masks[name] = m
    return masks


@pytest.mark.parametrize("op", OPS)
def test_gradient_impulse_response_is_the_printed_mask(orc, op):
    """Impulse responses recover all three 3x3x3 masks: the x mask equals
    the golden (printed) one, y and z are it turned onto their axes, and the
    tap counts are the paper's 6 (CD) and 54 (Sobel3D, Zucker-Hummel)."""
    mx = _golden_masks()[op]
    expect = [mx, np.transpose(mx, (2, 0, 1)), np.transpose(mx, (1, 2, 0))]
    got = np.zeros((3, 3, 3, 3))
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                arr = np.zeros((5, 5, 5))
                arr[2 - dz, 2 - dy, 2 - dx] = 1.0   # V(p + o) = 1 at o = -(dx,dy,dz)
                _, raw = orc.gradient(_vol(orc, arr), op, [2.0, 2.0, 2.0])
                # raw_a = sum_o W_a(o) V(p+o) = W_a(-(dx,dy,dz))
                got[:, 1 - dx, 1 - dy, 1 - dz] = raw
    for a in range(3):
        np.testing.assert_allclose(got[a], expect[a], atol=1e-11)
    n_taps = int(np.count_nonzero(np.abs(got) > 1e-12))
    assert n_taps == (6 if op == "central" else 54)


GAINS = {"central": 2.0, "sobel3d": 44.0,
         "zucker_hummel": 2.0 * (1.0 + 2.0 * math.sqrt(2.0) + 4.0 / math.sqrt(3.0))}


@pytest.mark.parametrize("op", OPS)
def test_gradient_exact_on_linear_fields(orc, op):
    """V = 10 + 3i + 5j + 7k: raw = gain * (3, 5, 7) at any interior point,
    scaled G = slope / spacing / (vmax - vmin), outward normal -G/|G|."""
    spacing = (1.0, 2.0, 0.5)
    vol = _vol(orc, _field((9, 9, 9), lambda i, j, k: 10 + 3 * i + 5 * j + 7 * k),
               spacing, 0.0, 255.0)
    rng = np.random.default_rng(4)
    assert abs(GAINS["zucker_hummel"] - 12.2756564) < 1e-7
    for _ in range(20):
        p = rng.uniform(2.0, 6.0, 3)
        g, raw = orc.gradient(vol, op, p)
        np.testing.assert_allclose(raw, GAINS[op] * np.array([3.0, 5.0, 7.0]), rtol=1e-12)
        np.testing.assert_allclose(g, np.array([3.0, 5.0, 7.0]) / np.array(spacing) / 255.0,
                                   rtol=1e-12)


@pytest.mark.parametrize("op", OPS)
def test_gradient_zero_on_constant_field(orc, op):
    vol = _vol(orc, np.full((6, 6, 6), 42.0))
    for p in ([2.5, 2.5, 2.5], [0.0, 0.0, 0.0], [5.0, 3.3, 0.1]):
        g, raw = orc.gradient(vol, op, p)
        assert np.all(raw == 0.0)


def _moments(op):
    """S_pq = sum_{b,c} w(b,c) b^p c^q of the smoothing weights of an operator."""
    if op == "sobel3d":
        return 22.0, 10.0, 4.0
    r2, r3 = 1 / math.sqrt(2), 1 / math.sqrt(3)
    return 1 + 4 * r2 + 4 * r3, 2 * (r2 + 2 * r3), 4 * r3


@pytest.mark.parametrize("op", ["sobel3d", "zucker_hummel"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gradient_weight_distribution(orc, op, axis):
    """x * y^2 * z^2 (and its axis rotations) at integer points:
    raw_x = 2 [y^2 z^2 S00 + y^2 S02 + z^2 S20 + S22].  The three moments
    fix centre, edge and corner weights separately, which a linear field
    (only the weight sum) cannot."""
    S00, S20, S22 = _moments(op)

    def fn(i, j, k):
        c = [i, j, k]
        a, b, g = c[axis], c[(axis + 1) % 3], c[(axis + 2) % 3]
        return a * b * b * g * g

    vol = _vol(orc, _field((8, 8, 8), fn))
    for p in ([3, 4, 2], [4, 2, 5], [2, 5, 3]):
        _, raw = orc.gradient(vol, op, [float(x) for x in p])
        b, g = p[(axis + 1) % 3], p[(axis + 2) % 3]
        expect = 2 * (b * b * g * g * S00 + b * b * S20 + g * g * S20 + S22)
        assert abs(raw[axis] - expect) < 1e-9 * max(1.0, abs(expect))


def test_gradient_central_on_quadratic(orc):
    vol = _vol(orc, _field((8, 8, 8), lambda i, j, k: i * i + 2 * j * j - k * k))
    _, raw = orc.gradient(vol, "central", [3.0, 4.0, 2.0])
    np.testing.assert_allclose(raw, [4 * 3, 2 * 4 * 4, -4 * 2], rtol=1e-13)


@pytest.mark.parametrize("op", OPS)
def test_gradient_tap_form_equals_corner_blend(orc, op):
    """Tap form (oracle) == corner-blend form (bruteforce), clamped edges included."""
    rng = np.random.default_rng(5)
    arr = rng.integers(0, 4096, (4, 5, 6)).astype(float)
    vol, grid = _vol(orc, arr, (1.0, 1.5, 0.75), 0, 4095), BF.Grid(arr, (1.0, 1.5, 0.75), 0, 4095)
    for _ in range(60):
        p = rng.uniform(-0.3, [5.3, 4.3, 3.3])
        g1, r1 = orc.gradient(vol, op, p)
        g2, r2 = grid.gradient(op, p)
        np.testing.assert_allclose(r1, r2, atol=1e-8 * 4095)
        np.testing.assert_allclose(g1, g2, atol=1e-12)


# ------------------------------------------------------------ transfer function (Section 3.7)
def test_tf_entries_and_midpoints(orc):
    rng = np.random.default_rng(6)
    tf = rng.uniform(0, 1, (16, 4))
    for i in range(16):
        np.testing.assert_array_equal(orc.tf_lookup(tf, float(i)), tf[i])
    for i in range(15):
        np.testing.assert_allclose(orc.tf_lookup(tf, i + 0.5), 0.5 * (tf[i] + tf[i + 1]),
                                   rtol=1e-14)
        np.testing.assert_allclose(orc.tf_lookup(tf, i + 0.25),
                                   [np.interp(i + 0.25, np.arange(16), tf[:, c]) for c in range(4)],
                                   rtol=1e-13)


# ------------------------------------------------------------ camera and box (Section 3.3)
def test_camera_centre_pixel_looks_at_target(orc):
    cam = W.orbit_camera((9, 9, 9), (1, 1, 1), 37.0, 22.0, 31, 17)
    o, d = orc.camera_ray(cam, 15, 8)
    f = np.subtract(cam["target"], cam["eye"])
    np.testing.assert_allclose(d, f / np.linalg.norm(f), atol=1e-15)
    np.testing.assert_allclose(o, cam["eye"])


def test_camera_perspective_edges_span_the_fov(orc):
    """The top and bottom pixel rows' centre rays make fov/2 * (H-1)/H
    (in tangent) with the view axis."""
    cam = W.orbit_camera((9, 9, 9), (1, 1, 1), 0.0, 0.0, 21, 10, fov_y_deg=50.0)
    _, d_top = orc.camera_ray(cam, 10, 0)
    f = np.subtract(cam["target"], cam["eye"])
    f /= np.linalg.norm(f)
    tan_expect = math.tan(math.radians(25.0)) * (1 - 1 / 10)
    cosang = float(np.dot(d_top, f))
    assert abs(math.tan(math.acos(cosang)) - tan_expect) < 1e-12
    assert d_top[2] > 0  # row 0 is the top of the image (up = +z)


def test_camera_orthographic_pixel_centres(orc):
    cam = {"projection": "ortho", "eye": (20.0, 3.5, 3.5), "target": (0.0, 3.5, 3.5),
           "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 8.0, "width": 8,
           "height": 8}
    for px in range(8):
        for py in range(8):
            o, d = orc.camera_ray(cam, px, py)
            np.testing.assert_array_equal(d, [-1.0, 0.0, 0.0])
            np.testing.assert_allclose(o, [20.0, px, 7 - py], atol=1e-14)


def test_ray_box_axis_aligned(orc):
    hit, t0, t1 = orc.ray_box([20.0, 2.0, 3.0], [-1.0, 0.0, 0.0], [0, 0, 0], [7, 7, 7])
    assert hit and t0 == 13.0 and t1 == 20.0
    hit, _, _ = orc.ray_box([20.0, 8.0, 3.0], [-1.0, 0.0, 0.0], [0, 0, 0], [7, 7, 7])
    assert not hit
    hit, t0, t1 = orc.ray_box([3.0, 3.0, 3.0], [0.0, 0.6, 0.8], [0, 0, 0], [7, 7, 7])
    assert hit and t0 == 0.0 and abs(t1 - 5.0) < 1e-14   # eye inside: t_in clamps to 0


# ------------------------------------------------------------ shading (Section 3.8)
def test_blinn_phong_special_geometry(orc):
    sh = W.default_shading(light=(-1.0, 0.0, 0.0))
    rgb = np.array([0.2, 0.5, 0.9])
    # G along +x -> outward normal -x, light from -x, viewer looking +x: N.L = N.H = 1
    c = orc.shade(sh, rgb, [5.0, 0, 0], [0, 0, 0], [1.0, 0, 0])
    np.testing.assert_allclose(c, rgb * (0.1 + 0.7) + 0.2, rtol=1e-14)
    # light perpendicular to the normal, viewer along the normal: diffuse 0, N.H = cos 45
    sh2 = W.default_shading(light=(0.0, 1.0, 0.0))
    c = orc.shade(sh2, rgb, [5.0, 0, 0], [0, 0, 0], [1.0, 0, 0])
    np.testing.assert_allclose(c, rgb * 0.1 + 0.2 * math.cos(math.pi / 4) ** 32, rtol=1e-12)
    # light behind the surface: ambient only, no specular
    sh3 = W.default_shading(light=(1.0, 0.0, 0.0))
    c = orc.shade(sh3, rgb, [5.0, 0, 0], [0, 0, 0], [1.0, 0, 0])
    np.testing.assert_allclose(c, rgb * 0.1, rtol=1e-14)


def test_blinn_phong_soft_normalisation(orc):
    """|G| below eps: N = -G/eps, so the cosine terms scale with |G|/eps."""
    sh = W.default_shading(light=(-1.0, 0.0, 0.0), ks=0.0, grad_eps=1e-3)
    c = orc.shade(sh, [1.0, 1.0, 1.0], [2.5e-4, 0, 0], [0, 0, 0], [1.0, 0, 0])
    np.testing.assert_allclose(c, [0.1 + 0.7 * 0.25] * 3, rtol=1e-13)


def test_paper_lambert_listing3(orc):
    """Listing 3: illum = cos(light - p, G), unclamped, colour = rgb * illum."""
    sh = W.default_shading("paper_lambert", light=(10.0, 7.0, 3.0), light_is_point=True)
    p = np.array([10.0, 2.0, 3.0])            # light straight along +y from p
    rgb = np.array([0.3, 0.6, 0.9])
    np.testing.assert_allclose(orc.shade(sh, rgb, [0, 4.0, 0], p, [1, 0, 0]), rgb, rtol=1e-14)
    np.testing.assert_allclose(orc.shade(sh, rgb, [0, -4.0, 0], p, [1, 0, 0]), -rgb, rtol=1e-14)
    np.testing.assert_allclose(orc.shade(sh, rgb, [3.0, 3.0, 0], p, [1, 0, 0]),
                               rgb * math.cos(math.pi / 4), rtol=1e-13)


# ------------------------------------------------------------ compositing (Section 3.9)
def _axis_camera(n, W_=None):
    """Orthographic camera looking down -x whose pixel centres sit on voxel rows."""
    W_ = W_ or n
    c = (n - 1) / 2.0
    return {"projection": "ortho", "eye": (n - 1 + 10.0, c, c), "target": (0.0, c, c),
            "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": float(n),
            "width": W_, "height": W_}


@pytest.mark.parametrize("step", [0.5, 1.0, 0.37])
def test_constant_slab_closed_form(orc, step):
    """Constant density, TF alpha = a, rgb = c, unshaded: A = 1-(1-a)^n, C = c A."""
    n = 8
    a, col = 0.13, np.array([0.25, 0.5, 0.75])
    tf = np.tile(np.concatenate([col, [a]]), (4, 1))
    vol = _vol(orc, np.full((n, n, n), 0.5))
    cam = _axis_camera(n)
    opt = W.default_options(step, "central")
    res = orc.render(vol, cam, tf, W.default_shading("none"), opt)
    n_samples = math.floor((n - 1) / step) + 1
    A = 1 - (1 - a) ** n_samples
    np.testing.assert_allclose(res["rgba"][..., 3], A, rtol=1e-13)
    np.testing.assert_allclose(res["rgba"][..., :3], np.broadcast_to(col * A, (n, n, 3)),
                               rtol=1e-13)


def test_line_integral(orc):
    """Orthographic axis-aligned rays, step 1, samples on voxel centres, unit
    colour, alpha_i = 1 - exp(-kappa i/255) on a u8 grid with a 256-entry
    table: -ln T = kappa/255 * sum of the voxel row, and C = 1 - T."""
    n, kappa = 8, 0.9
    rng = np.random.default_rng(7)
    arr = rng.integers(0, 256, (n, n, n)).astype(np.uint8)
    ent = np.arange(256)
    tf = np.stack([np.ones(256)] * 3 + [1 - np.exp(-kappa * ent / 255.0)], axis=1)
    vol = _vol(orc, arr, (1, 1, 1), 0.0, 255.0)
    cam = _axis_camera(n)
    res = orc.render(vol, cam, tf, W.default_shading("none"), W.default_options(1.0, "central"))
    assert np.all(res["flags"] & 2)          # (t_out - t_in)/step = 7 exactly: a lattice tie
    for py in range(n):
        for px in range(n):
            y, z = px, n - 1 - py
            T = 1 - res["rgba"][py, px, 3]
            line = kappa / 255.0 * arr[z, y, :].astype(float).sum()
            assert abs(-math.log(T) - line) < 1e-12
            np.testing.assert_allclose(res["rgba"][py, px, :3], 1 - T, rtol=1e-12)


def test_half_step_samples_are_column_lerps(orc):
    """Step 0.5 on the same rays: samples alternate between voxel values and
    the midpoints of neighbouring voxels (eq. 2 at x0 + 1/2)."""
    n = 6
    rng = np.random.default_rng(8)
    arr = rng.integers(0, 256, (n, n, n)).astype(float)
    ent = np.arange(256)
    kappa = 0.5
    tf = np.stack([np.ones(256)] * 3 + [1 - np.exp(-kappa * ent / 255.0)], axis=1)
    vol = _vol(orc, arr, (1, 1, 1), 0.0, 255.0)
    res = orc.render(vol, _axis_camera(n), tf, W.default_shading("none"),
                     W.default_options(0.5, "central"))
    row = arr[2, 3, :]                  # z = 2, y = 3  -> px = 3, py = n-1-2
    samples = []
    for x in range(n - 1, 0, -1):
        samples += [row[x], 0.5 * (row[x] + row[x - 1])]
    samples.append(row[0])
    # half-integer values fall between table entries: alpha is the entry lerp
    alphas = [np.interp(u, ent, tf[:, 3]) for u in samples]
    T_expect = float(np.prod([1 - a for a in alphas]))
    assert abs((1 - res["rgba"][n - 1 - 2, 3, 3]) - T_expect) < 1e-13


def test_miss_is_black(orc):
    vol = _vol(orc, np.full((4, 4, 4), 200.0), (1, 1, 1), 0, 255)
    cam = {"projection": "ortho", "eye": (30.0, 30.0, 30.0), "target": (40.0, 30.0, 30.0),
           "up": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "ortho_height": 2.0, "width": 4,
           "height": 4}
    tf = np.ones((8, 4))
    res = orc.render(vol, cam, tf, W.default_shading("none"), W.default_options())
    assert np.all(res["rgba"] == 0.0) and np.all(res["k_last"] == -1)


def test_early_termination_bound(orc):
    sc = W.config_small(seed=3, dims=(12, 12, 12), image=(24, 24))
    vol = _vol(orc, sc.volume, sc.spacing, sc.vmin, sc.vmax)
    full = orc.render(vol, sc.cameras[0], sc.tf, sc.shading, sc.options)
    tau = 0.6
    ert = orc.render(vol, sc.cameras[0], sc.tf, sc.shading, dict(sc.options, ert_threshold=tau))
    assert np.all(np.abs(full["rgba"] - ert["rgba"]) <= 1 - tau + 1e-12)
    stopped = ert["k_last"] < full["k_last"]
    assert stopped.any()
    assert np.all(ert["rgba"][..., 3][stopped] >= tau)


# ------------------------------------------------------------ full pipeline vs bruteforce
CASES = [
    dict(op="central", shading="blinn_phong", projection="persp", ert=0.0),
    dict(op="sobel3d", shading="blinn_phong", projection="ortho", ert=0.0),
    dict(op="zucker_hummel", shading="paper_lambert", projection="persp", ert=0.0),
    dict(op="sobel3d", shading="none", projection="persp", ert=0.5),
    dict(op="central", shading="blinn_phong", projection="persp", ert=0.7),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [11, 12])
def test_oracle_matches_bruteforce_on_4cubed(orc, case, seed):
    rng = np.random.default_rng(seed)
    arr = rng.integers(0, 256, (4, 4, 4)).astype(np.uint8)
    tf = W.tf_ramps(256, seed=seed, alpha_max=0.6)
    cam = W.orbit_camera((4, 4, 4), (1, 1, 1), rng.uniform(0, 360), rng.uniform(-60, 60), 9, 7,
                         projection=case["projection"])
    sh = W.default_shading(case["shading"], light=(0.3, -0.7, 0.5),
                           light_is_point=case["shading"] == "paper_lambert")
    if sh["light_is_point"]:
        sh["light"] = (10.0, -6.0, 8.0)
    opt = W.default_options(0.37, case["op"], case["ert"])
    if seed == 12:
        opt["clip_lo"], opt["clip_hi"] = (0.5, 0.0, 0.2), (3.0, 2.6, 3.0)
    vol = _vol(orc, arr, (1, 1, 1), 0, 255)
    res = orc.render(vol, cam, tf, sh, opt)
    bf = BF.render(arr, (1, 1, 1), 0, 255, tf, cam, sh, opt)
    got = res["rgba"].reshape(-1, 4)
    alt = res["rgba_alt"].reshape(-1, 4)
    ok = np.all(np.abs(got - bf) < 1e-9, axis=1) | np.all(np.abs(alt - bf) < 1e-9, axis=1)
    assert ok.all(), np.abs(got - bf).max()
    assert (res["flags"] & 1).sum() > 10


def test_back_to_front_equals_front_to_back_random(orc):
    """Eq. (6) run back to front == the front-to-back sum, per ray."""
    rng = np.random.default_rng(9)
    for _ in range(50):
        n = rng.integers(1, 40)
        a = rng.uniform(0, 0.5, n)
        c = rng.uniform(0, 1, (n, 3))
        Cb, Ab = np.zeros(3), 0.0
        for k in reversed(range(n)):
            Cb = Cb * (1 - a[k]) + c[k] * a[k]
            Ab = Ab * (1 - a[k]) + a[k]
        T = np.concatenate([[1.0], np.cumprod(1 - a)[:-1]])
        Cf = (T[:, None] * a[:, None] * c).sum(0)
        np.testing.assert_allclose(Cb, Cf, rtol=1e-13)
        assert abs(Ab - (1 - np.prod(1 - a))) < 1e-14
