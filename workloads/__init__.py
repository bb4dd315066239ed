"""Seeded synthetic inputs for the volume raycaster.

This module only *generates inputs*: voxel grids, transfer-function tables,
camera placements and option sets.  It holds none of the raycasting
arithmetic (ray setup, sampling, gradients, shading, compositing), so both
the GPU path and the FP64 oracle can take their inputs from here without
sharing any of the method.

The volumes stand in for the CT scans the paper renders (Section 3.2: a
512^3 cube of 16-bit voxels holding 12-bit values).  Those scans are not
available, so the generators reproduce their *shape*: sizes, storage type,
value range and the mix of empty space and nested structure.

Conventions shared by every consumer (they are interface, not method):
  * a volume is a numpy array indexed ``[z][y][x]`` (x fastest);
  * a camera, shading set and option set are plain dicts whose keys mirror
    the C structs of the library (see ``include/rc.h``);
  * every generator takes an explicit integer seed and uses
    ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "blob_volume", "phantom_volume", "tf_ramps", "orbit_camera",
    "default_shading", "default_options", "default_surface_options", "value_range",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5",
    "config_small",
]


# --------------------------------------------------------------------------
# scene container
# --------------------------------------------------------------------------
@dataclass
class Scene:
    """One render job: a volume plus everything needed to draw it."""

    name: str
    volume: np.ndarray                    # [nz][ny][nx], uint8 / uint16 / float32
    spacing: tuple                        # world units per voxel step (sx, sy, sz)
    vmin: float                           # raw value mapped to TF coordinate 0
    vmax: float                           # raw value mapped to TF coordinate 1
    tf: np.ndarray                        # [M][4] float32 RGBA table
    cameras: list                         # list of camera dicts
    shading: dict
    options: dict
    extra: dict = field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.volume.shape
        return nx, ny, nz


def value_range(dtype) -> tuple:
    """Default (vmin, vmax): u8 -> (0,255), u16 12-bit -> (0,4095), f32 -> (0,1)."""
    dt = np.dtype(dtype)
    if dt == np.uint8:
        return 0.0, 255.0
    if dt == np.uint16:
        return 0.0, 4095.0
    return 0.0, 1.0


# --------------------------------------------------------------------------
# volumes
# --------------------------------------------------------------------------
def blob_volume(shape_zyx, n_blobs, seed, dtype=np.uint8, sigma=(4.0, 12.0),
                amp=(80.0, 255.0), centre_lo=0.25, centre_hi=0.75, normalise=False):
    """Sum of isotropic Gaussian blobs.

    Centres are uniform in the box [centre_lo, centre_hi] of each axis, sigmas
    and amplitudes uniform in the given ranges.  Integer outputs are rounded
    and clamped to the type's 12/8-bit range; ``normalise`` divides a float
    field by its maximum so that it spans [0, 1].
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape_zyx
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    acc = np.zeros(shape_zyx, dtype=np.float64)
    for _ in range(n_blobs):
        c = rng.uniform(centre_lo, centre_hi, 3) * (np.array([nx, ny, nz]) - 1)
        s = rng.uniform(*sigma)
        a = rng.uniform(*amp)
        acc += a * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
    dt = np.dtype(dtype)
    if dt == np.float32:
        if normalise:
            acc /= acc.max()
        return acc.astype(np.float32)
    hi = 255 if dt == np.uint8 else 4095
    return np.clip(np.rint(acc), 0, hi).astype(dt)


def _random_rotation(rng):
    """Rotation matrix from a uniformly random unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, 3)
    q = np.array([
        math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
        math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
        math.sqrt(u1) * math.sin(2 * math.pi * u3),
        math.sqrt(u1) * math.cos(2 * math.pi * u3),
    ])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def phantom_volume(shape_zyx, n_ellipsoids, seed, dtype=np.uint16, noise_sigma=20.0,
                   n_cavities=3):
    """CT-like phantom of nested, overlapping, rotated ellipsoids.

    * ellipsoid 0 is large (semi-axes 0.36-0.45 of each edge) and centred,
      so it encloses most of the others;
    * the rest have semi-axes 0.05-0.25 of the edge and centres in the
      central 60 % box;
    * intensities are additive, U[200, 1500], except ``n_cavities`` of them
      which are negative, U[-400, -100] (cavities);
    * Gaussian noise N(0, noise_sigma^2) is added, then values are rounded
      and clamped to the 12-bit range [0, 4095] (u16) or [0, 255] (u8).

    Each ellipsoid is evaluated only inside its bounding box, so 512^3
    phantoms take seconds.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape_zyx
    n = np.array([nx, ny, nz], dtype=np.float64)
    acc = np.zeros(shape_zyx, dtype=np.float32)
    cav = set(rng.choice(np.arange(1, n_ellipsoids), size=min(n_cavities, n_ellipsoids - 1),
                         replace=False).tolist()) if n_ellipsoids > 1 else set()
    for e in range(n_ellipsoids):
        if e == 0:
            axes = rng.uniform(0.36, 0.45, 3) * n
            centre = (n - 1) / 2 + rng.uniform(-0.02, 0.02, 3) * n
        else:
            axes = rng.uniform(0.05, 0.25, 3) * n
            centre = rng.uniform(0.2, 0.8, 3) * (n - 1)
        rot = _random_rotation(rng)
        inten = -rng.uniform(100, 400) if e in cav else rng.uniform(200, 1500)
        # bounding box of the rotated ellipsoid: half-extent_i = |R_ij| a_j summed in quadrature
        ext = np.sqrt(((rot * axes[None, :]) ** 2).sum(axis=1))
        lo = np.maximum(np.floor(centre - ext), 0).astype(int)
        hi = np.minimum(np.ceil(centre + ext), n - 1).astype(int)
        if np.any(hi < lo):
            continue
        zs = np.arange(lo[2], hi[2] + 1, dtype=np.float32)[:, None, None] - centre[2]
        ys = np.arange(lo[1], hi[1] + 1, dtype=np.float32)[None, :, None] - centre[1]
        xs = np.arange(lo[0], hi[0] + 1, dtype=np.float32)[None, None, :] - centre[0]
        # coordinates in the ellipsoid frame: q = R^T (p - c)
        q0 = rot[0, 0] * xs + rot[1, 0] * ys + rot[2, 0] * zs
        q1 = rot[0, 1] * xs + rot[1, 1] * ys + rot[2, 1] * zs
        q2 = rot[0, 2] * xs + rot[1, 2] * ys + rot[2, 2] * zs
        inside = (q0 / axes[0]) ** 2 + (q1 / axes[1]) ** 2 + (q2 / axes[2]) ** 2 <= 1.0
        acc[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += np.float32(inten) * inside
    if noise_sigma > 0:
        acc += rng.normal(0.0, noise_sigma, size=shape_zyx).astype(np.float32)
    dt = np.dtype(dtype)
    hi = 255 if dt == np.uint8 else 4095
    if dt == np.uint8:
        acc *= 255.0 / 4095.0
    return np.clip(np.rint(acc), 0, hi).astype(dt)


# --------------------------------------------------------------------------
# transfer functions
# --------------------------------------------------------------------------
def tf_ramps(M, seed, n_break=5, alpha_max=0.15, alpha_min=0.0, lo=0.0, hi=1.0):
    """Piecewise-linear RGBA table through ``n_break`` seeded sorted breakpoints.

    Breakpoint positions are uniform in [lo, hi] (TF coordinate in [0, 1]);
    rgb is uniform in [0, 1], alpha uniform in [alpha_min, alpha_max].
    Alpha is exactly 0 at and below the first breakpoint (and the first
    breakpoint's alpha is forced to 0), constant after the last one.
    """
    rng = np.random.default_rng(seed)
    pos = np.sort(rng.uniform(lo, hi, n_break))
    rgb = rng.uniform(0.0, 1.0, (n_break, 3))
    alpha = rng.uniform(alpha_min, alpha_max, n_break)
    alpha[0] = 0.0
    xs = np.linspace(0.0, 1.0, M)
    out = np.zeros((M, 4), dtype=np.float64)
    for c in range(3):
        out[:, c] = np.interp(xs, pos, rgb[:, c])
    out[:, 3] = np.interp(xs, pos, alpha)
    out[xs <= pos[0], 3] = 0.0
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# cameras, shading, options
# --------------------------------------------------------------------------
def orbit_camera(dims_xyz, spacing, azimuth_deg, elevation_deg, width, height,
                 projection="persp", fov_y_deg=60.0, zoom=1.0):
    """Camera on a sphere around the volume centre, looking at the centre.

    The bounding sphere (radius r = half the box diagonal) is fitted to the
    vertical field of view: perspective eyes sit at r / sin(fov/2) from the
    centre, orthographic views use an image height of 2r.  ``up`` is +z.
    """
    ext = (np.asarray(dims_xyz, dtype=np.float64) - 1.0) * np.asarray(spacing, dtype=np.float64)
    centre = ext / 2.0
    r = max(float(np.linalg.norm(ext)) / 2.0, 0.5)
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    dirv = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    if projection == "persp":
        dist = r / math.sin(math.radians(fov_y_deg) / 2.0) / zoom
    else:
        dist = 2.0 * r
    eye = centre + dist * dirv
    return {
        "projection": projection,
        "eye": tuple(float(v) for v in eye),
        "target": tuple(float(v) for v in centre),
        "up": (0.0, 0.0, 1.0),
        "fov_y_deg": float(fov_y_deg),
        "ortho_height": float(2.0 * r / zoom),
        "width": int(width),
        "height": int(height),
    }


def default_shading(model="blinn_phong", light=(-0.4, -0.5, 0.75), light_is_point=False,
                    ka=0.1, kd=0.7, ks=0.2, shininess=32.0, grad_eps=1e-3):
    return {"model": model, "ka": ka, "kd": kd, "ks": ks, "shininess": shininess,
            "light_is_point": bool(light_is_point), "light": tuple(float(v) for v in light),
            "grad_eps": grad_eps}


def default_options(step=0.5, gradient_op="central", ert_threshold=0.0, skip_empty=False,
                    clip_lo=(-1e30, -1e30, -1e30), clip_hi=(1e30, 1e30, 1e30), nearest=False,
                    ref_step=0.0, adapt_factor=0, adapt_range=0.0):
    return {"step": float(step), "gradient_op": gradient_op, "ert_threshold": float(ert_threshold),
            "skip_empty": bool(skip_empty), "clip_lo": tuple(float(v) for v in clip_lo),
            "clip_hi": tuple(float(v) for v in clip_hi), "nearest": bool(nearest),
            "ref_step": float(ref_step), "adapt_factor": int(adapt_factor),
            "adapt_range": float(adapt_range)}


def default_surface_options(step=2.0, gradient_op="central", iso_lo=0.0, iso_hi=1e30, refine=6,
                            skip_empty=False, clip_lo=(-1e30, -1e30, -1e30),
                            clip_hi=(1e30, 1e30, 1e30)):
    """First-hit surface mode: a raw-value window, a coarse step (the
    hitpoint-refinement section allows 4-5x the volume-mode step) and the
    number of refinement halvings (5 to 6 in the paper)."""
    return {"step": float(step), "gradient_op": gradient_op, "iso_lo": float(iso_lo),
            "iso_hi": float(iso_hi), "refine": int(refine), "skip_empty": bool(skip_empty),
            "clip_lo": tuple(float(v) for v in clip_lo), "clip_hi": tuple(float(v) for v in clip_hi)}


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config_c1():
    """64^3 u8 blobs -> 128^2 orthographic, central difference, Blinn-Phong, no ERT/skip."""
    vol = blob_volume((64, 64, 64), 3, seed=1, dtype=np.uint8)
    tf = tf_ramps(256, seed=101, alpha_max=0.15)
    cam = orbit_camera((64, 64, 64), (1, 1, 1), 30.0, 20.0, 128, 128, projection="ortho")
    return Scene("c1_64_u8_ortho128_cd", vol, (1.0, 1.0, 1.0), 0.0, 255.0, tf, [cam],
                 default_shading(), default_options(0.5, "central"))


def _ct_tf(M, seed):
    """4096-entry CT table: alpha 0 below raw 300, seeded ramps above."""
    return tf_ramps(M, seed=seed, n_break=6, alpha_min=0.02, alpha_max=0.25,
                    lo=300.0 / 4095.0, hi=1.0)


def config_c2():
    """256^3 u16 phantom (10 ellipsoids) -> 512^2 perspective, Sobel3D, ERT 0.99, skip."""
    vol = phantom_volume((256, 256, 256), 10, seed=2)
    tf = _ct_tf(4096, seed=102)
    cam = orbit_camera((256, 256, 256), (1, 1, 1), 30.0, 20.0, 512, 512)
    return Scene("c2_256_u16_persp512_sobel", vol, (1.0, 1.0, 1.0), 0.0, 4095.0, tf, [cam],
                 default_shading(), default_options(0.5, "sobel3d", 0.99, True))


def config_c3(n_views=36, size=512, image=1024):
    """512^3 u16 phantom (24 ellipsoids) -> 1024^2, 36-view orbit, ERT 0.99, skip."""
    vol = phantom_volume((size, size, size), 24, seed=3)
    tf = _ct_tf(4096, seed=103)
    cams = [orbit_camera((size, size, size), (1, 1, 1), 10.0 * i, 20.0, image, image)
            for i in range(n_views)]
    return Scene("c3_512_u16_persp1024_orbit36", vol, (1.0, 1.0, 1.0), 0.0, 4095.0, tf, cams,
                 default_shading(), default_options(0.5, "sobel3d", 0.99, True))


def config_c4(n_volumes=64, seed=4):
    """64 uneven volumes, each with its own camera, image size and 256-entry TF."""
    rng = np.random.default_rng(seed)
    scenes = []
    for i in range(n_volumes):
        nx, ny = (int(v) for v in rng.integers(32, 257, 2))
        nz = int(rng.integers(32, 97))
        u16 = bool(rng.integers(0, 2))
        dt = np.uint16 if u16 else np.uint8
        sub = int(rng.integers(0, 2**31 - 1))
        if rng.integers(0, 2):
            vol = blob_volume((nz, ny, nx), 4, seed=sub, dtype=dt,
                              amp=(80.0, 255.0) if not u16 else (600.0, 4000.0))
        else:
            vol = phantom_volume((nz, ny, nx), 6, seed=sub, dtype=dt)
        vmin, vmax = value_range(dt)
        tf = tf_ramps(256, seed=sub + 1, alpha_min=0.02, alpha_max=0.25, lo=0.1, hi=1.0)
        side = int(rng.integers(8, 33)) * 16
        az = float(rng.uniform(0, 360))
        el = float(rng.uniform(-60, 60))
        cam = orbit_camera((nx, ny, nz), (1, 1, 1), az, el, side, side)
        scenes.append(Scene(f"c4_{i:02d}", vol, (1.0, 1.0, 1.0), vmin, vmax, tf, [cam],
                            default_shading(), default_options(0.5, "central", 0.99, True)))
    return scenes


def config_c5(n_views=16, size=128, image=256, target_seed=55):
    """128^3 f32 blobs in [0,1], learnable 256-entry TF, 16 views at 256^2, unshaded."""
    vol = blob_volume((size, size, size), 6, seed=5, dtype=np.float32, sigma=(6.0, 20.0),
                      amp=(0.3, 1.0), normalise=True)
    target = blob_volume((size, size, size), 6, seed=target_seed, dtype=np.float32,
                         sigma=(6.0, 20.0), amp=(0.3, 1.0), normalise=True)
    tf = tf_ramps(256, seed=101, alpha_max=0.15)
    cams = [orbit_camera((size, size, size), (1, 1, 1), 22.5 * i, 20.0 if i % 2 == 0 else -20.0,
                         image, image) for i in range(n_views)]
    return Scene("c5_128_f32_persp256_x16", vol, (1.0, 1.0, 1.0), 0.0, 1.0, tf, cams,
                 default_shading("none"), default_options(0.5, "central", 1.0 - 1e-4, False),
                 extra={"target_volume": target})


def config_small(seed=7, dims=(24, 20, 18), dtype=np.uint8, image=(40, 32), op="central",
                 shading="blinn_phong", projection="persp", ert=0.0, skip=False, step=0.5,
                 spacing=(1.0, 1.0, 1.0)):
    """Small randomised scene for parity tests: several tiles plus a ragged tail."""
    nx, ny, nz = dims
    vmin, vmax = value_range(dtype)
    if np.dtype(dtype) == np.float32:
        vol = blob_volume((nz, ny, nx), 3, seed=seed, dtype=np.float32, sigma=(2.0, 5.0),
                          amp=(0.3, 1.0), normalise=True)
    elif np.dtype(dtype) == np.uint16:
        vol = phantom_volume((nz, ny, nx), 4, seed=seed, dtype=np.uint16)
    else:
        vol = blob_volume((nz, ny, nx), 3, seed=seed, dtype=np.uint8, sigma=(2.0, 6.0))
    if np.dtype(dtype) == np.uint16:
        # breakpoints inside the small phantom's own value range (a few
        # ellipsoids reach a few hundred to ~1500 of the 12-bit scale)
        top = max(0.06, 0.9 * float(vol.max()) / 4095.0)
        tf = tf_ramps(4096, seed=seed + 11, alpha_min=0.02, alpha_max=0.3, lo=0.03, hi=top)
    else:
        tf = tf_ramps(256, seed=seed + 11, alpha_min=0.02, alpha_max=0.3, lo=0.08, hi=0.9)
    cam = orbit_camera(dims, spacing, 35.0 + seed, 25.0, image[0], image[1],
                       projection=projection)
    return Scene(f"small_{seed}", vol, tuple(float(s) for s in spacing), vmin, vmax, tf, [cam],
                 default_shading(shading), default_options(step, op, ert, skip))
