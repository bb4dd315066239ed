"""Independent NumPy raycaster for tiny grids -- a second formulation that
pins the C oracle.  It is written differently on purpose:

* trilinear interpolation as the explicit 8-term sum  sum_c V_c prod_a w_a
  (not the 7-lerp cascade of Section 3.4);
* gradients in *corner-blend* form: the integer 3x3x3 stencil is applied at
  the 8 cell corners (taps clamped to the grid) and the results are blended
  with the trilinear weights.  By linearity this equals the tap form the
  oracle uses (each tap a trilinear sample), so agreement checks both;
* the masks are explicit 3x3x3 arrays, the Sobel3D x mask typed from the
  printed slices of eq. (4) and the other components obtained by rotating
  the array, the Zucker-Hummel mask from its defining formula;
* the table lookup uses numpy.interp over entry indices;
* compositing runs *back to front* with eq. (6) of Section 3.9,
  C_out = C_in (1 - a) + C a, starting from black behind the last sample.

Slow (Python loop over pixels); meant for grids of a few voxels per edge.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- masks
def sobel_x_mask():
    """Eq. (4): slices x-1, x, x+1 of the x-derivative mask, indexed [dx][dy][dz]."""
    w = np.array([[1, 3, 1], [3, 6, 3], [1, 3, 1]], dtype=np.float64)
    m = np.zeros((3, 3, 3))
    m[0] = -w
    m[2] = w
    return m


def zh_x_mask():
    m = np.zeros((3, 3, 3))
    for dx in (-1, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                m[dx + 1, dy + 1, dz + 1] = dx / math.sqrt(dx * dx + dy * dy + dz * dz)
    return m


def cd_x_mask():
    m = np.zeros((3, 3, 3))
    m[0, 1, 1], m[2, 1, 1] = -1.0, 1.0
    return m


def masks(op):
    """Three masks [component][dx][dy][dz] for an operator name."""
    mx = {"central": cd_x_mask, "sobel3d": sobel_x_mask, "zucker_hummel": zh_x_mask}[op]()
    # y mask: the x mask with its axes (x, y, z) moved to (y, z, x): m_y[dx,dy,dz] = m_x[dy,dz,dx]
    my = np.transpose(mx, (2, 0, 1))
    mz = np.transpose(mx, (1, 2, 0))
    return np.stack([mx, my, mz])


def gain(op):
    """Response of the x mask to the unit-slope field V = x."""
    m = masks(op)[0]
    return float(sum(m[i, j, k] * (i - 1) for i in range(3) for j in range(3) for k in range(3)))


# ---------------------------------------------------------------- volume access
class Grid:
    def __init__(self, vol_zyx, spacing, vmin, vmax):
        self.v = np.asarray(vol_zyx, dtype=np.float64)
        self.nz, self.ny, self.nx = self.v.shape
        self.s = np.asarray(spacing, dtype=np.float64)
        self.vmin, self.vmax = float(vmin), float(vmax)

    def at(self, i, j, k):
        i = min(max(i, 0), self.nx - 1)
        j = min(max(j, 0), self.ny - 1)
        k = min(max(k, 0), self.nz - 1)
        return self.v[k, j, i]

    def corners(self, p):
        base = np.floor(p).astype(np.int64)
        f = p - base
        out = []
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    w = ((f[0] if cx else 1 - f[0]) * (f[1] if cy else 1 - f[1])
                         * (f[2] if cz else 1 - f[2]))
                    out.append((w, base[0] + cx, base[1] + cy, base[2] + cz))
        return out

    def sample(self, p):
        return sum(w * self.at(i, j, k) for w, i, j, k in self.corners(p))

    def stencil(self, masks3, i, j, k):
        g = np.zeros(3)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    val = self.at(i + dx, j + dy, k + dz)
                    g += masks3[:, dx + 1, dy + 1, dz + 1] * val
        return g

    def gradient(self, op, p):
        m = masks(op)
        raw = np.zeros(3)
        for w, i, j, k in self.corners(p):
            if w != 0.0:
                raw += w * self.stencil(m, i, j, k)
        return raw / gain(op) / self.s / (self.vmax - self.vmin), raw


# ---------------------------------------------------------------- camera and box
def camera_frame(cam):
    eye = np.asarray(cam["eye"], dtype=np.float64)
    fwd = np.asarray(cam["target"], dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(cam["up"], dtype=np.float64))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return eye, fwd, right, up


def pixel_ray(cam, px, py):
    eye, fwd, right, up = camera_frame(cam)
    W, H = cam["width"], cam["height"]
    sx = ((px + 0.5) / W * 2.0 - 1.0) * (W / H)
    sy = 1.0 - (py + 0.5) / H * 2.0
    if cam["projection"] == "persp":
        half = math.tan(math.radians(cam["fov_y_deg"]) / 2.0)
        point = eye + fwd + half * (sx * right + sy * up)   # image plane at distance 1
        d = point - eye
        return eye.copy(), d / np.linalg.norm(d)
    h = cam["ortho_height"] / 2.0
    return eye + h * (sx * right + sy * up), fwd


def box_span(o, d, lo, hi):
    """(t_in, t_out) of the slab intersection clamped to t >= 0, or None."""
    t_near, t_far = 0.0, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (lo[a] <= o[a] <= hi[a]):
                return None
            continue
        ta, tb = sorted(((lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]))
        t_near, t_far = max(t_near, ta), min(t_far, tb)
    return (t_near, t_far) if t_near <= t_far else None


# ---------------------------------------------------------------- shading
def shade(sh, rgb, g, pw, d):
    if sh["model"] == "none":
        return np.asarray(rgb[:3], dtype=np.float64)
    gl = float(np.linalg.norm(g))
    gh = np.asarray(g) / max(gl, sh["grad_eps"])
    light = np.asarray(sh["light"], dtype=np.float64)
    L = light - pw if sh["light_is_point"] else light.copy()
    L = L / np.linalg.norm(L)
    if sh["model"] == "paper_lambert":
        return np.asarray(rgb[:3]) * float(np.dot(L, gh))
    N = -gh
    Hh = L - d
    Hh = Hh / np.linalg.norm(Hh)
    diff = max(0.0, float(np.dot(N, L)))
    spec = max(0.0, float(np.dot(N, Hh))) ** sh["shininess"]
    return np.asarray(rgb[:3]) * (sh["ka"] + sh["kd"] * diff) + sh["ks"] * spec


# ---------------------------------------------------------------- render
def render(vol_zyx, spacing, vmin, vmax, tf, cam, sh, opt, pixels=None, n_override=None):
    """rgba [n,4] for linear pixel ids (all pixels by default).

    ``n_override`` maps pixel id -> sample count to force (used where the
    lattice end is a tie).
    """
    g = Grid(vol_zyx, spacing, vmin, vmax)
    tf = np.asarray(tf, dtype=np.float64)
    M = tf.shape[0]
    ent = np.arange(M, dtype=np.float64)
    W, H = cam["width"], cam["height"]
    ext = (np.array([g.nx, g.ny, g.nz]) - 1) * g.s
    lo = np.maximum(np.asarray(opt["clip_lo"]), 0.0)
    hi = np.minimum(np.asarray(opt["clip_hi"]), ext)
    ids = range(W * H) if pixels is None else pixels
    out = []
    for pid in ids:
        px, py = pid % W, pid // W
        o, d = pixel_ray(cam, px, py)
        span = box_span(o, d, lo, hi) if np.all(lo <= hi) else None
        if n_override is not None and pid in n_override:
            n = n_override[pid]
            if n > 0 and span is None:
                raise ValueError("forced samples on a missing ray")
        else:
            n = 0 if span is None else int(math.floor((span[1] - span[0]) / opt["step"])) + 1
        alphas, cols = [], []
        nearest = opt.get("nearest", False)
        ref = opt.get("ref_step", 0.0)
        for k in range(n):
            t = span[0] + k * opt["step"]
            pw = o + t * d
            pv = pw / g.s
            if nearest:
                idx = [int(math.floor(c + 0.5)) for c in pv]
                val = g.at(*idx)
            else:
                val = g.sample(pv)
            u = min(max((val - vmin) / (vmax - vmin), 0.0), 1.0) * (M - 1)
            rgba = np.array([np.interp(u, ent, tf[:, c]) for c in range(4)])
            if ref > 0 and rgba[3] < 1.0:
                # the same opacity per unit length: -log(1-a) scales with the step
                rgba[3] = -math.expm1(math.log1p(-rgba[3]) * opt["step"] / ref)
            if sh["model"] != "none" and rgba[3] != 0.0:
                if nearest:
                    raw = g.stencil(masks(opt["gradient_op"]), *idx)
                    grad = raw / gain(opt["gradient_op"]) / g.s / (g.vmax - g.vmin)
                else:
                    grad, _ = g.gradient(opt["gradient_op"], pv)
                col = shade(sh, rgba, grad, pw, d)
            else:
                col = rgba[:3]
            alphas.append(rgba[3])
            cols.append(col)
        # early termination is defined front to back: find the last sample kept
        keep = len(alphas)
        tau = opt["ert_threshold"]
        if tau > 0:
            T = 1.0
            for k, a in enumerate(alphas):
                T *= (1.0 - a)
                if 1.0 - T >= tau:
                    keep = k + 1
                    break
        # eq. (6), back to front over the kept samples
        C = np.zeros(3)
        A = 0.0
        for k in reversed(range(keep)):
            a = alphas[k]
            C = C * (1.0 - a) + cols[k] * a
            A = A * (1.0 - a) + a
        out.append(np.concatenate([C, [A]]))
    return np.array(out).reshape(-1, 4)


# ---------------------------------------------------------------- first-hit surface
def render_surface(vol_zyx, spacing, vmin, vmax, tf, cam, sh, opt, pixels=None):
    """(rgba [n,4], t_hit [n]) of the first-hit surface mode, written as an
    interval bisection: the last coarse interval [t_{k-1}, t_k] is halved
    refine-1 times by the window test at its midpoint, and the hit is the
    midpoint of what is left (refine = 0 keeps t_k; a ray that starts inside
    the window keeps t_in)."""
    g = Grid(vol_zyx, spacing, vmin, vmax)
    tf = np.asarray(tf, dtype=np.float64)
    M = tf.shape[0]
    ent = np.arange(M, dtype=np.float64)
    W, H = cam["width"], cam["height"]
    ext = (np.array([g.nx, g.ny, g.nz]) - 1) * g.s
    lo_b = np.maximum(np.asarray(opt["clip_lo"]), 0.0)
    hi_b = np.minimum(np.asarray(opt["clip_hi"]), ext)
    ids = range(W * H) if pixels is None else pixels
    step = opt["step"]

    def value(o, d, t):
        return g.sample((o + t * d) / g.s)

    def inside(val):
        return opt["iso_lo"] <= val <= opt["iso_hi"]

    out, th = [], []
    for pid in ids:
        px, py = pid % W, pid // W
        o, d = pixel_ray(cam, px, py)
        span = box_span(o, d, lo_b, hi_b) if np.all(lo_b <= hi_b) else None
        n = 0 if span is None else int(math.floor((span[1] - span[0]) / step)) + 1
        hit = next((k for k in range(n) if inside(value(o, d, span[0] + k * step))), None)
        if hit is None:
            out.append(np.zeros(4))
            th.append(math.inf)
            continue
        t_k = span[0] + hit * step
        if hit == 0 or opt["refine"] == 0:
            t = t_k
        else:
            a, b = t_k - step, t_k
            for _ in range(opt["refine"] - 1):
                m = 0.5 * (a + b)
                if inside(value(o, d, m)):
                    b = m
                else:
                    a = m
            t = 0.5 * (a + b)
        pw = o + t * d
        pv = pw / g.s
        val = g.sample(pv)
        u = min(max((val - vmin) / (vmax - vmin), 0.0), 1.0) * (M - 1)
        rgb = np.array([np.interp(u, ent, tf[:, c]) for c in range(3)])
        if sh["model"] != "none":
            grad, _ = g.gradient(opt["gradient_op"], pv)
            rgb = shade(sh, rgb, grad, pw, d)
        out.append(np.concatenate([rgb, [1.0]]))
        th.append(t)
    return np.array(out).reshape(-1, 4), np.array(th)


# ---------------------------------------------------------------- adaptive sampling
def poor_brick_flags(vol_zyx, adapt_range):
    """Detail-poor flags of the 8^3 bricks: value range over the brick plus
    its one-voxel high apron (edge-replicated), via numpy slicing."""
    v = np.asarray(vol_zyx, dtype=np.float64)
    nz, ny, nx = v.shape
    nbz, nby, nbx = (nz + 7) // 8, (ny + 7) // 8, (nx + 7) // 8
    pad = np.pad(v, ((0, 8 * nbz + 1 - nz), (0, 8 * nby + 1 - ny), (0, 8 * nbx + 1 - nx)),
                 mode="edge")
    flags = np.zeros((nbz, nby, nbx), dtype=bool)
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                blk = pad[8 * bz:8 * bz + 9, 8 * by:8 * by + 9, 8 * bx:8 * bx + 9]
                flags[bz, by, bx] = blk.max() - blk.min() <= adapt_range
    return flags


def render_adaptive(vol_zyx, spacing, vmin, vmax, tf, cam, sh, opt, pixels=None):
    """rgba [n,4] of the adaptive march, written as a list of (t, step)
    pairs built first and composited afterwards (front to back)."""
    g = Grid(vol_zyx, spacing, vmin, vmax)
    flags = poor_brick_flags(vol_zyx, opt["adapt_range"])
    tf = np.asarray(tf, dtype=np.float64)
    M = tf.shape[0]
    ent = np.arange(M, dtype=np.float64)
    W, H = cam["width"], cam["height"]
    ext = (np.array([g.nx, g.ny, g.nz]) - 1) * g.s
    lo = np.maximum(np.asarray(opt["clip_lo"]), 0.0)
    hi = np.minimum(np.asarray(opt["clip_hi"]), ext)
    ref = opt.get("ref_step", 0.0) or opt["step"]
    m = opt["adapt_factor"]
    ids = range(W * H) if pixels is None else pixels
    out = []
    for pid in ids:
        px, py = pid % W, pid // W
        o, d = pixel_ray(cam, px, py)
        span = box_span(o, d, lo, hi) if np.all(lo <= hi) else None
        plan = []
        if span is not None:
            t = span[0]
            while t <= span[1]:
                pv = (o + t * d) / g.s
                b = [min(max(int(math.floor(c)), 0), n - 1) // 8
                     for c, n in zip(pv, (g.nx, g.ny, g.nz))]
                step = m * opt["step"] if flags[b[2], b[1], b[0]] else opt["step"]
                plan.append((t, step))
                t += step
        C, T = np.zeros(3), 1.0
        for t, step in plan:
            pw = o + t * d
            pv = pw / g.s
            val = g.sample(pv)
            u = min(max((val - vmin) / (vmax - vmin), 0.0), 1.0) * (M - 1)
            rgba = np.array([np.interp(u, ent, tf[:, c]) for c in range(4)])
            a = rgba[3]
            if 0.0 < a < 1.0:
                a = -math.expm1(math.log1p(-a) * step / ref)
            col = rgba[:3]
            if sh["model"] != "none" and a != 0.0:
                grad, _ = g.gradient(opt["gradient_op"], pv)
                col = shade(sh, rgba, grad, pw, d)
            C = C + T * a * np.asarray(col)
            T *= 1.0 - a
            if opt["ert_threshold"] > 0 and 1.0 - T >= opt["ert_threshold"]:
                break
        out.append(np.concatenate([C, [1.0 - T]]))
    return np.array(out).reshape(-1, 4)
