"""ctypes front end of the FP64 CPU raycaster in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product package
never imports this module, and this module imports nothing from it.

Inputs are the plain dicts produced by :mod:`workloads` (camera, shading,
options) plus a numpy volume ``[nz][ny][nx]`` and an ``[M][4]`` table.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OP = {"central": 0, "sobel3d": 1, "zucker_hummel": 2}
SHADE = {"none": 0, "blinn_phong": 1, "paper_lambert": 2}
FLAG_HIT, FLAG_TIE, FLAG_ERT_NEAR, FLAG_ISO_NEAR, FLAG_ADAPT_NEAR = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-shared", "-fPIC",
               "-Wall", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class _Volume(C.Structure):
    _fields_ = [("data", C.POINTER(C.c_double)), ("nx", C.c_int), ("ny", C.c_int),
                ("nz", C.c_int), ("spacing", C.c_double * 3), ("vmin", C.c_double),
                ("vmax", C.c_double)]


class _Camera(C.Structure):
    _fields_ = [("projection", C.c_int), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("fov_y_deg", C.c_double), ("ortho_height", C.c_double),
                ("width", C.c_int), ("height", C.c_int)]


class _Shading(C.Structure):
    _fields_ = [("model", C.c_int), ("ka", C.c_double), ("kd", C.c_double), ("ks", C.c_double),
                ("shininess", C.c_double), ("light_is_point", C.c_int),
                ("light", C.c_double * 3), ("grad_eps", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("step", C.c_double), ("gradient_op", C.c_int), ("ert_threshold", C.c_double),
                ("clip_lo", C.c_double * 3), ("clip_hi", C.c_double * 3), ("nearest", C.c_int),
                ("ref_step", C.c_double), ("adapt_factor", C.c_int), ("adapt_range", C.c_double)]


class _SurfaceOptions(C.Structure):
    _fields_ = [("step", C.c_double), ("gradient_op", C.c_int), ("iso_lo", C.c_double),
                ("iso_hi", C.c_double), ("refine", C.c_int), ("clip_lo", C.c_double * 3),
                ("clip_hi", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_long)
        L.orc_sample.restype = C.c_double
        L.orc_sample.argtypes = [C.POINTER(_Volume), dp]
        L.orc_sample_nearest.restype = C.c_double
        L.orc_sample_nearest.argtypes = [C.POINTER(_Volume), dp]
        L.orc_gradient.restype = None
        L.orc_gradient.argtypes = [C.POINTER(_Volume), C.c_int, dp, dp, dp]
        L.orc_tf.restype = None
        L.orc_tf.argtypes = [dp, C.c_int, C.c_double, dp]
        L.orc_camera_ray.restype = None
        L.orc_camera_ray.argtypes = [C.POINTER(_Camera), C.c_int, C.c_int, dp, dp]
        L.orc_ray_box.restype = C.c_int
        L.orc_ray_box.argtypes = [dp, dp, dp, dp, dp, dp]
        L.orc_shade.restype = None
        L.orc_shade.argtypes = [C.POINTER(_Shading), dp, dp, dp, dp, dp]
        L.orc_render.restype = C.c_int
        L.orc_render.argtypes = [C.POINTER(_Volume), C.POINTER(_Camera), dp, C.c_int,
                                 C.POINTER(_Shading), C.POINTER(_Options), lp, C.c_long,
                                 dp, dp, ip, ip, dp, C.c_int]
        L.orc_render_grad.restype = C.c_int
        L.orc_render_grad.argtypes = [C.POINTER(_Volume), C.POINTER(_Camera), dp, C.c_int,
                                      C.POINTER(_Shading), C.POINTER(_Options), lp, C.c_long,
                                      dp, dp, dp, dp]
        L.orc_render_surface.restype = C.c_int
        L.orc_render_surface.argtypes = [C.POINTER(_Volume), C.POINTER(_Camera), dp, C.c_int,
                                         C.POINTER(_Shading), C.POINTER(_SurfaceOptions), lp,
                                         C.c_long, dp, dp, ip, ip, C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Volume:
    """Keeps the FP64 copy of the voxels alive while the struct points at it."""

    def __init__(self, vol, spacing=(1.0, 1.0, 1.0), vmin=0.0, vmax=1.0):
        self.data = np.ascontiguousarray(vol, dtype=np.float64)
        nz, ny, nx = self.data.shape
        self.s = _Volume(_dp(self.data), nx, ny, nz, (C.c_double * 3)(*spacing),
                         float(vmin), float(vmax))


def _camera(cam):
    return _Camera(1 if cam["projection"] == "persp" else 0, (C.c_double * 3)(*cam["eye"]),
                   (C.c_double * 3)(*cam["target"]), (C.c_double * 3)(*cam["up"]),
                   float(cam["fov_y_deg"]), float(cam["ortho_height"]), int(cam["width"]),
                   int(cam["height"]))


def _shading(sh):
    return _Shading(SHADE[sh["model"]], sh["ka"], sh["kd"], sh["ks"], sh["shininess"],
                    int(sh["light_is_point"]), (C.c_double * 3)(*sh["light"]), sh["grad_eps"])


def _options(opt):
    return _Options(opt["step"], OP[opt["gradient_op"]], opt["ert_threshold"],
                    (C.c_double * 3)(*opt["clip_lo"]), (C.c_double * 3)(*opt["clip_hi"]),
                    int(bool(opt.get("nearest", False))), float(opt.get("ref_step", 0.0)),
                    int(opt.get("adapt_factor", 0)), float(opt.get("adapt_range", 0.0)))


def sample(vol: Volume, p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_sample(C.byref(vol.s), _dp(p))


def sample_nearest(vol: Volume, p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_sample_nearest(C.byref(vol.s), _dp(p))


def gradient(vol: Volume, op: str, p):
    """(scaled gradient, raw stencil sum) at voxel-space point p."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    g, raw = np.zeros(3), np.zeros(3)
    lib().orc_gradient(C.byref(vol.s), OP[op], _dp(p), _dp(g), _dp(raw))
    return g, raw


def tf_lookup(tf, u):
    t = np.ascontiguousarray(tf, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_tf(_dp(t), t.shape[0], float(u), _dp(out))
    return out


def camera_ray(cam, px, py):
    o, d = np.zeros(3), np.zeros(3)
    c = _camera(cam)
    lib().orc_camera_ray(C.byref(c), int(px), int(py), _dp(o), _dp(d))
    return o, d


def ray_box(o, d, lo, hi):
    o, d, lo, hi = (np.ascontiguousarray(a, dtype=np.float64) for a in (o, d, lo, hi))
    t0, t1 = C.c_double(), C.c_double()
    hit = lib().orc_ray_box(_dp(o), _dp(d), _dp(lo), _dp(hi), C.byref(t0), C.byref(t1))
    return bool(hit), t0.value, t1.value


def shade(sh, rgb, g, p_world, d):
    s = _shading(sh)
    rgb, g, pw, d = (np.ascontiguousarray(a, dtype=np.float64) for a in (rgb, g, p_world, d))
    c = np.zeros(3)
    lib().orc_shade(C.byref(s), _dp(rgb), _dp(g), _dp(pw), _dp(d), _dp(c))
    return c


def render(vol: Volume, cam, tf, shading, options, pixels=None, threads=0):
    """Render all pixels (``pixels=None``) or the listed linear pixel indices.

    Returns a dict with rgba [n,4] (or [H,W,4] for a full frame), rgba_alt,
    flags, k_last and t_final.
    """
    L = lib()
    c, s, o = _camera(cam), _shading(shading), _options(options)
    t = np.ascontiguousarray(tf, dtype=np.float64)
    W, H = cam["width"], cam["height"]
    if pixels is None:
        n, pix_p, full = W * H, None, True
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n, pix_p, full = pix.size, pix.ctypes.data_as(C.POINTER(C.c_long)), False
    rgba, alt = np.zeros((n, 4)), np.zeros((n, 4))
    flags, kl = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
    tfin = np.zeros(n)
    rc = L.orc_render(C.byref(vol.s), C.byref(c), _dp(t), t.shape[0], C.byref(s), C.byref(o),
                      pix_p, n, _dp(rgba), _dp(alt), flags.ctypes.data_as(C.POINTER(C.c_int)),
                      kl.ctypes.data_as(C.POINTER(C.c_int)), _dp(tfin), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out = {"rgba": rgba, "rgba_alt": alt, "flags": flags, "k_last": kl, "t_final": tfin}
    if full:
        out = {k: v.reshape((H, W) + v.shape[1:]) for k, v in out.items()}
    return out


def render_grad(vol: Volume, cam, tf, options, g_rgba, pixels=None, shading=None,
                abs_sum=False):
    """dL/dvolume [nz,ny,nx] and dL/dTF [M,4]; shading None means NONE.

    With abs_sum, a third array [nz,ny,nx]: per voxel, the sum of the
    magnitudes of the terms that make up its dL/dvolume entry (how much
    cancellation the entry carries)."""
    L = lib()
    c, o = _camera(cam), _options(options)
    s = C.byref(_shading(shading)) if shading is not None else None
    t = np.ascontiguousarray(tf, dtype=np.float64)
    g = np.ascontiguousarray(g_rgba, dtype=np.float64).reshape(-1, 4)
    if pixels is None:
        n, pix_p = cam["width"] * cam["height"], None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n, pix_p = pix.size, pix.ctypes.data_as(C.POINTER(C.c_long))
    assert g.shape[0] == n
    dvol = np.zeros(vol.data.shape)
    dtf = np.zeros(t.shape)
    dabs = np.zeros(vol.data.shape) if abs_sum else None
    rc = L.orc_render_grad(C.byref(vol.s), C.byref(c), _dp(t), t.shape[0], s, C.byref(o), pix_p,
                           n, _dp(g), _dp(dvol), _dp(dtf), _dp(dabs) if abs_sum else None)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return (dvol, dtf, dabs) if abs_sum else (dvol, dtf)


def _surface_options(opt):
    return _SurfaceOptions(opt["step"], OP[opt["gradient_op"]], float(opt["iso_lo"]),
                           float(opt["iso_hi"]), int(opt["refine"]),
                           (C.c_double * 3)(*opt["clip_lo"]), (C.c_double * 3)(*opt["clip_hi"]))


def render_surface(vol: Volume, cam, tf, shading, options, pixels=None, threads=0):
    """First-hit surface render of all pixels or the listed linear indices.

    Returns rgba [n,4], t_hit [n] (+inf without a surface), k_hit [n] (-1)
    and flags [n]; full frames come back as [H,W,...].
    """
    L = lib()
    c, s, o = _camera(cam), _shading(shading), _surface_options(options)
    t = np.ascontiguousarray(tf, dtype=np.float64)
    W, H = cam["width"], cam["height"]
    if pixels is None:
        n, pix_p, full = W * H, None, True
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n, pix_p, full = pix.size, pix.ctypes.data_as(C.POINTER(C.c_long)), False
    rgba, th = np.zeros((n, 4)), np.zeros(n)
    kh, flags = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
    rc = L.orc_render_surface(C.byref(vol.s), C.byref(c), _dp(t), t.shape[0], C.byref(s),
                              C.byref(o), pix_p, n, _dp(rgba), _dp(th),
                              kh.ctypes.data_as(C.POINTER(C.c_int)),
                              flags.ctypes.data_as(C.POINTER(C.c_int)), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out = {"rgba": rgba, "t_hit": th, "k_hit": kh, "flags": flags}
    if full:
        out = {k: v.reshape((H, W) + v.shape[1:]) for k, v in out.items()}
    return out
