"""Python binding of ``librc.so``, the gfx950 volume raycaster.

Argument marshalling only: every step of the render runs in the HIP
kernels behind the C ABI declared in ``include/rc.h``.  PyTorch provides
device memory and the current stream.  The functions carry the C names;
cameras, shading and options are plain dicts with the C struct field
names (see ``include/rc.h``).  If the shared library is missing the
import still works, but every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

__all__ = [
    "RCError", "Volume", "rc_create_volume", "rc_update_volume", "rc_build_bricks",
    "rc_render", "rc_render_backward", "rc_destroy_volume", "rc_last_error", "RenderFn",
    "camera_struct", "shading_struct", "options_struct", "library_path",
    "Batch", "rc_batch_create", "rc_batch_render", "rc_batch_destroy", "rc_render_batch",
    "rc_batch_autotune", "rc_render_views", "rc_render_backward_views", "RenderViewsFn",
    "rc_render_surface", "surface_options_struct", "rc_debug_bounds_violations",
    "rc_debug_bounds_reset", "rc_render_views_noalloc", "NOALLOC_SCRATCH_BYTES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# RC_LIBRARY=debug selects the bounds-checked build (librc_debug.so), for tests
_LIB_NAMES = {"": "librc.so", "product": "librc.so", "debug": "librc_debug.so"}
if os.environ.get("RC_LIBRARY", "") not in _LIB_NAMES:
    raise RuntimeError(f"RC_LIBRARY must be one of {sorted(_LIB_NAMES)[1:]}")
_LIB_PATH = os.path.join(_HERE, _LIB_NAMES[os.environ.get("RC_LIBRARY", "")])

RC_OK, RC_E_INVALID, RC_E_OOM, RC_E_DEVICE, RC_E_STATE, RC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
RC_U8, RC_U16, RC_F32 = 0, 1, 2
GRADIENT_OPS = {"central": 0, "sobel3d": 1, "zucker_hummel": 2}
SHADING_MODELS = {"none": 0, "blinn_phong": 1, "paper_lambert": 2}
PROJECTIONS = {"ortho": 0, "persp": 1}


class RCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"rc status {status}: {message}")
        self.status = status


# ---------------------------------------------------------------- C structs
class rc_camera(C.Structure):
    _fields_ = [("projection", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("reserved", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("fov_y_deg", C.c_double), ("ortho_height", C.c_double)]


class rc_shading(C.Structure):
    _fields_ = [("model", C.c_int32), ("light_is_point", C.c_int32), ("ka", C.c_float),
                ("kd", C.c_float), ("ks", C.c_float), ("shininess", C.c_float),
                ("light", C.c_float * 3), ("grad_eps", C.c_float)]


class rc_options(C.Structure):
    _fields_ = [("step", C.c_double), ("clip_lo", C.c_double * 3), ("clip_hi", C.c_double * 3),
                ("ert_threshold", C.c_float), ("gradient_op", C.c_int32),
                ("skip_empty", C.c_int32), ("reserved", C.c_int32), ("sampling", C.c_int32),
                ("opacity_ref_step", C.c_float), ("adapt_factor", C.c_int32),
                ("adapt_range", C.c_float)]


class rc_surface_options(C.Structure):
    _fields_ = [("step", C.c_double), ("clip_lo", C.c_double * 3), ("clip_hi", C.c_double * 3),
                ("iso_lo", C.c_float), ("iso_hi", C.c_float), ("refine_steps", C.c_int32),
                ("gradient_op", C.c_int32), ("skip_empty", C.c_int32), ("reserved", C.c_int32)]


class rc_stats(C.Structure):
    _fields_ = [("lattice_samples", C.c_ulonglong), ("evaluated_samples", C.c_ulonglong),
                ("shaded_samples", C.c_ulonglong), ("rays_hit", C.c_ulonglong),
                ("chunks_staged", C.c_ulonglong), ("chunks_empty", C.c_ulonglong),
                ("chunks_direct", C.c_ulonglong), ("samples_direct", C.c_ulonglong)]


STATS_FIELDS = [f for f, _ in rc_stats._fields_]


def new_stats(device="cuda") -> torch.Tensor:
    """Zeroed int64 tensor laid out as rc_stats (see STATS_FIELDS)."""
    return torch.zeros(len(STATS_FIELDS), dtype=torch.int64, device=device)


class rc_batch_item(C.Structure):
    _fields_ = [("vol", C.c_void_p), ("cam", rc_camera), ("tf_rgba_dev", C.c_void_p),
                ("tf_len", C.c_int32), ("reserved", C.c_int32), ("sh", rc_shading),
                ("opt", rc_options), ("out_rgba_dev", C.c_void_p), ("aux_dev", C.c_void_p)]


class rc_batch_config(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("waves_per_wg", C.c_int32), ("wg_per_cu", C.c_int32),
                ("order", C.c_int32), ("box_bytes_grad", C.c_int32), ("box_bytes_cd", C.c_int32),
                ("chunk_len", C.c_int32)]


BATCH_CONFIG_FIELDS = [f for f, _ in rc_batch_config._fields_]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build() "
                               "(there is no non-HIP fallback)")
        L = C.CDLL(_LIB_PATH)
        vp, cp = C.c_void_p, C.c_char_p
        L.rc_last_error.restype = cp
        L.rc_last_error.argtypes = []
        L.rc_create_volume.restype = C.c_int
        L.rc_create_volume.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.POINTER(C.c_double), C.c_float, C.c_float, vp,
                                       C.POINTER(vp)]
        L.rc_update_volume.restype = C.c_int
        L.rc_update_volume.argtypes = [vp, vp, vp]
        L.rc_build_bricks.restype = C.c_int
        L.rc_build_bricks.argtypes = [vp, C.c_int, vp]
        L.rc_render.restype = C.c_int
        L.rc_render.argtypes = [vp, C.POINTER(rc_camera), vp, C.c_int, C.POINTER(rc_shading),
                                C.POINTER(rc_options), vp, vp, vp, vp]
        L.rc_render_backward.restype = C.c_int
        L.rc_render_backward.argtypes = [vp, C.POINTER(rc_camera), vp, C.c_int,
                                         C.POINTER(rc_shading), C.POINTER(rc_options), vp, vp,
                                         vp, vp, vp]
        L.rc_destroy_volume.restype = None
        L.rc_destroy_volume.argtypes = [vp]
        bi, bc = C.POINTER(rc_batch_item), C.POINTER(rc_batch_config)
        L.rc_batch_create.restype = C.c_int
        L.rc_batch_create.argtypes = [bi, C.c_int, bc, vp, C.POINTER(vp)]
        L.rc_batch_render.restype = C.c_int
        L.rc_batch_render.argtypes = [vp, C.c_int, vp]
        L.rc_batch_destroy.restype = None
        L.rc_batch_destroy.argtypes = [vp]
        L.rc_render_batch.restype = C.c_int
        L.rc_render_batch.argtypes = [bi, C.c_int, bc, vp]
        L.rc_batch_autotune.restype = C.c_int
        L.rc_batch_autotune.argtypes = [bi, C.c_int, C.c_char_p, vp, bc]
        pp = C.POINTER(vp)
        L.rc_render_views.restype = C.c_int
        L.rc_render_views.argtypes = [vp, C.POINTER(rc_camera), C.c_int, vp, C.c_int,
                                      C.POINTER(rc_shading), C.POINTER(rc_options), pp, pp, vp]
        L.rc_render_views_noalloc.restype = C.c_int
        L.rc_render_views_noalloc.argtypes = L.rc_render_views.argtypes
        L.rc_render_backward_views.restype = C.c_int
        L.rc_render_backward_views.argtypes = [vp, C.POINTER(rc_camera), C.c_int, vp, C.c_int,
                                               C.POINTER(rc_shading), C.POINTER(rc_options), pp,
                                               pp, vp, vp, vp]
        L.rc_render_surface.restype = C.c_int
        L.rc_render_surface.argtypes = [vp, C.POINTER(rc_camera), vp, C.c_int,
                                        C.POINTER(rc_shading), C.POINTER(rc_surface_options), vp,
                                        vp, vp]
        L.rc_debug_bounds_violations.restype = C.c_int
        L.rc_debug_bounds_violations.argtypes = [C.POINTER(C.c_ulonglong)]
        L.rc_debug_bounds_reset.restype = C.c_int
        L.rc_debug_bounds_reset.argtypes = []
        _lib = L
    return _lib


def rc_last_error() -> str:
    return _L().rc_last_error().decode()


def _check(st):
    if st != RC_OK:
        raise RCError(st, rc_last_error())


def rc_debug_bounds_violations() -> int:
    """Device-side index violations counted by the bounds-checked build since
    the last reset (synchronises the device); RCError(RC_E_UNSUPPORTED) in
    the product build."""
    n = C.c_ulonglong(0)
    _check(_L().rc_debug_bounds_violations(C.byref(n)))
    return int(n.value)


def rc_debug_bounds_reset():
    _check(_L().rc_debug_bounds_reset())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------- dict -> struct
def camera_struct(cam: dict) -> rc_camera:
    return rc_camera(PROJECTIONS[cam["projection"]], int(cam["width"]), int(cam["height"]), 0,
                     (C.c_double * 3)(*cam["eye"]), (C.c_double * 3)(*cam["target"]),
                     (C.c_double * 3)(*cam["up"]), float(cam["fov_y_deg"]),
                     float(cam["ortho_height"]))


def shading_struct(sh: dict) -> rc_shading:
    return rc_shading(SHADING_MODELS[sh["model"]], int(bool(sh["light_is_point"])), sh["ka"],
                      sh["kd"], sh["ks"], sh["shininess"], (C.c_float * 3)(*sh["light"]),
                      sh["grad_eps"])


def options_struct(opt: dict) -> rc_options:
    return rc_options(float(opt["step"]), (C.c_double * 3)(*opt["clip_lo"]),
                      (C.c_double * 3)(*opt["clip_hi"]), float(opt["ert_threshold"]),
                      GRADIENT_OPS[opt["gradient_op"]], int(bool(opt["skip_empty"])), 0,
                      int(bool(opt.get("nearest", False))), float(opt.get("ref_step", 0.0)),
                      int(opt.get("adapt_factor", 0)), float(opt.get("adapt_range", 0.0)))


def surface_options_struct(opt: dict) -> rc_surface_options:
    return rc_surface_options(float(opt["step"]), (C.c_double * 3)(*opt["clip_lo"]),
                              (C.c_double * 3)(*opt["clip_hi"]), float(opt["iso_lo"]),
                              float(opt["iso_hi"]), int(opt["refine"]),
                              GRADIENT_OPS[opt["gradient_op"]], int(bool(opt["skip_empty"])), 0)


# ---------------------------------------------------------------- volumes
_DT = {torch.uint8: RC_U8, torch.uint16: RC_U16, torch.int16: RC_U16, torch.float32: RC_F32}


class Volume:
    """Owns an ``rc_volume*``; keeps the last source tensor alive."""

    def __init__(self, handle, shape_zyx, dtype, spacing, vmin, vmax, src):
        self.handle = handle
        self.shape = tuple(shape_zyx)
        self.dtype = dtype
        self.spacing = tuple(spacing)
        self.vmin, self.vmax = vmin, vmax
        self._src = src
        self.has_bricks = False

    def __del__(self):
        try:
            if self.handle:
                rc_destroy_volume(self)
        except Exception:
            pass


def _check_src(src):
    if not isinstance(src, torch.Tensor) or not src.is_cuda:
        raise TypeError("volume source must be a CUDA tensor")
    if src.dim() != 3 or not src.is_contiguous():
        raise ValueError("volume source must be a contiguous [nz][ny][nx] tensor")
    if src.dtype not in _DT:
        raise TypeError(f"unsupported voxel dtype {src.dtype} (uint8, uint16/int16 bits, float32)")


def rc_create_volume(src: torch.Tensor, spacing=(1.0, 1.0, 1.0), vmin=0.0, vmax=1.0,
                     stream=None) -> Volume:
    _check_src(src)
    nz, ny, nx = src.shape
    h = C.c_void_p()
    sp = (C.c_double * 3)(*spacing)
    _check(_L().rc_create_volume(_ptr(src), nx, ny, nz, _DT[src.dtype], sp, float(vmin),
                                 float(vmax), _stream(stream), C.byref(h)))
    return Volume(h, (nz, ny, nx), _DT[src.dtype], spacing, vmin, vmax, src)


def rc_update_volume(vol: Volume, src: torch.Tensor, stream=None):
    _check_src(src)
    if tuple(src.shape) != vol.shape or _DT[src.dtype] != vol.dtype:
        raise ValueError("rc_update_volume: shape/dtype differ from the volume")
    _check(_L().rc_update_volume(vol.handle, _ptr(src), _stream(stream)))
    vol._src = src


def rc_build_bricks(vol: Volume, brick_edge=8, stream=None):
    _check(_L().rc_build_bricks(vol.handle, int(brick_edge), _stream(stream)))
    vol.has_bricks = True


def rc_destroy_volume(vol: Volume):
    if vol.handle:
        _L().rc_destroy_volume(vol.handle)
        vol.handle = None


# ---------------------------------------------------------------- render
def _check_tf(tf):
    if not (isinstance(tf, torch.Tensor) and tf.is_cuda and tf.dtype == torch.float32
            and tf.dim() == 2 and tf.shape[1] == 4 and tf.is_contiguous()):
        raise ValueError("transfer function must be a contiguous CUDA float32 [M,4] tensor")


def rc_render(vol: Volume, camera: dict, tf: torch.Tensor, shading: dict, options: dict,
              out: torch.Tensor = None, aux: torch.Tensor = None, stats: torch.Tensor = None,
              stream=None) -> torch.Tensor:
    """Render one image; returns ``out`` ([H,W,4] float32).

    ``aux``: optional int64 [H,W] tensor receiving rc_aux records
    (k_last int32, t_final float32 packed per pixel).  ``stats``: optional
    int64 [8] tensor accumulating rc_stats (new_stats())."""
    _check_tf(tf)
    H, W = int(camera["height"]), int(camera["width"])
    if out is None:
        out = torch.empty((H, W, 4), dtype=torch.float32, device=tf.device)
    if out.shape != (H, W, 4) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [H,W,4] tensor")
    if aux is not None and (aux.numel() != H * W or aux.element_size() * aux.numel() != 8 * H * W):
        raise ValueError("aux must hold H*W 8-byte records")
    if stats is not None and stats.numel() * stats.element_size() != C.sizeof(rc_stats):
        raise ValueError(f"stats must be {C.sizeof(rc_stats)} bytes (rc_stats)")
    cam, sh, opt = camera_struct(camera), shading_struct(shading), options_struct(options)
    _check(_L().rc_render(vol.handle, C.byref(cam), _ptr(tf), tf.shape[0], C.byref(sh),
                          C.byref(opt), _ptr(out), _ptr(aux), _ptr(stats), _stream(stream)))
    return out


def rc_render_backward(vol: Volume, camera: dict, tf: torch.Tensor, shading: dict, options: dict,
                       aux: torch.Tensor, grad_rgba: torch.Tensor, grad_volume=None, grad_tf=None,
                       stream=None):
    """Accumulate dL/dvolume ([nz,ny,nx] float32) and dL/dtf ([M,4]); returns both."""
    _check_tf(tf)
    if grad_volume is None:
        grad_volume = torch.zeros(vol.shape, dtype=torch.float32, device=tf.device)
    if grad_tf is None:
        grad_tf = torch.zeros_like(tf)
    H, W = int(camera["height"]), int(camera["width"])
    grad_rgba = grad_rgba.contiguous()
    if grad_rgba.shape != (H, W, 4) or grad_rgba.dtype != torch.float32:
        raise ValueError("grad_rgba must be float32 [H,W,4]")
    if grad_volume.shape != vol.shape or grad_volume.dtype != torch.float32:
        raise ValueError("grad_volume must be float32 with the volume's shape")
    cam, sh, opt = camera_struct(camera), shading_struct(shading), options_struct(options)
    _check(_L().rc_render_backward(vol.handle, C.byref(cam), _ptr(tf), tf.shape[0], C.byref(sh),
                                   C.byref(opt), _ptr(aux), _ptr(grad_rgba), _ptr(grad_volume),
                                   _ptr(grad_tf), _stream(stream)))
    return grad_volume, grad_tf


def new_aux(camera: dict, device="cuda") -> torch.Tensor:
    return torch.empty((int(camera["height"]), int(camera["width"])), dtype=torch.int64,
                       device=device)


def aux_fields(aux: torch.Tensor):
    """(k_last int32 [H,W], t_final float32 [H,W]) views of an aux tensor."""
    pair = aux.view(torch.int32).view(*aux.shape, 2)
    return pair[..., 0], pair[..., 1].view(torch.float32)


class RenderFn(torch.autograd.Function):
    """Differentiable unshaded render: (volume float32, tf) -> rgba.

    forward: rc_update_volume with the volume tensor, then rc_render with
    aux; backward: rc_render_backward (adjoint march, transmittance
    recovered from aux)."""

    @staticmethod
    def forward(ctx, volume, tf, handle, camera, shading, options):
        volume = volume.contiguous()
        tf = tf.contiguous()
        rc_update_volume(handle, volume)
        aux = new_aux(camera, device=tf.device)
        out = rc_render(handle, camera, tf, shading, options, aux=aux)
        ctx.save_for_backward(tf, aux)
        ctx.handle, ctx.camera, ctx.shading, ctx.options = handle, camera, shading, options
        return out

    @staticmethod
    def backward(ctx, grad_out):
        tf, aux = ctx.saved_tensors
        gv, gtf = rc_render_backward(ctx.handle, ctx.camera, tf, ctx.shading, ctx.options, aux,
                                     grad_out.float())
        return gv, gtf, None, None, None, None


# ---------------------------------------------------------------- batches
def _batch_items(items):
    """items: list of dicts with keys vol, camera, tf, shading, options, out, aux (optional)."""
    arr = (rc_batch_item * len(items))()
    keep = []
    for i, it in enumerate(items):
        _check_tf(it["tf"])
        cam = it["camera"]
        H, W = int(cam["height"]), int(cam["width"])
        out = it["out"]
        if out.shape != (H, W, 4) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError(f"item {i}: out must be a contiguous float32 [H,W,4] tensor")
        aux = it.get("aux")
        arr[i] = rc_batch_item(it["vol"].handle, camera_struct(cam), it["tf"].data_ptr(),
                               it["tf"].shape[0], 0, shading_struct(it["shading"]),
                               options_struct(it["options"]), out.data_ptr(),
                               aux.data_ptr() if aux is not None else None)
        keep.append((it["vol"], it["tf"], out, aux))
    return arr, keep


def _config(cfg):
    """dict -> rc_batch_config; the box budgets and chunk length default to 0
    (the library's defaults)."""
    if cfg is None:
        return None
    return C.byref(rc_batch_config(*[int(cfg.get(f, 0)) for f in BATCH_CONFIG_FIELDS]))


class Batch:
    """Owns an ``rc_batch*`` and keeps its items' tensors alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        try:
            rc_batch_destroy(self)
        except Exception:
            pass


def rc_batch_create(items, config=None, stream=None) -> Batch:
    arr, keep = _batch_items(items)
    h = C.c_void_p()
    _check(_L().rc_batch_create(arr, len(items), _config(config), _stream(stream), C.byref(h)))
    return Batch(h, keep)


def rc_batch_render(batch: Batch, use_graph=False, stream=None):
    _check(_L().rc_batch_render(batch.handle, int(bool(use_graph)), _stream(stream)))


def rc_batch_destroy(batch: Batch):
    if batch.handle:
        _L().rc_batch_destroy(batch.handle)
        batch.handle = None


def rc_render_batch(items, config=None, stream=None):
    arr, keep = _batch_items(items)
    _check(_L().rc_render_batch(arr, len(items), _config(config), _stream(stream)))


def rc_batch_autotune(items, cache_path=None, stream=None) -> dict:
    arr, keep = _batch_items(items)
    out = rc_batch_config()
    path = cache_path.encode() if cache_path else None
    _check(_L().rc_batch_autotune(arr, len(items), path, _stream(stream), C.byref(out)))
    return {f: int(getattr(out, f)) for f in BATCH_CONFIG_FIELDS}


# ---------------------------------------------------------------- several views of one volume
def _ptr_array(tensors):
    return (C.c_void_p * len(tensors))(*[t.data_ptr() if t is not None else None for t in tensors])


def rc_render_views(vol: Volume, cameras, tf: torch.Tensor, shading: dict, options: dict,
                    outs=None, auxes=None, stream=None):
    """Render len(cameras) views in as few launches as possible; returns the
    list of [H,W,4] outputs."""
    return _render_views("rc_render_views", vol, cameras, tf, shading, options, outs, auxes,
                         stream)


# size of the library's fixed scratch array (RC_NOALLOC_SCRATCH_BYTES in rc.h)
NOALLOC_SCRATCH_BYTES = 4 << 20


def rc_render_views_noalloc(vol: Volume, cameras, tf: torch.Tensor, shading: dict,
                            options: dict, outs, auxes=None, stream=None):
    """rc_render_views with the library's fixed scratch array instead of any
    device allocation; `outs` (and `auxes`) must be supplied by the caller."""
    if outs is None:
        raise ValueError("rc_render_views_noalloc: the caller supplies the outputs")
    return _render_views("rc_render_views_noalloc", vol, cameras, tf, shading, options, outs,
                         auxes, stream)


def _render_views(fn, vol, cameras, tf, shading, options, outs, auxes, stream):
    _check_tf(tf)
    n = len(cameras)
    if outs is None:
        outs = [torch.empty((int(c["height"]), int(c["width"]), 4), dtype=torch.float32,
                            device=tf.device) for c in cameras]
    for c, o in zip(cameras, outs):
        if o.shape != (int(c["height"]), int(c["width"]), 4) or o.dtype != torch.float32 \
                or not o.is_contiguous():
            raise ValueError("each output must be a contiguous float32 [H,W,4] tensor")
    cams = (rc_camera * n)(*[camera_struct(c) for c in cameras])
    sh, opt = shading_struct(shading), options_struct(options)
    aux_arr = _ptr_array(auxes) if auxes is not None else None
    _check(getattr(_L(), fn)(vol.handle, cams, n, _ptr(tf), tf.shape[0], C.byref(sh),
                             C.byref(opt), _ptr_array(outs), aux_arr, _stream(stream)))
    return outs


def rc_render_backward_views(vol: Volume, cameras, tf: torch.Tensor, shading: dict, options: dict,
                             auxes, grads, grad_volume=None, grad_tf=None, stream=None):
    """Accumulate dL/dvolume and dL/dtf over all views; returns both."""
    _check_tf(tf)
    n = len(cameras)
    if grad_volume is None:
        grad_volume = torch.zeros(vol.shape, dtype=torch.float32, device=tf.device)
    if grad_tf is None:
        grad_tf = torch.zeros_like(tf)
    grads = [g.contiguous().float() for g in grads]
    cams = (rc_camera * n)(*[camera_struct(c) for c in cameras])
    sh, opt = shading_struct(shading), options_struct(options)
    _check(_L().rc_render_backward_views(vol.handle, cams, n, _ptr(tf), tf.shape[0], C.byref(sh),
                                         C.byref(opt), _ptr_array(auxes), _ptr_array(grads),
                                         _ptr(grad_volume), _ptr(grad_tf), _stream(stream)))
    return grad_volume, grad_tf


class RenderViewsFn(torch.autograd.Function):
    """Differentiable unshaded render of several views of one volume, all of
    one image size: (volume float32, tf) -> rgba [V,H,W,4].  One launch for
    the forward, one for the reverse pass (per 16 views)."""

    @staticmethod
    def forward(ctx, volume, tf, handle, cameras, shading, options):
        volume = volume.contiguous()
        tf = tf.contiguous()
        rc_update_volume(handle, volume)
        H, W = int(cameras[0]["height"]), int(cameras[0]["width"])
        out = torch.empty((len(cameras), H, W, 4), dtype=torch.float32, device=tf.device)
        aux = torch.empty((len(cameras), H, W), dtype=torch.int64, device=tf.device)
        rc_render_views(handle, cameras, tf, shading, options, outs=list(out.unbind(0)),
                        auxes=list(aux.unbind(0)))
        ctx.save_for_backward(tf, aux)
        ctx.handle, ctx.cameras, ctx.shading, ctx.options = handle, cameras, shading, options
        return out

    @staticmethod
    def backward(ctx, grad_out):
        tf, aux = ctx.saved_tensors
        g = grad_out.float().contiguous()
        gv, gtf = rc_render_backward_views(ctx.handle, ctx.cameras, tf, ctx.shading, ctx.options,
                                           list(aux.unbind(0)), list(g.unbind(0)))
        return gv, gtf, None, None, None, None


# ---------------------------------------------------------------- first-hit surface mode
def rc_render_surface(vol: Volume, camera: dict, tf: torch.Tensor, shading: dict, options: dict,
                      out: torch.Tensor = None, t_hit: torch.Tensor = None, stream=None):
    """First-hit surface render; returns ``(out [H,W,4], t_hit [H,W] or None)``.

    ``options``: step, gradient_op, iso_lo, iso_hi, refine, skip_empty,
    clip_lo, clip_hi (rc_surface_options)."""
    _check_tf(tf)
    H, W = int(camera["height"]), int(camera["width"])
    if out is None:
        out = torch.empty((H, W, 4), dtype=torch.float32, device=tf.device)
    if out.shape != (H, W, 4) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [H,W,4] tensor")
    if t_hit is not None and (t_hit.shape != (H, W) or t_hit.dtype != torch.float32
                              or not t_hit.is_contiguous()):
        raise ValueError("t_hit must be a contiguous float32 [H,W] tensor")
    cam, sh, opt = camera_struct(camera), shading_struct(shading), surface_options_struct(options)
    _check(_L().rc_render_surface(vol.handle, C.byref(cam), _ptr(tf), tf.shape[0], C.byref(sh),
                                  C.byref(opt), _ptr(out), _ptr(t_hit), _stream(stream)))
    return out, t_hit
