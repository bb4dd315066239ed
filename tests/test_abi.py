"""C-ABI checks that need no GPU: the library loads, exports every function
``include/rc.h`` declares, and rejects bad arguments on the host before any
device work (these calls never reach the HIP runtime)."""
import ctypes as C
import os
import re

import pytest

import paper_1609_01317_amd as rc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(rc_[a-z_0-9]+)\s*\(", src))
    return names


def _lib():
    if not os.path.exists(rc.library_path()):
        pytest.skip("librc.so not built")
    return C.CDLL(rc.library_path())


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = _declared()
    assert {"rc_create_volume", "rc_build_bricks", "rc_render", "rc_render_backward"} <= names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_struct_layouts_match_header():
    assert C.sizeof(rc.rc_camera) == 16 + 11 * 8
    assert C.sizeof(rc.rc_shading) == 8 + 4 * 4 + 3 * 4 + 4
    assert C.sizeof(rc.rc_options) == 8 + 6 * 8 + 8 * 4
    assert C.sizeof(rc.rc_stats) == 64
    assert C.sizeof(rc.rc_batch_item) == 272
    assert C.sizeof(rc.rc_batch_config) == 28
    assert C.sizeof(rc.rc_surface_options) == 8 + 6 * 8 + 2 * 4 + 4 * 4


def _status(fn, *args):
    L = rc._L()
    return getattr(L, fn)(*args), L.rc_last_error().decode()


def test_create_rejects_bad_arguments_on_host():
    out = C.c_void_p()
    sp = (C.c_double * 3)(1.0, 1.0, 1.0)
    st, msg = _status("rc_create_volume", None, 4, 4, 4, 0, sp, 0.0, 1.0, None, C.byref(out))
    assert st == rc.RC_E_INVALID and "src_dev" in msg
    fake = C.c_void_p(0x1000)
    st, msg = _status("rc_create_volume", fake, 0, 4, 4, 0, sp, 0.0, 1.0, None, C.byref(out))
    assert st == rc.RC_E_INVALID and "dims" in msg
    st, msg = _status("rc_create_volume", fake, 4, 4, 4, 7, sp, 0.0, 1.0, None, C.byref(out))
    assert st == rc.RC_E_INVALID and "dtype" in msg
    bad = (C.c_double * 3)(1.0, 0.0, 1.0)
    st, msg = _status("rc_create_volume", fake, 4, 4, 4, 0, bad, 0.0, 1.0, None, C.byref(out))
    assert st == rc.RC_E_INVALID and "spacing" in msg
    st, msg = _status("rc_create_volume", fake, 4, 4, 4, 0, sp, 1.0, 1.0, None, C.byref(out))
    assert st == rc.RC_E_INVALID and "vmin" in msg
    st, _ = _status("rc_create_volume", fake, 4, 4, 4, 0, sp, 0.0, 1.0, None, None)
    assert st == rc.RC_E_INVALID


def test_render_rejects_null_volume_on_host():
    import workloads as W
    cam = rc.camera_struct(W.orbit_camera((8, 8, 8), (1, 1, 1), 0, 0, 8, 8))
    sh = rc.shading_struct(W.default_shading())
    opt = rc.options_struct(W.default_options())
    st, msg = _status("rc_render", None, C.byref(cam), C.c_void_p(0x1000), 256, C.byref(sh),
                      C.byref(opt), C.c_void_p(0x2000), None, None, None)
    assert st == rc.RC_E_INVALID and "volume" in msg
    st, msg = _status("rc_render_backward", None, C.byref(cam), C.c_void_p(0x1000), 256,
                      C.byref(sh), C.byref(opt), None, None, None, None, None)
    assert st == rc.RC_E_INVALID
    st, _ = _status("rc_build_bricks", None, 8, None)
    assert st == rc.RC_E_INVALID
    rc._L().rc_destroy_volume(None)     # NULL is ignored


def test_batch_rejects_bad_arguments_on_host():
    out = C.c_void_p()
    st, _ = _status("rc_batch_create", None, 1, None, None, C.byref(out))
    assert st == rc.RC_E_INVALID
    items = (rc.rc_batch_item * 1)()
    st, msg = _status("rc_batch_create", items, 1, None, None, C.byref(out))
    assert st == rc.RC_E_INVALID and "item 0" in msg
    bad = rc.rc_batch_config(7, 1, 8, 1)
    st, msg = _status("rc_batch_create", items, 1, C.byref(bad), None, C.byref(out))
    assert st == rc.RC_E_INVALID and "tile_w" in msg
    st, _ = _status("rc_batch_render", None, 0, None)
    assert st == rc.RC_E_INVALID
    st, _ = _status("rc_batch_autotune", items, 1, None, None, C.byref(rc.rc_batch_config()))
    assert st == rc.RC_E_INVALID
    rc._L().rc_batch_destroy(None)


def test_surface_rejects_bad_arguments_on_host():
    import workloads as W
    cam = rc.camera_struct(W.orbit_camera((8, 8, 8), (1, 1, 1), 0, 0, 8, 8))
    sh = rc.shading_struct(W.default_shading())
    tf, out = C.c_void_p(0x1000), C.c_void_p(0x2000)
    st, msg = _status("rc_render_surface", None, C.byref(cam), tf, 256, C.byref(sh), None, out,
                      None, None)
    assert st == rc.RC_E_INVALID and "options" in msg
    good = W.default_surface_options(iso_lo=10.0, iso_hi=20.0)
    for bad, word in [(dict(good, iso_lo=float("nan")), "iso"), (dict(good, iso_lo=30.0), "iso"),
                      (dict(good, refine=31), "refine"), (dict(good, refine=-1), "refine")]:
        opt = rc.surface_options_struct(bad)
        st, msg = _status("rc_render_surface", None, C.byref(cam), tf, 256, C.byref(sh),
                          C.byref(opt), out, None, None)
        assert st == rc.RC_E_INVALID and word in msg, msg
    opt = rc.surface_options_struct(good)
    st, msg = _status("rc_render_surface", None, C.byref(cam), tf, 256, C.byref(sh), C.byref(opt),
                      out, None, None)
    assert st == rc.RC_E_INVALID and "volume" in msg


def test_batch_config_rejected_on_host():
    """Box budgets and chunk lengths outside their ranges are refused before
    any item is looked at (no device work)."""
    items = (rc.rc_batch_item * 1)()
    out = C.c_void_p()
    base = dict(tile_w=8, waves_per_wg=1, wg_per_cu=8, order=1)
    for bad in (dict(box_bytes_grad=1000), dict(box_bytes_grad=1024), dict(box_bytes_cd=33792),
                dict(box_bytes_cd=-2048), dict(chunk_len=3), dict(chunk_len=65)):
        cfg = rc.rc_batch_config(*[int(dict(base, **bad).get(f, 0))
                                   for f in rc.BATCH_CONFIG_FIELDS])
        st, msg = _status("rc_batch_create", items, 1, C.byref(cfg), None, C.byref(out))
        assert st == rc.RC_E_INVALID and "batch config" in msg, (bad, msg)


def test_noalloc_scratch_size_matches_header():
    src = open(os.path.join(ROOT, "include", "rc.h")).read()
    m = re.search(r"#define\s+RC_NOALLOC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", src)
    assert m, "RC_NOALLOC_SCRATCH_BYTES not found"
    assert rc.NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
