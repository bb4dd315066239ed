"""Benchmark of the volume raycaster on one MI355X.

Headline workload (the paper's 512^3, 16-bit case at 1024^2): a 512^3 u16
CT-like phantom rendered to 1024x1024 over a 36-view orbit with each of the
three gradient operators (central difference, Sobel3D, Zucker-Hummel),
step 0.5, early ray termination at 0.99 and 8^3-brick empty-space skipping.

One step = the whole hot path over that input: re-ingest the resident
linear volume into the brick layout (which rebuilds the brick value
ranges), then
render the 108 views (36 views x 3 operators): one render list built once
before timing and rendered in one persistent batched launch per step, with
its empty-brick masks recomputed.  `value` =
lattice samples of one step / step time (Gsamples/s).  The single-image
path (one rc_render per view) is timed beside it, and two views per
operator are checked bit for bit against it.

Also reported (outside `value`): per-operator rates and frame rates, the
differentiable form (16 views of a 128^3 f32 volume, forward and
forward+backward against the plain forward; and four 1024^2 views of the
512^3 phantom with Sobel3D shading), the batched form (64 uneven
volumes), the first-hit surface form, adaptive sampling on the orbit
against the fixed step, the dominant kernel's roofline
position beside peaks measured on this GPU by plain probes, and the FP64
CPU oracle timed on a bounded sample (all threads, and one thread).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_1609_01317_amd as rc  # noqa: E402
import workloads as W  # noqa: E402

OPS = ["central", "sobel3d", "zucker_hummel"]
METRIC = "Gsamples/s fwd and fwd+bwd vs plain, 512³ vol→1024² img; % HBM/L2 roofline"

# Algorithmic work per sample (the roofline's unit of work):
# every evaluated sample pays the value path (8 voxels, trilinear + table
# lookup); a sample with alpha != 0 additionally pays the gradient operator,
# normalisation, shading and compositing.
FLOPS_VALUE = 28
FLOPS_SHADED = {"central": 145, "sobel3d": 550, "zucker_hummel": 550}
VOXELS_VALUE = 8
VOXELS_SHADED = {"central": 32, "sobel3d": 64, "zucker_hummel": 64}
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "raycast_batch_c3_orbit.txt")


def kernel_source_hash() -> str:
    """Hash of the sources that define the measured forward kernels
    (raycast_batch and raycast_fwd: the batch and render sources, the march,
    the shared parameter structs and the C header): HBM counters recorded in
    the profile summary describe these sources only."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_01317_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("batch.hip", "march.h", "rc_internal.h",
                                               "render.hip", "persist.h", "persist.hip",
                                               "adaptive.h")]
    files.append(os.path.join(ROOT, "include", "rc.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(views_per_launch):
    """HBM bytes per launch of raycast_batch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources changed
    since the counters were taken or the summary's launches rendered a
    different number of views."""
    if not os.path.exists(PROFILE):
        return None
    text = open(PROFILE).read()
    m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"views_per_launch:\s*(\d+)", text)
    if not m or int(m.group(1)) != views_per_launch:
        return None
    m = re.search(r"hbm_bytes_per_launch\s+raycast_batch:\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def recorded_l2(views_per_launch):
    """L2 figures of one raycast_batch launch from the committed counter
    summary (TCC_READ_SECTORS x 32 B read through L2, TCC_HIT / (TCC_HIT +
    TCC_MISS)), or (None, None) under the same conditions as
    recorded_traffic."""
    if recorded_traffic(views_per_launch) is None:
        return None, None
    text = open(PROFILE).read()
    b = re.search(r"l2_read_bytes_per_launch\s+raycast_batch:\s*([0-9.eE+]+)", text)
    h = re.search(r"l2_hit_rate\s+raycast_batch:\s*([0-9.eE+]+)", text)
    return (float(b.group(1)) if b else None), (float(h.group(1)) if h else None)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def c3_options(sc, op):
    return dict(sc.options, gradient_op=op)


def timed_pass(fn):
    """One call of fn bracketed by HIP events on the current stream (ms)."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    return e0, e1


AUTOTUNE_CACHE = os.path.join(ROOT, "_build", "batch_autotune.jsonl")


def c3_render_list(sc, vol, tf):
    """The headline render list: for each operator one item per orbit view
    (its own output image), and ``all_items``, the 108 items in launch order
    (view i of the three operators next to each other)."""
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    opts = {op: c3_options(sc, op) for op in OPS}
    items = {op: [{"vol": vol, "camera": cam, "tf": tf, "shading": sc.shading,
                   "options": opts[op],
                   "out": torch.empty((H, Wd, 4), dtype=torch.float32, device="cuda")}
                  for cam in sc.cameras] for op in OPS}
    all_items = [items[op][i] for i in range(len(sc.cameras)) for op in OPS]
    return items, all_items


def c3_batch(all_items):
    """The launch the step times: the autotuned configuration (cached as
    JSON lines under _build/) and the batch built with it."""
    os.makedirs(os.path.dirname(AUTOTUNE_CACHE), exist_ok=True)
    cfg = rc.rc_batch_autotune(all_items, AUTOTUNE_CACHE)
    return cfg, rc.rc_batch_create(all_items, cfg)


def run_c3(args):
    """The 108 views (36 per operator) are one render list (an rc_batch built
    once, before timing: cameras, outputs and options are fixed; view i of
    the three operators next to each other); a step re-ingests the volume,
    rebuilds the brick ranges and renders the list in one persistent launch
    (empty masks recomputed per render, as rc_render does).  Each operator's
    orbit is also timed as a launch of its own, outside the step."""
    sc = W.config_c3(n_views=args.views)
    log(f"bench: c3 volume {sc.volume.shape} {sc.volume.dtype}, {len(sc.cameras)} views")
    src = to_dev(sc.volume)
    vol = rc.rc_create_volume(src, sc.spacing, sc.vmin, sc.vmax)
    rc.rc_build_bricks(vol, 8)
    tf = to_dev(sc.tf)
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    out = torch.empty((H, Wd, 4), dtype=torch.float32, device="cuda")
    opts = {op: c3_options(sc, op) for op in OPS}
    items, all_items = c3_render_list(sc, vol, tf)
    outs = {op: [it["out"] for it in items[op]] for op in OPS}
    cache = AUTOTUNE_CACHE
    cfg_all, batch_all = c3_batch(all_items)

    def step(events=None):
        # re-ingest; the brick ranges exist, so rc_update_volume rebuilds them
        rc.rc_update_volume(vol, src)
        if events is None:
            rc.rc_batch_render(batch_all)
        else:
            events.append(timed_pass(lambda: rc.rc_batch_render(batch_all)))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(events)
        log(f"bench: step {s + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    render_ms = [a.elapsed_time(b) for a, b in events]

    # untimed: the single-image path (one rc_render per view), and the
    # counting pass (lattice / evaluated / shaded samples per view)
    single = {op: [] for op in OPS}
    for op in OPS:
        for cam in sc.cameras:
            single[op].append(timed_pass(
                lambda: rc.rc_render(vol, cam, tf, sc.shading, opts[op], out=out)))
    torch.cuda.synchronize()
    single_ms = {op: [a.elapsed_time(b) for a, b in single[op]] for op in OPS}
    counts = {}
    for op in OPS:
        st = rc.new_stats()
        per_view = []
        for cam in sc.cameras:
            st.zero_()
            rc.rc_render(vol, cam, tf, sc.shading, opts[op], out=out, stats=st)
            per_view.append(st.cpu().numpy().astype(np.int64))
        counts[op] = np.array(per_view)
    torch.cuda.synchronize()
    # the orbit renders are checked bit for bit against single renders
    for op in OPS:
        for i in (0, len(sc.cameras) // 2):
            rc.rc_render(vol, sc.cameras[i], tf, sc.shading, opts[op], out=out)
            if not torch.equal(out, outs[op][i]):
                raise RuntimeError(f"bench: batched {op} view {i} differs from rc_render")
    # untimed: each operator's orbit as a launch of its own
    cfgs, op_ms = {"all": cfg_all}, {}
    if not args.no_per_op:
        for op in OPS:
            cfgs[op] = rc.rc_batch_autotune(items[op], cache)
            b = rc.rc_batch_create(items[op], cfgs[op])
            rc.rc_batch_render(b)
            ev = [timed_pass(lambda: rc.rc_batch_render(b)) for _ in range(2)]
            torch.cuda.synchronize()
            op_ms[op] = float(np.mean([x.elapsed_time(y) for x, y in ev]))
            rc.rc_batch_destroy(b)
    return sc, vol, tf, ms_per_step, render_ms, op_ms, single_ms, counts, cfgs


def roofline(render_ms, counts, views_per_launch):
    """Dominant kernel: raycast_batch, one launch per step rendering the 108
    views of the three operators; the figures are per launch, averaged over
    the timed steps."""
    flops_total = 0.0
    bytes_total = 0.0
    for op in OPS:
        c = counts[op]
        evaluated, shaded = c[:, 1].astype(float), c[:, 2].astype(float)
        flops_total += float((FLOPS_VALUE * (evaluated - shaded) + FLOPS_SHADED[op] * shaded).sum())
        bytes_total += float(
            2 * (VOXELS_VALUE * (evaluated - shaded) + VOXELS_SHADED[op] * shaded).sum())
    launches = 1
    avg_ms = float(np.mean(render_ms))
    flops = flops_total / launches
    achieved = flops / (avg_ms * 1e-3) / 1e12
    traffic = recorded_traffic(views_per_launch)
    l2_bytes, l2_hit = recorded_l2(views_per_launch)
    return {
        "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
        "traffic": traffic,
        # achieved HBM and L2 rates of the same launch: counter bytes per
        # launch over the launch time measured here
        "hbm_gbs": round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None,
        "hbm_frac": round(traffic / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if traffic else None,
        "l2_gbs": round(l2_bytes / (avg_ms * 1e-3) / 1e9, 1) if l2_bytes else None,
        "l2_hit": l2_hit,
        "kernel": "raycast_batch (one launch = the 108 views of the three operators' orbits)",
        "avg_launch_ms": round(avg_ms, 4),
        "algorithmic_flops_per_launch": flops,
        "algorithmic_voxel_bytes_per_launch": bytes_total / launches,
    }


def run_c5(args):
    """Differentiable form: 16 views 256^2 of a 128^3 f32 volume, L2 loss."""
    sc = W.config_c5()
    vol_t = to_dev(sc.volume)
    h = rc.rc_create_volume(vol_t, sc.spacing, sc.vmin, sc.vmax)
    ht = rc.rc_create_volume(to_dev(sc.extra["target_volume"]), sc.spacing, sc.vmin, sc.vmax)
    tf0 = to_dev(sc.tf)
    targets = [rc.rc_render(ht, cam, tf0, sc.shading, sc.options).clone() for cam in sc.cameras]
    vp = vol_t.clone().requires_grad_(True)
    tp = tf0.clone().requires_grad_(True)

    target = torch.stack(targets)
    outs = torch.empty_like(target)
    out_list = list(outs.unbind(0))

    def fwd_only():
        with torch.no_grad():
            rc.rc_update_volume(h, vp.detach())
            rc.rc_render_views(h, sc.cameras, tp.detach(), sc.shading, sc.options, outs=out_list)

    def fwd_bwd():
        img = rc.RenderViewsFn.apply(vp, tp, h, sc.cameras, sc.shading, sc.options)
        ((img - target) ** 2).sum().backward()
        vp.grad = None
        tp.grad = None

    def timeit(fn, n):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    auxes = [rc.new_aux(cam) for cam in sc.cameras]
    grads = [torch.randn((cam["height"], cam["width"], 4), device="cuda") for cam in sc.cameras]
    gv = torch.zeros_like(vol_t)
    gt = torch.zeros_like(tf0)

    def bwd_only():
        rc.rc_render_backward_views(h, sc.cameras, tf0, sc.shading, sc.options, auxes, grads, gv,
                                    gt)

    st = rc.new_stats()
    rc.rc_update_volume(h, vol_t)
    for cam, aux in zip(sc.cameras, auxes):
        rc.rc_render(h, cam, tf0, sc.shading, sc.options, aux=aux, stats=st)
    lattice = int(st[0].item())
    ms_f = timeit(fwd_only, args.c5_iters)
    ms_fb = timeit(fwd_bwd, args.c5_iters)
    ms_b = timeit(bwd_only, args.c5_iters)
    return {
        "workload": "128^3 f32 blobs, learnable 256-entry TF, 16 views 256^2, step 0.5, unshaded, "
                    "L2 loss vs seed-55 target; all views in one launch (forward and backward)",
        "lattice_samples": lattice,
        "fwd_ms": round(ms_f, 3), "fwd_bwd_ms": round(ms_fb, 3),
        "fwd_gsamples_s": round(lattice / ms_f / 1e6, 3),
        "fwd_bwd_gsamples_s": round(lattice / ms_fb / 1e6, 3),
        "fwd_bwd_over_fwd_time": round(ms_fb / ms_f, 2),
        "bwd_kernels_ms": round(ms_b, 3),
    }


def run_c3_grad(args, sc, vol, tf):
    """Forward + backward at the metric's size: four views (every ninth of the
    orbit) of the 512^3 u16 phantom at 1024^2, Sobel3D with Blinn-Phong,
    step 0.5, ERT 0.99.  Loss: L2 against the same views rendered with a
    second table; dL/dvolume (float32, 512^3) and dL/dtable through the
    hand-written adjoint, which lights every sample (an opacity-0 sample
    still has a gradient in the table's opacity entries) and scatters the
    64-tap stencil adjoint.  All views in one launch each way."""
    cams = sc.cameras[::9][:4]
    opt = c3_options(sc, "sobel3d")
    H, Wd = cams[0]["height"], cams[0]["width"]
    tf2 = to_dev(W.tf_ramps(sc.tf.shape[0], seed=303, alpha_max=0.25, lo=0.1, hi=0.8))
    targets = rc.rc_render_views(vol, cams, tf2, sc.shading, opt)
    outs = [torch.empty((H, Wd, 4), dtype=torch.float32, device="cuda") for _ in cams]
    auxes = [rc.new_aux(c) for c in cams]
    grads = [torch.empty_like(o) for o in outs]
    gv = torch.zeros((512, 512, 512), dtype=torch.float32, device="cuda")
    gt = torch.zeros_like(tf)

    def fwd():
        rc.rc_render_views(vol, cams, tf, sc.shading, opt, outs=outs, auxes=auxes)

    def fwd_bwd():
        fwd()
        for g, o, t in zip(grads, outs, targets):
            torch.sub(o, t, out=g).mul_(2.0)
        gv.zero_()
        gt.zero_()
        rc.rc_render_backward_views(vol, cams, tf, sc.shading, opt, auxes, grads, gv, gt)

    def timeit(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    st = rc.new_stats()
    for cam in cams:
        rc.rc_render(vol, cam, tf, sc.shading, opt, stats=st)
    lattice = int(st[0].item())
    ms_f = timeit(fwd, 3)
    ms_fb = timeit(fwd_bwd, 2)
    nz = int((gv != 0).sum().item())
    return {"workload": "512^3 u16 phantom -> 1024^2, 4 orbit views (0, 90, 180, 270 deg), "
                        "Sobel3D Blinn-Phong, step 0.5, ERT 0.99; L2 loss vs a second table's "
                        "images; dL/dvolume 512^3 f32 and dL/dtable 4096x4",
            "views": len(cams), "lattice_samples": lattice,
            "fwd_ms": round(ms_f, 3), "fwd_bwd_ms": round(ms_fb, 3),
            "fwd_gsamples_s": round(lattice / ms_f / 1e6, 3),
            "fwd_bwd_gsamples_s": round(lattice / ms_fb / 1e6, 3),
            "fwd_bwd_over_fwd_time": round(ms_fb / ms_f, 2),
            "grad_volume_nonzero": nz}


def run_adaptive(args, sc, vol, tf):
    """Adaptive sampling on the headline orbit: Sobel3D, samples in bricks
    whose value range is at most adapt_range raw units advance 4 steps, with
    opacity corrected to the distance; all 36 views in one persistent launch,
    against the fixed-step orbit launch of the same views.  adapt_range is
    swept: 120 (about six noise sigmas: a brick of pure noise is poor about
    half the time), 200 (ten sigmas: every noise-only brick is poor) and 400
    (also the weakest material edges).  Error = |adaptive - fixed step| per
    channel over all pixels of all views."""
    opt_f = c3_options(sc, "sobel3d")
    H, Wd = sc.cameras[0]["height"], sc.cameras[0]["width"]
    outs_f = [torch.empty((H, Wd, 4), dtype=torch.float32, device="cuda") for _ in sc.cameras]
    outs_a = [torch.empty_like(o) for o in outs_f]

    def timeit(fn, n=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    def counters(opt):
        st = rc.new_stats()
        for cam in sc.cameras:
            rc.rc_render(vol, cam, tf, sc.shading, opt, stats=st)
        return [int(x) for x in st.tolist()]

    ms_f = timeit(lambda: rc.rc_render_views(vol, sc.cameras, tf, sc.shading, opt_f, outs=outs_f))
    st_f = counters(opt_f)
    nv = len(sc.cameras)
    sweep = []
    for rng in (120.0, 200.0, 400.0):
        opt_a = dict(opt_f, adapt_factor=4, adapt_range=rng)
        ms_a = timeit(lambda: rc.rc_render_views(vol, sc.cameras, tf, sc.shading, opt_a,
                                                 outs=outs_a))
        st_a = counters(opt_a)
        err_max, err_sum, n = 0.0, 0.0, 0
        for a, f in zip(outs_a, outs_f):
            d = (a - f).abs()
            err_max = max(err_max, float(d.max().item()))
            err_sum += float(d.sum().item())
            n += d.numel()
        sweep.append({"adapt_range": rng, "ms_per_view": round(ms_a / nv, 4),
                      "speedup_vs_fixed": round(ms_f / ms_a, 3),
                      "samples": st_a[0], "gsamples_s": round(st_a[0] / ms_a / 1e6, 3),
                      "counters": dict(zip(rc.STATS_FIELDS[1:], st_a[1:])),
                      "max_abs_err_vs_fixed": round(err_max, 5),
                      "mean_abs_err_vs_fixed": round(err_sum / n, 7)})
    return {"workload": "512^3 u16 phantom -> 1024^2, 36-view orbit, Sobel3D Blinn-Phong, step 0.5, "
                        "ERT 0.99, skipping; adaptive factor 4 in bricks of range <= adapt_range",
            "fixed_ms_per_view": round(ms_f / nv, 4),
            "fixed_lattice_samples": st_f[0],
            "fixed_gsamples_s": round(st_f[0] / ms_f / 1e6, 3),
            "fixed_counters": dict(zip(rc.STATS_FIELDS[1:], st_f[1:])),
            "adaptive": sweep}


def run_c4(args):
    """Batched form: 64 uneven volumes, one persistent launch (graph-replayed)
    against 64 sequential rc_render launches on the same stream."""
    scenes = W.config_c4()
    items = []
    for sc in scenes:
        cam = sc.cameras[0]
        vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
        rc.rc_build_bricks(vol, 8)
        items.append({"vol": vol, "camera": cam, "tf": to_dev(sc.tf), "shading": sc.shading,
                      "options": sc.options,
                      "out": torch.empty((cam["height"], cam["width"], 4), device="cuda")})
    st = rc.new_stats()
    for it in items:
        rc.rc_render(it["vol"], it["camera"], it["tf"], it["shading"], it["options"], stats=st)
    lattice = int(st[0].item())
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    cfg = rc.rc_batch_autotune(items, os.path.join(ROOT, "_build", "batch_autotune.jsonl"))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = rc.rc_batch_create(items, cfg, stream=s)

        def batched():
            rc.rc_batch_render(b, use_graph=True, stream=s)

        def sequential():
            for it in items:
                rc.rc_render(it["vol"], it["camera"], it["tf"], it["shading"], it["options"],
                             out=it["out"], stream=s)

        def timeit(fn, n):
            for _ in range(2):
                fn()
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(n):
                fn()
            e1.record(s)
            s.synchronize()
            return e0.elapsed_time(e1) / n

        ms_b = timeit(batched, args.c4_iters)
        ms_s = timeit(sequential, args.c4_iters)
        rc.rc_batch_destroy(b)
    return {
        "workload": "64 volumes 32^3..256x256x96 u8/u16 (blobs or phantoms), own perspective "
                    "camera, square images 128..512, own 256-entry TF, CD, Blinn-Phong, ERT 0.99, "
                    "skip",
        "lattice_samples": lattice, "autotuned_config": cfg,
        "batch_graph_ms": round(ms_b, 3), "sequential_64_ms": round(ms_s, 3),
        "batch_gsamples_s": round(lattice / ms_b / 1e6, 3),
        "sequential_gsamples_s": round(lattice / ms_s / 1e6, 3),
        "speedup_vs_sequential": round(ms_s / ms_b, 2),
    }


def run_surface(args, sc=None, vol=None, tf=None):
    """First-hit surface mode over the headline orbit: coarse step 2.0 (4x
    the volume-mode step, as hitpoint refinement allows), 6 refinement
    steps, window [500, 4095], Sobel3D Blinn-Phong, brick skipping."""
    if sc is None:
        sc = W.config_c3(n_views=args.views)
        vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
        rc.rc_build_bricks(vol, 8)
        tf = to_dev(sc.tf)
    opt = W.default_surface_options(step=2.0, gradient_op="sobel3d", iso_lo=500.0, iso_hi=4095.0,
                                    refine=6, skip_empty=True)
    cam0 = sc.cameras[0]
    out = torch.empty((cam0["height"], cam0["width"], 4), dtype=torch.float32, device="cuda")
    t_hit = torch.empty((cam0["height"], cam0["width"]), dtype=torch.float32, device="cuda")
    for cam in sc.cameras[:2]:
        rc.rc_render_surface(vol, cam, tf, sc.shading, opt, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for cam in sc.cameras:
        rc.rc_render_surface(vol, cam, tf, sc.shading, opt, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / len(sc.cameras)
    rc.rc_render_surface(vol, cam0, tf, sc.shading, opt, out=out, t_hit=t_hit)
    hits = int(torch.isfinite(t_hit).sum().item())
    return {"workload": "512^3 u16 phantom -> 1024^2, 36-view orbit, first-hit surface: window "
                        "[500, 4095], coarse step 2.0, 6 refinement steps, Sobel3D Blinn-Phong, "
                        "brick skipping",
            "ms_per_view": round(ms, 4), "fps": round(1e3 / ms, 1),
            "surface_pixels_view0": hits}


def cpu_baseline(sc, counts):
    """FP64 oracle on six full Sobel3D views of the headline workload (every
    sixth view of the orbit), in the metric's unit: the views' lattice samples
    (the workload size the GPU figure counts, from the counting pass) over the
    oracle's wall time."""
    import oracle
    v = oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    opt = c3_options(sc, "sobel3d")
    views = list(range(0, len(sc.cameras), 6))
    t0 = time.perf_counter()
    for i in views:
        oracle.render(v, sc.cameras[i], sc.tf, sc.shading, opt)
    dt = time.perf_counter() - t0
    lattice = int(sum(counts["sobel3d"][i, 0] for i in views))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # one thread on every sixteenth row of view 0; lattice samples from the
    # oracle's own last lattice index per ray
    cam = sc.cameras[0]
    pix = np.concatenate([np.arange(r * cam["width"], (r + 1) * cam["width"])
                          for r in range(0, cam["height"], 16)])
    t0 = time.perf_counter()
    r1 = oracle.render(v, cam, sc.tf, sc.shading, opt, pixels=pix, threads=1)
    dt1 = time.perf_counter() - t0
    hit = (r1["flags"] & oracle.FLAG_HIT) != 0
    lattice1 = int((r1["k_last"][hit].astype(np.int64) + 1).sum())
    return {"value": round(lattice / dt / 1e9, 6), "unit": "Gsamples/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(views)} full 1024x1024 Sobel3D views (every sixth view of the "
                      f"orbit) of the 512^3 u16 workload: {lattice} lattice samples in "
                      f"{dt:.1f} s",
            "single_thread_value": round(lattice1 / dt1 / 1e9, 6),
            "single_thread_sample": f"every 16th row of view 0, one thread: {lattice1} lattice "
                                    f"samples in {dt1:.1f} s"}


def measured_peaks():
    """Rates this GPU reaches on plain probes (``libpeaks.so``), beside the
    datasheet peaks: FP32 FMA built like the raycaster (no packed FP32), reads
    of a 2 MiB buffer that stays in each XCD's L2, reads of a 1 GiB buffer
    (HBM), and a 1 GiB device copy (read + write).  Best of five each."""
    path = os.path.join(ROOT, "paper_1609_01317_amd", "libpeaks.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    lib.pk_fma.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.pk_read.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int, ctypes.c_int,
                            ctypes.c_void_p, ctypes.c_void_p]
    stream = torch.cuda.current_stream().cuda_stream

    def best_ms(fn, n=5):
        fn()
        ts = []
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    def check(rc_):
        if rc_ != 0:
            raise RuntimeError(f"peak probe failed with HIP error {rc_}")

    fma_blocks, fma_iters = 4096, 2048
    out = torch.empty(fma_blocks * 256, dtype=torch.float32, device="cuda")
    ms = best_ms(lambda: check(lib.pk_fma(out.data_ptr(), fma_blocks, fma_iters, stream)))
    fma_tflops = 2 * 16 * fma_iters * fma_blocks * 256 / (ms * 1e-3) / 1e12

    rd_blocks = 2048
    out = torch.empty(rd_blocks * 256, dtype=torch.float32, device="cuda")
    rates = {}
    # 2 MiB: 512 chunks of 4 KiB, inside each XCD's 4 MB L2; 1 GiB: 262144
    # chunks, two passes over it (2048 workgroups x 256 repetitions)
    for name, nbytes, reps in (("l2", 2 << 20, 512), ("hbm", 1 << 30, 256)):
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        ms = best_ms(lambda: check(lib.pk_read(buf.data_ptr(), nbytes, rd_blocks, reps,
                                               out.data_ptr(), stream)))
        rates[name] = rd_blocks * reps * 4096 / (ms * 1e-3) / 1e12
        del buf
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = best_ms(lambda: b.copy_(a))
    copy_tbs = 2 * a.numel() * 4 / (ms * 1e-3) / 1e12
    del a, b
    return {"fp32_fma_tflops": round(fma_tflops, 2), "l2_read_tb_s": round(rates["l2"], 2),
            "hbm_read_tb_s": round(rates["hbm"], 2), "hbm_copy_tb_s": round(copy_tbs, 2),
            "probe": "FP32 FMA: 16 independent chains x 2048 steps per lane, 4096 x 256 lanes, "
                     "no packed FP32; reads: 2048 workgroups each reading one 4 KiB chunk per "
                     "repetition, walking a 2 MiB (L2, 512 repetitions) or 1 GiB (HBM, two "
                     "passes) buffer; copy: 1 GiB float32, read + write "
                     "bytes"}


def calib_copy():
    """A plain copy of known size, for scaling HBM counters in a --pmc run."""
    n = 1 << 28                         # 1 GiB of float32
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--views", type=int, default=36)
    ap.add_argument("--c5-iters", type=int, default=5)
    ap.add_argument("--c4-iters", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the differentiable form")
    ap.add_argument("--calib-copy", action="store_true", help="run a 1 GiB copy first")
    ap.add_argument("--no-per-op", action="store_true",
                    help="skip the per-operator orbit launches (profiling runs: every "
                         "raycast_batch dispatch is then the step's)")
    ap.add_argument("--only", choices=["c4", "c5", "surface", "adaptive", "c3grad"],
                    default=None,
                    help="run only the batched (c4), differentiable (c5 or c3grad), first-hit "
                         "surface or adaptive form and print it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: WORLD_SIZE > 1 is not supported on this one-GPU build", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.calib_copy:
        calib_copy()
    if args.only:
        if args.only in ("adaptive", "c3grad"):
            sc = W.config_c3(n_views=args.views)
            vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
            rc.rc_build_bricks(vol, 8)
            fn = run_adaptive if args.only == "adaptive" else run_c3_grad
            print(json.dumps(fn(args, sc, vol, to_dev(sc.tf))), flush=True)
            return
        fn = {"c4": run_c4, "c5": run_c5, "surface": run_surface}[args.only]
        print(json.dumps(fn(args)), flush=True)
        return

    sc, vol, tf, ms_per_step, render_ms, op_ms, single_ms, counts, cfgs = run_c3(args)
    lattice_step = int(sum(counts[op][:, 0].sum() for op in OPS))
    value = lattice_step / (ms_per_step * 1e-3) / 1e9
    per_op = {}
    for op in OPS:
        lat = int(counts[op][:, 0].sum())
        ev = int(counts[op][:, 1].sum())
        ms1 = float(np.sum(single_ms[op]))
        per_op[op] = {"single_image_orbit_ms": round(ms1, 3),
                      "single_image_ms_per_view": round(ms1 / len(sc.cameras), 4),
                      "lattice_samples": lat, "evaluated_samples": ev,
                      "shaded_samples": int(counts[op][:, 2].sum()),
                      "chunks_staged": int(counts[op][:, 4].sum()),
                      "chunks_empty": int(counts[op][:, 5].sum()),
                      "chunks_direct": int(counts[op][:, 6].sum()),
                      "samples_direct": int(counts[op][:, 7].sum())}
        if op in op_ms:         # the operator's orbit as a launch of its own
            ms = op_ms[op]
            per_op[op].update({"orbit_ms": round(ms, 3),
                               "fps": round(len(sc.cameras) / (ms * 1e-3), 1),
                               "batch_config": cfgs[op],
                               "lattice_gsamples_s": round(lat / (ms * 1e-3) / 1e9, 3),
                               "evaluated_gsamples_s": round(ev / (ms * 1e-3) / 1e9, 3)})
    roof = roofline(render_ms, counts, len(OPS) * len(sc.cameras))
    log("bench: measured peaks")
    peaks = measured_peaks()
    roof["measured_peaks"] = peaks
    roof["frac_of_measured_fp32_fma"] = round(roof["achieved"] / peaks["fp32_fma_tflops"], 4)
    result = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gsamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 u16 CT-like phantom (24 ellipsoids, 12-bit, noise 20) -> "
                               "1024^2 perspective 60 deg, 36-view orbit at 10 deg steps x "
                               "{central difference, Sobel3D, Zucker-Hummel}, step 0.5, ERT 0.99, "
                               "8^3-brick skipping; step = ingest + brick ranges + the three "
                               "operators' orbits (108 views) in one persistent batched launch",
                   "views": len(sc.cameras), "image": [1024, 1024], "volume": [512, 512, 512],
                   "lattice_samples_per_step": lattice_step, "batch_config": cfgs["all"],
                   "render_ms_per_step": round(float(np.mean(render_ms)), 3)},
        "per_operator": per_op,
        "roofline": roof,
    }
    if not args.no_forms:
        log("bench: differentiable form")
        result["differentiable"] = run_c5(args)
        log("bench: batched form")
        result["batched"] = run_c4(args)
        log("bench: first-hit surface form")
        result["surface"] = run_surface(args, sc, vol, tf)
        log("bench: adaptive sampling")
        result["adaptive"] = run_adaptive(args, sc, vol, tf)
        log("bench: forward + backward at 512^3 -> 1024^2")
        result["differentiable_c3"] = run_c3_grad(args, sc, vol, tf)
    if not args.no_cpu:
        log("bench: cpu oracle baseline")
        result["cpu_baseline"] = cpu_baseline(sc, counts)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
