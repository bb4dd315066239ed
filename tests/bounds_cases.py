"""Renders through every entry point, for the bounds-checked build test:
``run_cases()`` returns a digest per case (summary sums for the reverse
mode, whose float atomics land in no fixed order), computed with whichever
library the process loaded (``RC_LIBRARY``).  Run as a script it prints the digests
and the bounds-checked build's violation count as one JSON line."""
import hashlib
import json
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import paper_1609_01317_amd as rc  # noqa: E402
import workloads as W  # noqa: E402


def _digest(*ts):
    h = hashlib.sha1()
    for t in ts:
        h.update(t.detach().cpu().numpy().tobytes())
    return h.hexdigest()


def _sums(*ts):
    """Order-independent summaries of gradients accumulated with float
    atomics (their bits depend on the order the atomics land in)."""
    vals = []
    for t in ts:
        d = t.detach().double().flatten()
        w = torch.linspace(-1.0, 1.0, d.numel(), device=d.device, dtype=torch.float64)
        vals += [float(d.abs().sum()), float(d.sum()), float((d * w).sum())]
    return vals


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_cases():
    out = {}
    # single renders: every dtype, operator and shading model, skipping on
    # and off, ERT, nearest sampling, opacity correction, adaptive sampling,
    # orthographic cameras; volumes with ragged bricks
    cases = [
        dict(seed=71, dims=(21, 19, 17), dtype=np.uint8, op="central", shading="blinn_phong"),
        dict(seed=72, dims=(33, 18, 25), dtype=np.uint16, op="sobel3d", shading="blinn_phong",
             ert=0.95, skip=True),
        dict(seed=73, dims=(17, 29, 23), dtype=np.float32, op="zucker_hummel",
             shading="paper_lambert", skip=True),
        dict(seed=74, dims=(40, 36, 12), dtype=np.uint16, op="central", shading="none",
             ert=0.99, skip=True, projection="ortho"),
        dict(seed=75, dims=(26, 22, 30), dtype=np.float32, op="sobel3d", shading="blinn_phong",
             skip=True, image=(61, 47)),
    ]
    for k, c in enumerate(cases):
        sc = W.config_small(**c)
        vol = rc.rc_create_volume(_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
        rc.rc_build_bricks(vol, 8)
        # re-ingest: the brick ranges are rebuilt in the ingest pass
        rc.rc_update_volume(vol, _dev(sc.volume))
        tf = _dev(sc.tf)
        cam = sc.cameras[0]
        variants = [("plain", {}), ("nearest", {"nearest": True}),
                    ("ocorr", {"ref_step": 0.7})]
        if sc.options["skip_empty"]:
            variants.append(("adaptive", {"adapt_factor": 2, "adapt_range": 0.05 * (sc.vmax - sc.vmin)}))
        for name, extra in variants:
            opt = dict(sc.options, **extra)
            aux = rc.new_aux(cam)
            img = rc.rc_render(vol, cam, tf, sc.shading, opt, aux=aux)
            out[f"render{k}_{name}"] = _digest(img, aux)
        # several views in one call (their forward goes through the batched kernel)
        cams = [W.orbit_camera(c["dims"], sc.spacing, 40.0 * i, 20.0 - 8 * i, 24 + 8 * i, 20 + 4 * i)
                for i in range(5)]
        auxes = [rc.new_aux(cm) for cm in cams]
        imgs = rc.rc_render_views(vol, cams, tf, sc.shading, sc.options, auxes=auxes)
        out[f"views{k}"] = _digest(*imgs, *auxes)
        # reverse mode, single and multi-view
        g = torch.linspace(-1.0, 1.0, cam["height"] * cam["width"] * 4,
                           device="cuda").view(cam["height"], cam["width"], 4)
        aux = rc.new_aux(cam)
        rc.rc_render(vol, cam, tf, sc.shading, sc.options, aux=aux)
        gv, gt = rc.rc_render_backward(vol, cam, tf, sc.shading, sc.options, aux, g)
        out[f"backward{k}"] = _sums(gv, gt)
        grads = [torch.full((cm["height"], cm["width"], 4), 0.25, device="cuda") for cm in cams]
        gv, gt = rc.rc_render_backward_views(vol, cams, tf, sc.shading, sc.options, auxes, grads)
        out[f"backward_views{k}"] = _sums(gv, gt)
        # first-hit surface mode
        so = W.default_surface_options(step=1.5, gradient_op=c["op"],
                                       iso_lo=sc.vmin + 0.3 * (sc.vmax - sc.vmin))
        so["skip_empty"] = bool(sc.options["skip_empty"])
        simg, th = rc.rc_render_surface(vol, cam, tf, sc.shading, so,
                                        t_hit=torch.empty((cam["height"], cam["width"]),
                                                          device="cuda"))
        out[f"surface{k}"] = _digest(simg, th)
    # a batch of uneven items, eager and graph-replayed
    items = []
    for k, c in enumerate(cases[:4]):
        sc = W.config_small(**c)
        vol = rc.rc_create_volume(_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
        rc.rc_build_bricks(vol, 8)
        cam = sc.cameras[0]
        items.append({"vol": vol, "camera": cam, "tf": _dev(sc.tf), "shading": sc.shading,
                      "options": sc.options,
                      "out": torch.empty((cam["height"], cam["width"], 4), device="cuda")})
    torch.cuda.synchronize()
    s = torch.cuda.Stream()             # graph capture needs a stream of its own
    for cfg in (dict(tile_w=8, waves_per_wg=1, wg_per_cu=12, order=0),
                dict(tile_w=4, waves_per_wg=4, wg_per_cu=2, order=1)):
        b = rc.rc_batch_create(items, cfg, stream=s)
        rc.rc_batch_render(b, stream=s)
        rc.rc_batch_render(b, use_graph=True, stream=s)
        rc.rc_batch_render(b, use_graph=True, stream=s)
        s.synchronize()
        out[f"batch_tw{cfg['tile_w']}"] = _digest(*[it["out"] for it in items])
        rc.rc_batch_destroy(b)
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    torch.cuda.set_device(0)
    res = {"digests": run_cases()}
    try:
        res["violations"] = rc.rc_debug_bounds_violations()
    except rc.RCError as e:
        res["violations"] = None
        res["error"] = str(e)
    print(json.dumps(res), flush=True)
