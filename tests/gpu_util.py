"""Helpers shared by the GPU tests: render through the C ABI binding and
compare with the oracle under the admissible-result rules (lattice-end
ties have two correct answers; early-termination near-ties are allowed
1 - tau)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_1609_01317_amd as rc

TOL = 2e-4


def to_dev(arr):
    t = torch.from_numpy(np.ascontiguousarray(arr))
    return t.cuda()


def gpu_volume(sc, bricks=None):
    vol = rc.rc_create_volume(to_dev(sc.volume), sc.spacing, sc.vmin, sc.vmax)
    if bricks or (bricks is None and sc.options["skip_empty"]):
        rc.rc_build_bricks(vol, 8)
    return vol


def gpu_render(sc, cam=None, vol=None, options=None, shading=None, stats=False):
    cam = cam or sc.cameras[0]
    options = options or sc.options
    shading = shading or sc.shading
    vol = vol or gpu_volume(sc, bricks=options["skip_empty"])
    tf = to_dev(sc.tf)
    aux = rc.new_aux(cam)
    st = rc.new_stats() if stats else None
    out = rc.rc_render(vol, cam, tf, shading, options, aux=aux, stats=st)
    torch.cuda.synchronize()
    k_last, t_final = rc.aux_fields(aux)
    res = {"rgba": out.cpu().numpy(), "k_last": k_last.cpu().numpy(),
           "t_final": t_final.cpu().numpy()}
    if stats:
        res["stats"] = st.cpu().numpy()
    return res


def oracle_render(sc, cam=None, options=None, shading=None, pixels=None, threads=0):
    cam = cam or sc.cameras[0]
    v = oracle.Volume(sc.volume, sc.spacing, sc.vmin, sc.vmax)
    return oracle.render(v, cam, sc.tf, shading or sc.shading, options or sc.options,
                         pixels=pixels, threads=threads)


def compare(gpu_rgba, ref, tau=0.0, tol=TOL):
    """Per-pixel admissible error; returns (max error, mask of failing pixels)."""
    g = gpu_rgba.reshape(-1, 4).astype(np.float64)
    p = ref["rgba"].reshape(-1, 4)
    a = ref["rgba_alt"].reshape(-1, 4)
    err = np.minimum(np.abs(g - p).max(axis=1), np.abs(g - a).max(axis=1))
    lim = np.full(err.shape, tol)
    near = (ref["flags"].reshape(-1) & oracle.FLAG_ERT_NEAR) != 0
    lim[near] = (1.0 - tau) + tol
    # adaptive sampling: a sample on a brick plane may take either brick's step
    lim[(ref["flags"].reshape(-1) & oracle.FLAG_ADAPT_NEAR) != 0] = np.inf
    return float(err.max()) if err.size else 0.0, err > lim
