"""The allocation-free form of the several-views render
(rc_render_views_noalloc): its scratch is the library's fixed device array
instead of a stream-ordered allocation.  Two calls in a row, the second
with a smaller input (a smaller volume with fewer bricks, fewer and smaller
views, another table), must each give images and aux bit-identical to
rc_render_views on the same views -- both run the same kernels, so any
difference would be stale or misplaced scratch -- and the second is also
compared with the FP64 oracle.  A call that needs more scratch than the
array holds is rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

import paper_1609_01317_amd as rc
import workloads as W
from tests.gpu_util import compare, gpu_volume, oracle_render, to_dev

pytestmark = pytest.mark.gpu


def _cams(sc, n, image):
    return [W.orbit_camera(sc.dims, sc.spacing, 20.0 + 37.0 * i, 15.0 + 5.0 * (i % 3), image[0],
                           image[1]) for i in range(n)]


def _noalloc_then_views(sc, vol, cams):
    tf = to_dev(sc.tf)
    outs = [torch.full((c["height"], c["width"], 4), float("nan"), device="cuda") for c in cams]
    auxes = [torch.full((c["height"], c["width"]), -1, dtype=torch.int64, device="cuda")
             for c in cams]
    print(f"no-alloc: {sc.name}, {len(cams)} views", flush=True)
    rc.rc_render_views_noalloc(vol, cams, tf, sc.shading, sc.options, outs, auxes)
    ref_aux = [rc.new_aux(c) for c in cams]
    ref = rc.rc_render_views(vol, cams, tf, sc.shading, sc.options, auxes=ref_aux)
    torch.cuda.synchronize()
    for v in range(len(cams)):
        assert torch.equal(outs[v], ref[v]), (sc.name, v)
        assert torch.equal(auxes[v], ref_aux[v]), (sc.name, v)
    return [o.cpu().numpy() for o in outs]


def test_noalloc_views_match_views_twice_second_smaller():
    big = W.config_small(seed=93, dims=(70, 61, 52), dtype=np.uint16, image=(8, 8),
                         op="sobel3d", ert=0.99, skip=True)
    vol_big = gpu_volume(big, bricks=True)
    _noalloc_then_views(big, vol_big, _cams(big, 6, (96, 80)))

    small = W.config_small(seed=94, dims=(21, 18, 15), dtype=np.uint8, image=(8, 8),
                           op="central", skip=True)
    vol_small = gpu_volume(small, bricks=True)
    cams = _cams(small, 2, (24, 20))
    got = _noalloc_then_views(small, vol_small, cams)
    for v, c in enumerate(cams):
        ref = oracle_render(small, cam=c)
        err, bad = compare(got[v], ref, small.options["ert_threshold"])
        assert not bad.any(), (v, err)


def test_noalloc_rejects_scratch_beyond_its_array():
    # 4096 x 4088 x 128 u8: 4,186,112 bricks, just under 2^31 padded voxels;
    # its brick mask alone is about 4 MiB, so with the super-brick mask,
    # the table counts and the descriptors it exceeds the array
    src = torch.zeros((128, 4088, 4096), dtype=torch.uint8, device="cuda")
    src[60:70, 2000:2100, 2000:2100] = 200
    vol = rc.rc_create_volume(src, (1.0, 1.0, 1.0), 0.0, 255.0)
    rc.rc_build_bricks(vol, 8)
    # table, shading and options of a small scene (its own volume is unused)
    sc = W.config_small(seed=95, dims=(16, 16, 16), dtype=np.uint8, image=(8, 8), skip=True)
    cam = W.orbit_camera((4096, 4088, 128), (1.0, 1.0, 1.0), 30.0, 20.0, 8, 8)
    out = [torch.zeros((8, 8, 4), device="cuda")]
    with pytest.raises(rc.RCError) as e:
        rc.rc_render_views_noalloc(vol, [cam], to_dev(sc.tf), sc.shading, sc.options, out)
    assert e.value.status == rc.RC_E_INVALID and "scratch" in str(e.value)
    # the same views through the allocating form still render
    rc.rc_render_views(vol, [cam], to_dev(sc.tf), sc.shading, sc.options, outs=out)
    torch.cuda.synchronize()
    assert torch.isfinite(out[0]).all()
    del vol, src
