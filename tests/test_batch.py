"""Batched persistent rendering vs one rc_render per item (the same arithmetic,
so outputs must be bit-identical), hipGraph replay vs eager, the autotuner,
and the full 64-volume workload."""
import json
import os

import numpy as np
import pytest
import torch

import paper_1609_01317_amd as rc
import workloads as W
from tests.gpu_util import compare, gpu_volume, oracle_render, to_dev

pytestmark = pytest.mark.gpu


def _scenes():
    out = []
    specs = [
        dict(seed=41, dims=(26, 21, 19), dtype=np.uint8, image=(37, 29), op="central"),
        dict(seed=42, dims=(40, 17, 33), dtype=np.uint16, image=(64, 48), op="sobel3d",
             ert=0.99, skip=True),
        dict(seed=43, dims=(12, 30, 9), dtype=np.float32, image=(16, 40), op="zucker_hummel",
             shading="none"),
        dict(seed=44, dims=(33, 33, 33), dtype=np.uint8, image=(8, 8), op="sobel3d",
             projection="ortho", skip=True),
        dict(seed=45, dims=(50, 44, 20), dtype=np.uint16, image=(128, 96), op="central",
             ert=0.95, skip=True),
        dict(seed=46, dims=(9, 9, 9), dtype=np.uint8, image=(3, 130), op="zucker_hummel",
             shading="paper_lambert"),
        dict(seed=47, dims=(30, 25, 22), dtype=np.uint16, image=(40, 24), op="sobel3d",
             skip=True, ert=0.98),
    ]
    for sp in specs:
        sc = W.config_small(**sp)
        if sc.shading["model"] == "paper_lambert":
            sc.shading["light_is_point"] = True
            sc.shading["light"] = (40.0, -30.0, 35.0)
        if sp["seed"] == 47:
            sc.options.update(nearest=True, ref_step=0.8)
        out.append(sc)
    return out


def _items(scenes):
    items = []
    for sc in scenes:
        cam = sc.cameras[0]
        items.append({"vol": gpu_volume(sc), "camera": cam, "tf": to_dev(sc.tf),
                      "shading": sc.shading, "options": sc.options,
                      "out": torch.full((cam["height"], cam["width"], 4), -1.0, device="cuda"),
                      "aux": rc.new_aux(cam)})
    return items


def _reference(items):
    refs = []
    for it in items:
        aux = rc.new_aux(it["camera"])
        img = rc.rc_render(it["vol"], it["camera"], it["tf"], it["shading"], it["options"],
                           aux=aux)
        refs.append((img.clone(), aux.clone()))
    torch.cuda.synchronize()
    return refs


@pytest.mark.parametrize("cfg", [None, dict(tile_w=16, waves_per_wg=4, wg_per_cu=2, order=0),
                                 dict(tile_w=4, waves_per_wg=2, wg_per_cu=1, order=1),
                                 dict(tile_w=32, waves_per_wg=1, wg_per_cu=32, order=1),
                                 # the smallest boxes and first chunks (chunks halve to fit)
                                 dict(tile_w=8, waves_per_wg=1, wg_per_cu=8, order=1,
                                      box_bytes_grad=2048, box_bytes_cd=2048, chunk_len=4),
                                 # the largest boxes and first chunks
                                 dict(tile_w=8, waves_per_wg=2, wg_per_cu=4, order=0,
                                      box_bytes_grad=32768, box_bytes_cd=32768, chunk_len=64)])
def test_batch_equals_single_renders(cfg):
    scenes = _scenes()
    items = _items(scenes)
    refs = _reference(items)
    rc.rc_render_batch(items, cfg)
    torch.cuda.synchronize()
    for it, (img, aux) in zip(items, refs):
        assert torch.equal(it["out"], img)
        assert torch.equal(it["aux"], aux)
    # and against the oracle for one item of each dtype
    for k in (0, 1, 2):
        r = oracle_render(scenes[k])
        err, bad = compare(items[k]["out"].cpu().numpy(), r, scenes[k].options["ert_threshold"])
        assert not bad.any(), err


@pytest.mark.parametrize("images", [[(1, 1)], [(1, 1), (3, 2)], [(8, 8)] * 3 + [(9, 1)],
                                    [(70, 9)] * 5])
def test_batches_smaller_than_the_work_queues(images):
    """The launch's tiles go to eight per-XCD queues in groups of 8: a batch
    of one tile (seven queues empty from the start), a few tiles, and one
    that fills some groups partly.  Every output equals rc_render bit for
    bit; the pixels were all written (they start at -1)."""
    sc = W.config_small(seed=51, dims=(21, 18, 16), dtype=np.uint16, image=(8, 8),
                        op="sobel3d", ert=0.97, skip=True)
    vol = gpu_volume(sc, bricks=True)
    tf = to_dev(sc.tf)
    items = []
    for j, (w, h) in enumerate(images):
        cam = W.orbit_camera((21, 18, 16), sc.spacing, 23.0 * j, 15.0, w, h)
        items.append({"vol": vol, "camera": cam, "tf": tf, "shading": sc.shading,
                      "options": sc.options,
                      "out": torch.full((h, w, 4), -1.0, device="cuda"), "aux": rc.new_aux(cam)})
    refs = _reference(items)
    for cfg in (None, dict(tile_w=4, waves_per_wg=2, wg_per_cu=1, order=0)):
        for it in items:
            it["out"].fill_(-1.0)
        rc.rc_render_batch(items, cfg)
        torch.cuda.synchronize()
        for it, (img, aux) in zip(items, refs):
            assert torch.equal(it["out"], img)
            assert torch.equal(it["aux"], aux)


def test_items_sharing_volume_and_table():
    """Orbit-style batches: several views of one volume and table (their
    empty-brick masks are computed once and shared), mixed with items that
    share only the volume or only the table.  Every output equals its own
    rc_render bit for bit."""
    sc = W.config_small(seed=48, dims=(45, 38, 33), dtype=np.uint16, image=(48, 40),
                        op="sobel3d", ert=0.99, skip=True)
    vol = gpu_volume(sc, bricks=True)
    tf = to_dev(sc.tf)
    tf2 = to_dev(W.tf_ramps(sc.tf.shape[0], seed=148, alpha_max=0.3,
                            hi=max(0.06, 0.9 * float(sc.volume.max()) / 4095.0)))
    sc2 = W.config_small(seed=49, dims=(30, 28, 26), dtype=np.uint16, image=(32, 32),
                         op="sobel3d", skip=True)
    vol2 = gpu_volume(sc2, bricks=True)
    items = []
    for az, v, t in ((0.0, vol, tf), (40.0, vol, tf), (95.0, vol, tf2), (150.0, vol, tf),
                     (200.0, vol2, tf), (260.0, vol, tf2), (300.0, vol, tf)):
        dims = sc.volume.shape[::-1] if v is vol else sc2.volume.shape[::-1]
        cam = W.orbit_camera(tuple(dims), (1, 1, 1), az, 20.0, 48, 40)
        items.append({"vol": v, "camera": cam, "tf": t, "shading": sc.shading,
                      "options": sc.options,
                      "out": torch.full((40, 48, 4), -1.0, device="cuda"),
                      "aux": rc.new_aux(cam)})
    refs = _reference(items)
    rc.rc_render_batch(items)
    torch.cuda.synchronize()
    lit = 0
    for it, (img, aux) in zip(items, refs):
        assert torch.equal(it["out"], img)
        assert torch.equal(it["aux"], aux)
        lit += int((img[..., 3] > 1e-3).sum())
    assert lit > 500


def test_graph_replay_matches_eager():
    scenes = _scenes()
    items = _items(scenes)
    refs = _reference(items)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = rc.rc_batch_create(items, stream=s)
        for rep in range(4):
            for it in items:
                it["out"].fill_(float(rep))           # eager work between replays
            rc.rc_batch_render(b, use_graph=True, stream=s)
            s.synchronize()
            for it, (img, aux) in zip(items, refs):
                assert torch.equal(it["out"], img), f"replay {rep}"
            # unrelated eager render on the same stream between replays
            rc.rc_render(items[0]["vol"], items[0]["camera"], items[0]["tf"],
                         items[0]["shading"], items[0]["options"])
            s.synchronize()
        rc.rc_batch_render(b, use_graph=False, stream=s)
        s.synchronize()
        for it, (img, aux) in zip(items, refs):
            assert torch.equal(it["out"], img)
        rc.rc_batch_destroy(b)


def test_autotune_and_cache(tmp_path):
    """Launch shape, LDS box budgets and first chunk length are searched and
    cached together (one JSON line per item set); a cache hit returns the
    same configuration without timing."""
    items = _items(_scenes())
    path = str(tmp_path / "tune.jsonl")
    cfg = rc.rc_batch_autotune(items, path)
    assert cfg["tile_w"] in (4, 8, 16, 32) and cfg["wg_per_cu"] >= 1
    # the scenes hold Sobel3D / Zucker-Hummel and central-difference items:
    # both budgets are chosen
    assert cfg["box_bytes_grad"] in (0, 8192, 12288, 16384, 20480)
    assert cfg["box_bytes_cd"] in (0, 4096, 8192, 12288)
    assert cfg["chunk_len"] in (0, 8, 32)
    lines = open(path).read().strip().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert all(rec[k] == cfg[k] for k in cfg)
    cfg2 = rc.rc_batch_autotune(items, path)       # cache hit: no new line
    assert cfg2 == cfg and len(open(path).read().strip().splitlines()) == 1
    refs = _reference(items)
    rc.rc_render_batch(items, cfg)
    torch.cuda.synchronize()
    for it, (img, _) in zip(items, refs):
        assert torch.equal(it["out"], img)


def test_batch_rejects_box_budget_beyond_the_workgroup():
    """4 waves x 32 KiB boxes would need 128 KiB of LDS per workgroup."""
    items = _items(_scenes()[:2])
    with pytest.raises(rc.RCError) as e:
        rc.rc_batch_create(items, dict(tile_w=8, waves_per_wg=4, wg_per_cu=2, order=0,
                                       box_bytes_grad=32768, box_bytes_cd=32768))
    assert e.value.status == rc.RC_E_INVALID and "64 KiB" in str(e.value)


def test_batch_rejects_bad_item():
    items = _items(_scenes()[:2])
    items[1]["options"] = dict(items[1]["options"], step=-1.0)
    with pytest.raises(rc.RCError) as e:
        rc.rc_batch_create(items)
    assert e.value.status == rc.RC_E_INVALID and "item 1" in str(e.value)


def test_c4_sixty_four_volumes():
    """The 64-volume workload: one persistent launch (graph-replayed) equals 64
    sequential renders bit for bit; 4 items are also checked on sampled
    pixels against the oracle."""
    scenes = W.config_c4()
    items = _items(scenes)
    refs = _reference(items)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = rc.rc_batch_create(items, stream=s)
        for _ in range(2):
            rc.rc_batch_render(b, use_graph=True, stream=s)
        s.synchronize()
    for it, (img, aux) in zip(items, refs):
        assert torch.equal(it["out"], img)
    rng = np.random.default_rng(404)
    for k in (0, 17, 40, 63):
        sc = scenes[k]
        cam = sc.cameras[0]
        pix = rng.choice(cam["width"] * cam["height"], size=2000, replace=False)
        r = oracle_render(sc, pixels=pix)
        err, bad = compare(items[k]["out"].cpu().numpy().reshape(-1, 4)[pix], r,
                           sc.options["ert_threshold"])
        assert not bad.any(), (k, err)
