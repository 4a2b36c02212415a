"""Tile-bucket binning + per-tile depth sort (the default frame path) against
the emission + LSD radix path, which the oracle parity tests pin: identical
tile ranges, sorted splat indices and images, on scenes built to reach the
bucket sort's harder branches — tile segments far beyond one workgroup's LDS
capacity (multi-level splits), long runs of exactly equal depth (splits on
the splat-index bits, the full-key fallback of the LDS sort), and frames with
more tiles than the bucket path takes (radix fallback)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from paper_2501_17792_amd import synth

from .gpu_common import check_sorted_pairs, gpu_frame_buffers

pytestmark = pytest.mark.gpu


def _render(scene, algo, tile=(16, 16), mode=None, thresholds=(), ranks=0, blocks=(0, 0)):
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    mode = cs.CS_LOD_FULL if mode is None else mode
    r = cs.Renderer(0, tile=tile, sort_algo=algo, sort_ranks=ranks, blocks=blocks)
    r.upload_templates(scene.templates)
    r.set_crowd(scene.crowd)
    img = r.frame(scene.camera, mode, thresholds, stats=True)
    torch.cuda.synchronize()
    st = r.last_stats
    assert st.overflow == 0
    # no LDS-sorted segment failed its order check (a failure would have been
    # re-sorted with ballot ranks and counted here)
    assert st.sort_fallbacks == 0
    cam = scene.camera
    n_tiles = -(-cam.width // tile[0]) * -(-cam.height // tile[1])
    ranges = r.debug("RANGES", np.uint32, 2 * n_tiles).reshape(n_tiles, 2)
    svals = r.debug("SVALS", np.uint32, int(st.n_pairs)) if st.n_pairs else np.zeros(0, np.uint32)
    return r, img.cpu().numpy(), ranges, svals


def _same_as_radix(scene, tile=(16, 16), **kw):
    from paper_2501_17792_amd import crowdsplat as cs

    rb, img_b, rg_b, sv_b = _render(scene, cs.CS_SORT_TILE_BUCKET, tile, **kw)
    _, img_r, rg_r, sv_r = _render(scene, cs.CS_SORT_REDUCE_SCAN, tile, **kw)
    assert np.array_equal(rg_b, rg_r)
    assert np.array_equal(sv_b, sv_r)
    assert np.array_equal(img_b, img_r)
    # the LDS sort with ballot ranks in every pass (documented behaviour only)
    # gives the same order as its checked LDS-atomic ranks
    _, img_q, rg_q, sv_q = _render(scene, cs.CS_SORT_TILE_BUCKET, tile, ranks=cs.CS_SORT_RANKS_BALLOT, **kw)
    assert np.array_equal(rg_q, rg_b)
    assert np.array_equal(sv_q, sv_b)
    assert np.array_equal(img_q, img_b)
    g = gpu_frame_buffers(rb, scene.crowd.n)
    check_sorted_pairs(g, g["n_splats"])
    return rg_b


def _clustered(t: synth.Template, seed: int, n_clusters: int, frac: float) -> synth.Template:
    """``frac`` of the Gaussians moved onto ``n_clusters`` shared means (with the
    representative's skin binding), so each cluster skins and projects to one
    exact depth."""
    rng = np.random.default_rng(seed)
    mean, idx, w = t.mean.copy(), t.skin_idx.copy(), t.skin_w.copy()
    pick = rng.uniform(size=t.n) < frac
    rep = rng.integers(0, n_clusters, size=t.n)
    mean[pick] = mean[rep[pick]]
    idx[pick] = idx[rep[pick]]
    w[pick] = w[rep[pick]]
    return dataclasses.replace(t, mean=mean, skin_idx=idx, skin_w=w)


def test_long_segments_multi_level_split():
    """A dense far crowd piles >100k pairs into single tiles."""
    templates = [synth.make_template(t, 40000, 1, (1.0, 0.25)) for t in range(2)]
    rng = np.random.default_rng(7)
    n = 40
    pos = np.stack([rng.uniform(-2.0, 2.0, n), rng.uniform(18.0, 26.0, n)], 1).astype(np.float32)
    crowd = synth.Crowd(tid=rng.integers(0, 2, n).astype(np.int32), yaw=rng.uniform(0, 6.28, n).astype(np.float32),
                        pos=pos, pose=rng.normal(0, 0.3, (n, 24, 3)).astype(np.float32))
    cam = synth.look_at((0.0, 1.5, 0.0), (0.0, 1.0, 22.0), 640, 360)
    sc = synth.Scene("dense", templates, crowd, cam, lod_thresholds=())
    rg = _same_as_radix(sc)
    seg = (rg[:, 1] - rg[:, 0]).astype(np.int64)
    assert seg.max() > 4 * 16384  # far beyond one workgroup's LDS capacity: the split path ran
    print("max tile segment", seg.max(), "pairs", seg.sum())
    # the workgroup counts the autotuner may pick leave every list and pixel unchanged
    from paper_2501_17792_amd import crowdsplat as cs

    _, img0, rg0, sv0 = _render(sc, cs.CS_SORT_TILE_BUCKET)
    for blocks in [(64, 64), (256, 1024), (1024, 4096), (777, 333)]:
        _, img1, rg1, sv1 = _render(sc, cs.CS_SORT_TILE_BUCKET, blocks=blocks)
        assert np.array_equal(rg1, rg0) and np.array_equal(sv1, sv0) and np.array_equal(img1, img0), blocks
    with pytest.raises(cs.CrowdSplatError):
        cs.Renderer(0, blocks=(2048, 0))


def test_equal_depth_runs():
    """Clusters of Gaussians at one exact depth, four identical instances on
    one spot: equal-depth runs of tens of thousands of pairs in a tile."""
    t = _clustered(synth.make_template(3, 30000, 0, (1.0,)), 1, 3, 0.7)
    rng = np.random.default_rng(2)
    pose = np.repeat(rng.normal(0, 0.2, (1, 24, 3)), 4, axis=0).astype(np.float32)
    crowd = synth.Crowd(tid=np.zeros(4, np.int32), yaw=np.full(4, 0.3, np.float32),
                        pos=np.zeros((4, 2), np.float32), pose=pose)
    cam = synth.look_at((0.0, 1.0, -3.0), (0.0, 0.9, 0.0), 256, 256)
    sc = synth.Scene("ties", [t], crowd, cam, lod_thresholds=())
    _same_as_radix(sc)


def test_short_equal_depth_runs_in_lds():
    """Equal depths inside segments that fit the LDS sort (tie runs shorter
    and longer than the per-thread fix-up handles)."""
    t = _clustered(synth.make_template(4, 6000, 0, (1.0,)), 2, 40, 0.5)
    rng = np.random.default_rng(3)
    crowd = synth.Crowd(tid=np.zeros(2, np.int32), yaw=np.zeros(2, np.float32),
                        pos=np.array([[0.0, 0.0], [0.0, 0.0]], np.float32),
                        pose=np.repeat(rng.normal(0, 0.2, (1, 24, 3)), 2, axis=0).astype(np.float32))
    cam = synth.look_at((0.0, 1.0, -4.0), (0.0, 0.9, 0.0), 192, 160)
    sc = synth.Scene("ties_small", [t], crowd, cam, lod_thresholds=())
    for tile in [(8, 8), (16, 16), (32, 32)]:
        _same_as_radix(sc, tile)


def test_many_short_equal_depth_runs():
    """Thousands of small clusters (a few Gaussians on one mean): tie runs of
    2 to a few dozen keys all through the LDS-sorted segments, next to each
    other and across wave and segment boundaries."""
    t = _clustered(synth.make_template(5, 40000, 0, (1.0,)), 4, 4000, 0.6)
    rng = np.random.default_rng(5)
    crowd = synth.Crowd(tid=np.zeros(3, np.int32), yaw=np.array([0.0, 0.4, -0.3], np.float32),
                        pos=np.array([[0.0, 0.0], [0.35, 0.6], [-0.4, 1.1]], np.float32),
                        pose=rng.normal(0, 0.2, (3, 24, 3)).astype(np.float32))
    cam = synth.look_at((0.0, 1.0, -3.5), (0.0, 0.9, 0.0), 320, 256)
    sc = synth.Scene("ties_short", [t], crowd, cam, lod_thresholds=())
    for tile in [(16, 16), (32, 16)]:
        _same_as_radix(sc, tile)


def test_radix_fallback_beyond_bucket_tiles():
    """A frame with more than 8192 tiles takes the radix path by itself and
    draws the same image as with 16x16 tiles."""
    from paper_2501_17792_amd import crowdsplat as cs

    templates = [synth.make_template(t, 8000, 0, (1.0,)) for t in range(2)]
    crowd = synth.make_crowd(5, 10, 2, 8.0, 0.3)
    cam = synth.look_at((4.0, 1.7, -6.0), (4.0, 1.0, 4.0), 800, 680)  # 100 x 85 tiles of 8x8
    sc = synth.Scene("many_tiles", templates, crowd, cam, lod_thresholds=())
    _, img8, _, _ = _render(sc, cs.CS_SORT_TILE_BUCKET, (8, 8))
    _, img16, _, _ = _render(sc, cs.CS_SORT_TILE_BUCKET, (16, 16))
    assert np.array_equal(img8, img16)


def test_bucket_graph_replay_and_backward_offsets():
    """Captured bucket frames replay bit-exactly; the pair offsets the backward
    pass builds on demand equal the scan of the tile counts."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    templates = [synth.make_template(t, 12000, 0, (1.0, 0.25)) for t in range(2)]
    crowd = synth.make_crowd(9, 16, 2, 10.0, 0.3)
    cam = synth.look_at((5.0, 1.7, -4.0), (5.0, 1.0, 6.0), 320, 240)
    sc = synth.Scene("replay", templates, crowd, cam, lod_thresholds=(6.0,))
    r, ref, _, _ = _render(sc, cs.CS_SORT_TILE_BUCKET, mode=cs.CS_LOD_FIXED, thresholds=(6.0,))
    g = gpu_frame_buffers(r, sc.crowd.n)
    cnt = g["count"].astype(np.int64)
    np.testing.assert_array_equal(g["pair_off"].astype(np.int64), np.concatenate([[0], np.cumsum(cnt)[:-1]]))
    stream = torch.cuda.Stream()
    r2 = cs.Renderer(0, stream=stream)
    r2.upload_templates(sc.templates)
    r2.set_crowd(sc.crowd)
    with torch.cuda.stream(stream):
        r2.frame(sc.camera, cs.CS_LOD_FIXED, (6.0,))
        out = torch.zeros((3, cam.height, cam.width), device="cuda")
        r2.capture(sc.camera, out, cs.CS_LOD_FIXED, (6.0,))
        for k in range(3):
            out.zero_()
            r2.launch()
            assert r2.poll().overflow == 0
            assert np.array_equal(out.cpu().numpy(), ref), k
    stream.synchronize()


def test_frames_in_flight_on_separate_contexts():
    """Contexts on separate streams replay their captured frames concurrently
    (the bench's frames in flight) and each draws exactly what one context
    draws alone for the same pose."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    templates = [synth.make_template(t, 12000, 0, (1.0, 0.25)) for t in range(2)]
    crowd = synth.make_crowd(11, 24, 2, 10.0, 0.3)
    cam = synth.look_at((5.0, 1.7, -4.0), (5.0, 1.0, 6.0), 320, 240)
    rng = np.random.default_rng(5)
    poses = [torch.from_numpy(rng.normal(0, 0.3, (crowd.n, 24, 3)).astype(np.float32)).cuda() for _ in range(4)]
    ref = []
    r0 = cs.Renderer(0)
    r0.upload_templates(templates)
    r0.set_crowd(crowd)
    for p in poses:
        r0.pose_dev.copy_(p)
        ref.append(r0.frame(cam, cs.CS_LOD_FIXED, (6.0,)).cpu().numpy())
    r0.close()
    streams = [torch.cuda.Stream() for _ in range(2)]
    rs, outs = [], []
    for st in streams:
        with torch.cuda.stream(st):
            r = cs.Renderer(0, stream=st)
            r.upload_templates(templates)
            r.set_crowd(crowd)
            r.frame(cam, cs.CS_LOD_FIXED, (6.0,))
            out = torch.zeros((3, cam.height, cam.width), device="cuda")
            r.capture(cam, out, cs.CS_LOD_FIXED, (6.0,))
            rs.append(r)
            outs.append(out)
    torch.cuda.synchronize()
    for rnd in range(2):
        for i, (r, st) in enumerate(zip(rs, streams)):
            with torch.cuda.stream(st):
                r.pose_dev.copy_(poses[2 * rnd + i])
                r.launch()
        torch.cuda.synchronize()
        for i, r in enumerate(rs):
            assert r.poll().overflow == 0
            assert np.array_equal(outs[i].cpu().numpy(), ref[2 * rnd + i]), (rnd, i)
    for r in rs:
        r.close()
