"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances (FP32 kernel vs FP64 oracle on the same FP32 inputs):
* bone matrices, posed means / covariances: relative 2e-5 of the largest
  entry magnitude (a few FP32 ulps through the 24-joint chain);
* screen position u, v: 2e-3 px; conic, 2D covariance, depth: relative 1e-4;
  colour: 1e-4 absolute;
* tile rects and visibility against the FP64 footprint: equal except where
  the oracle's bound lies within 2e-3 px of a pixel edge (both decisions are
  then correct);
* keys, rects, per-tile lists and ranges: bit-exact against the integer key
  oracle, which takes the device's own float32 records (u, v, rx, ry, depth)
  and decides in float32 like the kernel (the order of the frame path's
  sorted splat indices and its tile ranges, not rebuilt keys);
* per-tile splat sets against the FP64 oracle's own lists: equal except the
  rect-fragile splats; order consistent with the FP64 depths except among
  depths equal to 2e-6 relative;
* pixels, two ways, both over the device's per-tile lists (membership and
  order are integer decisions the kernel takes in float32, pinned bit-exactly
  above):
  - compositing alone: the device's own records, upcast, composited in FP64:
    max-abs 2e-3 outside the pixels where an evaluated splat has alpha
    within the float32 error of the kernel's alpha of 1/255, or T' within
    1e-4 (relative) of 1e-4. That error: dx = (x + 1/2) - u is exact near
    the splat (Sterbenz), the exponent's float32 terms err by a few ulps of
    their magnitude (allowed: 8 ulps of (A dx^2 + 2|B dx dy| + C dy^2)/2,
    which matters for thin splats whose terms cancel) and __expf by a few
    ulps (allowed: 1e-5 relative, about 30 ulps);
  - end to end: the FP64 oracle's records composited in FP64: max-abs 2e-3
    outside the same bands widened splat by splat by how far the FP64 and
    the device's records put that alpha and T' apart (there the two records
    may legitimately decide differently);
  a flagged pixel may miss the 2e-3 bar, but by at most
  cmax (2/255 + 1.01e-2) + 2e-3 (one skip flip moves a pixel by at most
  2 cmax / 255, one stop flip by at most cmax T <= cmax 1e-2 plus the 1e-4
  left after it), and such pixels are at most 1e-3 of those compared. (How
  many pixels are flagged grows with the splats a pixel evaluates; nearly
  all of them still meet 2e-3.)
"""
import numpy as np
import pytest

from oracle import frame as oframe
from oracle import skinning as oskin
from oracle import splat as osplat
from paper_2501_17792_amd import synth

from .gpu_common import (check_sorted_pairs, gpu_frame_buffers, rect_fragile, run_gpu,
                         unpack_rect)

pytestmark = pytest.mark.gpu

BAND_ALPHA = 1e-5
BAND_T = 1e-4
POWER_ULPS = 8.0
BEYOND_MAX = 1e-3  # share of the compared pixels that may miss 2e-3 (flagged ones only)


def flag_bound(rgb):
    cmax = float(np.max(rgb)) if np.size(rgb) else 1.0
    return cmax * (2.0 / 255.0 + 1.01e-2) + 2e-3


def device_records(R):
    """The device's float32 records as the oracle's record dict (FP64)."""
    R = R.astype(np.float64)
    return dict(u=R[:, 0], v=R[:, 1], A=R[:, 4], B=R[:, 5], C=R[:, 6], opacity=R[:, 7],
                rgb=R[:, 8:11], depth=R[:, 11])


def integer_key_oracle(R, cam, tw, th):
    """Rects, counts, sorted splat indices and ranges from the device's own
    float32 records (u, v, rx, ry, depth), decided in float32."""
    ntx, nty = -(-cam.width // tw), -(-cam.height // th)
    rect, cnt, vis = osplat.footprint_rect_f32(R[:, 0], R[:, 1], R[:, 2], R[:, 3], R[:, 11], cam.width,
                                               cam.height, tw, th)
    keys, vals = osplat.emit_pairs(rect, cnt, vis, R[:, 11].astype(np.float64), ntx)
    sk, sv = osplat.sort_pairs(keys, vals)
    return rect, cnt, vis, sk, sv, osplat.tile_ranges(sk, ntx * nty)


def check_pixels(img, sp, svals, ranges, cam, tw, th, tiles=None, label="", sp_alt=None):
    """FP64 compositing of records ``sp`` over the device's lists against the
    device image (on ``tiles`` or all); ``sp_alt`` (the device's records)
    widens the fragile bands by its distance from ``sp``. Returns (max-abs
    outside the mask, flagged pixels, pixels beyond 2e-3, pixels compared)."""
    ref, _, frag = osplat.composite_tiled(sp, svals.astype(np.int64), ranges.astype(np.int64), cam.width,
                                          cam.height, tw, th, cam.bg, BAND_ALPHA, BAND_T, tiles=tiles,
                                          chunked=True, sp_alt=sp_alt, power_ulps=POWER_ULPS)
    return judge_pixels(img, ref, frag, tiles, cam.width, cam.height, tw, th, flag_bound(sp["rgb"]), label)


def judge_pixels(img, ref, frag, tiles, W, H, tw, th, bound, label):
    if tiles is None:
        sel = np.ones((H, W), bool)
    else:
        sel = np.zeros((H, W), bool)
        ntx = -(-W // tw)
        for t in tiles:
            ty, tx = divmod(int(t), ntx)
            sel[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw] = True
    diff = np.abs(img - ref).max(axis=0)
    clean = sel & ~frag
    worst = float(diff[clean].max()) if clean.any() else 0.0
    nf = int((frag & sel).sum())
    beyond = int((sel & (diff > 2e-3)).sum())
    fmax = float(diff[frag & sel].max()) if nf else 0.0
    print(f"  {label}: max-abs {worst:.2e} outside the mask; {nf} of {int(sel.sum())} pixels flagged "
          f"(max-abs {fmax:.2e}), {beyond} beyond 2e-3", flush=True)
    assert worst <= 2e-3, f"{label}: max-abs {worst} outside the fragile mask"
    assert fmax <= bound, f"{label}: flagged pixel off by {fmax}"
    assert beyond <= BEYOND_MAX * sel.sum() + 1, f"{label}: {beyond} pixels beyond 2e-3"
    return worst, nf, beyond, int(sel.sum())


def _small_c2_scene(n_inst=12, n_gauss=20000, width=480, height=270):
    """A slice of the 14-template SH3 crowd: fewer, smaller templates and
    instances, a 480x270 image (ragged last tile row) and the C2 camera rig."""
    templates = [synth.make_template(t, n_gauss, 3, synth.C2_LEVELS) for t in range(3)]
    crowd = synth.make_crowd(100, n_inst, 3, 12.0, 0.3)
    cam = synth.look_at((6.0, 1.7, -3.0), (6.0, 1.0, 8.0), width, height)
    return synth.Scene("c2slice", templates, crowd, cam, lod_thresholds=(6.0, 11.0))


def _compare_frame(scene, mode, thresholds, tile=(16, 16), setup=None, mean_fn=None, **kw):
    """The HIP frame against the FP64 oracle, stage by stage. ``setup(r)``
    runs on the renderer before the frame; ``mean_fn(i, n)`` gives the
    oracle instance i's canonical means when they depend on the instance."""
    from paper_2501_17792_amd import crowdsplat as cs

    r, img = run_gpu(scene, mode, thresholds, tile=tile, setup=setup, **kw)
    n_inst = scene.crowd.n
    g = gpu_frame_buffers(r, n_inst)
    cam = scene.camera
    tw, th = tile
    ntx, nty = -(-cam.width // tw), -(-cam.height // th)
    # ---- LoD levels: same decision unless the distance sits on a threshold
    if mode == cs.CS_LOD_FULL:
        levels = np.zeros(n_inst, np.int64)
    else:
        levels = oframe.fixed_levels(scene.crowd.pos, cam.eye, thresholds)
        dist = oframe.instance_distance(scene.crowd.pos, cam.eye)
        near = np.min(np.abs(dist[:, None] - np.asarray(thresholds)[None]), axis=1) < 1e-4
        assert np.all((g["level"] == levels) | near)
        levels = g["level"].astype(np.int64)  # decided identically within FP32 ties
    rec = oframe.frame_records(scene.templates, scene.crowd, cam, levels, tw, th, mean_fn=mean_fn)
    # ---- forward kinematics
    for i in range(n_inst):
        t = scene.templates[int(scene.crowd.tid[i])]
        B = oskin.bone_matrices(scene.crowd.pose[i], t.joints_rest, t.parents, scene.crowd.yaw[i],
                                scene.crowd.pos[i, 0], scene.crowd.pos[i, 1])
        scale = np.abs(B).max()
        np.testing.assert_allclose(g["bones"][i], B, atol=2e-5 * scale, rtol=0)
    # ---- work list
    np.testing.assert_array_equal(g["offset"].astype(np.int64), rec["offsets"])
    n = g["n_splats"]
    assert n == rec["offsets"][-1]
    # ---- skinning (posed means, covariances)
    mu = r.debug("SKIN_MU", np.float32, 4 * n).reshape(n, 4) if not kw.get("fuse") else None
    if mu is not None:
        scale = np.abs(rec["mu"]).max()
        np.testing.assert_allclose(mu[:, :3], rec["mu"], atol=2e-5 * scale, rtol=0)
        cov = r.debug("SKIN_COV", np.float32, 4 * n).reshape(n, 4)
        czz = r.debug("SKIN_COV2", np.float32, n)
        gcov = np.stack([mu[:, 3], cov[:, 0], cov[:, 1], cov[:, 2], cov[:, 3], czz], 1)
        ocov = rec["cov"][:, [0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
        cscale = np.abs(ocov).max(axis=1, keepdims=True)
        assert np.all(np.abs(gcov - ocov) <= 2e-5 * cscale + 1e-12)
    # ---- projection records against FP64
    frag_rect = rect_fragile(rec, tw, th, cam.width, cam.height)
    gvis = g["count"] > 0
    ovis = rec["visible"]
    assert np.all((gvis == ovis) | frag_rect), np.nonzero((gvis != ovis) & ~frag_rect)[0][:10]
    both = gvis & ovis
    R = g["rec"][both]
    np.testing.assert_allclose(R[:, 0], rec["u"][both], atol=2e-3)
    np.testing.assert_allclose(R[:, 1], rec["v"][both], atol=2e-3)
    np.testing.assert_allclose(R[:, 11], rec["depth"][both], rtol=1e-5)
    # record columns: u v rx ry | A B C o | r g b depth
    for k, name in [(4, "A"), (5, "B"), (6, "C")]:
        ref = rec[name][both]
        tol = 1e-4 * np.maximum(np.abs(rec["A"][both]), np.abs(rec["C"][both]))
        assert np.all(np.abs(R[:, k] - ref) <= tol), name
    np.testing.assert_allclose(R[:, 7], rec["opacity"][both], rtol=0, atol=0)
    np.testing.assert_allclose(R[:, [8, 9, 10]], rec["rgb"][both], atol=1e-4)
    np.testing.assert_allclose(R[:, 2], rec["rx"][both], rtol=1e-4)
    np.testing.assert_allclose(R[:, 3], rec["ry"][both], rtol=1e-4)
    grect = unpack_rect(g["rect"][both])
    ok = np.all(grect == rec["rect"][both], axis=1) | frag_rect[both]
    assert ok.all(), np.nonzero(~ok)[0][:10]
    # ---- O6: the integer key oracle on the device's own float32 records
    irect, icnt, ivis, isk, isv, irg = integer_key_oracle(g["rec"], cam, tw, th)
    np.testing.assert_array_equal(icnt, g["count"].astype(np.int64))
    np.testing.assert_array_equal(irect[ivis], unpack_rect(g["rect"][ivis]))
    assert int(icnt.sum()) == g["n_pairs"]
    np.testing.assert_array_equal(irg, g["ranges"].astype(np.int64))
    if g["n_pairs"]:
        np.testing.assert_array_equal(isv, g["svals"])
        check_sorted_pairs(g, n)
        # ---- per-tile sets against the FP64 oracle's own lists
        okeys, ovals = osplat.emit_pairs(rec["rect"], rec["count"], rec["visible"], rec["depth"], ntx)
        osk, osv = osplat.sort_pairs(okeys, ovals)
        org = osplat.tile_ranges(osk, ntx * nty)
        gv, ov = g["svals"].astype(np.int64), osv.astype(np.int64)
        fr = set(np.nonzero(frag_rect)[0].tolist())
        for tt in range(ntx * nty):
            a = gv[g["ranges"][tt, 0]:g["ranges"][tt, 1]]
            b = ov[org[tt, 0]:org[tt, 1]]
            assert set(a.tolist()) - fr == set(b.tolist()) - fr, f"tile {tt}"
            d = rec["depth"][a]  # order consistent with FP64 depth except near ties
            assert not (d[1:] < d[:-1] * (1 - 2e-6)).any(), f"tile {tt} depth order"
    # ---- pixels over the device's lists: end to end, then compositing alone
    drec = device_records(g["rec"])
    e2e = check_pixels(img, rec, g["svals"], g["ranges"], cam, tw, th, label="end to end", sp_alt=drec)
    comp = check_pixels(img, drec, g["svals"], g["ranges"], cam, tw, th, label="compositing")
    return r, img, rec, g, dict(e2e_max_abs=e2e[0], e2e_fragile=e2e[1], e2e_beyond=e2e[2], composite_max_abs=comp[0],
                                composite_fragile=comp[1], composite_beyond=comp[2], pixels=e2e[3])


def test_c1_plain_full_detail():
    from paper_2501_17792_amd import crowdsplat as cs

    sc = synth.scene_c1()
    _, img, rec, g, info = _compare_frame(sc, cs.CS_LOD_FULL, ())
    assert g["n_pairs"] > 1000
    print("C1", info)


def test_c2_slice_fixed_lod():
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene()
    _, img, rec, g, info = _compare_frame(sc, cs.CS_LOD_FIXED, sc.lod_thresholds)
    assert len(set(g["level"].tolist())) >= 2  # several levels in play
    print("C2 slice", info)


@pytest.mark.parametrize("tile", [(8, 8), (32, 8), (16, 32)])
def test_c2_slice_other_tiles(tile):
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene(n_inst=6)
    _compare_frame(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, tile=tile)


def test_tile_shape_launch_and_fusion_invariance():
    """The image is bit-identical across tile shapes, per-instance vs batched
    launches and sort forms, with skinning separate and with skinning fused
    into projection (which works in the camera frame and rounds differently:
    it is held to the oracle on its own, below and in the Tab. 2 cells)."""
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene(n_inst=8)
    for fuse in (False, True):
        _, ref = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=fuse)
        for kw in [dict(tile=(8, 8)), dict(tile=(32, 32)), dict(tile=(8, 32)),
                   dict(launch_mode=cs.CS_LAUNCH_PER_INSTANCE),
                   dict(sort_algo=cs.CS_SORT_ONESWEEP), dict(sort_algo=cs.CS_SORT_REDUCE_SCAN)]:
            _, img = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=fuse, **kw)
            assert np.array_equal(img, ref), (fuse, kw)


def test_blend_split_compositing_invariance():
    """A binning tile's rows composited by 2 or 4 workgroups (blend_split)
    give the bit-identical image, plain and with the compositing counters on;
    splits that leave fewer than 8 rows per workgroup, or other counts, are
    refused at creation."""
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene(n_inst=8)
    _, ref = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=True)
    for tile, split in [((16, 16), 2), ((16, 32), 2), ((16, 32), 4), ((32, 32), 2), ((32, 32), 4), ((8, 32), 4),
                        ((32, 16), 2)]:
        r, img = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=True, tile=tile, blend_split=split)
        assert np.array_equal(img, ref), (tile, split)
        assert r.last_stats.overflow == 0
        rc, img_c = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=True, tile=tile, blend_split=split,
                            profile=True, count_blend=True)
        assert np.array_equal(img_c, ref), (tile, split, "counting")
        assert rc.last_stats.blend_evals > 0
    for tile, split in [((16, 16), 4), ((8, 8), 2), ((16, 32), 3), ((32, 32), 8), ((16, 16), -1)]:
        with pytest.raises(cs.CrowdSplatError):
            cs.Renderer(0, tile=tile, blend_split=split)


def test_c2_slice_fused_matches_oracle():
    """Skinning fused into projection (camera-frame algebra) against the FP64
    oracle, records to pixels."""
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene()
    _, img, rec, g, info = _compare_frame(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=True)
    print("C2 slice fused", info)


def test_blend_evaluation_counters():
    """Instrumented frames count the compositing evaluations without changing
    the image: every splat a pixel adds was evaluated live for it (the FP64
    oracle's count over the device's lists bounds the count from below), no
    pixel evaluates more than its tile's list, and lane slots cover the live
    evaluations. Uninstrumented frames report none."""
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene(n_inst=6)
    rp, img_p = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, profile=True, count_blend=True)
    st = rp.last_stats
    _, img = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds)
    assert np.array_equal(img_p, img)
    g = gpu_frame_buffers(rp, sc.crowd.n)
    cam = sc.camera
    tw, th = 16, 16
    ntx = -(-cam.width // tw)
    lens = (g["ranges"][:, 1] - g["ranges"][:, 0]).astype(np.int64)
    upper = 0
    for t in range(len(lens)):
        ty, tx = divmod(t, ntx)
        w = min(tw, cam.width - tx * tw)
        h = min(th, cam.height - ty * th)
        upper += int(lens[t]) * w * h
    added = 0
    drec = device_records(g["rec"])
    for t in np.nonzero(lens)[0]:
        ty, tx = divmod(int(t), ntx)
        gy, gx = np.mgrid[ty * th:min((ty + 1) * th, cam.height), tx * tw:min((tx + 1) * tw, cam.width)]
        s0, s1 = g["ranges"][t]
        _, _, _, n_added = osplat._blend_list_chunked(gx.ravel() * 1.0, gy.ravel() * 1.0,
                                                       g["svals"][s0:s1].astype(np.int64), drec, cam.bg, 0, 0)
        added += int(n_added.sum())
    print(f"evals {st.blend_evals}, slots {st.blend_eval_slots} ({st.blend_done_slots} of finished pixels), "
          f"adds {st.blend_adds}, oracle adds {added}, list bound {upper}")
    assert 0 < added <= st.blend_evals <= min(upper, st.blend_eval_slots)
    assert st.blend_evals + st.blend_done_slots <= st.blend_eval_slots
    # the device's adds against the FP64 oracle's over the same lists: equal
    # but for pixels whose alpha or stopping test sits within rounding of its
    # threshold (each moves a pixel's count by about one)
    assert 0 < st.blend_adds <= st.blend_evals
    assert abs(st.blend_adds - added) <= 1e-3 * added + 16
    for kw in ({}, dict(profile=True)):
        r = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, **kw)[0]
        assert r.last_stats.blend_evals == 0 and r.last_stats.blend_eval_slots == 0
        assert r.last_stats.blend_done_slots == 0 and r.last_stats.blend_adds == 0


def test_determinism_and_graph_replay():
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    sc = _small_c2_scene(n_inst=8)
    r, ref = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds)
    img2 = r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds).cpu().numpy()
    assert np.array_equal(img2, ref)
    # graph capture of the whole frame, replayed with eager work in between
    stream = torch.cuda.Stream()
    r2 = cs.Renderer(0, stream=stream)
    r2.upload_templates(sc.templates)
    r2.set_crowd(sc.crowd)
    with torch.cuda.stream(stream):
        r2.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds)
        out = torch.zeros((3, sc.camera.height, sc.camera.width), device="cuda")
        r2.capture(sc.camera, out, cs.CS_LOD_FIXED, sc.lod_thresholds)
        for k in range(3):
            out.zero_()
            r2.launch()
            st = r2.poll()
            assert st.overflow == 0
            assert np.array_equal(out.cpu().numpy(), ref), k
            r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds)  # unrelated eager work
    stream.synchronize()


@pytest.mark.parametrize("algo", [0, 1])
@pytest.mark.parametrize("n,bits", [(1, 44), (1000, 44), (4096, 44), (4097, 46), (123457, 44),
                                    (2_000_000, 44), (70000, 13), (8192 * 512 + 77, 44)])
def test_standalone_sort_bit_exact(n, bits, algo):
    """The onesweep sort against numpy's stable argsort on tile-pair-shaped keys:
    few distinct tiles (heavy duplicates), FP32 depth bits, ragged sizes."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    rng = np.random.default_rng(n + bits)
    tiles = rng.integers(0, min(1 << max(bits - 31, 1), 300), size=n).astype(np.uint64)
    depth = rng.uniform(0.2, 90.0, size=n).astype(np.float32)
    depth[rng.uniform(size=n) < 0.2] = 7.5  # exact ties
    if bits > 31:
        keys = (tiles << np.uint64(31)) | depth.view(np.uint32).astype(np.uint64)
    else:
        keys = rng.integers(0, 1 << bits, size=n).astype(np.uint64)
    vals = np.arange(n, dtype=np.uint32)
    r = cs.Renderer(0, sort_algo=algo)
    kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    r.sort_pairs(kd, vd, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(vd.cpu().numpy().view(np.uint32), vals[order])


def test_copy_kernel():
    """The bandwidth-reference copy: exact, ragged sizes, misaligned refused."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    r = cs.Renderer(0)
    for nb in (16, 1000 * 16 + 7, (1 << 22) + 3):
        a = torch.randint(0, 255, (nb,), dtype=torch.uint8, device="cuda")
        b = torch.zeros_like(a)
        r.copy(b, a)
        torch.cuda.synchronize()
        assert torch.equal(a, b), nb
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(cs.CrowdSplatError) as e:
        r.copy(a[1:], a[:32], 16)
    assert e.value.code == cs.CS_ERR_INVALID
    r.close()


def test_empty_frame_and_bad_calls():
    """A crowd entirely behind the camera renders the background; calls out of
    order and bad arguments return status codes."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    sc = synth.scene_c1()
    sc.camera.bg[:] = (0.25, 0.5, 0.75)
    sc.crowd.pos[:] = (0.0, -20.0)  # behind the camera
    r, img = run_gpu(sc, cs.CS_LOD_FULL, ())
    assert r.last_stats.n_pairs == 0
    assert np.all(img[0] == 0.25) and np.all(img[1] == 0.5) and np.all(img[2] == 0.75)
    r2 = cs.Renderer(0)
    with pytest.raises(cs.CrowdSplatError) as e:
        r2.set_crowd(sc.crowd)
        r2.select_lod(sc.camera, cs.CS_LOD_FULL)
    assert e.value.code == cs.CS_ERR_STATE
    r2.upload_templates(sc.templates)
    with pytest.raises(cs.CrowdSplatError) as e:
        r2.render(sc.camera)
    assert e.value.code == cs.CS_ERR_STATE
