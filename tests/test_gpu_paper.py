"""The paper's own crowd set-ups against the FP64 oracle (through the C ABI).

* Tab. 2 cells (CrowdSplat §3): duplicates of one 3,176-Gaussian template on
  the grid, 1280x720, camera 3 m from the first row, with and without motion.
  The animated cell is a full captured frame per replay (poses from looping
  clips); the static cell skins once and captures rendering alone. Both are
  compared with the oracle on their first frame (records, keys, lists and
  pixels as in the parity tests) and the replays with eager frames.
* The paper's LoD schedule (§2 last paragraph): 202,738 / 12,661 / 3,176
  Gaussians chosen at 5 m and 10 m, on characters placed so every level is
  drawn.
"""
import numpy as np
import pytest

from paper_2501_17792_amd import synth

from .test_gpu_parity import _compare_frame

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tab2_template():
    return synth.make_template(600 + synth.PAPER_SIZES.index(3176), 3176, 3)


@pytest.mark.parametrize("n_chars", [1, 100])
def test_tab2_animated_cell_matches_oracle(tab2_template, n_chars):
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    sc = synth.scene_tab2(3176, n_chars, True, template=tab2_template, frames=8)
    print(f"tab2 animated cell: 3176 x {n_chars}", flush=True)
    r, img0, rec, g, info = _compare_frame(sc, cs.CS_LOD_FULL, (), fuse=True)
    print("tab2 animated", n_chars, info)
    assert g["n_pairs"] > 0
    # captured frames animate from a pose ring (pinned host memory for one
    # cell, device memory for the other): replay k draws ring frame
    # (first + k) % 8, equal to an eager frame of those poses
    poses = torch.from_numpy(sc.frame_poses)
    ring = poses.pin_memory() if n_chars == 1 else poses.cuda()
    # the eager reference runs on the capturing context's stream: its pose
    # copy (enqueued on the current stream) is then ordered before its frame
    stream = torch.cuda.Stream()
    re = cs.Renderer(0, stream=stream, fuse=True)
    re.upload_templates(sc.templates)
    re.set_crowd(sc.crowd)
    rc = cs.Renderer(0, stream=stream, fuse=True)
    rc.upload_templates(sc.templates)
    rc.set_crowd(sc.crowd)
    first = 5
    with torch.cuda.stream(stream):
        out = torch.zeros((3, sc.camera.height, sc.camera.width), device="cuda")
        rc.frame(sc.camera, cs.CS_LOD_FULL, (), image=out)
        rc.reserve(0, g["n_splats"] + 4096, 4 * max(g["n_pairs"], 1) + 65536)
        rc.set_pose_ring(ring, first=first)
        rc.capture(sc.camera, out, cs.CS_LOD_FULL, ())
        for k in range(5):
            f = (first + k) % poses.shape[0]
            rc.launch()
            assert rc.poll().overflow == 0
            got = out.cpu().numpy()
            re.pose_dev.copy_(poses[f].cuda())
            want = re.frame(sc.camera, cs.CS_LOD_FULL, ()).cpu().numpy()
            assert np.array_equal(got, want), (k, f)
            if f == 0:
                assert np.array_equal(got, img0)
    stream.synchronize()
    rc.close()
    re.close()


@pytest.mark.parametrize("n_chars", [1, 100])
def test_tab2_static_cell_matches_oracle(tab2_template, n_chars):
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    sc = synth.scene_tab2(3176, n_chars, False, template=tab2_template)
    print(f"tab2 static cell: 3176 x {n_chars}", flush=True)
    r, img0, rec, g, info = _compare_frame(sc, cs.CS_LOD_FULL, ())
    print("tab2 static", n_chars, info)
    # skin once, then replay rendering alone: every replay draws the same frame
    stream = torch.cuda.Stream()
    rs = cs.Renderer(0, stream=stream)
    rs.upload_templates(sc.templates)
    rs.set_crowd(sc.crowd)
    with torch.cuda.stream(stream):
        rs.reserve(sc.crowd.n, g["n_splats"] + 4096, 2 * max(g["n_pairs"], 1) + 65536)
        out = torch.zeros((3, sc.camera.height, sc.camera.width), device="cuda")
        rs.frame(sc.camera, cs.CS_LOD_FULL, (), image=out)
        rs.capture_render(sc.camera, out)
        for k in range(3):
            out.zero_()
            rs.launch()
            assert rs.poll().overflow == 0
            assert np.array_equal(out.cpu().numpy(), img0), k
    stream.synchronize()
    rs.close()
    # a fused context cannot capture a static crowd
    rf = cs.Renderer(0, fuse=True)
    rf.upload_templates(sc.templates)
    rf.set_crowd(sc.crowd)
    rf.frame(sc.camera, cs.CS_LOD_FULL, ())
    with pytest.raises(cs.CrowdSplatError) as e:
        rf.capture_render(sc.camera, torch.zeros((3, sc.camera.height, sc.camera.width), device="cuda"))
    assert e.value.code == cs.CS_ERR_UNSUPPORTED
    rf.close()


def test_paper_lod_schedule_matches_oracle():
    """Two 202,738-Gaussian templates with the paper's 12,661 and 3,176
    prefixes; six characters at 3.5 to 14 m from the camera, so the 5 m and
    10 m thresholds give every level."""
    from paper_2501_17792_amd import crowdsplat as cs

    templates = [synth.make_template_counts(900 + t, synth.PAPER_SIZES) for t in range(2)]
    cam = synth.paper_camera(480, 270)
    # ground positions at the wanted distances from the eye (0, 1.7, -3)
    dist = np.array([3.6, 4.6, 6.0, 8.5, 11.0, 14.0])
    x = np.array([-0.8, 0.9, -1.5, 1.4, -2.0, 2.5])
    z = -3.0 + np.sqrt(dist ** 2 - 1.7 ** 2 - x ** 2)
    rng = np.random.default_rng(5)
    clips = synth.looping_clips(1001)
    clip_of, phase = synth.clip_assignment(1002, 6)
    crowd = synth.Crowd(tid=np.array([0, 1, 0, 1, 0, 1], np.int32),
                        yaw=rng.uniform(0, 2 * np.pi, 6).astype(np.float32),
                        pos=np.stack([x, z], 1).astype(np.float32),
                        pose=synth.clip_poses(clips, clip_of, phase, 0))
    sc = synth.Scene("paper_lod_slice", templates, crowd, cam, lod_thresholds=(5.0, 10.0))
    r, img, rec, g, info = _compare_frame(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=True)
    assert sorted(set(g["level"].tolist())) == [0, 1, 2]
    counts = np.diff(g["offset"].astype(np.int64))
    assert set(counts.tolist()) == set(synth.PAPER_SIZES)
    print("paper LoD slice", info)
