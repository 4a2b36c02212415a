"""Pose-dependent Gaussian offsets (the offset network on the matrix cores)
against the FP64 oracle, through the C ABI.

Tolerance (derived from the arithmetic): both sides round the same bfloat16
weights and inputs; the device accumulates in FP32 where the oracle uses
FP64, so a hidden value lying at a bfloat16 rounding boundary may round one
step the other way. Every offset must lie within the oracle's one-step bound
(sum over hidden units of |W3| times the step, through W2 for the first
layer) plus 1e-6 of the largest offset; and all but a small fraction (the
Gaussians that hit such a boundary) agree to 2e-5 of the largest offset,
which a conversion that truncated instead of rounding to nearest even would
fail for most Gaussians. The frame drawn with offsets is then checked
against the oracle frame skinned from the oracle's offset means, stage by
stage, as in the parity tests (the offsets move positions by well under the
2e-3 px screen tolerance when they differ by one rounding step).
"""
import numpy as np
import pytest

from oracle import posenet as opn
from paper_2501_17792_amd import synth

from .gpu_common import run_gpu
from .test_gpu_parity import _compare_frame

pytestmark = pytest.mark.gpu


def _scene(n_inst=8, n_gauss=20000):
    templates = [synth.make_template(t, n_gauss, 3, synth.C2_LEVELS) for t in range(3)]
    crowd = synth.make_crowd(100, n_inst, 3, 12.0, 0.3)
    cam = synth.look_at((6.0, 1.7, -3.0), (6.0, 1.0, 8.0), 480, 270)
    return synth.Scene("c2slice", templates, crowd, cam, lod_thresholds=(6.0, 11.0))


def _net_and_embeds(sc):
    net = synth.pose_net_weights()
    embeds = [synth.pose_embeddings(1200 + t, tpl.n) for t, tpl in enumerate(sc.templates)]
    return net, embeds


def test_offsets_match_oracle():
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _scene()
    net, embeds = _net_and_embeds(sc)
    r, _ = run_gpu(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, setup=lambda rr: rr.upload_pose_net(net, embeds))
    n = int(r.last_stats.n_splats)
    got = r.debug("OFFSETS", np.float32, 4 * n).reshape(n, 4)
    off = r.debug("OFFSET", np.uint32, sc.crowd.n + 1).astype(np.int64)
    ref, bound = [], []
    for i in range(sc.crowd.n):
        t = int(sc.crowd.tid[i])
        k = off[i + 1] - off[i]
        d, b = opn.forward(net, embeds[t][:k], sc.crowd.pose[i], with_bound=True)
        ref.append(d)
        bound.append(b)
    ref, bound = np.concatenate(ref), np.concatenate(bound)
    assert got.shape[0] == ref.shape[0]
    assert np.all(got[:, 3] == 0)
    err = np.abs(got[:, :3] - ref)
    scale = np.abs(ref).max()
    assert 1e-3 < scale < 0.2, scale  # offsets of about a centimetre
    assert np.all(err <= bound + 1e-6 * scale), (err - bound).max()
    tight = np.all(err <= 2e-5 * scale, axis=1)
    print(f"offsets: {n} Gaussians, max err {err.max():.3e} (scale {scale:.3e}), "
          f"{int((~tight).sum())} beyond 2e-5 of the scale")
    assert tight.mean() >= 0.98


def test_frame_with_offsets_matches_oracle():
    from paper_2501_17792_amd import crowdsplat as cs

    sc = _scene()
    net, embeds = _net_and_embeds(sc)

    def mean_fn(i, n):
        t = sc.templates[int(sc.crowd.tid[i])]
        return opn.offset_template(t, embeds[int(sc.crowd.tid[i])], net, sc.crowd.pose[i], n)

    for fuse in (False, True):
        _, img, rec, g, info = _compare_frame(sc, cs.CS_LOD_FIXED, sc.lod_thresholds, fuse=fuse,
                                              setup=lambda rr: rr.upload_pose_net(net, embeds), mean_fn=mean_fn)
        print("offsets frame", "fused" if fuse else "unfused", info)


def test_offsets_move_the_frame_and_can_be_removed():
    """With the network the image differs from the plain frame; removing it
    gives the plain frame back bit for bit; the backward is refused while it
    is set."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    sc = _scene(n_inst=4)
    net, embeds = _net_and_embeds(sc)
    r = cs.Renderer(0, fuse=True)
    r.upload_templates(sc.templates)
    r.set_crowd(sc.crowd)
    plain = r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds).cpu().numpy()
    r.upload_pose_net(net, embeds)
    moved = r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds).cpu().numpy()
    assert np.abs(moved - plain).max() > 1e-3
    with pytest.raises(cs.CrowdSplatError) as e:
        r.render_backward(torch.ones((3, sc.camera.height, sc.camera.width), device="cuda"))
    assert e.value.code == cs.CS_ERR_UNSUPPORTED
    r.upload_pose_net(None, None)
    again = r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds).cpu().numpy()
    assert np.array_equal(again, plain)
    r.close()


def test_captured_frame_with_offsets_equals_eager():
    """The whole frame with the offset network captured as a graph: every
    replay (with unrelated eager work in between) gives the eager frame's
    image and offsets bit for bit. A captured frame launches the offset
    kernel over the chunk capacity (here several times the frame's chunks);
    the workgroups past the frame's chunks must leave without effect."""
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    sc = _scene()
    net, embeds = _net_and_embeds(sc)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        r = cs.Renderer(0, stream=stream, fuse=True)
        r.upload_templates(sc.templates)
        r.set_crowd(sc.crowd)
        r.upload_pose_net(net, embeds)
        ref = r.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds, stats=True).clone()
        n = int(r.last_stats.n_splats)
        stream.synchronize()
        off_ref = r.debug("OFFSETS", np.float32, 4 * n)
        other = cs.Renderer(0, stream=stream)
        other.upload_templates(sc.templates)
        other.set_crowd(sc.crowd)
        out = torch.zeros_like(ref)
        r.capture(sc.camera, out, cs.CS_LOD_FIXED, sc.lod_thresholds)
        for k in range(3):
            out.zero_()
            r.launch()
            assert r.poll().overflow == 0
            stream.synchronize()
            assert torch.equal(out, ref), k
            assert np.array_equal(r.debug("OFFSETS", np.float32, 4 * n), off_ref), k
            other.frame(sc.camera, cs.CS_LOD_FIXED, sc.lod_thresholds)  # unrelated eager work
        stream.synchronize()
        other.close()
        r.close()
