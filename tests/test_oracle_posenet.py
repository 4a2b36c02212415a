"""Pins of the pose-dependent offset oracle (oracle/posenet.py) against what
the definition fixes: bfloat16 rounding by torch's own conversion, single-path
networks with closed-form outputs, ReLU gating, the pose code's layout and
root invariance, the rounding bound, and skinning of the offset means."""
import numpy as np
import pytest

from oracle import posenet as opn
from oracle import skinning as oskin
from paper_2501_17792_amd import synth


def _zero_net():
    return dict(w1=np.zeros((64, 112), np.float32), b1=np.zeros(64, np.float32),
                w2=np.zeros((64, 64), np.float32), b2=np.zeros(64, np.float32),
                w3=np.zeros((3, 64), np.float32), b3=np.zeros(3, np.float32))


def test_bf16_matches_torch():
    import torch

    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.uniform(-1e-3, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, -2.5, 65504.0]]).astype(np.float32)
    # exact ties: values halfway between two bfloat16 numbers
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(opn.bf16(x), want)


def test_single_path_networks_have_closed_forms():
    """One nonzero weight per layer routes input k through hidden units j and m
    to output c: d_c = max(x_k, 0) * a * b * w (all other outputs 0)."""
    rng = np.random.default_rng(1)
    embed = rng.normal(0, 1, (7, 32)).astype(np.float32)
    pose = rng.normal(0, 0.3, (24, 3)).astype(np.float32)
    x = np.concatenate([embed, np.broadcast_to(opn.pose_code(pose), (7, 80))], axis=1)
    for k, j, m, c in [(0, 5, 9, 0), (31, 63, 0, 2), (32, 1, 17, 1), (100, 40, 63, 2), (111, 0, 1, 0)]:
        net = _zero_net()
        net["w1"][j, k], net["w2"][m, j], net["w3"][c, m] = 2.0, 0.5, -4.0
        d = opn.forward(net, embed, pose, rounded=False)
        want = np.zeros((7, 3))
        want[:, c] = np.maximum(x[:, k].astype(np.float64), 0.0) * 2.0 * 0.5 * -4.0
        np.testing.assert_allclose(d, want, rtol=1e-15, atol=0)


def test_biases_and_relu_gating():
    rng = np.random.default_rng(2)
    embed = rng.normal(0, 1, (5, 32)).astype(np.float32)
    pose = rng.normal(0, 0.3, (24, 3)).astype(np.float32)
    net = _zero_net()
    net["b3"][:] = (0.25, -0.5, 0.125)
    np.testing.assert_array_equal(opn.forward(net, embed, pose), np.tile([0.25, -0.5, 0.125], (5, 1)))
    # every first-layer unit off: only b2 passes (through its ReLU)
    net["w1"][:] = rng.normal(0, 0.01, (64, 112)).astype(np.float32)
    net["b1"][:] = -100.0
    net["b2"][:] = np.linspace(-1, 1, 64).astype(np.float32)
    net["w3"][:] = rng.normal(0, 1, (3, 64)).astype(np.float32)
    w3 = opn.bf16(net["w3"])
    want = w3 @ opn.bf16(np.maximum(net["b2"], 0)) + net["b3"]
    np.testing.assert_allclose(opn.forward(net, embed, pose), np.tile(want, (5, 1)), rtol=1e-14)


def test_pose_code_layout_and_root_invariance():
    rng = np.random.default_rng(3)
    pose = rng.normal(0, 0.3, (24, 3)).astype(np.float32)
    p = opn.pose_code(pose)
    assert p.shape == (80,)
    for j in (1, 7, 23):
        for a in range(3):
            assert p[3 * (j - 1) + a] == pose[j, a]
    assert np.all(p[69:] == 0)
    net = {k: v for k, v in _zero_net().items()}
    net["w1"][:] = rng.normal(0, 0.2, (64, 112)).astype(np.float32)
    net["b1"][:] = 0.1
    net["w2"][:] = rng.normal(0, 0.2, (64, 64)).astype(np.float32)
    net["w3"][:] = rng.normal(0, 0.2, (3, 64)).astype(np.float32)
    embed = rng.normal(0, 1, (9, 32)).astype(np.float32)
    d0 = opn.forward(net, embed, pose)
    p2 = pose.copy()
    p2[0] += (0.7, -0.2, 1.1)  # the root's global orientation: no effect
    np.testing.assert_array_equal(opn.forward(net, embed, p2), d0)
    p3 = pose.copy()
    p3[12, 1] += 0.5  # a body joint: the offsets change
    assert np.abs(opn.forward(net, embed, p3) - d0).max() > 1e-4


def test_rounding_bound_covers_one_step_moves():
    """Moving one hidden value one bfloat16 step changes the output by no more
    than the bound the oracle reports."""
    rng = np.random.default_rng(4)
    net = dict(w1=rng.normal(0, 0.15, (64, 112)).astype(np.float32), b1=rng.normal(0, 0.1, 64).astype(np.float32),
               w2=rng.normal(0, 0.15, (64, 64)).astype(np.float32), b2=rng.normal(0, 0.1, 64).astype(np.float32),
               w3=rng.normal(0, 0.05, (3, 64)).astype(np.float32), b3=np.zeros(3, np.float32))
    embed = rng.normal(0, 1, (50, 32)).astype(np.float32)
    pose = rng.normal(0, 0.3, (24, 3)).astype(np.float32)
    d, bound = opn.forward(net, embed, pose, with_bound=True)
    assert np.all(bound > 0)
    W2, W3 = opn.bf16(net["w2"]), opn.bf16(net["w3"])
    # recompute the hidden values of one Gaussian and nudge each h2 value
    e = opn.bf16(embed[:1])
    x = np.concatenate([e, opn.bf16(opn.pose_code(pose).astype(np.float32))[None]], axis=1)
    h1 = opn.bf16(np.maximum(x @ opn.bf16(net["w1"]).T + net["b1"], 0).astype(np.float32))
    h2 = opn.bf16(np.maximum(h1 @ W2.T + net["b2"], 0).astype(np.float32))
    for j in range(64):
        h = h2.copy()
        h[0, j] += opn._bf16_step(h2[0, j])
        moved = np.abs((h @ W3.T + net["b3"]) - d[:1])
        assert np.all(moved <= bound[:1] * (1 + 1e-12))


def test_offsets_are_skinned_with_the_mean():
    """Identity pose at the origin: the skinned mean is the offset canonical
    mean; all weight on one bone: it moves rigidly with that bone."""
    t = synth.make_template(3, 64, 0)
    rng = np.random.default_rng(5)
    d = rng.normal(0, 0.01, (64, 3))
    B = oskin.bone_matrices(np.zeros((24, 3)), t.joints_rest, t.parents, 0.0, 0.0, 0.0)
    cov = oskin.canonical_covariance(t.log_scale, t.quat)
    mu, _, _ = oskin.lbs(B, t.mean.astype(np.float64) + d, cov, t.skin_idx, t.skin_w)
    np.testing.assert_allclose(mu, t.mean.astype(np.float64) + d, atol=1e-12)
    pose = rng.normal(0, 0.4, (24, 3))
    B = oskin.bone_matrices(pose, t.joints_rest, t.parents, 0.3, 1.0, -2.0)
    idx = np.full((64, 4), 7, np.uint8)
    w = np.tile([1.0, 0.0, 0.0, 0.0], (64, 1)).astype(np.float32)
    mu, _, _ = oskin.lbs(B, t.mean.astype(np.float64) + d, cov, idx, w)
    np.testing.assert_allclose(mu, (t.mean + d) @ B[7][:, :3].T + B[7][:, 3], atol=1e-12)


@pytest.mark.parametrize("n", [1, 33])
def test_offset_template_adds_the_forward(n):
    t = synth.make_template(4, 40, 0)
    rng = np.random.default_rng(6)
    net = dict(w1=rng.normal(0, 0.1, (64, 112)).astype(np.float32), b1=np.zeros(64, np.float32),
               w2=rng.normal(0, 0.1, (64, 64)).astype(np.float32), b2=np.zeros(64, np.float32),
               w3=rng.normal(0, 0.01, (3, 64)).astype(np.float32), b3=np.full(3, 0.001, np.float32))
    emb = rng.normal(0, 1, (40, 32)).astype(np.float32)
    pose = rng.normal(0, 0.3, (24, 3)).astype(np.float32)
    m = opn.offset_template(t, emb, net, pose, n)
    assert m.shape == (n, 3)
    np.testing.assert_array_equal(m - t.mean[:n].astype(np.float64), opn.forward(net, emb[:n], pose))
