"""Pins of the learned-LoD oracle: bfloat16 rounding against torch, the MLP
gradient against central finite differences, Adam's closed-form first step,
the selection rule, the view box and features in closed-form set-ups."""
import math

import numpy as np
import pytest

from oracle import lod
from paper_2501_17792_amd import synth


def test_bf16_rounding_matches_torch():
    import torch

    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.normal(0, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, -3.0e-5]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(lod.bf16(x), ref)


def _params(rng):
    return dict(W1=rng.normal(0, 0.3, (32, 64)), b1=rng.normal(0, 0.1, 64),
                W2=rng.normal(0, 0.2, (64, 64)), b2=rng.normal(0, 0.1, 64),
                W3=rng.normal(0, 0.2, (64, 5)), b3=rng.normal(0, 0.1, 5),
                mu=rng.normal(0, 1, 32), sd=rng.uniform(0.5, 2.0, 32))


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(rng)
    x = rng.normal(0, 1, (16, 32))
    t = rng.normal(40, 5, (16, 5))
    loss, g = lod.mlp_loss_grad(p, x, t, rounded=False)
    h = 1e-6
    for name in ["W1", "b1", "W2", "b2", "W3", "b3"]:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = lod.mlp_loss_grad(p, x, t, rounded=False)
            flat[idx] = old - h
            lm, _ = lod.mlp_loss_grad(p, x, t, rounded=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_mlp_forward_is_the_layered_definition():
    rng = np.random.default_rng(2)
    p = _params(rng)
    x = rng.normal(0, 1, (4, 32))
    y, _ = lod.mlp_forward(p, x, rounded=False)
    z = (x - p["mu"]) / p["sd"]
    ref = np.zeros((4, 5))
    for b in range(4):  # plain loops over the units
        h1 = [max(0.0, sum(z[b, i] * p["W1"][i, j] for i in range(32)) + p["b1"][j]) for j in range(64)]
        h2 = [max(0.0, sum(h1[i] * p["W2"][i, j] for i in range(64)) + p["b2"][j]) for j in range(64)]
        ref[b] = [sum(h2[i] * p["W3"][i, k] for i in range(64)) + p["b3"][k] for k in range(5)]
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-9, 0.0])
    w = np.ones(4)
    w1, m, v = lod.adam_step(w, g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    np.testing.assert_allclose(w1, 1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_select_levels():
    pred = np.array([[60, 45, 41.5, 39, 30], [60, 40.9, 30, 20, 10], [60, 20, 20, 20, 42],
                     [10, 10, 10, 10, 10]])
    np.testing.assert_array_equal(lod.select_levels(pred, 40, 1), [2, 0, 4, 0])


def test_view_box_single_joint_closed_form():
    cam = synth.Camera(width=100, height=80, fx=50.0, fy=50.0, cx=50.0, cy=40.0,
                       eye=np.zeros(3, np.float32), R=np.eye(3, dtype=np.float32))
    box, clip = lod.view_box(np.array([[0.2, -0.1, 2.0]]), 0.4, cam)
    u, v, r = 50 * 0.1 + 50, 50 * -0.05 + 40, 50 * 0.4 / 2
    np.testing.assert_allclose(box, [u - r, v - r, u + r, v + r])
    np.testing.assert_allclose(clip, [u - r, v - r, u + r, v + r])
    box, clip = lod.view_box(np.array([[0.0, 0.0, -1.0]]), 0.4, cam)
    assert box is None
    assert lod.crop_window(np.array([3.5, 0.0, 17.2, 9.0]), 8, 8, 100, 80) == (0, 0, 24, 16)
    assert lod.crop_window(np.array([95.0, 70.0, 100.0, 80.0]), 16, 16, 100, 80) == (80, 64, 100, 80)


def test_features_closed_forms():
    t = synth.make_template(0, 512, 0)
    cam = synth.look_at((0.0, 1.7, -3.0), (0.0, 1.0, 10.0), 320, 180)
    pose = np.zeros((24, 3))
    basis = np.eye(72)[:8]
    # facing the camera: +z after R_y(pi) points to -z, towards the eye
    f = lod.instance_features(t, 3, 14, pose, math.pi, 0.0, 7.0, 0.3, cam, np.zeros(72), basis)
    np.testing.assert_allclose(f[0], math.sqrt(10 ** 2 + 1.7 ** 2))
    np.testing.assert_allclose(f[24], math.log(f[0]))
    np.testing.assert_allclose([f[28], f[29]], [1.0, 0.0], atol=1e-12)
    assert f[13] == 1.0 and f[10:24].sum() == 1.0
    assert 0 < f[1] < 1 and f[30] == 1.0 and f[31] == 0.0
    np.testing.assert_allclose(f[25], math.log(f[1] + 1e-6))
    # facing away, offset to the side: relative yaw turns
    f2 = lod.instance_features(t, 3, 14, pose, 0.0, 3.0, 7.0, 0.3, cam, np.zeros(72), basis)
    to_cam = np.array([-3.0, -10.0]) / math.hypot(3, 10)
    np.testing.assert_allclose([f2[28], f2[29]], [to_cam[1], to_cam[0]], atol=1e-12)
    # PCA coordinates are the projection on the basis
    pose3 = np.random.default_rng(3).normal(0, 0.3, (24, 3))
    f3 = lod.instance_features(t, 0, 14, pose3, 0.0, 0.0, 7.0, 0.3, cam, np.zeros(72), basis)
    np.testing.assert_allclose(f3[2:10], pose3.reshape(-1)[:8])


def test_psnr_labels_known_mse():
    a = np.zeros((3, 4, 4))
    b = a.copy()
    b[:, 1:3, 1:3] = 0.1  # MSE over the 4x4 window = 0.01 * 4/16
    lab = lod.psnr_labels([a, b, a], (0, 0, 4, 4))
    np.testing.assert_allclose(lab, [60.0, -10 * math.log10(0.0025), 60.0])


def _one_joint_template(means, log_scales):
    """A template whose 24 joints all sit at the origin except joint 1 at
    (0, 2, 0), holding the given Gaussians."""
    n = len(means)
    J = np.zeros((24, 3), np.float32)
    J[1] = (0.0, 2.0, 0.0)
    return synth.Template(
        mean=np.asarray(means, np.float32), log_scale=np.asarray(log_scales, np.float32),
        quat=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), opacity=np.full(n, 0.5, np.float32),
        sh=np.zeros((n, 1, 3), np.float32), skin_idx=np.zeros((n, 4), np.uint8),
        skin_w=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), joints_rest=J,
        parents=np.array([-1] + [0] * 23, np.int32), sh_degree=0, level_count=np.array([n], np.int32))


def test_pad_radius_closed_form():
    """One Gaussian: its distance to the nearest joint plus 3 times its largest
    standard deviation. Three Gaussians: the largest of their three such sums,
    which here is neither that of the Gaussian farthest from a joint nor that
    of the widest one."""
    t = _one_joint_template([[3.0, 4.0, 0.0]], [[-2.0, -1.0, -3.0]])
    # nearest joint: (0, 2, 0) at sqrt(9 + 4) (the origin is 5 away)
    assert math.isclose(lod.pad_radius(t), math.sqrt(13.0) + 3.0 * math.exp(-1.0), rel_tol=1e-12)
    t = _one_joint_template([[0.0, 2.5, 0.0], [2.0, 0.0, 0.0], [0.0, 0.0, 1.5]],
                            [[0.0, -4.0, -4.0], [-4.0, -4.0, -4.0], [-0.375, -1.5, -3.0]])
    ref = 1.5 + 3.0 * math.exp(-0.375)  # the third: neither the farthest (2.0) nor the widest (e^0)
    assert ref > max(0.5 + 3.0 * math.exp(0.0), 2.0 + 3.0 * math.exp(-4.0))
    assert math.isclose(lod.pad_radius(t), ref, rel_tol=1e-12)


# ---------------------------------------------------------------- frame budget

def test_level_sse_is_the_windows_squared_error_and_adds_up_to_the_frame_psnr():
    """SSE from a label equals the summed squared difference over the label
    window, and for instances whose windows do not overlap the frame's PSNR
    against full detail is 10 log10(3 W H / sum of their SSE)."""
    rng = np.random.default_rng(3)
    W, H = 96, 64
    frame_full = np.zeros((3, H, W))
    frame_lod = np.zeros((3, H, W))
    sse_sum = 0.0
    for (x0, y0, x1, y1), noise in [((0, 0, 32, 32), 0.01), ((48, 16, 96, 64), 0.003)]:
        full = rng.uniform(0, 1, (3, H, W))
        coarse = full + rng.normal(0, noise, full.shape)
        lab = lod.psnr_labels([full, coarse], (x0, y0, x1, y1))
        pred = np.array([[lab[0], lab[1], 0, 0, 0]])
        s = lod.level_sse(pred, [(x1 - x0) * (y1 - y0)], np.array([1]))
        want = ((coarse - full)[:, y0:y1, x0:x1] ** 2).sum()
        np.testing.assert_allclose(s[0, 1], want, rtol=1e-12)
        assert s[0, 0] == 0 and np.all(s[0, 2:] == 0)  # level 0 and levels above the top
        frame_full[:, y0:y1, x0:x1] = full[:, y0:y1, x0:x1]
        frame_lod[:, y0:y1, x0:x1] = coarse[:, y0:y1, x0:x1]
        sse_sum += s[0, 1]
    psnr = -10 * math.log10(np.mean((frame_lod - frame_full) ** 2))
    np.testing.assert_allclose(psnr, 10 * math.log10(3 * W * H / sse_sum), rtol=1e-12)
    np.testing.assert_allclose(lod.frame_budget(W, H, psnr), sse_sum, rtol=1e-12)


def test_label_window_is_whole_16_tiles():
    assert lod.label_window_px(np.array([5.0, 3.0, 17.5, 30.0]), 100, 40) == 32 * 32
    assert lod.label_window_px(np.array([90.0, 30.0, 100.0, 40.0]), 100, 40) == (100 - 80) * (40 - 16)
    assert lod.label_window_px(None, 100, 40) == 0.0


def _budget_case(seed, n=4, levels=3):
    rng = np.random.default_rng(seed)
    counts = np.tile(np.array([1000.0, 500.0, 250.0, 125.0, 62.5])[None], (n, 1))
    pred = np.zeros((n, 5))
    pred[:, 0] = 60.0
    pred[:, 1:] = np.sort(rng.uniform(15, 60, (n, 4)), axis=1)[:, ::-1]
    win = rng.uniform(50, 5000, n)
    top = np.full(n, levels - 1)
    return lod.level_sse(pred, win, top), counts, top


def test_budget_selection_against_brute_force():
    """On tiny crowds (4 instances, 3 levels, every one of the 81 selections
    enumerated): the result keeps the summed SSE within the budget, no
    selection with at most its SSE draws fewer Gaussians (it minimises
    Gaussians + lambda SSE), and half a bisection step lower lambda is
    infeasible (the smallest such lambda was found)."""
    import itertools

    for seed in range(20):
        sse, counts, top = _budget_case(seed)
        n = sse.shape[0]
        allsel = np.array(list(itertools.product(range(3), repeat=n)))
        tot_sse = sse[np.arange(n)[None], allsel].sum(1)
        tot_n = counts[np.arange(n)[None], allsel].sum(1)
        for budget in np.quantile(tot_sse, [0.05, 0.3, 0.6, 0.95]):
            lv, t = lod.select_budget(sse, counts, top, budget)
            s_res = sse[np.arange(n), lv].sum()
            n_res = counts[np.arange(n), lv].sum()
            assert s_res <= budget
            assert np.all(tot_n[tot_sse <= s_res] >= n_res)
            step = (lod.BUDGET_T_HI - lod.BUDGET_T_LO) / 2 ** lod.BUDGET_ITERS
            lower = lod.choose_levels(sse, counts, top, 2.0 ** (t - step))
            assert t <= lod.BUDGET_T_LO + step or sse[np.arange(n), lower].sum() > budget


def test_budget_selection_limits_and_order():
    sse, counts, top = _budget_case(7, n=6, levels=5)
    lv, _ = lod.select_budget(sse, counts, top, np.inf)
    assert np.all(lv == 4)  # no limit: the coarsest level everywhere
    lv, _ = lod.select_budget(sse, counts, top, 0.0)
    assert np.all(lv == 0)  # no error allowed: full detail
    # an instance with no window (nothing on screen) costs nothing at any level
    sse2 = sse.copy()
    sse2[0] = 0.0
    lv, _ = lod.select_budget(sse2, counts, top, 0.0)
    assert lv[0] == 4 and np.all(lv[1:] == 0)
    # two equal instances except a 100x larger window: the small one coarsens first
    pred = np.array([[60.0, 45.0, 40.0, 35.0, 30.0]] * 2)
    s = lod.level_sse(pred, [100.0, 10000.0], np.array([4, 4]))
    c = np.tile(np.array([1000.0, 500.0, 250.0, 125.0, 62.5])[None], (2, 1))
    for budget in np.geomspace(1e-3, 1e2, 30):
        lv, _ = lod.select_budget(s, c, np.array([4, 4]), budget)
        assert lv[0] >= lv[1]
    # instances without a template draw level 0 and add nothing
    lv, _ = lod.select_budget(sse, counts, top, 0.0, valid=np.array([False] + [True] * 5))
    assert lv[0] == 0


def test_visible_share_scales_the_errors():
    """Seen in its whole window: the errors unchanged; never seen: none (the
    coarsest level is free); seen in a part: scaled by that share; more
    pixels than the window (a larger window earlier): capped at the whole."""
    sse, counts, top = _budget_case(3, n=4, levels=5)
    pred = np.array([[60.0, 45.0, 40.0, 35.0, 30.0]] * 4)
    win = np.array([1000.0, 1000.0, 1000.0, 0.0])
    base = lod.level_sse(pred, win, np.full(4, 4))
    got = lod.level_sse(pred, win, np.full(4, 4), visible_px=np.array([1000.0, 0.0, 250.0, 10.0]))
    np.testing.assert_allclose(got[0], base[0])
    assert np.all(got[1] == 0.0)
    np.testing.assert_allclose(got[2], 0.25 * base[2], rtol=1e-15)
    assert np.all(got[3] == 0.0)
    got = lod.level_sse(pred, win, np.full(4, 4), visible_px=np.array([5000.0, 0, 0, 0]))
    np.testing.assert_allclose(got[0], base[0])
    lv, _ = lod.select_budget(got, counts, top, 0.0)
    assert list(lv) == [0, 4, 4, 4]
