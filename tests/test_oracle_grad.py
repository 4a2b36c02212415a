"""Pins of the analytic FP64 backward: central finite differences of the
whole forward (skin -> project -> composite) on a 64-Gaussian template at
32x32, for every attribute family; entries whose perturbation changes a
discrete decision are detected (the differences at h and h/2 disagree) and
excluded. Plus closed forms of the SSIM loss."""
import dataclasses

import numpy as np
import pytest

from oracle import grad as ograd
from paper_2501_17792_amd import synth


def _setup(seed=0, n=64, size=32):
    t = synth.make_template(seed, n, 3)
    t = dataclasses.replace(t, mean=t.mean.astype(np.float64), log_scale=t.log_scale.astype(np.float64) + 1.2,
                            quat=t.quat.astype(np.float64), opacity=t.opacity.astype(np.float64),
                            sh=t.sh.astype(np.float64), skin_w=t.skin_w.astype(np.float64))
    rng = np.random.default_rng(seed + 1)
    pose = rng.normal(0, 0.2, (1, 24, 3))
    crowd = synth.Crowd(tid=np.zeros(1, np.int32), yaw=np.array([0.3]), pos=np.zeros((1, 2)), pose=pose)
    c = 0.5 * (t.mean.min(0) + t.mean.max(0))
    cam = synth.look_at(c + np.array([0.4, 0.3, -3.2]), c, size, size)
    cam.bg = np.array([0.1, 0.2, 0.3])
    w = rng.normal(0, 1, (3, size, size))
    return t, crowd, cam, w


def _loss(t, crowd, cam, w):
    out = ograd.forward([t], crowd, np.zeros(1, int), cam, 8, 8)
    return float((out["image"] * w).sum())


def _set(t, name, idx, val):
    arr = getattr(t, name).copy()
    arr.reshape(-1)[idx] = val
    return dataclasses.replace(t, **{name: arr})


@pytest.mark.parametrize("name", ["mean", "log_scale", "quat", "opacity_logit", "sh"])
def test_backward_matches_central_differences(name):
    t, crowd, cam, w = _setup()
    out = ograd.forward([t], crowd, np.zeros(1, int), cam, 8, 8)
    grads, _ = ograd.backward([t], crowd, np.zeros(1, int), cam, out, w, 8, 8)
    g = grads[0][name].reshape(-1)
    scale = np.abs(g).max()
    assert scale > 0
    rng = np.random.default_rng(hash(name) % 1000)
    src = "opacity" if name == "opacity_logit" else name
    base = getattr(t, src).reshape(-1)
    checked = 0
    for idx in rng.permutation(base.size)[:60]:
        vals = []
        for h in (1e-4, 5e-5):
            if name == "opacity_logit":
                lg = np.log(base[idx] / (1 - base[idx]))
                lp = _loss(_set(t, src, idx, 1 / (1 + np.exp(-(lg + h)))), crowd, cam, w)
                lm = _loss(_set(t, src, idx, 1 / (1 + np.exp(-(lg - h)))), crowd, cam, w)
            else:
                lp = _loss(_set(t, src, idx, base[idx] + h), crowd, cam, w)
                lm = _loss(_set(t, src, idx, base[idx] - h), crowd, cam, w)
            vals.append((lp - lm) / (2 * h))
        if abs(vals[0] - vals[1]) > 1e-6 * (abs(vals[0]) + scale):
            continue  # a discrete decision changed inside the interval
        assert abs(vals[0] - g[idx]) <= 1e-5 * (abs(vals[0]) + scale), (name, idx, vals[0], g[idx])
        checked += 1
        if checked >= 16:
            break
    assert checked >= 8


def test_ssim_closed_forms():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (3, 20, 24))
    assert abs(ograd.ssim(x, x) - 1.0) < 1e-12
    assert abs(ograd.fit_loss(x, x)) < 1e-12
    w = ograd.gaussian_window()
    np.testing.assert_allclose(w.sum(), 1.0)
    np.testing.assert_allclose(w[5] / w[6], np.exp(1 / (2 * 1.5 ** 2)))
    # constant images away from the zero padding: variances vanish and the map
    # is (2 m1 m2 + C1) / (m1^2 + m2^2 + C1)
    a = np.full((1, 40, 40), 0.3)
    b = np.full((1, 40, 40), 0.6)
    m = ograd.ssim_map(a, b)[0, 5:35, 5:35]
    np.testing.assert_allclose(m, (2 * 0.18 + 1e-4) / (0.09 + 0.36 + 1e-4), rtol=1e-9)
    # a pure offset changes only the luminance term; L1 is the offset
    assert abs(ograd.fit_loss(a + 0.1, a, lam=0.0) - 0.1) < 1e-12
