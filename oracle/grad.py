"""FP64 analytic backward of the renderer (oracle) and the fit loss.

The reconstruction stage of CrowdSplat (§2, Fig. 2 stage 1, following
GaussianAvatar) fits a template's Gaussian attributes by gradient descent
through the 3DGS renderer. This module differentiates the forward of
``splat``/``skinning`` with every discrete decision held fixed (culls, tile
rects, sort order, skipped contributions, the stopping splat, the 0.99 clamp
and the exponent clamp), with respect to the template attributes: canonical
means, log-scales, quaternions (before normalisation), opacity logits and SH
coefficients, summed over all instances of the template.

Compositing: with S_i the colour accumulated behind splat i (later
contributions plus T_final * background), d pixel / d alpha_i =
c_i T_i - S_i / (1 - alpha_i) and d pixel / d c_i = alpha_i T_i.

The fit loss is L1 + 0.2 (1 - SSIM), SSIM with an 11x11 Gaussian window
(sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, zero padding, per channel, averaged.
"""
from __future__ import annotations

import math

import numpy as np

from . import skinning, splat

SQ = {  # real SH constants, as in splat.sh_basis
    "c0": 0.5 * math.sqrt(1.0 / math.pi), "c1": math.sqrt(3.0 / (4.0 * math.pi)),
    "c2a": 0.5 * math.sqrt(15.0 / math.pi), "c2b": 0.25 * math.sqrt(5.0 / math.pi),
    "c2c": 0.25 * math.sqrt(15.0 / math.pi), "c3a": 0.25 * math.sqrt(35.0 / (2.0 * math.pi)),
    "c3b": 0.5 * math.sqrt(105.0 / math.pi), "c3c": 0.25 * math.sqrt(21.0 / (2.0 * math.pi)),
    "c3d": 0.25 * math.sqrt(7.0 / math.pi), "c3e": 0.25 * math.sqrt(105.0 / math.pi),
}


def sh_gradient(d, degree):
    """d Y_k / d (x, y, z) of the polynomial forms in splat.sh_basis: [N,K,3]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    n = d.shape[0]
    K = (degree + 1) ** 2
    G = np.zeros((n, K, 3))
    c = SQ
    if degree >= 1:
        G[:, 1, 1] = c["c1"]
        G[:, 2, 2] = c["c1"]
        G[:, 3, 0] = c["c1"]
    if degree >= 2:
        G[:, 4] = np.stack([c["c2a"] * y, c["c2a"] * x, 0 * x], 1)
        G[:, 5] = np.stack([0 * x, c["c2a"] * z, c["c2a"] * y], 1)
        G[:, 6] = np.stack([0 * x, 0 * x, 6 * c["c2b"] * z], 1)
        G[:, 7] = np.stack([c["c2a"] * z, 0 * x, c["c2a"] * x], 1)
        G[:, 8] = np.stack([2 * c["c2c"] * x, -2 * c["c2c"] * y, 0 * x], 1)
    if degree >= 3:
        G[:, 9] = np.stack([6 * c["c3a"] * x * y, c["c3a"] * (3 * x * x - 3 * y * y), 0 * x], 1)
        G[:, 10] = np.stack([c["c3b"] * y * z, c["c3b"] * x * z, c["c3b"] * x * y], 1)
        G[:, 11] = np.stack([0 * x, c["c3c"] * (5 * z * z - 1), 10 * c["c3c"] * y * z], 1)
        G[:, 12] = np.stack([0 * x, 0 * x, c["c3d"] * (15 * z * z - 3)], 1)
        G[:, 13] = np.stack([c["c3c"] * (5 * z * z - 1), 0 * x, 10 * c["c3c"] * x * z], 1)
        G[:, 14] = np.stack([2 * c["c3e"] * x * z, -2 * c["c3e"] * y * z, c["c3e"] * (x * x - y * y)], 1)
        G[:, 15] = np.stack([c["c3a"] * (3 * x * x - 3 * y * y), -6 * c["c3a"] * x * y, 0 * x], 1)
    return G


def quat_rot_jacobian(qn):
    """d R_ij / d (w, x, y, z) of the unit-quaternion rotation: [N,3,3,4]."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    o = 0 * w
    J = np.zeros(qn.shape[:1] + (3, 3, 4))
    J[:, 0, 0] = np.stack([o, o, -4 * y, -4 * z], 1)
    J[:, 0, 1] = np.stack([-2 * z, 2 * y, 2 * x, -2 * w], 1)
    J[:, 0, 2] = np.stack([2 * y, 2 * z, 2 * w, 2 * x], 1)
    J[:, 1, 0] = np.stack([2 * z, 2 * y, 2 * x, 2 * w], 1)
    J[:, 1, 1] = np.stack([o, -4 * x, o, -4 * z], 1)
    J[:, 1, 2] = np.stack([-2 * x, -2 * w, 2 * z, 2 * y], 1)
    J[:, 2, 0] = np.stack([-2 * y, 2 * z, -2 * w, 2 * x], 1)
    J[:, 2, 1] = np.stack([2 * x, 2 * w, 2 * z, 2 * y], 1)
    J[:, 2, 2] = np.stack([o, -4 * x, -4 * y, o], 1)
    return J


# ----------------------------------------------------------------------------
# forward with the cache the backward needs
# ----------------------------------------------------------------------------

def forward(templates, crowd, levels, cam, tw=16, th=16):
    """Whole-frame forward (as oracle.frame) keeping per-splat intermediates."""
    parts, per = [], []
    for i in range(crowd.n):
        t = templates[int(crowd.tid[i])]
        n = int(t.level_count[int(levels[i])])
        mu, cov, L, B = skinning.skin_instance(t, crowd.pose[i], crowd.yaw[i], crowd.pos[i, 0],
                                               crowd.pos[i, 1], n)
        rec = splat.splat_records(mu, cov, L, t.opacity[:n], t.sh[:n], t.sh_degree, cam, tw, th)
        rec["mu"] = mu
        rec["cov"] = cov
        rec["L"] = L
        rec["sh"] = np.asarray(t.sh[:n], np.float64)
        rec["deg"] = np.full(n, t.sh_degree)
        parts.append(rec)
        per.append((int(crowd.tid[i]), n))
    rec = splat.concat_records(parts)
    out = splat.render_records(rec, cam, tw, th)
    out["records"] = rec
    out["per_instance"] = per
    return out


# ----------------------------------------------------------------------------
# backward
# ----------------------------------------------------------------------------

def composite_backward(rec, sorted_vals, ranges, cam, tw, th, dimg):
    """dL/d (u, v, A, B, C, opacity, rgb) per splat from dL/d image [3,H,W]."""
    n = rec["u"].shape[0]
    g = {k: np.zeros(n) for k in ("u", "v", "A", "B", "C", "o")}
    g["rgb"] = np.zeros((n, 3))
    ntx = (cam.width + tw - 1) // tw
    bg = np.asarray(cam.bg, np.float64)
    for t in range(ranges.shape[0]):
        s0, s1 = ranges[t]
        if s1 <= s0:
            continue
        ty, tx = divmod(t, ntx)
        x0, y0 = tx * tw, ty * th
        x1, y1 = min(x0 + tw, cam.width), min(y0 + th, cam.height)
        gy, gx = np.mgrid[y0:y1, x0:x1]
        cx = gx.ravel() + 0.5
        cy = gy.ravel() + 0.5
        P = cx.shape[0]
        dpix = dimg[:, y0:y1, x0:x1].reshape(3, P)
        lst = sorted_vals[s0:s1]
        # forward, recording each pair's alpha, T before it, and whether it was added
        T = np.ones(P)
        done = np.zeros(P, bool)
        rec_a, rec_T, rec_add, rec_cl = [], [], [], []
        for s in lst:
            dx = cx - rec["u"][s]
            dy = cy - rec["v"][s]
            praw = -0.5 * (rec["A"][s] * dx * dx + 2 * rec["B"][s] * dx * dy + rec["C"][s] * dy * dy)
            p = np.minimum(0.0, praw)
            raw = rec["opacity"][s] * np.exp(p)
            a = np.minimum(splat.ALPHA_MAX, raw)
            use = ~done & (a >= splat.ALPHA_MIN)
            Tn = T * (1 - a)
            stop = use & (Tn < splat.T_MIN)
            done |= stop
            add = use & ~stop
            rec_a.append(a)
            rec_T.append(T.copy())
            rec_add.append(add)
            rec_cl.append((raw > splat.ALPHA_MAX, praw > 0, p))
            T = np.where(add, Tn, T)
        # backward, back to front: S = colour accumulated behind the current pair
        S = T[None, :] * bg[:, None]
        for k in range(len(lst) - 1, -1, -1):
            s = lst[k]
            add = rec_add[k]
            if not add.any():
                continue
            a, Tk = rec_a[k], rec_T[k]
            c = rec["rgb"][s]
            g["rgb"][s] += (dpix * (a * Tk * add)[None, :]).sum(1)
            dL_da = ((dpix * (c[:, None] * Tk[None, :] - S / (1 - a)[None, :])).sum(0)) * add
            S = S + np.where(add[None, :], c[:, None] * (a * Tk)[None, :], 0.0)
            clamped, pclamp, p = rec_cl[k]
            live = add & ~clamped
            g["o"][s] += (dL_da * np.exp(p) * live).sum()
            dL_dp = dL_da * a * live * ~pclamp
            dx = cx - rec["u"][s]
            dy = cy - rec["v"][s]
            g["A"][s] += (dL_dp * -0.5 * dx * dx).sum()
            g["B"][s] += (dL_dp * -dx * dy).sum()
            g["C"][s] += (dL_dp * -0.5 * dy * dy).sum()
            g["u"][s] += (dL_dp * (rec["A"][s] * dx + rec["B"][s] * dy)).sum()
            g["v"][s] += (dL_dp * (rec["B"][s] * dx + rec["C"][s] * dy)).sum()
    return g


def projection_backward(rec, gsp, cam):
    """dL/d mu' [N,3], dL/d Sigma' [N,3,3], dL/d sh [N,K,3] per splat."""
    n = rec["u"].shape[0]
    vis = rec["visible"]
    R = np.asarray(cam.R, np.float64)
    eye = np.asarray(cam.eye, np.float64)
    mu, cov, L = rec["mu"], rec["cov"], rec["L"]
    t = (mu - eye) @ R.T
    tx, ty, tz = t[:, 0], t[:, 1], np.where(vis, t[:, 2], 1.0)
    fx, fy = cam.fx, cam.fy
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = fx / tz
    J[:, 0, 2] = -fx * tx / tz ** 2
    J[:, 1, 1] = fy / tz
    J[:, 1, 2] = -fy * ty / tz ** 2
    T = J @ R
    # conic -> 2D covariance
    Q = np.stack([np.stack([rec["A"], rec["B"]], -1), np.stack([rec["B"], rec["C"]], -1)], -2)
    G = np.stack([np.stack([gsp["A"], 0.5 * gsp["B"]], -1), np.stack([0.5 * gsp["B"], gsp["C"]], -1)], -2)
    dS = -Q @ G @ Q
    G2 = np.stack([np.stack([dS[:, 0, 0], dS[:, 0, 1]], -1), np.stack([dS[:, 1, 0], dS[:, 1, 1]], -1)], -2)
    g_cov = np.transpose(T, (0, 2, 1)) @ G2 @ T
    gT = 2.0 * G2 @ T @ cov
    gJ = gT @ R.T
    gt = np.zeros((n, 3))
    gt[:, 0] = gJ[:, 0, 2] * (-fx / tz ** 2) + gsp["u"] * fx / tz
    gt[:, 1] = gJ[:, 1, 2] * (-fy / tz ** 2) + gsp["v"] * fy / tz
    gt[:, 2] = (gJ[:, 0, 0] * (-fx / tz ** 2) + gJ[:, 0, 2] * (2 * fx * tx / tz ** 3)
                + gJ[:, 1, 1] * (-fy / tz ** 2) + gJ[:, 1, 2] * (2 * fy * ty / tz ** 3)
                - gsp["u"] * fx * tx / tz ** 2 - gsp["v"] * fy * ty / tz ** 2)
    g_mu = gt @ R
    # colour
    deg = int(rec["deg"][0]) if n else 0
    K = (deg + 1) ** 2
    w = np.einsum("nji,nj->ni", L, mu - eye)
    wn = np.linalg.norm(w, axis=1, keepdims=True)
    d = w / wn
    Y = splat.sh_basis(d, deg)
    sh = rec["sh"][:, :K, :]
    raw = 0.5 + np.einsum("nk,nkc->nc", Y, sh)
    grgb = gsp["rgb"] * (raw > 0)
    g_sh = Y[:, :, None] * grgb[:, None, :]
    dY = sh_gradient(d, deg)
    gd = np.einsum("nkc,nc,nkx->nx", sh, grgb, dY)
    gw = (gd - d * (d * gd).sum(1, keepdims=True)) / wn
    g_mu = g_mu + np.einsum("nij,nj->ni", L, gw)
    z = ~vis
    g_mu[z] = 0
    g_cov[z] = 0
    g_sh[z] = 0
    return g_mu, g_cov, g_sh


def template_backward(template, n, L, g_mu, g_cov, g_sh, g_o):
    """Chain one instance's per-Gaussian gradients to the template attributes
    of its first n Gaussians."""
    gmean = np.einsum("nji,nj->ni", L, g_mu)
    gS = np.einsum("nji,njk,nkl->nil", L, g_cov, L)
    gS = 0.5 * (gS + np.transpose(gS, (0, 2, 1)))
    q = np.asarray(template.quat[:n], np.float64)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    R = skinning.quat_to_rot(qn)
    es = np.exp(np.asarray(template.log_scale[:n], np.float64))
    M = R * es[:, None, :]
    gM = 2.0 * gS @ M
    gls = np.einsum("nij,nij->nj", R, gM) * es
    gR = gM * es[:, None, :]
    gqn = np.einsum("nij,nijk->nk", gR, quat_rot_jacobian(qn))
    gq = (gqn - qn * (qn * gqn).sum(1, keepdims=True)) / np.linalg.norm(q, axis=1, keepdims=True)
    o = np.asarray(template.opacity[:n], np.float64)
    glogit = g_o * o * (1 - o)
    return dict(mean=gmean, log_scale=gls, quat=gq, opacity_logit=glogit, sh=g_sh)


def backward(templates, crowd, levels, cam, out, dimg, tw=16, th=16):
    """Gradients of sum(dimg * image) w.r.t. every template's attributes."""
    rec = out["records"]
    gsp = composite_backward(rec, out["sorted_vals"], out["ranges"], cam, tw, th, np.asarray(dimg, np.float64))
    g_mu, g_cov, g_sh = projection_backward(rec, gsp, cam)
    grads = {}
    for tid, t in enumerate(templates):
        K = (t.sh_degree + 1) ** 2
        grads[tid] = dict(mean=np.zeros((t.n, 3)), log_scale=np.zeros((t.n, 3)), quat=np.zeros((t.n, 4)),
                          opacity_logit=np.zeros(t.n), sh=np.zeros((t.n, K, 3)))
    off = 0
    for (tid, n) in out["per_instance"]:
        sl = slice(off, off + n)
        g = template_backward(templates[tid], n, rec["L"][sl], g_mu[sl], g_cov[sl], g_sh[sl], gsp["o"][sl])
        for k, v in g.items():
            grads[tid][k][:n] += v
        off += n
    return grads, gsp


# ----------------------------------------------------------------------------
# fit loss
# ----------------------------------------------------------------------------

def gaussian_window(size=11, sigma=1.5):
    x = np.arange(size) - size // 2
    g = np.exp(-x * x / (2 * sigma * sigma))
    return g / g.sum()


def _filter(img, w):
    """Separable zero-padded 'same' filtering of [C,H,W]."""
    r = len(w) // 2
    C, H, W = img.shape
    pad = np.zeros((C, H + 2 * r, W + 2 * r))
    pad[:, r:r + H, r:r + W] = img
    tmp = sum(w[k] * pad[:, :, k:k + W] for k in range(len(w)))
    return sum(w[k] * tmp[:, k:k + H, :] for k in range(len(w)))


def ssim_map(x, y, c1=0.01 ** 2, c2=0.03 ** 2):
    w = gaussian_window()
    mx, my = _filter(x, w), _filter(y, w)
    sxx = _filter(x * x, w) - mx * mx
    syy = _filter(y * y, w) - my * my
    sxy = _filter(x * y, w) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(x, y, c1=0.01 ** 2, c2=0.03 ** 2):
    return float(ssim_map(x, y, c1, c2).mean())


def fit_loss(x, y, lam=0.2):
    """L1 + lam * (1 - SSIM) of render x against target y ([3,H,W])."""
    return float(np.mean(np.abs(x - y))) + lam * (1.0 - ssim(x, y))
