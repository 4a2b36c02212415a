"""FP64 oracle of the learned level of detail.

CrowdSplat §2 (last paragraph) picks a template level per character from its
camera distance; §3 (Fig. 4) shows that the quality loss of a coarser level
depends on how large the character appears. The learned rule replaces the
distance thresholds by a small network that predicts, per instance, the PSNR
of every level against the full template, and picks the coarsest level whose
prediction clears a quality floor.

Definitions (readings where the paper is silent):
* view box: the screen rectangle covering every posed joint in front of the
  near plane, each padded by the template's rest pad radius projected at the
  joint's depth (fx * pad / depth); clipped to the image;
* features (31 used of 32): distance, clipped box area / (W H), 8 pose PCA
  coordinates, template one-hot (14), log distance, log(area + 1e-6), box
  centre / (W, H), cos and sin of the instance's facing relative to the
  direction to the camera, and the visible fraction of the box;
* network: z-scored features -> 31x64 -> ReLU -> 64x64 -> ReLU -> 64x5,
  BF16 weights and BF16 layer inputs (round to nearest even), FP32 (here
  FP64) accumulation and biases;
* label: PSNR of each level against level 0 over the instance's crop window
  (the view box widened to whole tiles), rendered alone on black, clamped to
  60 dB;
* selection: the coarsest level whose prediction is at least floor + margin,
  else level 0;
* frame-budget selection (the floor read as one for the whole frame against
  the full-detail frame): a level's predicted PSNR over the instance's label
  window (16x16 tiles, w x h pixels) gives its predicted squared error summed
  over the window's RGB values, SSE_l = 3 w h 10^(-PSNR_l / 10) (PSNR clamped
  to [0, 60], none at level 0); instances take the level minimising
  n_l + lambda SSE_l (ties to the finer level) for the smallest lambda on a
  30-step bisection of log2(lambda) in [-40, 60] whose summed SSE stays within
  3 W H 10^(-floor / 10); each instance's errors scaled by the share of its
  window it was seen in (pixels whose largest contribution it gave) in a
  previous frame, once one exists.
"""
from __future__ import annotations

import math

import numpy as np

from . import skinning

N_FEAT = 32
N_USED = 31
N_LEVELS = 5
PSNR_CAP = 60.0


# ----------------------------------------------------------------------------
# view box, features, crop windows
# ----------------------------------------------------------------------------

def pad_radius(template) -> float:
    """Rest-pose bound of the template around its joints: the largest distance
    from a mean to its nearest joint plus 3 of its largest standard deviations."""
    m = np.asarray(template.mean, np.float64)
    J = np.asarray(template.joints_rest, np.float64)
    d = np.sqrt(((m[:, None, :] - J[None]) ** 2).sum(-1)).min(1)
    smax = np.exp(np.asarray(template.log_scale, np.float64).max(1))
    return float((d + 3.0 * smax).max())


def posed_joints(template, pose, yaw, px, pz) -> np.ndarray:
    """World positions of the 24 posed joints: W G_j applied to the origin."""
    G = skinning.global_transforms(pose, template.joints_rest, template.parents)
    W = skinning.instance_transform(yaw, px, pz)
    return np.array([(W @ G[j])[:3, 3] for j in range(G.shape[0])])


def view_box(joints, pad, cam):
    """(x0, y0, x1, y1) unclipped, the clipped box, and whether any joint is in
    front of the near plane."""
    R = np.asarray(cam.R, np.float64)
    t = (np.asarray(joints, np.float64) - np.asarray(cam.eye, np.float64)) @ R.T
    front = t[:, 2] > cam.near
    if not front.any():
        return None, None
    t = t[front]
    u = cam.fx * t[:, 0] / t[:, 2] + cam.cx
    v = cam.fy * t[:, 1] / t[:, 2] + cam.cy
    ru = cam.fx * pad / t[:, 2]
    rv = cam.fy * pad / t[:, 2]
    box = np.array([np.min(u - ru), np.min(v - rv), np.max(u + ru), np.max(v + rv)])
    clip = np.array([max(box[0], 0.0), max(box[1], 0.0), min(box[2], cam.width),
                     min(box[3], cam.height)])
    return box, clip


def instance_features(template, tid, n_templates, pose, yaw, px, pz, pad, cam,
                      pca_mean, pca_basis) -> np.ndarray:
    f = np.zeros(N_FEAT)
    eye = np.asarray(cam.eye, np.float64)
    dist = math.sqrt((px - eye[0]) ** 2 + eye[1] ** 2 + (pz - eye[2]) ** 2)
    joints = posed_joints(template, pose, yaw, px, pz)
    box, clip = view_box(joints, pad, cam)
    W, H = cam.width, cam.height
    if box is None:
        area = vis = 0.0
        cu = cv = 0.5
    else:
        cw, ch = max(clip[2] - clip[0], 0.0), max(clip[3] - clip[1], 0.0)
        area = cw * ch / (W * H)
        full = (box[2] - box[0]) * (box[3] - box[1])
        vis = cw * ch / full if full > 0 else 0.0
        cu = 0.5 * (box[0] + box[2]) / W
        cv = 0.5 * (box[1] + box[3]) / H
    f[0] = dist
    f[1] = area
    f[2:10] = (np.asarray(pose, np.float64).reshape(-1) - pca_mean) @ np.asarray(pca_basis, np.float64).T
    f[10 + int(tid)] = 1.0
    f[24] = math.log(dist)
    f[25] = math.log(area + 1e-6)
    f[26] = cu
    f[27] = cv
    face = np.array([math.sin(yaw), math.cos(yaw)])          # (x, z) facing of +z after R_y
    to_cam = np.array([eye[0] - px, eye[2] - pz])
    to_cam /= np.linalg.norm(to_cam)
    f[28] = face @ to_cam
    f[29] = face[1] * to_cam[0] - face[0] * to_cam[1]
    f[30] = vis
    return f


def crop_window(clip, tw, th, width, height):
    """Whole-tile window (x0, y0, x1, y1) in pixels around a clipped box, or
    None if the box is empty."""
    if clip is None or clip[2] <= clip[0] or clip[3] <= clip[1]:
        return None
    tx = (width + tw - 1) // tw
    ty = (height + th - 1) // th
    x0 = int(math.floor(clip[0] / tw))
    y0 = int(math.floor(clip[1] / th))
    x1 = min(int(math.ceil(clip[2] / tw)), tx)
    y1 = min(int(math.ceil(clip[3] / th)), ty)
    if x1 <= x0 or y1 <= y0:
        return None
    return (x0 * tw, y0 * th, min(x1 * tw, width), min(y1 * th, height))


def psnr_labels(images, window) -> np.ndarray:
    """PSNR of each level's render against level 0 over the window, on [0,1]
    colours, clamped to 60 dB."""
    x0, y0, x1, y1 = window
    ref = images[0][:, y0:y1, x0:x1]
    out = np.zeros(len(images))
    for l, im in enumerate(images):
        mse = float(np.mean((im[:, y0:y1, x0:x1] - ref) ** 2))
        out[l] = PSNR_CAP if mse <= 10 ** (-PSNR_CAP / 10) else min(PSNR_CAP, -10 * math.log10(mse))
    return out


# ----------------------------------------------------------------------------
# the network
# ----------------------------------------------------------------------------

def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) and return as float64."""
    a = np.asarray(x, np.float64).astype(np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def mlp_forward(params, x, rounded=True):
    """x [B,32] raw features -> (y [B,5], cache). params: W1 [32,64], b1,
    W2 [64,64], b2, W3 [64,5], b3, mu [32], sd [32]."""
    q = bf16 if rounded else (lambda v: np.asarray(v, np.float64))
    z = (np.asarray(x, np.float64) - params["mu"]) / params["sd"]
    a0 = q(z)
    h1 = np.maximum(a0 @ q(params["W1"]) + params["b1"], 0.0)
    a1 = q(h1)
    h2 = np.maximum(a1 @ q(params["W2"]) + params["b2"], 0.0)
    a2 = q(h2)
    y = a2 @ q(params["W3"]) + params["b3"]
    return y, dict(a0=a0, h1=h1, a1=a1, h2=h2, a2=a2)


def mlp_loss_grad(params, x, target, rounded=True):
    """Mean squared error over the batch and the 5 outputs, and its gradient
    with respect to W1, b1, W2, b2, W3, b3. In the rounded network the
    backward's matrix-core inputs dY, dH2 and dH1 are bfloat16 too, and each
    rounding counts as the identity in the derivative."""
    q = bf16 if rounded else (lambda v: np.asarray(v, np.float64))
    y, c = mlp_forward(params, x, rounded)
    B, L = y.shape
    r = y - target
    loss = float(np.mean(r * r))
    dy = q(2.0 * r / (B * L))
    g = {}
    g["W3"] = c["a2"].T @ dy
    g["b3"] = dy.sum(0)
    dh2 = q((dy @ q(params["W3"]).T) * (c["h2"] > 0))
    g["W2"] = c["a1"].T @ dh2
    g["b2"] = dh2.sum(0)
    dh1 = q((dh2 @ q(params["W2"]).T) * (c["h1"] > 0))
    g["W1"] = c["a0"].T @ dh1
    g["b1"] = dh1.sum(0)
    return loss, g


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def select_levels(pred, floor=40.0, margin=1.0) -> np.ndarray:
    """Coarsest level whose predicted PSNR is >= floor + margin, else 0."""
    pred = np.asarray(pred, np.float64)
    ok = pred >= floor + margin
    ok[:, 0] = True
    L = pred.shape[1]
    return (L - 1) - np.argmax(ok[:, ::-1], axis=1)


# ----------------------------------------------------------------------------
# frame-budget selection
# ----------------------------------------------------------------------------

LABEL_TILE = 16
BUDGET_ITERS = 30
BUDGET_T_LO, BUDGET_T_HI = -40.0, 60.0


def label_window_px(clip, width, height) -> float:
    """Pixels of the label window: the clipped view box widened to whole
    16x16 tiles (the tiles the labels were rendered with), clipped to the
    image; 0 if the box is empty."""
    win = crop_window(clip, LABEL_TILE, LABEL_TILE, width, height)
    if win is None:
        return 0.0
    return float((win[2] - win[0]) * (win[3] - win[1]))


def level_sse(pred, window_px, top, visible_px=None) -> np.ndarray:
    """[n, 5] predicted squared error of each level summed over the window's
    RGB values: the PSNR over the window is 10 log10(1 / MSE) with MSE the
    mean over its 3 w h values, so SSE = 3 w h 10^(-PSNR / 10); level 0 and
    levels above the template's top have none. With ``visible_px`` (pixels
    the instance was seen in, in a previous frame of the crowd) the error is
    scaled by the visible share of its window, min(1, visible / (w h)): the
    label measures the avatar alone, and in the crowd only its visible
    pixels can show its error."""
    pred = np.clip(np.asarray(pred, np.float64)[:, :N_LEVELS], 0.0, PSNR_CAP)
    win = np.asarray(window_px, np.float64)
    sse = 3.0 * win[:, None] * 10.0 ** (-pred / 10.0)
    if visible_px is not None:
        vis = np.asarray(visible_px, np.float64)
        share = np.where(win > 0, np.minimum(1.0, vis / np.where(win > 0, win, 1.0)), 0.0)
        sse = sse * share[:, None]
    lv = np.arange(N_LEVELS)[None, :]
    sse[(lv == 0) | (lv > np.asarray(top)[:, None])] = 0.0
    return sse


def frame_budget(width, height, floor_db) -> float:
    """Summed squared error over the frame's 3 W H values at PSNR = floor."""
    return 3.0 * width * height * 10.0 ** (-floor_db / 10.0)


def choose_levels(sse, counts, top, lam) -> np.ndarray:
    """argmin over l <= top of counts[l] + lam sse[l], the first (finest) of
    equal costs."""
    cost = np.asarray(counts, np.float64) + lam * sse
    lv = np.arange(N_LEVELS)[None, :]
    cost = np.where(lv <= np.asarray(top)[:, None], cost, np.inf)
    return np.argmin(cost, axis=1)


def select_budget(sse, counts, top, budget, valid=None):
    """Levels and t = log2(lambda) of the frame-budget rule: bisection of t
    in [-40, 60] for 30 steps keeping the upper end feasible (summed SSE
    within the budget); the levels are those at the upper end. ``valid``
    marks instances with a template (others draw nothing: level 0, no SSE)."""
    n = sse.shape[0]
    valid = np.ones(n, bool) if valid is None else np.asarray(valid, bool)
    lo, hi = BUDGET_T_LO, BUDGET_T_HI
    for _ in range(BUDGET_ITERS):
        mid = 0.5 * (lo + hi)
        lv = choose_levels(sse, counts, top, 2.0 ** mid)
        total = sse[np.arange(n), lv][valid].sum()
        if total <= budget:
            hi = mid
        else:
            lo = mid
    lv = choose_levels(sse, counts, top, 2.0 ** hi)
    return np.where(valid, lv, 0), hi
