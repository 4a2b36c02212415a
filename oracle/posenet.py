"""FP64 oracle of the pose-dependent Gaussian offsets.

TEST INFRASTRUCTURE ONLY (see the package header).

CrowdSplat §2 builds on GaussianAvatar, whose second stage trains a network
that predicts pose-dependent changes of the template's 3D Gaussians (cloth
wrinkles) before the template is skinned. The paper gives neither the
network nor its inputs; the reading used here (listed in the design notes):

* every template Gaussian g carries an embedding e_g of 32 values;
* an instance's pose code p_i holds the axis-angles of joints 1..23 (69
  values, the root's global orientation excluded: it moves the body
  rigidly and cannot wrinkle cloth), followed by 11 zeros (80 values);
* a per-Gaussian MLP maps [e_g ; p_i] (112 values) to an offset of the
  canonical mean: h1 = relu(W1 [e; p] + b1) (64), h2 = relu(W2 h1 + b2) (64),
  d = W3 h2 + b3 (3);
* the skinned mean is then M (mu_g + d_g) (linear blend skinning of the
  offset canonical mean); covariances are unchanged;
* arithmetic: W1, W2, W3 and every layer input (e, p, h1, h2) are rounded
  to bfloat16 (round to nearest even) before their product; biases and
  accumulation are FP32 on the device (FP64 here).
"""
from __future__ import annotations

import numpy as np

N_EMBED = 32
N_POSE = 80
N_POSE_USED = 69
N_HIDDEN = 64


def bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float64. NaN and infinities do not occur in these inputs."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def pose_code(pose) -> np.ndarray:
    """[..., 24, 3] axis-angles -> [..., 80]: joints 1..23 flattened, then zeros."""
    p = np.asarray(pose, np.float64)
    flat = p[..., 1:, :].reshape(p.shape[:-2] + (N_POSE_USED,))
    out = np.zeros(p.shape[:-2] + (N_POSE,), np.float64)
    out[..., :N_POSE_USED] = flat
    return out


def forward(net, embed, pose, rounded=True, with_bound=False):
    """Offsets d [N, 3] of N Gaussians with embeddings ``embed`` [N, 32] for
    one instance of pose ``pose`` [24, 3]. ``net`` holds w1 [64, 112], b1,
    w2 [64, 64], b2, w3 [3, 64], b3 (float32 masters). With ``rounded`` the
    weights and layer inputs are rounded to bfloat16 first.

    With ``with_bound`` also returns, per Gaussian and output, how far the
    offset can move if each rounded hidden value (h1, h2) lands one bfloat16
    step away (a device that accumulates in FP32 may round a value lying at a
    rounding boundary the other way): sum_j |W3_cj| (u(h2_j) + sum_k |W2_jk|
    u(h1_k)), u = the bfloat16 step at that value."""
    q = bf16 if rounded else (lambda v: np.asarray(v, np.float64))
    W1, W2, W3 = q(net["w1"]), q(net["w2"]), q(net["w3"])
    b1, b2, b3 = (np.asarray(net[k], np.float64) for k in ("b1", "b2", "b3"))
    e = q(embed)
    p = q(pose_code(pose).astype(np.float32))
    x = np.concatenate([e, np.broadcast_to(p, (e.shape[0], N_POSE))], axis=1)
    z1 = x @ W1.T + b1
    h1 = q(np.maximum(z1, 0.0).astype(np.float32)) if rounded else np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = q(np.maximum(z2, 0.0).astype(np.float32)) if rounded else np.maximum(z2, 0.0)
    d = h2 @ W3.T + b3
    if not with_bound:
        return d
    u1 = _bf16_step(h1)
    u2 = _bf16_step(h2)
    bound = u2 @ np.abs(W3).T + (u1 @ np.abs(W2).T) @ np.abs(W3).T
    return d, bound


def _bf16_step(v) -> np.ndarray:
    """The gap between consecutive bfloat16 values around |v| (2^(e-7) for
    |v| in [2^e, 2^(e+1))); the smallest normal step for zero."""
    a = np.abs(np.asarray(v, np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def offset_template(template, embed, net, pose, n=None) -> np.ndarray:
    """The template's canonical means with this pose's offsets added (first
    ``n`` Gaussians)."""
    n = template.n if n is None else n
    d = forward(net, np.asarray(embed, np.float32)[:n], pose)
    return np.asarray(template.mean[:n], np.float64) + d
