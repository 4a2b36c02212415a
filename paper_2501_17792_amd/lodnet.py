"""Learned level of detail: the network's device layout, its training data
and its training loop, driven through the C ABI.

Labels: every training instance-view is rendered alone (cs_render_views) at
each level; its PSNR against level 0 over its window is the label
(cs_view_psnr). Pose PCA and the feature z-scoring are fitted on the training
set (a preprocessing step on the host); the network itself is trained on the
GPU by cs_mlp_train_step (forward, backward and Adam in the library's
kernels).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np

from . import crowdsplat as cs
from . import synth


def pack(params: dict, mu, sd, pca_mean, pca_basis) -> cs.CsMlp:
    """params: W1 [32,64], b1 [64], W2 [64,64], b2, W3 [64,5], b3 [5] (in-major)."""
    net = cs.CsMlp()
    flat = np.zeros(cs.CS_MLP_NPARAM, np.float32)

    def put(name, arr):
        off, shape = cs.MLP_OFF[name]
        a = np.zeros(shape, np.float32)
        arr = np.asarray(arr, np.float32)
        a[tuple(slice(0, d) for d in arr.shape)] = arr
        flat[off:off + a.size] = a.reshape(-1)

    put("w1", np.asarray(params["W1"]).T)
    put("b1", params["b1"])
    put("w2", np.asarray(params["W2"]).T)
    put("b2", params["b2"])
    put("w3", np.asarray(params["W3"]).T)
    put("b3", params["b3"])
    ctypes.memmove(net.params, flat.ctypes.data, flat.nbytes)
    # every source array is held in a name until its copy is done: a
    # temporary's buffer may be freed (and reused) before memmove reads it
    mu = np.ascontiguousarray(mu, np.float32)
    isd = (1.0 / np.asarray(sd, np.float64)).astype(np.float32)
    pm = np.ascontiguousarray(pca_mean, np.float32)
    pb = np.ascontiguousarray(pca_basis, np.float32)
    assert mu.size == 32 and isd.size == 32 and pm.size == 72 and pb.size == 8 * 72
    ctypes.memmove(net.mu, mu.ctypes.data, 128)
    ctypes.memmove(net.inv_sd, isd.ctypes.data, 128)
    ctypes.memmove(net.pca_mean, pm.ctypes.data, 72 * 4)
    ctypes.memmove(net.pca_basis, pb.ctypes.data, 8 * 72 * 4)
    return net


def unpack(raw: np.ndarray) -> dict:
    """Host copy of a device cs_mlp (uint8 bytes) -> dict of float64 arrays
    in the oracle's in-major convention, plus mu, sd and the PCA."""
    net = cs.CsMlp.from_buffer_copy(raw.tobytes())
    flat = np.frombuffer(bytes(net.params), np.float32).astype(np.float64)

    def get(name):
        off, shape = cs.MLP_OFF[name]
        return flat[off:off + int(np.prod(shape))].reshape(shape)

    out = dict(W1=get("w1").T.copy(), b1=get("b1").copy(), W2=get("w2").T.copy(), b2=get("b2").copy(),
               W3=get("w3")[:5].T.copy(), b3=get("b3")[:5].copy())
    out["mu"] = np.frombuffer(bytes(net.mu), np.float32).astype(np.float64)
    out["sd"] = 1.0 / np.frombuffer(bytes(net.inv_sd), np.float32).astype(np.float64)
    out["pca_mean"] = np.frombuffer(bytes(net.pca_mean), np.float32).astype(np.float64)
    out["pca_basis"] = np.frombuffer(bytes(net.pca_basis), np.float32).astype(np.float64).reshape(8, 72)
    return out


def init_params(seed: int = 0, out_bias: float = 50.0) -> dict:
    """He-initialised weights; the output bias starts near the label mean."""
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, np.sqrt(2 / 31), (32, 64)), b1=np.zeros(64),
                W2=rng.normal(0, np.sqrt(2 / 64), (64, 64)), b2=np.zeros(64),
                W3=rng.normal(0, np.sqrt(1 / 64), (64, 5)), b3=np.full(5, out_bias))


def fit_pca(poses: np.ndarray, k: int = 8):
    """Mean and the top-k principal directions of flattened poses [N,72]."""
    X = np.asarray(poses, np.float64).reshape(poses.shape[0], -1)
    mean = X.mean(0)
    _, _, vt = np.linalg.svd(X - mean, full_matrices=False)
    return mean, vt[:k]


def to_device(r: "cs.Renderer", net: cs.CsMlp):
    import torch

    buf = torch.from_numpy(np.frombuffer(bytes(net), np.uint8).copy()).to(r.device)
    r.mlp_sync(buf)
    return buf


@dataclasses.dataclass
class LabelSet:
    features: np.ndarray   # [N,32]
    psnr: np.ndarray       # [N,5]
    poses: np.ndarray      # [N,24,3]


def view_crowd(seed: int, n: int, n_templates: int = 14, extent: float = 80.0, sigma: float = 0.3):
    """Instance-views placed, posed and oriented like the crowd's instances."""
    """Training instance-views drawn like the 3,500-avatar crowd."""
    return synth.make_crowd(seed, n, n_templates, extent, sigma)


def generate_labels(r: "cs.Renderer", templates, cam, crowd, pca_mean, pca_basis, batch: int = 2500,
                    levels: int = 5, log=None) -> LabelSet:
    """Features and per-level PSNR labels of every instance of ``crowd``,
    each rendered alone, ``batch`` instances per launch."""
    import torch

    zero = init_params()
    net_dev = to_device(r, pack(zero, np.zeros(32), np.ones(32), pca_mean, pca_basis))
    feats, labels = [], []
    for b0 in range(0, crowd.n, batch):
        sub = synth.Crowd(tid=crowd.tid[b0:b0 + batch], yaw=crowd.yaw[b0:b0 + batch],
                          pos=crowd.pos[b0:b0 + batch], pose=crowd.pose[b0:b0 + batch])
        r.set_crowd(sub)
        feats.append(r.lod_features(cam, net_dev).cpu().numpy())
        atlases = []
        for lvl in range(levels):
            r.select_lod(cam, cs.CS_LOD_CONSTANT, (), level=lvl)
            r.skin()
            at, views = r.render_views(cam, atlases[0].clone() if atlases else None)
            atlases.append(at.clone())
        ps = [r.view_psnr(atlases[0], a).cpu().numpy() for a in atlases]
        labels.append(np.stack(ps, axis=1))
        if log:
            log(f"labels {b0 + sub.n}/{crowd.n}")
    torch.cuda.synchronize()
    return LabelSet(features=np.concatenate(feats), psnr=np.concatenate(labels), poses=crowd.pose)


def train(r: "cs.Renderer", features: np.ndarray, labels: np.ndarray, pca_mean, pca_basis,
          epochs: int = 30, batch: int = 1024, lr: float = 1e-3, seed: int = 0, log=None):
    """Fit the network on the GPU; returns (device cs_mlp buffer, losses)."""
    import torch

    mu = features.mean(0)
    sd = features.std(0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    params = init_params(seed, out_bias=float(labels.mean()))
    net = to_device(r, pack(params, mu, sd, pca_mean, pca_basis))
    m = torch.zeros(cs.CS_MLP_NPARAM, dtype=torch.float32, device=r.device)
    v = torch.zeros_like(m)
    fd = torch.from_numpy(np.ascontiguousarray(features, np.float32)).to(r.device)
    td = torch.from_numpy(np.ascontiguousarray(labels, np.float32)).to(r.device)
    n = (features.shape[0] // batch) * batch
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=r.device)
    losses = []
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(features.shape[0])[:n]).to(r.device)
        fe = fd[perm].contiguous()
        ta = td[perm].contiguous()
        acc = torch.zeros(1, dtype=torch.float32, device=r.device)
        for b0 in range(0, n, batch):
            step += 1
            r.mlp_train_step(net, m, v, fe[b0:b0 + batch], ta[b0:b0 + batch], step, lr, loss)
            acc += loss
        losses.append(float(acc.item()) / (n // batch))
        if log:
            log(f"epoch {ep} loss {losses[-1]:.4f}")
    return net, losses


def predict(r: "cs.Renderer", net, features: np.ndarray) -> np.ndarray:
    import torch

    fd = torch.from_numpy(np.ascontiguousarray(features, np.float32)).to(r.device)
    return r.mlp_predict(net, fd)[:, :5].cpu().numpy()
