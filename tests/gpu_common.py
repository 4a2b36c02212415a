"""Shared helpers of the GPU parity tests (no tests here)."""
from __future__ import annotations

import numpy as np

from oracle import frame as oframe
from oracle import splat as osplat
from paper_2501_17792_amd import synth


def run_gpu(scene, levels_mode, thresholds=(10.0, 25.0), tile=(16, 16), setup=None, **kw):
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    r = cs.Renderer(0, tile=tile, **kw)
    r.upload_templates(scene.templates)
    r.set_crowd(scene.crowd)
    if setup is not None:
        setup(r)
    img = r.frame(scene.camera, levels_mode, thresholds, stats=True)
    torch.cuda.synchronize()
    return r, img.cpu().numpy()


def gpu_frame_buffers(r, n_inst):
    st = r.last_stats
    n_s, n_p = int(st.n_splats), int(st.n_pairs)
    out = dict(stats=st, n_splats=n_s, n_pairs=n_p)
    out["bones"] = r.debug("BONES", np.float32, n_inst * 24 * 12).reshape(n_inst, 24, 3, 4)
    out["level"] = r.debug("LEVEL", np.int32, n_inst)
    out["offset"] = r.debug("OFFSET", np.uint32, n_inst + 1)
    cam = r.last_camera
    n_tiles = -(-cam.width // r.tile[0]) * -(-cam.height // r.tile[1])
    out["ranges"] = r.debug("RANGES", np.uint32, 2 * n_tiles).reshape(n_tiles, 2)
    if n_s:
        out["rec"] = r.debug("RECORD", np.float32, n_s * 12).reshape(n_s, 12)
        out["rect"] = r.debug("RECT", np.uint32, n_s)
        out["count"] = r.debug("COUNT", np.uint32, n_s)
        out["pair_off"] = r.debug("PAIR_OFF", np.uint32, n_s)
    if n_p:
        out["keys"] = r.debug("KEYS", np.uint64, n_p)
        out["vals"] = r.debug("VALS", np.uint32, n_p)
        out["skeys"] = r.debug("SKEYS", np.uint64, n_p)
        out["svals"] = r.debug("SVALS", np.uint32, n_p)
    return out


def unpack_rect(r):
    r = r.astype(np.int64)
    return np.stack([r & 255, (r >> 8) & 255, (r >> 16) & 255, (r >> 24) & 255], axis=1)


def rect_fragile(orc, tw, th, width, height, tol=2e-3):
    """Splats whose tile rect (or visibility) is decided within ``tol`` px of a
    boundary: the FP32 and FP64 decisions may legitimately differ there."""
    b = orc["bounds"]  # u-rx, v-ry, u+rx, v+ry
    frag = np.zeros(b.shape[0], bool)
    for k, t in enumerate((tw, th, tw, th)):
        x = b[:, k]
        frag |= np.abs(x - np.round(x)) < tol  # pixel floor flips
        lim = width if k % 2 == 0 else height
        frag |= np.abs(x) < tol
        frag |= np.abs(x - lim) < 1 + tol
    return frag


def check_sorted_pairs(g, n_splats):
    """Sort invariants on the device's own output: non-decreasing keys, a
    permutation of the emitted pairs, stable ties, counts = rect areas."""
    keys, vals, sk, sv = g["keys"], g["vals"], g["skeys"], g["svals"]
    assert np.all(sk[1:] >= sk[:-1])
    order = np.lexsort((np.arange(len(keys)), keys))
    assert np.array_equal(sk, keys[order])
    assert np.array_equal(sv, vals[order])
    np.testing.assert_array_equal(np.bincount(vals, minlength=n_splats).astype(np.uint32), g["count"])
    # emission layout: pair_off is the exclusive scan of count
    cs = np.concatenate([[0], np.cumsum(g["count"].astype(np.int64))[:-1]])
    np.testing.assert_array_equal(g["pair_off"].astype(np.int64), cs)
