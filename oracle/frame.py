"""FP64 whole-frame oracle: fixed-distance LoD, work list, skin, render.

CrowdSplat §2 (last paragraph): each character uses a template level chosen
by its distance to the camera (202k Gaussians within 5 m, 12k from 5 to 10 m,
3k beyond). Here the levels are importance-ordered prefixes of one template,
selected by distance thresholds; the finer level wins at a boundary
(distance strictly below a threshold). Instance-major concatenation of the
selected prefixes is the emission order of the frame.
"""
from __future__ import annotations

import numpy as np

from . import skinning, splat


def instance_distance(pos, eye) -> np.ndarray:
    """|| (px, 0, pz) - eye || per instance."""
    pos = np.asarray(pos, np.float64)
    p = np.stack([pos[:, 0], np.zeros(pos.shape[0]), pos[:, 1]], axis=1)
    return np.linalg.norm(p - np.asarray(eye, np.float64)[None], axis=1)


def fixed_levels(pos, eye, thresholds) -> np.ndarray:
    """Level = number of thresholds the distance is not below."""
    d = instance_distance(pos, eye)
    lvl = np.zeros(d.shape[0], np.int64)
    for t in thresholds:
        lvl += (d >= t)
    return lvl


def instance_counts(templates, tid, levels) -> np.ndarray:
    return np.array([int(templates[int(t)].level_count[int(l)])
                     for t, l in zip(tid, levels)], np.int64)


def skin_crowd(templates, crowd, levels, mean_fn=None):
    """Posed means / covariances / linear parts of every selected Gaussian,
    instance-major. Returns (mu, cov, L, opacity, sh(list), template ids).
    ``mean_fn(i, n)`` gives instance i's canonical means of its first n
    Gaussians when they depend on the instance (pose-dependent offsets)."""
    mus, covs, Ls, ops, shs = [], [], [], [], []
    counts = instance_counts(templates, crowd.tid, levels)
    for i in range(crowd.n):
        t = templates[int(crowd.tid[i])]
        n = int(counts[i])
        mean = mean_fn(i, n) if mean_fn is not None else None
        mu, cov, L, _ = skinning.skin_instance(t, crowd.pose[i], crowd.yaw[i],
                                               crowd.pos[i, 0], crowd.pos[i, 1], n, mean=mean)
        mus.append(mu)
        covs.append(cov)
        Ls.append(L)
        ops.append(t.opacity[:n].astype(np.float64))
        shs.append(t.sh[:n].astype(np.float64))
    return mus, covs, Ls, ops, shs, counts


def frame_records(templates, crowd, cam, levels, tw, th, mean_fn=None):
    """Splat records of a whole frame in emission order."""
    mus, covs, Ls, ops, shs, counts = skin_crowd(templates, crowd, levels, mean_fn)
    parts = []
    for i in range(crowd.n):
        deg = templates[int(crowd.tid[i])].sh_degree
        parts.append(splat.splat_records(mus[i], covs[i], Ls[i], ops[i], shs[i], deg,
                                         cam, tw, th))
    rec = splat.concat_records(parts)
    rec["mu"] = np.concatenate(mus)
    rec["cov"] = np.concatenate(covs)
    rec["offsets"] = np.concatenate([[0], np.cumsum(counts)])
    return rec


def render_frame(templates, crowd, cam, levels, tw=16, th=16,
                 fragile_alpha=1e-4, fragile_t=1e-4, tie_impact=None):
    rec = frame_records(templates, crowd, cam, levels, tw, th)
    out = splat.render_records(rec, cam, tw, th, fragile_alpha, fragile_t, tie_impact)
    out["records"] = rec
    return out
