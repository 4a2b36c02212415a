"""Train the learned-LoD network and tune the fixed-distance baseline.

1. Draw training instance-views like the 3,500-avatar crowd (seeded), render
   each alone at the 5 levels (100/50/25/12.5/6.25 %) and label it with the
   PSNR of every level against level 0 (library kernels).
2. Fit the pose PCA and the feature z-scoring on the training split (host
   preprocessing), train the network on the GPU (cs_mlp_train_step).
3. On the validation split: choose the margin so that at least ``coverage``
   of the views keep their true PSNR >= floor at the selected level; tune the
   4 thresholds of the fixed-distance 5-level rule to the same criterion.
4. Save the network bytes and the tuned constants (npz).

Usage: python -m paper_2501_17792_amd.train_lod [--views 200000] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from . import crowdsplat as cs
from . import lodnet, synth

FLOOR = 40.0


def fixed_levels(dist, thresholds):
    return np.searchsorted(np.asarray(thresholds), dist, side="right")


def tune_fixed(dist, psnr, floor=FLOOR, coverage=0.99):
    """Smallest increasing thresholds d_1..d_4 such that, for each level l, at
    least ``coverage`` of the views at distance >= d_l reach floor at level l."""
    L = psnr.shape[1]
    order = np.argsort(dist)
    d_sorted = dist[order]
    th = []
    for l in range(1, L):
        ok = (psnr[order, l] >= floor).astype(np.float64)
        # fraction of good views among those at index >= i (suffix means)
        suffix = np.cumsum(ok[::-1])[::-1] / np.arange(len(ok), 0, -1)
        cand = np.nonzero(suffix >= coverage)[0]
        d = d_sorted[cand[0]] if cand.size else np.inf
        th.append(max(d, th[-1] if th else 0.0))
    return np.array(th)


def gaussians(levels, counts):
    return counts[levels].sum()


def select(pred, floor, margin):
    ok = pred >= floor + margin
    ok[:, 0] = True
    L = pred.shape[1]
    return (L - 1) - np.argmax(ok[:, ::-1], axis=1)


def tune_margin(pred, psnr, floor=FLOOR, coverage=0.99):
    for m in np.arange(0.0, 20.01, 0.25):
        lv = select(pred, floor, m)
        good = psnr[np.arange(len(lv)), lv] >= floor
        if good.mean() >= coverage:
            return float(m)
    return 20.0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--views", type=int, default=200_000)
    ap.add_argument("--val", type=float, default=0.1)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--gauss", type=int, default=100_000)
    ap.add_argument("--coverage", type=float, default=0.99)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "lod_net.npz"))
    args = ap.parse_args(argv)
    import torch

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t0 = time.time()
    templates = [synth.make_template(t, args.gauss, 3, synth.C4_LEVELS) for t in range(14)]
    cam = synth.scene_c3(templates=templates, n_frames=0).camera
    views = lodnet.view_crowd(400, args.views)
    pca_mean, pca_basis = lodnet.fit_pca(views.pose[: int(args.views * (1 - args.val))])
    r = cs.Renderer(0)
    r.upload_templates(templates)
    lab = lodnet.generate_labels(r, templates, cam, views, pca_mean, pca_basis, batch=2500, log=log)
    log(f"labels in {time.time() - t0:.1f} s")
    n_tr = int(args.views * (1 - args.val))
    net, losses = lodnet.train(r, lab.features[:n_tr], lab.psnr[:n_tr], pca_mean, pca_basis,
                               epochs=args.epochs, log=log)
    pred = lodnet.predict(r, net, lab.features[n_tr:])
    psnr_v = lab.psnr[n_tr:]
    margin = tune_margin(pred, psnr_v, FLOOR, args.coverage)
    dist = lab.features[:, 0]
    th = tune_fixed(dist[:n_tr], lab.psnr[:n_tr], FLOOR, args.coverage)
    counts = np.array(templates[0].level_count, np.float64)
    lv_l = select(pred, FLOOR, margin)
    lv_f = fixed_levels(dist[n_tr:], th)
    good_l = (psnr_v[np.arange(len(lv_l)), lv_l] >= FLOOR).mean()
    good_f = (psnr_v[np.arange(len(lv_f)), lv_f] >= FLOOR).mean()
    rmse = float(np.sqrt(np.mean((pred - psnr_v) ** 2)))
    summary = dict(margin=margin, thresholds=th.tolist(), val_rmse_db=rmse,
                   val_gauss_learned=float(counts[lv_l].mean()), val_gauss_fixed=float(counts[lv_f].mean()),
                   val_ok_learned=float(good_l), val_ok_fixed=float(good_f), final_loss=losses[-1])
    log(summary)
    np.savez(args.out, net=net.cpu().numpy(), margin=margin, thresholds=th, floor=FLOOR,
             coverage=args.coverage, views=args.views, losses=np.array(losses), summary=str(summary))
    print(summary, flush=True)


if __name__ == "__main__":
    main()
