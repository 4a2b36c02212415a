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


# ----------------------------------------------------------------------------
# rules tuned to the frame's PSNR against the full-detail frame
# ----------------------------------------------------------------------------

HOLD_FRAMES = tuple(range(5, 300, 10))
TUNE_FRAMES = tuple(k for k in range(300) if k not in HOLD_FRAMES)  # every frame not held out
TUNE_EXTRA_DB = 0.5  # tuned to floor + this on the tuning frames, so held-out frames keep the floor
VISIBLE_LAG = 4  # the visible-share rule reads the counts of the frame this many frames back
FIXED_RATIOS = (1.0, 1.25, 1.5, 2.0, 3.0)


def frame_psnr(torch, img, ref) -> float:
    mse = float(torch.mean((img - ref) ** 2).item())
    return float("inf") if mse == 0.0 else -10.0 * np.log10(mse)


class FrameJudge:
    """Full-detail reference frames of an animated crowd and the PSNR of any
    LoD rule's frames against them (one fused context, eager frames). A
    frame of the visible-share rule is drawn right after frame k - ``lag``
    (clamped at 0), whose visible pixels it reads, as it is in a stream of
    frames with ``lag`` frames in flight on alternating contexts."""

    def __init__(self, torch, scene, frames, tile=(32, 16), lag=VISIBLE_LAG):
        self.torch, self.scene, self.lag = torch, scene, lag
        self.poses = torch.from_numpy(scene.frame_poses).cuda()
        self.r = cs.Renderer(0, fuse=True, tile=tile)
        self.r.upload_templates(scene.templates)
        self.r.set_crowd(scene.crowd)
        self.ref = {}
        for k in frames:
            self.ref[k] = self.render(k, (cs.CS_LOD_FULL, (), 0, 0.0)).clone()

    def render(self, k, lod, floor=FLOOR):
        mode, thr, mlp_ptr, margin = lod
        self.r.pose_dev.copy_(self.poses[k])
        self.r.select_lod(self.scene.camera, mode, thr, mlp_ptr=mlp_ptr, psnr_min=floor, margin=margin)
        self.r.skin()
        return self.r.render(self.scene.camera, stats=True)

    def evaluate(self, lod, frames, floor=FLOOR):
        """(min PSNR over the frames, mean drawn Gaussians per frame)."""
        ps, ns = [], []
        for k in frames:
            if lod[0] == cs.CS_LOD_BUDGET_VISIBLE:
                self.render(max(0, k - self.lag), lod, floor)
            img = self.render(k, lod, floor)
            ns.append(int(self.r.last_stats.n_splats))
            ps.append(frame_psnr(self.torch, img, self.ref[k]))
        return float(min(ps)), float(np.mean(ns))

    def close(self):
        self.r.close()


def tune_frame_rules(torch, scene, mlp_ptr, floor=FLOOR, tune=TUNE_FRAMES, hold=HOLD_FRAMES, tile=(32, 16),
                     extra_db=TUNE_EXTRA_DB, log=print):
    """Both rules tuned on the ``tune`` frames so that every one of them keeps
    PSNR >= floor + extra_db against full detail, then judged on the ``hold``
    frames (the floor itself):
    * fixed distance, 5 levels: thresholds d_k = d_1 r^(k-1); for each ratio r
      the smallest d_1 (bisection, 12 steps in [0.5, 400] m) meeting the
      target, and of those the one drawing the fewest Gaussians;
    * learned, frame budget: the smallest margin (bisection, 12 steps in
      [-40, 10] dB) meeting it. The predicted errors are those of each avatar
      alone on black over its whole window; in the crowd nearer avatars hide
      much of that, so the margin that calibrates the predicted total to the
      frame's error is negative;
    * learned, frame budget on the visible share: the same bisection in
      [-20, 40] dB, the errors scaled by each avatar's visible share of its
      window. Its margin comes out positive: the label's error is spread over
      the whole window, background included, while the visible pixels are
      all on the avatar, where its error lies."""
    judge = FrameJudge(torch, scene, tuple(tune) + tuple(hold), tile)
    target = floor + extra_db
    fixed = []
    for ratio in FIXED_RATIOS:
        lo, hi = 0.5, 400.0
        th = lambda d: tuple(float(d * ratio ** k) for k in range(4))  # noqa: E731
        if judge.evaluate((cs.CS_LOD_FIXED, th(hi), 0, 0.0), tune)[0] < target:
            continue
        for _ in range(12):
            mid = float(np.sqrt(lo * hi))
            if judge.evaluate((cs.CS_LOD_FIXED, th(mid), 0, 0.0), tune)[0] >= target:
                hi = mid
            else:
                lo = mid
        p, n = judge.evaluate((cs.CS_LOD_FIXED, th(hi), 0, 0.0), tune)
        fixed.append(dict(ratio=ratio, thresholds=list(th(hi)), tune_min_psnr=p, tune_gauss=n))
        log(f"fixed ratio {ratio}: d1 {hi:.2f} m, {n / 1e6:.1f}M Gaussians, min PSNR {p:.2f} dB")
    best = min(fixed, key=lambda f: f["tune_gauss"])
    out = dict(floor=floor, target_db=target, tune_frames=list(tune), hold_frames=list(hold),
               fixed_candidates=fixed, fixed_thresholds=best["thresholds"], fixed_tune_gauss=best["tune_gauss"],
               visible_lag=judge.lag)
    margins = {}
    for name, mode, lo, hi in (("budget", cs.CS_LOD_BUDGET, -40.0, 10.0),
                               ("budget_visible", cs.CS_LOD_BUDGET_VISIBLE, -20.0, 40.0)):
        for _ in range(12):
            mid = 0.5 * (lo + hi)
            p, n = judge.evaluate((mode, (), mlp_ptr, mid), tune, floor)
            log(f"{name} margin {mid:.3f} dB: {n / 1e6:.1f}M Gaussians, min PSNR {p:.2f} dB")
            if p >= target:
                hi = mid
            else:
                lo = mid
        margins[name] = hi
        p, n = judge.evaluate((mode, (), mlp_ptr, hi), tune, floor)
        out.update({f"{name}_margin": hi, f"{name}_tune_min_psnr": p, f"{name}_tune_gauss": n})
    for name, lod in [("fixed", (cs.CS_LOD_FIXED, tuple(best["thresholds"]), 0, 0.0)),
                      ("budget", (cs.CS_LOD_BUDGET, (), mlp_ptr, margins["budget"])),
                      ("budget_visible", (cs.CS_LOD_BUDGET_VISIBLE, (), mlp_ptr, margins["budget_visible"]))]:
        p, n = judge.evaluate(lod, hold, floor)
        out[f"{name}_hold_min_psnr"], out[f"{name}_hold_gauss"] = p, n
    judge.close()
    log(out)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--views", type=int, default=200_000)
    ap.add_argument("--val", type=float, default=0.1)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--gauss", type=int, default=100_000)
    ap.add_argument("--coverage", type=float, default=0.99)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "lod_net.npz"))
    ap.add_argument("--frame-rules", action="store_true",
                    help="with the saved network: tune the fixed-distance thresholds and the frame-budget "
                         "margin to the frame PSNR of the 3,500-avatar animation and write "
                         "lod_frame_rules.json next to the network")
    args = ap.parse_args(argv)
    import torch

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.frame_rules:
        import json

        templates = [synth.make_template(t, args.gauss, 3, synth.C4_LEVELS) for t in range(14)]
        scene = synth.scene_c3(templates=templates, n_frames=300)
        z = np.load(args.out, allow_pickle=False)
        net = torch.from_numpy(z["net"]).cuda()
        rules = tune_frame_rules(torch, scene, net.data_ptr(), log=log)
        path = os.path.join(os.path.dirname(args.out), "lod_frame_rules.json")
        with open(path, "w") as f:
            json.dump(rules, f, indent=1)
        print(json.dumps(rules), flush=True)
        return

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
