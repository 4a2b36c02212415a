"""Benchmark of the crowd-splatting hot path on one MI355X.

Workload: 3,500 animated avatars instancing 14 synthetic templates of 100k
Gaussians (SH degree 3) with 5 importance-ordered levels (100/50/25/12.5/6.25 %),
1920x1080, a 300-frame keyframed animation (poses interpolated at 30 Hz).
A step is one whole frame: pose upload (device copy), LoD selection and work
list (learned network, or distance thresholds), forward kinematics, skinning +
projection, tile binning, the per-tile depth sort and compositing, all
replayed as one captured hipGraph. Consecutive frames alternate between
``--inflight`` contexts (one stream and one set of buffers each), so that
that many frames are in flight; the head mode is also timed with one.

The headline value is the learned-LoD frame rate when a trained network is
present (paper_2501_17792_amd/lod_net.npz, written by train_lod.py), else the
10 m / 25 m fixed rule; every LoD rule is reported with its frame PSNR against
the full-detail frame.

Prints one JSON line (rank 0). ``--gpus`` above 1 is refused: this build
measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Frames in flight only overlap on distinct hardware queues. HIP shares its
# queues (4 per process by default) among every stream, torch's stream pool
# included, and two of the four frame streams could land on one queue (frames
# then alternated 3.5 / 6.7 ms: 215 instead of 237 FPS). The frame streams are
# picked by a concurrency probe and a short run of the frame that must advance
# evenly (autotune.pick_streams), from 8 queues (at least: a larger setting is
# kept), asked for before anything starts HIP.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

METRIC = "FPS @3,500 avatars 1080p, learned-LoD vs fixed-LoD at ≥40 dB PSNR vs full"
HBM_PEAK_GBS = 8000.0

N_CU = 256
CLOCK_HZ = 2.4e9
# Non-packed FP32 issue peak: 256 CUs x 4 SIMDs x 16 lanes per clock (a wave64
# VALU instruction occupies its SIMD 4 clocks; packed FP32 is disabled in this
# build): 39.3e12 lane-instructions/s, 78.6 TFLOP/s counting an FMA as two.
ISSUE_PEAK = N_CU * 64 * CLOCK_HZ
FP32_PEAK_TFLOPS = 2 * ISSUE_PEAK / 1e12
# FP32 operations of one live compositing evaluation (FMA = 2): dx, dy, the
# quadratic form and its clamp, o e^power and the 0.99 clamp, 1 - alpha,
# T' = T (1 - alpha), alpha T and three colour FMAs.
BLEND_FLOPS_PER_EVAL = 24

# Counter measurements of the headline frame (learned LoD, frame budget) for the kernel sources they were
# taken on (digest), per tile shape and blend split the autotuner may pick: HBM bytes per launch from two rocprofv3 --pmc
# runs (FETCH_SIZE scaled by 2.000 and WRITE_SIZE by 1.000, the factors a plain 1 GiB copy gives) and VALU
# lane-instructions per item (SQ_INSTS_VALU x 64 / items: splats for the projection, pairs for the sort and
# the blend), summarised under profiles/crowd3500_1080p_budget_<shape>_kernels.md. Other sources, shapes or
# workloads report null.
MEASURED = {"digest": "a3bad74c8ace29b0", "lod": "learned_budget",
            "tiles": {(32, 32, 4): {"traffic": {"blend": 3_308_388_057, "project_fused": 3_167_018_319,
                                                "segsort": 917_354_530},
                                    "valu_per_item": {"blend": 587.9, "project_fused": 422.7, "segsort": 119.9}}}}


def kernel_digest():
    import hashlib

    d = os.path.join(ROOT, "paper_2501_17792_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(stage, st, scene, uniq):
    """Algorithmic HBM bytes of one frame's pass through a stage: what the
    stage must read and write at least, from N splats, P tile pairs and U
    unique template Gaussians drawn this frame (the per-stage terms below)."""
    n, p = float(st["n_splats"]), float(st["n_pairs"])
    W, H = scene.camera.width, scene.camera.height
    sh_bytes = 16 * 12  # SH3: 48 floats per Gaussian
    if stage == "skin":  # template geometry in, posed mean + covariance out
        return 36 * n + 56 * uniq
    if stage == "project_fused":  # template in, record + rect + count out
        return 56 * n + (56 + 4 + sh_bytes) * uniq
    if stage == "project":  # posed Gaussians + template appearance in, record out
        return (36 + 56) * n + (32 + 4 + sh_bytes) * uniq
    if stage == "emit":  # tile-bucket binning: count + scatter read 12 B/splat each, 8 B per pair out
        return 24 * n + 8 * p
    if stage in ("sort", "segsort"):  # per-tile depth order: every pair's key in, its splat index out
        return 12 * p
    if stage == "blend":
        return 52 * p + 12 * W * H
    return 0.0


def unique_template_gaussians(scene, levels):
    tot = 0
    for t in range(len(scene.templates)):
        sel = scene.crowd.tid == t
        if sel.any():
            tot += int(max(scene.templates[t].level_count[int(l)] for l in levels[sel]))
    return tot


_CPU_CTX = {}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))  # the host share of one GPU


def _cpu_worker(pick):
    """One oracle worker: records (skin + project) of its instances, then
    binning + sort + compositing of those records; each timed."""
    from oracle import frame as oframe
    from oracle import splat as osplat
    from paper_2501_17792_amd import synth

    scene, levels = _CPU_CTX["scene"], _CPU_CTX["levels"]
    pick = np.asarray(pick)
    sub = synth.Crowd(tid=scene.crowd.tid[pick], yaw=scene.crowd.yaw[pick], pos=scene.crowd.pos[pick],
                      pose=scene.crowd.pose[pick])
    t0 = time.perf_counter()
    rec = oframe.frame_records(scene.templates, sub, scene.camera, levels[pick], 16, 16)
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    out = osplat.render_records(rec, scene.camera, 16, 16)
    return int(rec["offsets"][-1]), int(len(out["keys"])), t_rec, time.perf_counter() - t0


def oracle_levels(scene, host_net, margin, floor=40.0):
    """The frame-budget LoD selection of the whole crowd by the FP64 oracle
    (features, network, windows, bisection)."""
    from oracle import lod as olod

    cam = scene.camera
    n = scene.crowd.n
    feats = np.zeros((n, 32))
    win = np.zeros(n)
    counts = np.zeros((n, 5))
    top = np.zeros(n, np.int64)
    pads = [olod.pad_radius(t) for t in scene.templates]
    for i in range(n):
        tid = int(scene.crowd.tid[i])
        t = scene.templates[tid]
        yaw, px, pz = float(scene.crowd.yaw[i]), float(scene.crowd.pos[i, 0]), float(scene.crowd.pos[i, 1])
        feats[i] = olod.instance_features(t, tid, 14, scene.crowd.pose[i], yaw, px, pz, pads[tid], cam,
                                          host_net["pca_mean"], host_net["pca_basis"])
        joints = olod.posed_joints(t, scene.crowd.pose[i], yaw, px, pz)
        _, clip = olod.view_box(joints, pads[tid], cam)
        win[i] = olod.label_window_px(clip, cam.width, cam.height)
        lc = np.asarray(t.level_count, np.float64)
        counts[i, :len(lc)] = lc
        top[i] = min(len(lc), 5) - 1
    pred, _ = olod.mlp_forward(host_net, feats, rounded=True)
    sse = olod.level_sse(pred, win, top)
    levels, _ = olod.select_budget(sse, counts, top, olod.frame_budget(cam.width, cam.height, floor + margin))
    return levels, counts


def oracle_fixed_levels(scene, thresholds):
    """The fixed-distance LoD of the whole crowd by the FP64 oracle."""
    from oracle import frame as oframe

    levels = oframe.fixed_levels(scene.crowd.pos, scene.camera.eye, thresholds)
    counts = np.zeros((scene.crowd.n, 5))
    for i in range(scene.crowd.n):
        lc = np.asarray(scene.templates[int(scene.crowd.tid[i])].level_count, np.float64)
        counts[i, :len(lc)] = lc
    return np.asarray(levels, np.int64), counts


def cpu_baseline(scene, host_net, margin, per_worker=21, levels_fn=None, what="the learned-LoD (frame budget) crowd"):
    """The FP64 oracle on the host's cores (at most 16: the host share of one
    GPU), timed on a bounded sample of the frame (frame 0): LoD selection of
    all instances (the frame budget, or ``levels_fn()``), then skin + project
    and binning + sort + compositing of a seeded sample of instances
    (per_worker per core) in a process pool, each phase's wall time
    extrapolated per Gaussian and per tile pair to the oracle's own frame.
    Runs before the GPU is touched (the pool forks)."""
    import multiprocessing as mp

    cores = _cpu_cores()
    t0 = time.perf_counter()
    levels, counts = levels_fn() if levels_fn is not None else oracle_levels(scene, host_net, margin)
    t_lod = time.perf_counter() - t0
    n_splats = int(counts[np.arange(scene.crowd.n), levels].sum())
    rng = np.random.default_rng(7)
    pick = np.sort(rng.choice(scene.crowd.n, size=min(scene.crowd.n, per_worker * cores), replace=False))
    chunks = [pick[k::cores].tolist() for k in range(cores)]
    _CPU_CTX.update(scene=scene, levels=levels)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_cpu_worker, chunks)
        wall = time.perf_counter() - t0
    g = sum(r[0] for r in res)
    p = sum(r[1] for r in res)
    t_rec, t_ras = sum(r[2] for r in res), sum(r[3] for r in res)
    # the sample's pairs per Gaussian stand in for the frame's (instances rendered alone)
    n_pairs = int(round(n_splats * p / max(g, 1)))
    frame_s = t_lod + wall * n_splats / max(g, 1)
    return {"value": round(1.0 / frame_s, 8), "unit": "FPS", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": (f"FP64 oracle, frame 0 of {what}: LoD selection of all "
                       f"{scene.crowd.n} instances ({t_lod:.1f} s, one core), then {len(pick)} seeded instances "
                       f"({g} instance-Gaussians, {p} tile pairs) split over a pool of {cores} processes: "
                       f"{wall:.1f} s wall ({t_rec:.1f} CPU-s skin+project, {t_ras:.1f} CPU-s bin+sort+blend); "
                       f"extrapolated per Gaussian to the oracle frame's {n_splats} Gaussians "
                       f"(~{n_pairs} pairs) = {frame_s:.0f} s/frame"),
            "oracle_levels_hist": np.bincount(levels, minlength=5).tolist()}


def load_net(path):
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    return dict(net=z["net"], margin=float(z["margin"]), thresholds=[float(t) for t in z["thresholds"]],
                floor=float(z["floor"]))


def time_mode(torch, rs, scene, poses_all, imgs, streams, lod, steps, warmup):
    """Captured frames in flight over the contexts ``rs`` (one stream each):
    the autotuner's timing procedure, so tuned and reported rates agree."""
    from paper_2501_17792_amd import autotune

    return autotune.time_frames(torch, rs, scene, poses_all, imgs, streams, lod, steps, warmup)


# The paper's Tab. 2 (FPS, RTX 4090, 1280x720) and Tab. 1 (MiB unshared, shared): context, not targets.
PAPER_TAB2_FPS = {(202_738, False): {1: 728, 100: 50, 400: 22.2}, (202_738, True): {1: 617, 100: 18.2},
                  (12_661, False): {1: 1612, 100: 586, 400: 251, 1000: 125, 5000: 10.3},
                  (12_661, True): {1: 1370, 100: 312, 400: 76, 1000: 34, 5000: 6.1},
                  (3_176, False): {1: 1703, 100: 1240, 400: 673, 1000: 275, 5000: 38.6},
                  (3_176, True): {1: 1347, 100: 804, 400: 298, 1000: 121, 5000: 23.2}}
PAPER_TAB1_MIB = {202_738: {1: (651, 651), 100: (7929, 7075)},
                  12_661: {1: (567, 567), 100: (1005, 953), 400: (2335, 2121), 1000: (5127, 4593),
                           5000: (21340, 19625)},
                  3_176: {1: (557, 557), 100: (675, 639), 400: (993, 937), 1000: (1695, 1541),
                          5000: (5995, 5329)}}


def time_captured(torch, scene, animated, steps, warmup, tile=(16, 16), lod=None):
    """Frames of one crowd as captured graphs on their own stream, one frame
    in flight. Animated: the whole frame (pose upload from a device pose ring,
    LoD, FK, skinning fused into projection, binning, sort, blend) per replay.
    Static: skinned once, rendering alone per replay. Returns (ms per frame
    list, frame stats, image of the first replay)."""
    from paper_2501_17792_amd import crowdsplat as cs

    mode, thr = lod if lod is not None else (cs.CS_LOD_FULL, ())
    stream = torch.cuda.Stream()
    dev = torch.device("cuda", 0)
    with torch.cuda.stream(stream):
        r = cs.Renderer(0, stream=stream, fuse=animated, tile=tile)
        r.upload_templates(scene.templates)
        r.set_crowd(scene.crowd)
        img = torch.zeros((3, scene.camera.height, scene.camera.width), device=dev)
        ring = torch.from_numpy(scene.frame_poses).to(dev) if animated else None
        max_s = max_p = 0
        for f in ((0, ring.shape[0] // 3, 2 * ring.shape[0] // 3) if animated else (0,)):
            if animated:
                r.pose_dev.copy_(ring[f])
            r.frame(scene.camera, mode, thr, image=img, stats=True)
            max_s, max_p = max(max_s, int(r.last_stats.n_splats)), max(max_p, int(r.last_stats.n_pairs))
        r.reserve(scene.crowd.n, int(max_s * 1.02) + 4096, int(max_p * 1.3) + 65536)
        if animated:
            r.set_pose_ring(ring)
            r.capture(scene.camera, img, mode, thr)
        else:
            r.frame(scene.camera, mode, thr, image=img, stats=True)  # skinned once, after the reserve
            r.capture_render(scene.camera, img)
        st = r.last_stats
        for _ in range(warmup):
            r.launch()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        evs[0].record(stream)
        for k in range(steps):
            r.launch()
            evs[k + 1].record(stream)
        stream.synchronize()
        ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
        overflow = int(r.poll().overflow)
        r.close()
    return ms, st, overflow


def stage_frame(torch, scene, animated, tile=(16, 16), frames=3, lod=None):
    """Per-stage times of eager frames of the crowd (HIP events on the launch
    stream), the timed configuration's kernels; then one more frame on a
    context that counts the blend's live evaluations (slower: only its count
    is used), returned in ``out["blend_evals"]``."""
    from paper_2501_17792_amd import crowdsplat as cs

    mode, thr = lod if lod is not None else (cs.CS_LOD_FULL, ())
    evals = None
    with torch.cuda.stream(torch.cuda.Stream()):
        rc = cs.Renderer(0, fuse=animated, profile=True, tile=tile, count_blend=True)
        rc.upload_templates(scene.templates)
        rc.set_crowd(scene.crowd)
        rc.frame(scene.camera, mode, thr, stats=True)
        evals = int(rc.last_stats.blend_evals)
        rc.close()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        r = cs.Renderer(0, stream=stream, fuse=animated, profile=True, tile=tile)
        r.upload_templates(scene.templates)
        r.set_crowd(scene.crowd)
        img = torch.zeros((3, scene.camera.height, scene.camera.width), device="cuda")
        acc = {}
        if not animated:
            r.frame(scene.camera, mode, thr, image=img, stats=True)
        for k in range(frames + 1):
            if animated:
                r.frame(scene.camera, mode, thr, image=img, stats=True)
            else:
                r.render(scene.camera, img, stats=True)
            if k:
                for name, v in r.stage_times().items():
                    acc.setdefault(name, []).append(v)
        stream.synchronize()
        st = r.last_stats
        r.close()
    out = {k: float(np.median(v)) for k, v in acc.items()}
    if animated and "project" in out:
        out["project_fused"] = out.pop("project")
    out["blend_evals"] = evals
    return out, st


def dominant_roofline(stage_ms, st, scene, uniq):
    """Roofline of the longest single-launch kernel of a sweep cell: the
    projection or the LDS segment sort on algorithmic HBM bytes, the blend on
    its FP32 operations (24 per counted live evaluation)."""
    kernels = {"project_fused": "project_kernel (skinning fused)", "project": "project_kernel",
               "segsort": "seg_sort_kernel", "blend": "blend_kernel"}
    cand = {k: stage_ms[k] for k in kernels if stage_ms.get(k, 0.0) > 0}
    if not cand:
        return None
    dom = max(cand, key=cand.get)
    if dom == "blend":
        flops = float(stage_ms.get("blend_evals") or 0) * BLEND_FLOPS_PER_EVAL
        a = flops / (stage_ms[dom] * 1e-3) / 1e12
        return {"bound": "alu", "kernel": kernels[dom], "achieved": round(a, 3), "peak": round(FP32_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(a / FP32_PEAK_TFLOPS, 4), "launch_ms": round(stage_ms[dom], 4),
                "flops_per_launch": int(flops)}
    stats = dict(n_splats=int(st.n_splats), n_pairs=int(st.n_pairs))
    b = algorithmic_bytes(dom, stats, scene, uniq)
    a = b / (stage_ms[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernels[dom], "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(a / HBM_PEAK_GBS, 4), "launch_ms": round(stage_ms[dom], 4), "bytes_per_launch": int(b)}


def frame_roofline(stage_ms, stats, scene, uniq, tile, split, blend):
    """Roofline object of the dominant single-launch kernel of the timed
    frame (fused projection, LDS segment sort or compositing), timed with HIP
    events on its launch stream in the instrumented frames. Projection and
    sort: algorithmic HBM bytes against 8 TB/s and, where counters for these
    sources exist, VALU issue against the non-packed FP32 peak; the bound is
    the larger fraction. Compositing: FP32 operations of the evaluations it
    ran against the non-packed FP32 peak."""
    kernels = {"project_fused": "project_kernel (skinning fused)", "segsort": "seg_sort_kernel",
               "blend": "blend_kernel"}
    cand = {k: stage_ms[k] for k in kernels if stage_ms.get(k, 0.0) > 0}
    dom = max(cand, key=cand.get)
    t = stage_ms[dom] * 1e-3
    meas = MEASURED["tiles"].get((*tile, split)) if kernel_digest() == MEASURED["digest"] else None
    out = {"kernel": kernels[dom], "launch_ms": round(stage_ms[dom], 4),
           "traffic": meas["traffic"].get(dom) if meas else None}
    if dom == "blend":
        flops = blend["evals_per_frame"] * BLEND_FLOPS_PER_EVAL
        a = flops / t / 1e12
        out.update(bound="alu", achieved=round(a, 3), peak=round(FP32_PEAK_TFLOPS, 1), unit="TFLOP/s",
                   frac=round(a / FP32_PEAK_TFLOPS, 4), flops_per_launch=int(flops))
        # the instruction stream behind those operations: VALU issue (list compaction, staging, lanes of
        # finished or untouched pixels) against the non-packed issue peak
        valu = meas["valu_per_item"].get(dom) if meas else None
        if valu is not None:
            ai = valu * stats["n_pairs"] / t
            out["issue"] = {"achieved": round(ai / 1e12, 3), "peak": round(ISSUE_PEAK / 1e12, 2),
                            "unit": "Tlane-instr/s", "frac": round(ai / ISSUE_PEAK, 4), "valu_per_pair": valu}
        return out
    b = algorithmic_bytes(dom, stats, scene, uniq)
    a = b / t / 1e9
    hbm = {"achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(a / HBM_PEAK_GBS, 4),
           "bytes_per_launch": int(b)}
    items = stats["n_splats"] if dom == "project_fused" else stats["n_pairs"]
    valu = meas["valu_per_item"].get(dom) if meas else None
    issue = None
    if valu is not None:
        ai = valu * items / t
        issue = {"achieved": round(ai / 1e12, 3), "peak": round(ISSUE_PEAK / 1e12, 2), "unit": "Tlane-instr/s",
                 "frac": round(ai / ISSUE_PEAK, 4), "valu_per_item": valu}
    if issue is not None and issue["frac"] > hbm["frac"]:
        out.update(bound="alu", **{k: v for k, v in issue.items() if k != "valu_per_item"})
    else:
        out.update(bound="hbm", **{k: v for k, v in hbm.items() if k != "bytes_per_launch"})
    out["hbm"] = hbm
    out["issue"] = issue
    return out


def sweep_tab2(torch, steps, warmup, cells=None):
    """Tab. 2-shaped sweep: duplicates of one SH3 template of 202,738 / 12,661
    / 3,176 Gaussians, 1 to 5,000 characters on the grid, with and without
    motion, 1280x720. One JSON line per cell."""
    from paper_2501_17792_amd import synth

    out = []
    for n_gauss in synth.PAPER_SIZES:
        tpl = synth.make_template(600 + synth.PAPER_SIZES.index(n_gauss), n_gauss, 3)
        for animated in (False, True):
            for n_chars in synth.TAB2_CELLS[(n_gauss, animated)]:
                if cells and (n_gauss, n_chars, animated) not in cells:
                    continue
                sc = synth.scene_tab2(n_gauss, n_chars, animated, template=tpl)
                ms, st, overflow = time_captured(torch, sc, animated, steps, warmup)
                stage_ms, stp = stage_frame(torch, sc, animated)
                med = float(np.median(ms))
                fps = 1000.0 / med
                rec = {"sweep": "tab2", "gaussians": n_gauss, "characters": n_chars, "motion": animated,
                       "width": 1280, "height": 720, "fps": round(fps, 2), "frame_ms_median": round(med, 4),
                       "frame_ms_p95": round(float(np.percentile(ms, 95)), 4),
                       "gaussians_per_s": round(int(st.n_splats) * fps, 1), "n_splats": int(st.n_splats),
                       "n_pairs": int(st.n_pairs), "overflow": overflow,
                       "stage_ms": {k: round(v, 4) for k, v in stage_ms.items() if k != "blend_evals"},
                       "blend_evals": stage_ms["blend_evals"],
                       "roofline": dominant_roofline(stage_ms, stp, sc, n_gauss),
                       "paper_fps_rtx4090": PAPER_TAB2_FPS[(n_gauss, animated)][n_chars]}
                print(json.dumps(rec), flush=True)
                out.append(rec)
    return out


def sweep_tab1(torch):
    """Tab. 1-shaped memory accounting: device bytes of the context after one
    animated 1280x720 frame, templates shared (the default) against one copy
    per character, from the library's own accounting and from the device's
    free-memory counter. One JSON line per cell."""
    from paper_2501_17792_amd import crowdsplat as cs
    from paper_2501_17792_amd import synth

    out = []
    mib = 1024.0 * 1024.0
    for n_gauss, chars in synth.TAB1_CELLS.items():
        tpl = synth.make_template(600 + synth.PAPER_SIZES.index(n_gauss), n_gauss, 3)
        for n_chars in chars:
            sc = synth.scene_tab2(n_gauss, n_chars, True, template=tpl, frames=1)
            res = {}
            for mode in ("shared", "unshared"):
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                free0 = torch.cuda.mem_get_info()[0]
                r = cs.Renderer(0, fuse=True)
                r.upload_templates(sc.templates)
                r.set_crowd(sc.crowd)
                if mode == "unshared":
                    r.materialise(True)
                img = r.frame(sc.camera, cs.CS_LOD_FULL, (), stats=True)
                torch.cuda.synchronize()
                m = r.memory()
                used = free0 - torch.cuda.mem_get_info()[0]
                res[mode] = dict(m, device_used=int(used))
                r.close()
                del img
            sh, un = res["shared"], res["unshared"]
            rec = {"sweep": "tab1", "gaussians": n_gauss, "characters": n_chars,
                   "shared_mib": round(sh["total"] / mib, 1), "unshared_mib": round(un["total"] / mib, 1),
                   "saving_pct": round(100.0 * (1.0 - sh["total"] / un["total"]), 2),
                   "shared_device_used_mib": round(sh["device_used"] / mib, 1),
                   "unshared_device_used_mib": round(un["device_used"] / mib, 1),
                   "shared": {k: sh[k] for k in ("templates", "per_instance", "per_splat", "per_pair", "workspace")},
                   "copies_bytes_per_character": round(un["instance_copies"] / n_chars, 1),
                   "n_splats": int(sc.crowd.n * n_gauss),
                   "paper_mib_rtx4090": list(PAPER_TAB1_MIB[n_gauss][n_chars])}
            print(json.dumps(rec), flush=True)
            out.append(rec)
    return out


def paper_lod_leg(torch, steps, warmup, n_chars=3500, width=1920, height=1080):
    """The paper's own LoD schedule (§2): 3,500 characters from 14 templates of
    202,738 Gaussians with 12,661 / 3,176 prefixes chosen at 5 m and 10 m, on
    the grid 3 m in front of the camera, 15 looping motions, captured frames."""
    from paper_2501_17792_amd import crowdsplat as cs
    from paper_2501_17792_amd import synth

    t0 = time.perf_counter()
    sc = synth.scene_paper_lod(n_chars, width=width, height=height)
    log(f"paper LoD inputs in {time.perf_counter() - t0:.1f} s")
    lod = (cs.CS_LOD_FIXED, sc.lod_thresholds)
    ms, st, overflow = time_captured(torch, sc, True, steps, warmup, lod=lod)
    stage_ms, stp = stage_frame(torch, sc, True, lod=lod)
    med = float(np.median(ms))
    uniq = len(sc.templates) * synth.PAPER_SIZES[0]
    return {"workload": f"{n_chars} characters, 14 templates x 202,738 Gaussians SH3 with 12,661 / 3,176 "
                        f"prefixes at 5 m / 10 m, grid 3 m in front of the camera, 15 looping clips, "
                        f"{width}x{height}, captured frames, one in flight",
            "fps": round(1000.0 / med, 2), "frame_ms_median": round(med, 4),
            "frame_ms_p95": round(float(np.percentile(ms, 95)), 4),
            "gaussians_per_s": round(int(st.n_splats) * 1000.0 / med, 1), "n_splats": int(st.n_splats),
            "n_pairs": int(st.n_pairs), "level_hist": list(st.level_hist)[:3], "overflow": overflow,
            "stage_ms": {k: round(v, 4) for k, v in stage_ms.items() if k != "blend_evals"},
            "blend_evals": stage_ms["blend_evals"],
            "roofline": dominant_roofline(stage_ms, stp, sc, uniq), "paper_fps_rtx4090": 31}


def psnr(a, b):
    mse = float(np.mean((a.astype(np.float64) - b.astype(np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def fit_leg(torch, steps=2000, timed_steps=50):
    """The reconstruction-stage fit at its configuration: one 100k-Gaussian
    SH3 template, 512x512, 64 seeded cameras on a 3 m sphere, start
    perturbed (positions N(0, 1 cm), colours N(0, 0.1)), ``steps`` Adam steps
    at lr 1e-3 on every attribute, L1 + 0.2 D-SSIM, one camera per step.
    Reports the loss curve, the position error against the truth and the
    time per step (wall over the whole fit, and HIP-event times of each
    phase over ``timed_steps`` further steps). At lr 1e-3 Adam moves every
    mean about 1 mm per step whatever its gradient's size and the positions
    drift while the loss falls, so the same fit is run once more with the
    positions at lr 1e-4 (``positions_lr_1e-4``)."""
    from paper_2501_17792_amd import fit, synth

    truth, crowd, cams = synth.scene_c5()
    start = synth.perturb_template(truth, seed=502)
    # 8 views on the same sphere that the fit never sees
    center = 0.5 * (truth.mean.min(axis=0) + truth.mean.max(axis=0))
    held = synth.sphere_cameras(777, 8, center, 3.0, cams[0].width, cams[0].height)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params, losses, r = fit.fit(truth, start, crowd, cams, steps=steps, lr=1e-3, log_every=100)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r.close()
    mean = params["mean"].cpu().numpy().astype(np.float64)
    err0 = np.linalg.norm(start.mean.astype(np.float64) - truth.mean, axis=1)
    err1 = np.linalg.norm(mean - truth.mean, axis=1)
    view0, view1 = fit.view_psnr(truth, params, start, crowd, held)
    phases = {}
    _, _, r2 = fit.fit(truth, start, crowd, cams, steps=timed_steps, lr=1e-3, log_every=10 ** 9,
                       phase_times=phases)
    r2.close()
    ph = {k: round(float(np.median(v[1:])), 4) for k, v in phases.items()}
    lr = dict(mean=1e-4, log_scale=1e-3, quat=1e-3, opacity_logit=1e-3, sh=1e-3)
    params_b, losses_b, r3 = fit.fit(truth, start, crowd, cams, steps=steps, lr=lr, log_every=500)
    r3.close()
    err_b = np.linalg.norm(params_b["mean"].cpu().numpy().astype(np.float64) - truth.mean, axis=1)
    _, view_b = fit.view_psnr(truth, params_b, start, crowd, held)
    slow_pos = {"loss_curve": [[k, round(v, 6)] for k, v in losses_b],
                "held_out_view_psnr_db": {"start": round(view0, 3), "end": round(view_b, 3)},
                "position_rmse_m": {"start": round(float(np.sqrt(np.mean(err0 ** 2))), 6),
                                    "end": round(float(np.sqrt(np.mean(err_b ** 2))), 6)},
                "closer_fraction": round(float(np.mean(err_b < err0)), 4)}
    return {"workload": "one 100k-Gaussian SH3 template, 512x512, 64 cameras on a 3 m sphere, start perturbed "
                        "(positions N(0, 0.01 m), colours N(0, 0.1)), Adam lr 1e-3, L1 + 0.2 D-SSIM",
            "steps": steps, "ms_per_step_wall": round(1000.0 * wall / steps, 4),
            "phase_ms_median": ph, "loss_curve": [[k, round(v, 6)] for k, v in losses],
            "position_rmse_m": {"start": round(float(np.sqrt(np.mean(err0 ** 2))), 6),
                                "end": round(float(np.sqrt(np.mean(err1 ** 2))), 6)},
            "position_median_m": {"start": round(float(np.median(err0)), 6), "end": round(float(np.median(err1)), 6)},
            "closer_fraction": round(float(np.mean(err1 < err0)), 4),
            "held_out_view_psnr_db": {"start": round(view0, 3), "end": round(view1, 3), "views": len(held)},
            "positions_lr_1e-4": slow_pos}


# useful FLOPs of the offset network per instance-Gaussian (its per-Gaussian layers: 32 embedding inputs
# to 64, 64 to 64, 64 to 3; FMA = 2) and per instance (the pose part of the first layer, 80 to 64)
OFFSET_FLOPS_PER_SPLAT = 2 * (32 * 64 + 64 * 64 + 64 * 3)
OFFSET_FLOPS_PER_INSTANCE = 2 * 80 * 64
BF16_PEAK_TFLOPS = 2500.0  # dense bf16 matrix-core peak of one MI355X


def offsets_leg(torch, scene, poses_all, lod, tile, pose_net, timed, frames=3, blocks=(0, 0), split=1):
    """The headline frame with pose-dependent offsets: frame rate as timed
    (``timed``: captured frames in flight), then the offsets stage of eager
    instrumented frames (HIP events) against the matrix cores' bf16 peak on
    the network's useful operations, and against HBM on its compulsory bytes
    (the offsets written, 16 B per instance-Gaussian, and every template's
    embeddings read once, 64 B per Gaussian)."""
    from paper_2501_17792_amd import crowdsplat as cs

    mode, thr, mlp_ptr, margin = lod
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        r = cs.Renderer(0, stream=stream, fuse=True, profile=True, tile=tile, blocks=blocks, blend_split=split)
        r.upload_templates(scene.templates)
        r.set_crowd(scene.crowd)
        r.upload_pose_net(*pose_net)
        img = torch.zeros((3, scene.camera.height, scene.camera.width), device=poses_all.device)
        ts = []
        for k in range(frames + 1):
            r.pose_dev.copy_(poses_all[k % poses_all.shape[0]])
            r.select_lod(scene.camera, mode, thr, mlp_ptr=mlp_ptr, margin=margin)
            r.skin()
            r.render(scene.camera, img, stats=True)
            if k:
                ts.append(r.stage_times()["offsets"])
        stream.synchronize()
        n_splats = int(r.last_stats.n_splats)
        r.close()
    t = float(np.mean(ts)) * 1e-3
    flops = n_splats * OFFSET_FLOPS_PER_SPLAT + scene.crowd.n * OFFSET_FLOPS_PER_INSTANCE
    nbytes = 16 * n_splats + 64 * sum(tpl.n for tpl in scene.templates)
    mfma = flops / t / 1e12
    hbm = nbytes / t / 1e9
    return {"fps": round(1000.0 / timed["ms"], 2), "frame_ms_p95": round(float(np.percentile(timed["per"], 95)), 4),
            "overflow": timed["overflow"], "n_splats": n_splats, "offsets_ms": round(t * 1e3, 4),
            "mfma": {"achieved": round(mfma, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(mfma / BF16_PEAK_TFLOPS, 4), "flops_per_launch": int(flops)},
            "hbm": {"achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4),
                    "bytes_per_launch": int(nbytes)}}


def copy_bandwidth(torch, stream, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: the library's copy kernel over 1 GiB (read +
    write bytes per second), HIP events on its stream."""
    from paper_2501_17792_amd import crowdsplat as cs

    with torch.cuda.stream(stream):
        r = cs.Renderer(0, stream=stream)
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        r.copy(b, a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            r.copy(b, a)
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ok = bool(torch.equal(a, b))
        r.close()
        del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ok


def load_rules(path):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--stage-frames", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-offsets", action="store_true", help="skip the headline frame with pose-dependent offsets")
    ap.add_argument("--no-psnr", action="store_true", help="skip the PSNR of every rule on the held-out frames")
    ap.add_argument("--instances", type=int, default=3500)
    ap.add_argument("--net", default=os.path.join(ROOT, "paper_2501_17792_amd", "lod_net.npz"))
    ap.add_argument("--rules", default=os.path.join(ROOT, "paper_2501_17792_amd", "lod_frame_rules.json"))
    ap.add_argument("--tile", default="auto",
                    help="WxH, WxHsK (K workgroups composite each tile's rows) or 'auto' (autotuned per run)")
    ap.add_argument("--modes", default="", help="comma list of LoD modes to time (default: all)")
    ap.add_argument("--sweep", default="", choices=["", "tab2", "tab1", "paper_lod", "fit"],
                    help="instead of the headline: the Tab. 2 FPS sweep, the Tab. 1 memory sweep, the "
                         "paper's LoD schedule (one JSON line per cell), or the template fit alone")
    ap.add_argument("--no-c2", action="store_true", help="skip the 500-avatar crowd")
    ap.add_argument("--fit-steps", type=int, default=2000, help="steps of the template fit (0: skip it)")
    ap.add_argument("--frames", type=int, default=300,
                    help="frames of the animation the timed replays cycle through (1: every replay draws frame 0, "
                         "a fixed workload for counter runs)")
    ap.add_argument("--inflight", type=int, default=0,
                    help="frames in flight: contexts (one stream each) that consecutive frames alternate between "
                         "(0: from the autotuner)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner's cache (and rewrite it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    from paper_2501_17792_amd import synth

    if args.sweep:
        import torch

        if args.sweep == "tab2":
            sweep_tab2(torch, args.steps, args.warmup)
        elif args.sweep == "tab1":
            sweep_tab1(torch)
        elif args.sweep == "fit":
            print(json.dumps(dict(sweep="fit", **fit_leg(torch, args.fit_steps))), flush=True)
        else:
            print(json.dumps(dict(sweep="paper_lod", **paper_lod_leg(torch, args.steps, args.warmup))), flush=True)
        return

    t0 = time.perf_counter()
    templates = [synth.make_template(t, 100_000, 3, synth.C4_LEVELS) for t in range(14)]
    scene = synth.scene_c3(templates=templates, n_frames=300, n_inst=args.instances)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")
    netinfo = load_net(args.net)
    rules = load_rules(args.rules)
    if netinfo is None or rules is None:
        raise SystemExit("the trained network and the frame-tuned rules are needed (train_lod.py)")
    # the oracle baseline first: its process pool forks, before anything touches the GPU
    cpu = cpu_c2 = None
    if not args.no_cpu_baseline:
        from paper_2501_17792_amd import lodnet

        t0 = time.perf_counter()
        cpu = cpu_baseline(scene, lodnet.unpack(netinfo["net"]), rules["budget_margin"])
        log(f"cpu baseline in {time.perf_counter() - t0:.1f} s: {cpu['value']:.3g} FPS on {cpu['cores']} cores")
        if not args.no_c2:  # the oracle on C2's frame 0 too (500 avatars, fixed 10 / 25 m)
            sc2c = synth.scene_c2(templates=templates)
            t0 = time.perf_counter()
            cpu_c2 = cpu_baseline(sc2c, None, 0.0, levels_fn=lambda: oracle_fixed_levels(sc2c, (10.0, 10.0, 25.0, 25.0)),
                                  what="the 500-avatar crowd, fixed 10 / 25 m")
            log(f"cpu baseline (C2) in {time.perf_counter() - t0:.1f} s: {cpu_c2['value']:.3g} FPS")

    import torch

    from paper_2501_17792_amd import crowdsplat as cs
    from paper_2501_17792_amd import train_lod

    stream = torch.cuda.Stream()
    dev = torch.device("cuda", 0)
    with torch.cuda.stream(stream):
        poses_all = torch.from_numpy(scene.frame_poses[:max(1, args.frames)]).to(dev)
        net_dev = torch.from_numpy(netinfo["net"]).to(dev)
    # LoD rules, each at >= 40 dB frame PSNR against full detail on held-out frames
    modes = {
        "learned_budget": (cs.CS_LOD_BUDGET, (), net_dev.data_ptr(), rules["budget_margin"]),
        "learned_budget_visible": (cs.CS_LOD_BUDGET_VISIBLE, (), net_dev.data_ptr(),
                                   rules.get("budget_visible_margin")),
        "fixed_frame_tuned": (cs.CS_LOD_FIXED, tuple(rules["fixed_thresholds"]), 0, 0.0),
        "learned_instance_floor": (cs.CS_LOD_LEARNED, (), net_dev.data_ptr(), netinfo["margin"]),
        "fixed_10_25m": (cs.CS_LOD_FIXED, (10.0, 10.0, 25.0, 25.0), 0, 0.0),
        "full": (cs.CS_LOD_FULL, (), 0, 0.0),
    }
    if modes["learned_budget_visible"][3] is None:  # rules tuned before the visible-share rule existed
        del modes["learned_budget_visible"]
    head = "learned_budget"
    if args.modes:  # timing a subset (e.g. for a profiler run); the headline mode is always kept
        keep = set(args.modes.split(",")) | {head}
        modes = {k: v for k, v in modes.items() if k in keep}
    tile_timing = None
    blocks = (0, 0)  # (bin_blocks, sort_blocks): library defaults unless the autotuner picked others
    split = 1  # workgroups compositing one binning tile's rows (blend_split)
    inflight = args.inflight
    from paper_2501_17792_amd import autotune

    if args.tile == "auto":
        cache = os.path.join(ROOT, "paper_2501_17792_amd", "autotune_cache.json")
        if args.retune and os.path.exists(cache):
            os.remove(cache)
        tile, tuned_inflight, tile_timing = autotune.tune_frame(torch, scene, poses_all, stream, modes[head],
                                                                rule=head, cache_path=cache, log=log)
        inflight = inflight or tuned_inflight
        blocks = tuple(int(b) for b in tile_timing.get("blocks", (0, 0)))
        split = int(tile_timing.get("split", 1))
    else:
        tile, split = autotune.parse_shape(args.tile)
    inflight = inflight or 3
    log(f"tile {tile}, blend split {split}, {inflight} frames in flight")
    # frame streams: a set on which the frames in flight advance evenly (short runs of the headline frame)
    def trial(sts):
        return autotune.frames_on(torch, scene, poses_all, modes[head], tile, sts, 80, 10, blocks, split)

    streams, stream_sets = autotune.pick_streams(torch, dev, inflight, trial, log=log)

    def run(lod, n, sc=scene, poses=poses_all, pose_net=None):  # fresh contexts: capacities are fixed at capture
        with torch.cuda.stream(stream):
            imgs = [torch.zeros((3, sc.camera.height, sc.camera.width), device=dev) for _ in range(n)]
            rs = []
            for st in streams[:n]:
                r = cs.Renderer(0, stream=st, fuse=True, tile=tile, blocks=blocks, blend_split=split)
                r.upload_templates(sc.templates)
                r.set_crowd(sc.crowd)
                if pose_net is not None:
                    r.upload_pose_net(*pose_net)
                rs.append(r)
            torch.cuda.synchronize()
            out = time_mode(torch, rs, sc, poses, imgs, streams[:n], lod, args.steps, args.warmup)
            for r in rs:
                r.close()
            del imgs
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        return out

    results = {}
    for name, lod in modes.items():
        results[name] = run(lod, len(streams))
        log(f"{name}: {1000.0 / results[name]['ms']:.1f} FPS, {results[name]['stats'].n_splats} splats, "
            f"{results[name]['stats'].n_pairs} pairs")
    single = run(modes[head], 1) if len(streams) > 1 else results[head]
    log(f"{head}, one frame in flight: {1000.0 / single['ms']:.1f} FPS")
    # the fixed 10 / 25 m rule on the 500-avatar, 50 x 50 m crowd (3 of the 5 levels: 100 / 25 / 6.25 %)
    c2 = None
    if not args.no_c2:
        sc2 = synth.scene_c2(templates=templates)
        with torch.cuda.stream(stream):
            poses2 = torch.from_numpy(np.ascontiguousarray(sc2.crowd.pose[None], np.float32)).to(dev)
        c2 = run((cs.CS_LOD_FIXED, (10.0, 10.0, 25.0, 25.0), 0, 0.0), len(streams), sc=sc2, poses=poses2)
        log(f"500 avatars, 10/25 m: {1000.0 / c2['ms']:.1f} FPS")

    # the headline frame with pose-dependent offsets (synthetic offset network and embeddings)
    offsets = None
    if not args.no_offsets:
        pn = (synth.pose_net_weights(), [synth.pose_embeddings(1200 + t, tpl.n) for t, tpl in enumerate(scene.templates)])
        ro = run(modes[head], len(streams), pose_net=pn)
        offsets = offsets_leg(torch, scene, poses_all, modes[head], tile, pn, ro, blocks=blocks, split=split)
        log(f"{head} with pose-dependent offsets: {offsets['fps']:.1f} FPS, offsets stage {offsets['offsets_ms']:.3f} ms")

    res = results[head]
    ms = res["ms"]
    fps = 1000.0 / ms
    st0 = res["stats"]
    n_splats, n_pairs = int(st0.n_splats), int(st0.n_pairs)
    lod_head = modes[head]

    # ---- per-stage timing: instrumented eager frames (HIP events on the launch
    # stream around each stage, blend evaluations counted). First the timed
    # configuration (skinning fused into projection), then separate skinning.
    def stage_profile(fuse, count=False):
        with torch.cuda.stream(stream):
            img = torch.zeros((3, scene.camera.height, scene.camera.width), device=dev)
            rp = cs.Renderer(0, stream=stream, fuse=fuse, profile=True, tile=tile, count_blend=count, blocks=blocks,
                             blend_split=split)
            rp.upload_templates(scene.templates)
            rp.set_crowd(scene.crowd)
            lvl_out = torch.zeros(scene.crowd.n, dtype=torch.int32, device=dev)
            acc, evals = {}, []
            for k in range(args.stage_frames + 1):
                rp.pose_dev.copy_(poses_all[k % poses_all.shape[0]])
                rp.select_lod(scene.camera, lod_head[0], lod_head[1], level_out=lvl_out, mlp_ptr=lod_head[2],
                              margin=lod_head[3])
                rp.skin()
                rp.render(scene.camera, img, stats=True)
                t = rp.stage_times()
                if k > 0:
                    for name, v in t.items():
                        acc.setdefault(name, []).append(v)
                    evals.append((int(rp.last_stats.blend_evals), int(rp.last_stats.blend_eval_slots),
                                  int(rp.last_stats.n_pairs), t.get("blend", 0.0),
                                  int(rp.last_stats.blend_done_slots), int(rp.last_stats.blend_adds)))
            stream.synchronize()
            stp = rp.last_stats
            rp.close()
        return {k: float(np.mean(v)) for k, v in acc.items()}, lvl_out.cpu().numpy().astype(np.int64), stp, evals

    stage_ms, levels, stp, _ = stage_profile(True)
    stage_unfused, _, _, _ = stage_profile(False)
    _, _, _, evals = stage_profile(True, count=True)  # the counting blend is slower: only its counts are used
    uniq = unique_template_gaussians(scene, levels)
    stats = dict(n_splats=int(stp.n_splats), n_pairs=int(stp.n_pairs))
    stage_ms = {("project_fused" if k == "project" else k): v for k, v in stage_ms.items()}
    stage_ms["skin"] = stage_unfused.get("skin", 0.0)
    stage_ms["project"] = stage_unfused.get("project", 0.0)
    stage_gbs = {}
    for name in ("skin", "project", "project_fused", "emit", "sort", "segsort"):
        if stage_ms.get(name, 0.0) > 0:
            stage_gbs[name] = algorithmic_bytes(name, stats, scene, uniq) / (stage_ms[name] * 1e-3) / 1e9
    ev = np.array(evals, np.float64)
    blend_ms = stage_ms["blend"]  # the uncounting kernel of the same frames
    blend = {"evals_per_frame": int(ev[:, 0].mean()), "eval_slots_per_frame": int(ev[:, 1].mean()),
             "pairs_per_frame": int(ev[:, 2].mean()), "blend_ms": round(blend_ms, 4),
             "evals_per_s_per_cu": round(float(ev[:, 0].mean() / (blend_ms * 1e-3)) / N_CU, 1),
             "eval_slots_per_s_per_cu": round(float(ev[:, 1].mean() / (blend_ms * 1e-3)) / N_CU, 1),
             "live_fraction_of_slots": round(float(ev[:, 0].sum() / max(ev[:, 1].sum(), 1.0)), 4),
             "evals_per_pair": round(float(ev[:, 0].sum() / max(ev[:, 2].sum(), 1.0)), 3),
             # idle slots: lanes of finished pixels, and lanes past their group's list while another
             # group of the wave still walks its own
             "finished_fraction_of_slots": round(float(ev[:, 4].sum() / max(ev[:, 1].sum(), 1.0)), 4),
             "past_list_fraction_of_slots": round(float((ev[:, 1] - ev[:, 0] - ev[:, 4]).sum()
                                                        / max(ev[:, 1].sum(), 1.0)), 4),
             "adds_per_frame": int(ev[:, 5].mean())}
    roofline = frame_roofline(stage_ms, stats, scene, uniq, tile, split, blend)
    copy_gbs, copy_ok = copy_bandwidth(torch, stream)
    fit_res = None
    if args.fit_steps > 0:
        t0 = time.perf_counter()
        fit_res = fit_leg(torch, args.fit_steps)
        log(f"fit: {fit_res['ms_per_step_wall']:.2f} ms/step, position RMSE {fit_res['position_rmse_m']} "
            f"({time.perf_counter() - t0:.1f} s)")
    if roofline.get("hbm"):
        roofline["hbm"]["frac_of_copy"] = round(roofline["hbm"]["achieved"] / copy_gbs, 4)
    stage_copy_frac = {k: round(v / copy_gbs, 4) for k, v in stage_gbs.items()}

    # ---- quality: every rule's frames against full-detail frames, on the
    # frames the rules were not tuned on (and on frame 0)
    quality = {}
    if not args.no_psnr:
        hold = tuple(rules["hold_frames"])
        judge = train_lod.FrameJudge(torch, scene, hold + (0,), tile, lag=len(streams))
        for name, lod in modes.items():
            p_min, g_mean = judge.evaluate(lod, hold)
            p0, _ = judge.evaluate(lod, (0,))
            quality[name] = {"min_psnr_held_out_db": round(p_min, 2), "psnr_frame0_db": round(p0, 2),
                             "held_out_frames": len(hold)}
        judge.close()

    lod_cmp = {}
    for name, rr in results.items():
        lod_cmp[name] = {"fps": round(1000.0 / rr["ms"], 2), "frame_ms_p95": round(float(np.percentile(rr["per"], 95)), 4),
                         "n_splats": int(rr["stats"].n_splats), "n_pairs": int(rr["stats"].n_pairs),
                         "level_hist": list(rr["stats"].level_hist)[:5], "overflow": rr["overflow"]}
        lod_cmp[name].update(quality.get(name, {}))
    out = {
        "metric": METRIC, "value": round(fps, 2), "unit": "FPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3,500 animated avatars, 14 templates x 100k Gaussians SH3 with 5 LoD levels "
                               "(100/50/25/12.5/6.25%), 1920x1080, 300-frame keyframed animation, learned LoD "
                               "with a frame budget of 40 dB PSNR against full detail, hipGraph-captured frame "
                               "(pose upload inside), frames in flight on separate contexts",
                   "lod": head, "instances": scene.crowd.n, "width": scene.camera.width,
                   "height": scene.camera.height, "tile": list(tile), "blend_split": split,
                   "blocks": list(blocks)},
        "autotune": tile_timing,
        "frames_in_flight": len(streams), "frame_stream_sets_tried": stream_sets,
        "frame_ms_median": round(float(np.median(res["per"])), 4),
        "frame_ms_p95": round(float(np.percentile(res["per"], 95)), 4),
        "one_frame_in_flight": {"fps": round(1000.0 / single["ms"], 2), "frame_ms": round(single["ms"], 4)},
        "gaussians_per_s": round(n_splats * fps, 1), "n_splats": n_splats, "n_pairs": n_pairs,
        "n_visible": int(st0.n_visible), "level_hist": list(st0.level_hist)[:5],
        "lod_comparison": lod_cmp,
        "lod_rules": {"budget_margin_db": rules["budget_margin"], "fixed_thresholds_m": rules["fixed_thresholds"],
                      "tuned_on_frames": rules["tune_frames"], "target_db": rules.get("target_db")},
        "c2_500_avatars_fixed_10_25m": None if c2 is None else {
            "fps": round(1000.0 / c2["ms"], 2), "n_splats": int(c2["stats"].n_splats),
            "n_pairs": int(c2["stats"].n_pairs), "overflow": c2["overflow"],
            "level_hist": list(c2["stats"].level_hist)[:5]},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_gbs": {k: round(v, 1) for k, v in stage_gbs.items()},
        "copy_gbs": round(copy_gbs, 1), "copy_ok": copy_ok, "stage_frac_of_copy": stage_copy_frac,
        "blend": blend, "fit": fit_res, "pose_offsets": offsets,
        "roofline": roofline, "cpu_baseline": cpu, "cpu_baseline_c2": cpu_c2,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
