"""Tile-shape autotuner for the captured frame.

The image does not depend on the tile shape (the footprint is the exact
alpha >= 1/255 box, so every pixel walks the same splats in the same order
whatever the tiling), so the tuner is free to pick the fastest shape: it
captures the whole frame once per candidate, times a few replays with HIP
events on the frame's stream, and keeps the fastest. Results are cached in a
JSON file keyed by (device name, width, height, instance count bucket).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import crowdsplat as cs

CANDIDATES = [(16, 16), (8, 8), (16, 8), (8, 16), (32, 8), (32, 16), (16, 32)]


def cache_key(torch, width, height, n_inst):
    name = torch.cuda.get_device_name(0).replace(" ", "_")
    bucket = 1 << int(np.ceil(np.log2(max(n_inst, 1))))
    return f"{name}:{width}x{height}:n{bucket}"


def tune(torch, scene, poses_all, stream, lod, frames: int = 20, candidates=CANDIDATES,
         cache_path: str | None = None, log=None):
    """Returns (best tile, {tile: ms per frame})."""
    key = cache_key(torch, scene.camera.width, scene.camera.height, scene.crowd.n)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return tuple(cache[key]["tile"]), cache[key]["ms"]
    mode, thr, mlp_ptr, margin = lod
    timing = {}
    for tile in candidates:
        with torch.cuda.stream(stream):
            r = cs.Renderer(0, stream=stream, tile=tile, fuse=True)
            r.upload_templates(scene.templates)
            r.set_crowd(scene.crowd)
            img = torch.zeros((3, scene.camera.height, scene.camera.width), device=poses_all.device)
            r.pose_dev.copy_(poses_all[0])
            try:
                r.select_lod(scene.camera, mode, thr, mlp_ptr=mlp_ptr, margin=margin)
                r.skin()
                r.render(scene.camera, img, stats=True)
                st = r.last_stats
                r.reserve(0, int(st.n_splats * 1.05) + 1024, int(st.n_pairs * 1.2) + 65536)
                r.capture(scene.camera, img, mode, thr, mlp_ptr=mlp_ptr, margin=margin)
            except cs.CrowdSplatError as e:  # the shape does not fit (e.g. too many tile pairs)
                r.close()
                timing[f"{tile[0]}x{tile[1]}"] = None
                if log:
                    log(f"tile {tile}: skipped ({e})")
                continue
            for k in range(3):
                r.launch()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for k in range(frames):
                r.pose_dev.copy_(poses_all[k % poses_all.shape[0]])
                r.launch()
            e1.record(stream)
            stream.synchronize()
            ok = r.poll().overflow == 0
            r.close()
        ms = e0.elapsed_time(e1) / frames
        timing[f"{tile[0]}x{tile[1]}"] = round(ms, 4) if ok else None
        if log:
            log(f"tile {tile}: {ms:.3f} ms/frame{'' if ok else ' (overflow, discarded)'}")
    valid = {k: v for k, v in timing.items() if v is not None}
    best = min(valid, key=valid.get)
    tile = tuple(int(x) for x in best.split("x"))
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {"tile": list(tile), "ms": timing}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return tile, timing
