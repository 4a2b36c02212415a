"""Differentiable rendering of one template and the template fit.

``CrowdSplatFn`` is a torch.autograd.Function whose forward renders a frame
through the C ABI (skin -> project -> sort -> blend) from the template's
attribute tensors and whose backward is the library's hand-written backward
rasteriser (cs_render_backward). ``fit`` reproduces the reconstruction
stage's optimisation on synthetic targets: each step renders the template
from one camera, evaluates L1 + 0.2 (1 - SSIM) against the target render
(cs_fit_loss), back-propagates through CrowdSplatFn and applies Adam
(cs_adam). Every arithmetic step runs in the library's kernels; torch holds
the tensors and the autograd bookkeeping.
"""
from __future__ import annotations

import math

import numpy as np

from . import crowdsplat as cs
from . import synth

PARAMS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def _torch():
    import torch

    return torch


def make_function():
    torch = _torch()

    class CrowdSplatFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, renderer, cam, skin_idx, skin_w, mean, log_scale, quat, opacity_logit, sh):
            renderer.update_template(0, mean.detach(), log_scale.detach(), quat.detach(), opacity_logit.detach(),
                                     sh.detach(), skin_idx, skin_w, opacity_is_logit=True)
            renderer.select_lod(cam, cs.CS_LOD_FULL, ())
            renderer.skin()
            img = renderer.render(cam)
            ctx.renderer = renderer
            return img

        @staticmethod
        def backward(ctx, dimg):
            g = ctx.renderer.render_backward(dimg.contiguous(), 0)
            return (None, None, None, None, g["mean"], g["log_scale"], g["quat"], g["opacity_logit"], g["sh"])

    return CrowdSplatFn


def template_tensors(t: synth.Template, device):
    torch = _torch()
    o = np.clip(t.opacity.astype(np.float64), 1e-6, 1 - 1e-6)
    logit = np.log(o / (1 - o)).astype(np.float32)
    out = dict(mean=t.mean, log_scale=t.log_scale, quat=t.quat, opacity_logit=logit, sh=t.sh)
    out = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device) for k, v in out.items()}
    out["skin_idx"] = torch.from_numpy(np.ascontiguousarray(t.skin_idx)).to(device)
    out["skin_w"] = torch.from_numpy(np.ascontiguousarray(t.skin_w, np.float32)).to(device)
    return out


def render_targets(r, cams):
    return [r.frame(c, cs.CS_LOD_FULL, ()).clone() for c in cams]


def fit(truth: synth.Template, start: synth.Template, crowd, cams, steps=2000, lr=1e-3, lam=0.2, seed=503,
        log=None, log_every=100, phase_times=None, tile=(8, 8)):
    """Fit ``start`` to renders of ``truth`` from ``cams``; returns the fitted
    tensors and the loss history. ``lr`` is one rate for every attribute or a
    dict per attribute (mean, log_scale, quat, opacity_logit, sh). With a
    dict ``phase_times``, every step's forward render, loss, backward and Adam
    update are timed with HIP events on the renderer's stream (ms lists).
    ``tile``: the tile shape of the forward and backward rasterisers (8x8:
    the backward walks each tile's list once per wave, pair after pair, so
    its longest tiles set the step time; at 512x512 a 100k-Gaussian step
    measured 4.5 ms at 8x8 against 6.6 ms at 16x16)."""
    lrs = lr if isinstance(lr, dict) else {k: lr for k in PARAMS}
    torch = _torch()
    r = cs.Renderer(0, tile=tile)
    r.upload_templates([truth])
    r.set_crowd(crowd)
    targets = render_targets(r, cams)
    r.upload_templates([start])
    P = template_tensors(start, r.device)
    params = {k: P[k].clone().requires_grad_(True) for k in PARAMS}
    m = {k: torch.zeros_like(params[k]) for k in PARAMS}
    v = {k: torch.zeros_like(params[k]) for k in PARAMS}
    Fn = make_function()
    order = np.random.default_rng(seed).permutation(len(cams))
    losses = []
    ev = None
    if phase_times is not None:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        for name in ("forward", "loss", "backward", "adam"):
            phase_times.setdefault(name, [])
    for step in range(1, steps + 1):
        c = int(order[(step - 1) % len(cams)])
        if ev:
            ev[0].record(r.stream)
        img = Fn.apply(r, cams[c], P["skin_idx"], P["skin_w"], *[params[k] for k in PARAMS])
        if ev:
            ev[1].record(r.stream)
        loss, dimg = r.fit_loss(img.detach(), targets[c], lam)
        if ev:
            ev[2].record(r.stream)
        for k in PARAMS:
            params[k].grad = None
        img.backward(dimg)
        if ev:
            ev[3].record(r.stream)
        with torch.no_grad():
            for k in PARAMS:
                r.adam(params[k], params[k].grad.contiguous(), m[k], v[k], step, lrs[k])
        if ev:
            ev[4].record(r.stream)
            ev[4].synchronize()
            for i, name in enumerate(("forward", "loss", "backward", "adam")):
                phase_times[name].append(ev[i].elapsed_time(ev[i + 1]))
        if step % log_every == 0 or step == 1:
            losses.append((step, float(loss.item())))
            if log:
                log(f"step {step} loss {losses[-1][1]:.5f}")
    return {k: params[k].detach() for k in PARAMS}, losses, r


def view_psnr(truth: synth.Template, fitted, start: synth.Template, crowd, cams):
    """PSNR (dB, over all pixels of ``cams``) of renders of the fitted
    attribute tensors ``fitted`` (as ``fit`` returns them) and of ``start``
    against renders of ``truth``: the image-space measure of a fit, on views
    it was not fitted to. Returns (start dB, fitted dB)."""
    torch = _torch()
    r = cs.Renderer(0)
    try:
        r.upload_templates([truth])
        r.set_crowd(crowd)
        refs = render_targets(r, cams)
        r.upload_templates([start])
        first = render_targets(r, cams)
        P = template_tensors(start, r.device)
        r.update_template(0, fitted["mean"], fitted["log_scale"], fitted["quat"], fitted["opacity_logit"],
                          fitted["sh"], P["skin_idx"], P["skin_w"], opacity_is_logit=True)
        last = render_targets(r, cams)

        def db(imgs):
            mse = sum(float(torch.mean((a - b) ** 2).item()) for a, b in zip(imgs, refs)) / len(refs)
            return float("inf") if mse == 0.0 else -10.0 * math.log10(mse)

        return db(first), db(last)
    finally:
        r.close()
