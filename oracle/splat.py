"""FP64 Gaussian-splatting renderer (oracle).

CrowdSplat §2 renders all characters with the 3D Gaussian Splatting
rasteriser (Kerbl et al. 2023): project each 3D Gaussian to a 2D screen-space
Gaussian (EWA splatting, the local affine approximation of the perspective
map), bin it into the screen tiles its footprint touches, sort every tile's
list front to back, and alpha-composite per pixel. The constants are that
renderer's: alpha clamped to 0.99, contributions below 1/255 skipped, and a
pixel stops before its transmittance would fall below 1e-4.

Readings where the paper is silent (the same ones the GPU library takes):
* pinhole camera, vertical field of view, pixel centres at +1/2, near plane
  0.2 m, a 1.5x guard band on the normalised image coordinates;
* the screen-space covariance gets +0.3 px^2 on its diagonal (low-pass
  filter) with no opacity compensation;
* the footprint is the exact bounding box of the alpha >= 1/255 ellipse,
  widened by 1e-4 relative and 0.01 px, so that the image does not depend on
  the tile shape;
* colour = max(0, 0.5 + sum_k sh_k Y_k(d)), with d the viewing direction in
  the Gaussian's canonical frame (L^T (mu' - eye), normalised) and Y_k the
  real orthonormal spherical harmonics without the Condon-Shortley phase;
* sort key = (tile << 31) | bits(float32(depth)); ties keep emission order
  (instance-major, then Gaussian, then tiles row-major);
* the exponent is clamped to <= 0; the splat that would take T below 1e-4 is
  not added.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4
LOWPASS = 0.3
GUARD = 1.5
RECT_REL = 1e-4
RECT_ABS = 0.01


# ----------------------------------------------------------------------------
# spherical harmonics
# ----------------------------------------------------------------------------

def sh_basis(d: np.ndarray, degree: int) -> np.ndarray:
    """Real orthonormal SH (no Condon-Shortley phase, polar axis +z) at unit
    directions d [N,3]; column k = l^2 + l + m. Returns [N,(degree+1)^2]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    cols = [np.full_like(x, 0.5 * math.sqrt(1.0 / pi))]
    if degree >= 1:
        c = math.sqrt(3.0 / (4.0 * pi))
        cols += [c * y, c * z, c * x]
    if degree >= 2:
        cols += [0.5 * math.sqrt(15.0 / pi) * x * y,
                 0.5 * math.sqrt(15.0 / pi) * y * z,
                 0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),
                 0.5 * math.sqrt(15.0 / pi) * x * z,
                 0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if degree >= 3:
        cols += [0.25 * math.sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y),
                 0.5 * math.sqrt(105.0 / pi) * x * y * z,
                 0.25 * math.sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0),
                 0.25 * math.sqrt(7.0 / pi) * (5.0 * z ** 3 - 3.0 * z),
                 0.25 * math.sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0),
                 0.25 * math.sqrt(105.0 / pi) * z * (x * x - y * y),
                 0.25 * math.sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y)]
    return np.stack(cols, axis=1)


def colour(sh, mu, L, eye, degree: int) -> np.ndarray:
    """rgb [N,3] = max(0, 0.5 + sum_k sh_k Y_k(normalise(L^T (mu - eye))))."""
    v = np.asarray(mu, np.float64) - np.asarray(eye, np.float64)
    d = np.einsum("nji,nj->ni", np.asarray(L, np.float64), v)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = sh_basis(d, degree)
    sh = np.asarray(sh, np.float64)[:, : (degree + 1) ** 2, :]
    return np.maximum(0.0, 0.5 + np.einsum("nk,nkc->nc", Y, sh))


# ----------------------------------------------------------------------------
# projection and footprint
# ----------------------------------------------------------------------------

def project(mu, cov, cam):
    """EWA projection of posed Gaussians. Returns a dict of FP64 arrays:
    t (camera-space mean), u, v, cov2d (a, b, c), conic (A, B, C) and the
    visibility mask after the near-plane, guard-band and determinant culls."""
    mu = np.asarray(mu, np.float64)
    cov = np.asarray(cov, np.float64)
    R = np.asarray(cam.R, np.float64)
    t = (mu - np.asarray(cam.eye, np.float64)) @ R.T
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    ok = tz > cam.near
    tzs = np.where(ok, tz, 1.0)
    xn, yn = tx / tzs, ty / tzs
    ok &= np.abs(xn) <= GUARD * cam.width / (2.0 * cam.fx)
    ok &= np.abs(yn) <= GUARD * cam.height / (2.0 * cam.fy)
    u = cam.fx * xn + cam.cx
    v = cam.fy * yn + cam.cy
    J = np.zeros((mu.shape[0], 2, 3))
    J[:, 0, 0] = cam.fx / tzs
    J[:, 0, 2] = -cam.fx * tx / (tzs * tzs)
    J[:, 1, 1] = cam.fy / tzs
    J[:, 1, 2] = -cam.fy * ty / (tzs * tzs)
    T = J @ R
    S = np.einsum("nij,njk,nlk->nil", T, cov, T)
    a = S[:, 0, 0] + LOWPASS
    b = S[:, 0, 1]
    c = S[:, 1, 1] + LOWPASS
    det = a * c - b * b
    ok &= det > 0
    dets = np.where(det > 0, det, 1.0)
    return dict(t=t, u=u, v=v, depth=tz, a=a, b=b, c=c,
                A=c / dets, B=-b / dets, C=a / dets, visible=ok)


def footprint(u, v, a, c, opacity, visible, width, height, tw, th):
    """Opacity-aware pixel AABB half-extents, tile rect [x0, y0, x1, y1]
    (inclusive, in tiles) and tile count; culls alpha-invisible and off-screen
    splats. Also returns the four pre-floor pixel bounds."""
    o = np.asarray(opacity, np.float64)
    vis = np.asarray(visible, bool) & (o >= ALPHA_MIN)
    k = 2.0 * np.log(np.maximum(255.0 * o, 1.0)) * (1.0 + RECT_REL)
    rx = np.sqrt(k * a) + RECT_ABS
    ry = np.sqrt(k * c) + RECT_ABS
    bounds = np.stack([u - rx, v - ry, u + rx, v + ry], axis=1)
    px0, py0 = np.floor(u - rx), np.floor(v - ry)
    px1, py1 = np.floor(u + rx), np.floor(v + ry)
    vis &= (px1 >= 0) & (px0 <= width - 1) & (py1 >= 0) & (py0 <= height - 1)
    px0 = np.clip(px0, 0, width - 1).astype(np.int64)
    px1 = np.clip(px1, 0, width - 1).astype(np.int64)
    py0 = np.clip(py0, 0, height - 1).astype(np.int64)
    py1 = np.clip(py1, 0, height - 1).astype(np.int64)
    rect = np.stack([px0 // tw, py0 // th, px1 // tw, py1 // th], axis=1)
    count = np.where(vis, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)
    return dict(rx=rx, ry=ry, rect=rect, count=count.astype(np.int64),
                visible=vis, bounds=bounds)


def footprint_rect_f32(u, v, rx, ry, depth, width, height, tw, th):
    """The integer part of the footprint taken in float32, the precision the
    renderer decides it in: from a splat's float32 screen centre (u, v), box
    half-extents (rx, ry) and depth (0 = culled before the footprint), the
    pixel bounds floor(u - rx), floor(u + rx), ... come from float32
    subtractions (IEEE round to nearest), then the off-screen cull, the clamp
    to the image and the integer division by the tile size of ``footprint``.
    Returns (rect [N,4], count [N], visible [N])."""
    f32 = np.float32
    u, v = np.asarray(u, f32), np.asarray(v, f32)
    rx, ry = np.asarray(rx, f32), np.asarray(ry, f32)
    vis = np.asarray(depth, np.float64) > 0.0
    px0 = np.floor(u - rx).astype(np.float64)
    px1 = np.floor(u + rx).astype(np.float64)
    py0 = np.floor(v - ry).astype(np.float64)
    py1 = np.floor(v + ry).astype(np.float64)
    vis &= (px1 >= 0) & (px0 <= width - 1) & (py1 >= 0) & (py0 <= height - 1)
    px0 = np.clip(px0, 0, width - 1).astype(np.int64)
    px1 = np.clip(px1, 0, width - 1).astype(np.int64)
    py0 = np.clip(py0, 0, height - 1).astype(np.int64)
    py1 = np.clip(py1, 0, height - 1).astype(np.int64)
    rect = np.stack([px0 // tw, py0 // th, px1 // tw, py1 // th], axis=1)
    rect[~vis] = 0
    count = np.where(vis, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)
    return rect, count.astype(np.int64), vis


# ----------------------------------------------------------------------------
# binning and the stable (tile | depth) sort
# ----------------------------------------------------------------------------

def depth_bits(depth) -> np.ndarray:
    """The IEEE-754 bit pattern of float32(depth) as uint64 (depth > 0)."""
    return np.asarray(depth, np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)


def emit_pairs(rect, count, visible, depth, n_tiles_x):
    """(key, value) pairs in emission order: splat-major, tiles row-major.
    key = (tile << 31) | depth bits; value = splat index."""
    rect = np.asarray(rect, np.int64)
    splats = np.nonzero(visible)[0]
    cnt = np.asarray(count, np.int64)[splats]
    s_rep = np.repeat(splats, cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(s_rep.shape[0], dtype=np.int64) - first
    width = rect[s_rep, 2] - rect[s_rep, 0] + 1
    ty = rect[s_rep, 1] + local // width
    tx = rect[s_rep, 0] + local % width
    tile = (ty * n_tiles_x + tx).astype(np.uint64)
    keys = (tile << np.uint64(31)) | depth_bits(depth)[s_rep]
    return keys, s_rep.astype(np.uint32)


def sort_pairs(keys, vals):
    """Stable ascending sort by key (ties keep emission order)."""
    order = np.argsort(keys, kind="stable")
    return keys[order], vals[order]


def tile_ranges(sorted_keys, n_tiles: int) -> np.ndarray:
    """[start, end) into the sorted pairs for every tile, [n_tiles, 2]."""
    tiles = (np.asarray(sorted_keys, np.uint64) >> np.uint64(31)).astype(np.int64)
    idx = np.arange(n_tiles)
    start = np.searchsorted(tiles, idx, side="left")
    end = np.searchsorted(tiles, idx, side="right")
    return np.stack([start, end], axis=1)


# ----------------------------------------------------------------------------
# compositing
# ----------------------------------------------------------------------------

def _blend_list(px, py, order, sp, bg, fragile_alpha, fragile_t, tie_impact=None):
    """Front-to-back compositing of the splats ``order`` at pixel centres
    (px + 1/2, py + 1/2). Returns colour [3,P], final T [P], fragile [P] and
    the number of splats added per pixel.

    The fragile mask marks pixels where a float32 renderer may legitimately
    take a different discrete decision: alpha within ``fragile_alpha``
    (relative) of 1/255, T' within ``fragile_t`` (relative) of 1e-4, and, if
    ``tie_impact`` is given, two consecutive alpha >= 1/255 splats whose depths
    agree within their float32 error bound ``sp["depth_eps"]`` (their order is
    then not fixed by float32 depths) when swapping them would move the pixel
    by more than ``tie_impact`` (a swap changes it by T a1 a2 |c1 - c2|) or one
    of them is the splat that stops the pixel."""
    P = px.shape[0]
    T = np.ones(P)
    C = np.zeros((3, P))
    done = np.zeros(P, bool)
    fragile = np.zeros(P, bool)
    n_added = np.zeros(P, np.int64)
    cx, cy = px + 0.5, py + 0.5
    last = np.full(P, -1, np.int64)      # previous alpha >= 1/255 splat
    last_a = np.zeros(P)
    last_T = np.ones(P)                  # T before that splat
    for s in order:
        if done.all():
            break
        dx = cx - sp["u"][s]
        dy = cy - sp["v"][s]
        power = -0.5 * (sp["A"][s] * dx * dx + 2.0 * sp["B"][s] * dx * dy
                        + sp["C"][s] * dy * dy)
        power = np.minimum(0.0, power)
        raw = sp["opacity"][s] * np.exp(power)
        alpha = np.minimum(ALPHA_MAX, raw)
        live = ~done
        fragile |= live & (np.abs(raw - ALPHA_MIN) <= fragile_alpha * ALPHA_MIN)
        use = live & (alpha >= ALPHA_MIN)
        Tn = T * (1.0 - alpha)
        fragile |= use & (np.abs(Tn - T_MIN) <= fragile_t * T_MIN)
        stop = use & (Tn < T_MIN)
        if tie_impact is not None:
            has = use & (last >= 0)
            if has.any():
                lp = np.where(has, last, 0)
                tie = has & (np.abs(sp["depth"][lp] - sp["depth"][s])
                             <= sp["depth_eps"][lp] + sp["depth_eps"][s])
                if tie.any():
                    dc = np.abs(sp["rgb"][lp] - sp["rgb"][s][None, :]).max(axis=1)
                    impact = last_T * last_a * alpha * dc
                    fragile |= tie & (stop | (impact > tie_impact))
            last = np.where(use, s, last)
            last_a = np.where(use, alpha, last_a)
            last_T = np.where(use, T, last_T)
        done |= stop
        add = use & ~stop
        C += np.where(add, sp["rgb"][s][:, None] * (alpha * T), 0.0)
        T = np.where(add, Tn, T)
        n_added += add
    C += T[None, :] * np.asarray(bg, np.float64)[:, None]
    return C, T, fragile, n_added


def _alpha_raw(sp, s, cx, cy):
    """Unclamped opacity o e^power of splats ``s`` at pixel centres (cx, cy)
    (pixels along axis 0, splats along axis 1)."""
    dx = cx[:, None] - sp["u"][s][None, :]
    dy = cy[:, None] - sp["v"][s][None, :]
    power = -0.5 * (sp["A"][s][None] * dx * dx + 2.0 * sp["B"][s][None] * dx * dy
                    + sp["C"][s][None] * dy * dy)
    return sp["opacity"][s][None] * np.exp(np.minimum(0.0, power))


def _blend_list_chunked(px, py, order, sp, bg, fragile_alpha, fragile_t, chunk=2048, sp_alt=None,
                        power_ulps=0.0):
    """The same front-to-back walk as ``_blend_list`` (without the tie test),
    taken ``chunk`` splats at a time for every still-unfinished pixel at once,
    for lists of millions of splats. Each pixel's transmittance before splat k
    is the running product T0 (1 - a_0) (1 - a_1) ... over the splats it adds,
    formed in the loop's order (np.cumprod multiplies left to right), and its
    colour the running sum of the added c a T, also in the loop's order
    (np.cumsum), so the results equal the loop's bit for bit.

    ``sp_alt``: a second record set for the same splats (e.g. a float32
    renderer's records, upcast). The walk follows ``sp``; the fragile bands
    then widen, splat by splat and pixel by pixel, by how far the two record
    sets put alpha and T' apart (T' of ``sp_alt`` taken under ``sp``'s
    decisions): a decision is fragile where the two record sets, or a
    renderer within the base band of either, could take it differently.

    ``power_ulps``: the alpha band also widens by that many float32 units in
    the last place (2^-24, relative) of the exponent's terms,
    (A dx^2 + 2 |B dx dy| + C dy^2) / 2: a float32 evaluation of the exponent
    errs by about that much, which is far more than the base band for thin
    splats whose terms cancel."""
    P = px.shape[0]
    T = np.ones(P)
    C = np.zeros((3, P))
    done = np.zeros(P, bool)
    fragile = np.zeros(P, bool)
    n_added = np.zeros(P, np.int64)
    T_alt = np.ones(P)
    cx, cy = px + 0.5, py + 0.5
    order = np.asarray(order, np.int64)
    for c0 in range(0, order.shape[0], chunk):
        live = np.nonzero(~done)[0]
        if live.size == 0:
            break
        s = order[c0:c0 + chunk]
        K = s.shape[0]
        dx = cx[live, None] - sp["u"][s][None, :]
        dy = cy[live, None] - sp["v"][s][None, :]
        power = -0.5 * (sp["A"][s][None] * dx * dx + 2.0 * sp["B"][s][None] * dx * dy
                        + sp["C"][s][None] * dy * dy)
        power = np.minimum(0.0, power)
        raw = sp["opacity"][s][None] * np.exp(power)
        alpha = np.minimum(ALPHA_MAX, raw)
        use = alpha >= ALPHA_MIN
        factor = np.where(use, 1.0 - alpha, 1.0)
        # transmittance before each splat (the first column is T itself)
        Tb = np.cumprod(np.concatenate([T[live, None], factor], axis=1), axis=1)
        Tn = Tb[:, :-1] * (1.0 - alpha)
        Tb = Tb[:, :-1]
        stop = use & (Tn < T_MIN)
        has_stop = stop.any(axis=1)
        k_stop = np.where(has_stop, np.argmax(stop, axis=1), K)
        k = np.arange(K)[None, :]
        evaluated = k <= k_stop[:, None]          # the stopping splat is evaluated, not added
        add = use & (k < k_stop[:, None])
        band_a = fragile_alpha * ALPHA_MIN
        band_t = fragile_t * T_MIN
        if power_ulps:
            mag = 0.5 * (sp["A"][s][None] * dx * dx + 2.0 * np.abs(sp["B"][s][None] * dx * dy)
                         + sp["C"][s][None] * dy * dy)
            band_a = band_a + ALPHA_MIN * power_ulps * 2.0 ** -24 * mag
        if sp_alt is not None:
            raw_alt = _alpha_raw(sp_alt, s, cx[live], cy[live])
            alpha_alt = np.minimum(ALPHA_MAX, raw_alt)
            fac_alt = np.where(use, 1.0 - alpha_alt, 1.0)
            Tb_alt = np.cumprod(np.concatenate([T_alt[live, None], fac_alt], axis=1), axis=1)
            Tn_alt = Tb_alt[:, :-1] * (1.0 - alpha_alt)
            band_a = band_a + np.abs(raw - raw_alt)
            band_t = band_t + np.abs(Tn - Tn_alt)
            T_alt[live] = np.cumprod(np.concatenate([T_alt[live, None], np.where(add, 1.0 - alpha_alt, 1.0)],
                                                    axis=1), axis=1)[:, -1]
        fragile[live] |= (evaluated & (np.abs(raw - ALPHA_MIN) <= band_a)).any(axis=1)
        fragile[live] |= (evaluated & use & (np.abs(Tn - T_MIN) <= band_t)).any(axis=1)
        wgt = np.where(add, alpha * Tb, 0.0)
        for ch in range(3):
            contrib = np.where(add, sp["rgb"][s, ch][None] * wgt, 0.0)
            C[ch, live] = np.cumsum(np.concatenate([C[ch, live][:, None], contrib], axis=1), axis=1)[:, -1]
        # new transmittance: the product up to the stop (exclusive) or over the whole chunk
        last = np.cumprod(np.concatenate([T[live, None], np.where(add, 1.0 - alpha, 1.0)], axis=1), axis=1)[:, -1]
        T[live] = last
        n_added[live] += add.sum(axis=1)
        done[live] = has_stop
    C += T[None, :] * np.asarray(bg, np.float64)[:, None]
    return C, T, fragile, n_added


def dominant_splats(px, py, order, sp, chunk=2048):
    """For each pixel, the splat of ``order`` with the largest contribution
    weight alpha T among those the front-to-back walk adds (the first of
    equal ones), or -1 if it adds none; the walk of ``_blend_list``."""
    P = px.shape[0]
    T = np.ones(P)
    done = np.zeros(P, bool)
    best_w = np.full(P, -1.0)
    best = np.full(P, -1, np.int64)
    cx, cy = px + 0.5, py + 0.5
    order = np.asarray(order, np.int64)
    for c0 in range(0, order.shape[0], chunk):
        live = np.nonzero(~done)[0]
        if live.size == 0:
            break
        s = order[c0:c0 + chunk]
        K = s.shape[0]
        alpha = np.minimum(ALPHA_MAX, _alpha_raw(sp, s, cx[live], cy[live]))
        use = alpha >= ALPHA_MIN
        Tb = np.cumprod(np.concatenate([T[live, None], np.where(use, 1.0 - alpha, 1.0)], axis=1), axis=1)
        Tn = Tb[:, :-1] * (1.0 - alpha)
        Tb = Tb[:, :-1]
        stop = use & (Tn < T_MIN)
        has_stop = stop.any(axis=1)
        k_stop = np.where(has_stop, np.argmax(stop, axis=1), K)
        add = use & (np.arange(K)[None, :] < k_stop[:, None])
        wgt = np.where(add, alpha * Tb, -1.0)
        kb = np.argmax(wgt, axis=1)  # the first of equal maxima
        wb = wgt[np.arange(live.size), kb]
        better = wb > best_w[live]
        best_w[live] = np.where(better, wb, best_w[live])
        best[live] = np.where(better, s[kb], best[live])
        T[live] = np.cumprod(np.concatenate([T[live, None], np.where(add, 1.0 - alpha, 1.0)], axis=1),
                             axis=1)[:, -1]
        done[live] = has_stop
    return best


def dominant_splats_tiled(sp, sorted_vals, ranges, width, height, tw, th, tiles=None):
    """``dominant_splats`` over each tile's sorted list: [H, W] splat indices."""
    ntx = (width + tw - 1) // tw
    nty = (height + th - 1) // th
    out = np.full((height, width), -1, np.int64)
    for t in (range(ntx * nty) if tiles is None else tiles):
        ty, tx = divmod(int(t), ntx)
        x0, y0 = tx * tw, ty * th
        x1, y1 = min(x0 + tw, width), min(y0 + th, height)
        gy, gx = np.mgrid[y0:y1, x0:x1]
        s0, s1 = ranges[t]
        out[y0:y1, x0:x1] = dominant_splats(gx.ravel().astype(np.float64), gy.ravel().astype(np.float64),
                                            sorted_vals[s0:s1], sp).reshape(y1 - y0, x1 - x0)
    return out


def composite_tiled(sp, sorted_vals, ranges, width, height, tw, th, bg,
                    fragile_alpha=1e-4, fragile_t=1e-4, tiles=None, tie_impact=None,
                    chunked=False, sp_alt=None, power_ulps=0.0):
    """Per-tile front-to-back compositing over each tile's sorted list.
    Returns image [3,H,W], final transmittance [H,W] and the fragile mask.
    ``chunked`` walks the lists with ``_blend_list_chunked`` (same results,
    for long lists; no tie test), which also takes ``sp_alt`` (a second record
    set that widens the fragile bands by its distance from ``sp``) and
    ``power_ulps`` (a float32 error allowance on the exponent)."""
    ntx = (width + tw - 1) // tw
    nty = (height + th - 1) // th
    img = np.zeros((3, height, width))
    Tfin = np.ones((height, width))
    frag = np.zeros((height, width), bool)
    tile_ids = range(ntx * nty) if tiles is None else tiles
    for t in tile_ids:
        ty, tx = divmod(int(t), ntx)
        x0, y0 = tx * tw, ty * th
        x1, y1 = min(x0 + tw, width), min(y0 + th, height)
        gy, gx = np.mgrid[y0:y1, x0:x1]
        s0, s1 = ranges[t]
        if chunked:
            C, T, f, _ = _blend_list_chunked(gx.ravel().astype(np.float64), gy.ravel().astype(np.float64),
                                             sorted_vals[s0:s1], sp, bg, fragile_alpha, fragile_t,
                                             sp_alt=sp_alt, power_ulps=power_ulps)
        else:
            C, T, f, _ = _blend_list(gx.ravel().astype(np.float64), gy.ravel().astype(np.float64),
                                     sorted_vals[s0:s1], sp, bg, fragile_alpha, fragile_t,
                                     tie_impact)
        img[:, y0:y1, x0:x1] = C.reshape(3, y1 - y0, x1 - x0)
        Tfin[y0:y1, x0:x1] = T.reshape(y1 - y0, x1 - x0)
        frag[y0:y1, x0:x1] = f.reshape(y1 - y0, x1 - x0)
    return img, Tfin, frag


def composite_bruteforce(sp, visible, depth, width, height, bg):
    """Untiled compositing: every pixel walks all visible splats in
    (float32 depth, splat index) order. Must equal the tiled result exactly."""
    vis = np.nonzero(visible)[0]
    order = vis[np.lexsort((vis, depth_bits(depth)[vis]))]
    gy, gx = np.mgrid[0:height, 0:width]
    C, T, _, _ = _blend_list(gx.ravel().astype(np.float64), gy.ravel().astype(np.float64),
                             order, sp, bg, 0.0, 0.0)
    return C.reshape(3, height, width), T.reshape(height, width)


# ----------------------------------------------------------------------------
# whole frames
# ----------------------------------------------------------------------------

def splat_records(mu, cov, L, opacity, sh, degree, cam, tw, th):
    """Project + colour + footprint for a batch of posed Gaussians."""
    pr = project(mu, cov, cam)
    fp = footprint(pr["u"], pr["v"], pr["a"], pr["c"], opacity, pr["visible"],
                   cam.width, cam.height, tw, th)
    rgb = colour(sh, mu, L, cam.eye, degree)
    rec = dict(pr)
    # float32 error bound of a depth computed from world coordinates of this size
    mag = np.linalg.norm(np.asarray(mu, np.float64), axis=1) + np.linalg.norm(
        np.asarray(cam.eye, np.float64))
    rec["depth_eps"] = 4e-7 * mag + np.spacing(np.abs(pr["depth"]).astype(np.float32)).astype(np.float64)
    rec.update(fp)
    rec["opacity"] = np.asarray(opacity, np.float64)
    rec["rgb"] = rgb
    return rec


def concat_records(parts):
    out = {}
    for k in parts[0]:
        out[k] = np.concatenate([p[k] for p in parts], axis=0)
    return out


def render_records(rec, cam, tw, th, fragile_alpha=1e-4, fragile_t=1e-4, tie_impact=None):
    """Bin, sort and composite concatenated splat records (in emission order)."""
    ntx = (cam.width + tw - 1) // tw
    nty = (cam.height + th - 1) // th
    keys, vals = emit_pairs(rec["rect"], rec["count"], rec["visible"], rec["depth"], ntx)
    skeys, svals = sort_pairs(keys, vals)
    ranges = tile_ranges(skeys, ntx * nty)
    img, T, frag = composite_tiled(rec, svals, ranges, cam.width, cam.height, tw, th,
                                   cam.bg, fragile_alpha, fragile_t, tie_impact=tie_impact)
    return dict(image=img, T=T, fragile=frag, keys=keys, vals=vals,
                sorted_keys=skeys, sorted_vals=svals, ranges=ranges)
