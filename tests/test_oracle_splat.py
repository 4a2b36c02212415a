"""Pins of the FP64 splatting oracle: SH against scipy and by quadrature,
projection against finite-difference Jacobians and closed forms, the
footprint against the ellipse it bounds, compositing against closed-form
stacks, tiled against untiled, and the sort against Python's sorted()."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import frame, splat
from paper_2501_17792_amd import synth


# ---------------------------------------------------------------- SH

def _real_sh_scipy(l, m, d):
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    if m == 0:
        return scipy.special.sph_harm_y(l, 0, theta, phi).real
    Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    # remove scipy's Condon-Shortley phase (-1)^m
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Y.real
    return math.sqrt(2) * (-1) ** m * Y.imag


def test_sh_basis_matches_scipy_real_transform():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = splat.sh_basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[:, l * l + l + m], _real_sh_scipy(l, m, d), atol=1e-12)


def test_sh_basis_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = np.repeat(wg, nphi) * (2 * np.pi / nphi)
    Y = splat.sh_basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_colour_degree0_is_rgb():
    t = synth.make_template(0, 100, 0)
    rgb = 0.5 + t.sh[:, 0, :].astype(np.float64) * synth.SH_C0
    rng = np.random.default_rng(1)
    mu = rng.normal(size=(100, 3))
    L = np.broadcast_to(np.eye(3), (100, 3, 3))
    c = splat.colour(t.sh, mu, L, np.array([0.0, 0, -3]), 0)
    np.testing.assert_allclose(c, np.maximum(rgb, 0), atol=1e-12)


def test_colour_direction_is_canonical_frame():
    """d = L^T (mu - eye), normalised; checked with scipy's inverse rotation."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(2)
    n = 50
    rots = Rotation.random(n, random_state=3)
    L = rots.as_matrix()
    mu = rng.normal(size=(n, 3))
    eye = np.array([0.2, 1.0, -3.0])
    sh = rng.normal(size=(n, 4, 3))
    c = splat.colour(sh, mu, L, eye, 1)
    d = rots.inv().apply(mu - eye)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c1 = math.sqrt(3 / (4 * math.pi))
    ref = 0.5 + 0.5 / math.sqrt(math.pi) * sh[:, 0] + c1 * (
        sh[:, 1] * d[:, 1:2] + sh[:, 2] * d[:, 2:3] + sh[:, 3] * d[:, 0:1])
    np.testing.assert_allclose(c, np.maximum(ref, 0), atol=1e-12)


# ---------------------------------------------------------------- projection

def _identity_cam(W=64, H=48, f=50.0):
    return synth.Camera(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2,
                        eye=np.zeros(3, np.float32), R=np.eye(3, dtype=np.float32))


def test_on_axis_isotropic_closed_form():
    cam = _identity_cam()
    for z, sig in [(2.0, 0.05), (5.0, 0.3), (0.5, 0.01)]:
        mu = np.array([[0.0, 0.0, z]])
        cov = (sig ** 2) * np.eye(3)[None]
        pr = splat.project(mu, cov, cam)
        assert pr["visible"][0]
        assert pr["u"][0] == cam.cx and pr["v"][0] == cam.cy
        ref = (cam.fx * sig / z) ** 2 + 0.3
        np.testing.assert_allclose([pr["a"][0], pr["c"][0]], [ref, ref], rtol=1e-14)
        assert pr["b"][0] == 0.0


def test_on_axis_anisotropic_has_no_depth_variance_term():
    cam = _identity_cam()
    mu = np.array([[0.0, 0.0, 3.0]])
    cov = np.diag([0.01, 0.04, 0.5])[None]
    pr = splat.project(mu, cov, cam)
    np.testing.assert_allclose([pr["a"][0], pr["c"][0]],
                               [(cam.fx / 3) ** 2 * 0.01 + 0.3, (cam.fy / 3) ** 2 * 0.04 + 0.3], rtol=1e-14)


def test_projection_jacobian_matches_finite_differences():
    rng = np.random.default_rng(3)
    cam = synth.look_at((0.3, 1.2, -3.0), (0.0, 0.8, 0.0), 320, 240)
    R = cam.R.astype(np.float64)
    eye = cam.eye.astype(np.float64)

    def pix(x):
        t = R @ (x - eye)
        return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])

    for _ in range(20):
        mu = np.array([rng.uniform(-0.8, 0.8), rng.uniform(0.2, 1.6), rng.uniform(-0.5, 0.5)])
        A = rng.normal(size=(3, 3)) * 0.05
        cov = A @ A.T + 1e-4 * np.eye(3)
        Jn = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (pix(mu + e) - pix(mu - e)) / (2 * h)
        ref = Jn @ cov @ Jn.T + 0.3 * np.eye(2)
        pr = splat.project(mu[None], cov[None], cam)
        np.testing.assert_allclose([pr["a"][0], pr["b"][0], pr["c"][0]],
                                   [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-6)
        S = np.array([[pr["a"][0], pr["b"][0]], [pr["b"][0], pr["c"][0]]])
        Si = np.linalg.inv(S)
        np.testing.assert_allclose([pr["A"][0], pr["B"][0], pr["C"][0]],
                                   [Si[0, 0], Si[0, 1], Si[1, 1]], rtol=1e-12)
        np.testing.assert_allclose([pr["u"][0], pr["v"][0]], pix(mu), rtol=1e-14)


def test_near_and_guard_band_culls():
    cam = _identity_cam()
    tan_x = 1.5 * cam.width / (2 * cam.fx)
    mu = np.array([[0, 0, 0.19], [0, 0, 0.21], [tan_x * 2 * 0.999, 0, 2], [tan_x * 2 * 1.001, 0, 2]])
    cov = np.broadcast_to(1e-4 * np.eye(3), (4, 3, 3))
    pr = splat.project(mu, cov, cam)
    assert list(pr["visible"]) == [False, True, True, False]


def test_footprint_is_the_exact_ellipse_box():
    rng = np.random.default_rng(5)
    for _ in range(30):
        A = rng.normal(size=(2, 2))
        S = A @ A.T * rng.uniform(0.5, 30) + 0.3 * np.eye(2)
        o = rng.uniform(0.02, 0.99)
        u, v = rng.uniform(20, 40), rng.uniform(20, 40)
        fp = splat.footprint(np.array([u]), np.array([v]), np.array([S[0, 0]]), np.array([S[1, 1]]),
                             np.array([o]), np.array([True]), 64, 64, 8, 8)
        k0 = 2 * math.log(255 * o)
        # boundary of the alpha = 1/255 ellipse: d = sqrt(k0) * chol(S) * (cos, sin)
        Lc = np.linalg.cholesky(S)
        th = np.linspace(0, 2 * np.pi, 20001)
        pts = math.sqrt(k0) * (Lc @ np.stack([np.cos(th), np.sin(th)]))
        Si = np.linalg.inv(S)
        alpha = o * np.exp(-0.5 * np.einsum("in,ij,jn->n", pts, Si, pts))
        np.testing.assert_allclose(alpha, 1 / 255, rtol=1e-9)
        assert np.abs(pts[0]).max() <= fp["rx"][0] - 0.01 + 1e-9
        assert np.abs(pts[0]).max() >= (fp["rx"][0] - 0.01) / (1 + 1e-4) ** 0.5 - 1e-6
        assert np.abs(pts[1]).max() <= fp["ry"][0] - 0.01 + 1e-9


def test_footprint_offscreen_and_opacity_culls():
    fp = splat.footprint(np.array([-5.0, 70.0, 10.0, 10.0]), np.array([10.0, 10.0, 10.0, 10.0]),
                         np.ones(4), np.ones(4), np.array([0.9, 0.9, 1 / 255 * 0.999, 0.9]),
                         np.ones(4, bool), 64, 64, 16, 16)
    assert list(fp["visible"]) == [False, False, False, True]
    assert list(fp["rect"][3]) == [0, 0, 0, 0]


# ---------------------------------------------------------------- compositing

def _records(us, vs, sig2, ops, rgbs, depth=None):
    n = len(us)
    a = np.array(sig2, np.float64) + 0.0
    rec = dict(u=np.array(us, np.float64), v=np.array(vs, np.float64),
               A=1 / a, B=np.zeros(n), C=1 / a, opacity=np.array(ops, np.float64),
               rgb=np.array(rgbs, np.float64))
    return rec


def test_single_splat_closed_form():
    rec = _records([10.5], [7.5], [4.0], [0.8], [[1.0, 0.5, 0.25]])
    gy, gx = np.mgrid[0:16, 0:20]
    C, T, frag, _ = splat._blend_list(gx.ravel() * 1.0, gy.ravel() * 1.0, [0], rec, np.zeros(3), 0, 0)
    r2 = (gx.ravel() + 0.5 - 10.5) ** 2 + (gy.ravel() + 0.5 - 7.5) ** 2
    a = np.minimum(0.99, 0.8 * np.exp(-r2 / 8.0))
    a = np.where(a >= 1 / 255, a, 0)
    np.testing.assert_allclose(C[0], a, atol=1e-15)
    np.testing.assert_allclose(C[1], 0.5 * a, atol=1e-15)


def test_anisotropic_splat_matches_quadratic_form():
    rng = np.random.default_rng(11)
    A = rng.normal(size=(2, 2)) * 2
    S = A @ A.T + 0.3 * np.eye(2)
    Si = np.linalg.inv(S)
    det = S[0, 0] * S[1, 1] - S[0, 1] ** 2
    rec = dict(u=np.array([8.3]), v=np.array([6.9]), A=np.array([S[1, 1] / det]),
               B=np.array([-S[0, 1] / det]), C=np.array([S[0, 0] / det]),
               opacity=np.array([0.7]), rgb=np.array([[1.0, 1.0, 1.0]]))
    gy, gx = np.mgrid[0:16, 0:16]
    C, T, _, _ = splat._blend_list(gx.ravel() * 1.0, gy.ravel() * 1.0, [0], rec, np.zeros(3), 0, 0)
    d = np.stack([gx.ravel() + 0.5 - 8.3, gy.ravel() + 0.5 - 6.9])
    a = 0.7 * np.exp(-0.5 * np.einsum("in,ij,jn->n", d, Si, d))
    a = np.where(a >= 1 / 255, np.minimum(a, 0.99), 0)
    np.testing.assert_allclose(C[0], a, atol=1e-14)


def test_two_and_three_splat_stacks():
    rec = _records([5.5] * 3, [5.5] * 3, [1.0] * 3, [0.9, 0.6, 0.3],
                   [[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    px = np.array([5.0])
    C, T, _, n = splat._blend_list(px, px, [0, 1], rec, np.zeros(3), 0, 0)
    np.testing.assert_allclose(C[:, 0], [0.9, 0.6 * 0.1, 0], atol=1e-15)
    C, T, _, n = splat._blend_list(px, px, [0, 1, 2], rec, np.zeros(3), 0, 0)
    np.testing.assert_allclose(C[:, 0], [0.9, 0.06, 0.3 * 0.1 * 0.4], atol=1e-15)
    np.testing.assert_allclose(T[0], 0.1 * 0.4 * 0.7, atol=1e-15)


def test_alpha_clamp_and_early_stop_without_adding():
    # o = 1.0 clamps to 0.99; T after 2 = 1e-4 exactly on the threshold (fragile)
    rec = _records([5.5] * 4, [5.5] * 4, [1.0] * 4, [0.95] * 4, [[1, 1, 1]] * 4)
    px = np.array([5.0])
    C, T, frag, n = splat._blend_list(px, px, [0, 1, 2, 3], rec, np.zeros(3), 1e-4, 1e-4)
    # T: 0.05, 0.0025, 1.25e-4, then 6.25e-6 < 1e-4 -> the 4th is not added
    assert n[0] == 3
    np.testing.assert_allclose(C[0, 0], 0.95 * (1 + 0.05 + 0.0025), atol=1e-15)
    np.testing.assert_allclose(T[0], 1.25e-4, rtol=1e-12)
    rec = _records([5.5] * 3, [5.5] * 3, [1.0] * 3, [1.0] * 3, [[1, 1, 1]] * 3)
    C, T, frag, n = splat._blend_list(px, px, [0, 1, 2], rec, np.zeros(3), 1e-4, 1e-4)
    assert frag[0]  # 0.01 * 0.01 sits on 1e-4: flagged fragile


def test_alpha_below_threshold_is_skipped():
    o = 0.5
    # pixel at distance r with o exp(-r^2/2) = (1/255)(1 -+ 1e-3)
    for factor, added in [(1 - 1e-3, False), (1 + 1e-3, True)]:
        r = math.sqrt(-2 * math.log(factor / (255 * o)))
        rec = _records([0.5 + r], [0.5], [1.0], [o], [[1, 1, 1]])
        C, T, frag, n = splat._blend_list(np.array([0.0]), np.array([0.0]), [0], rec,
                                          np.zeros(3), 1e-2, 1e-4)
        assert bool(n[0]) == added
        assert frag[0]


def _random_scene(seed, n=64, size=32):
    rng = np.random.default_rng(seed)
    cam = synth.Camera(width=size, height=size, fx=30.0, fy=30.0, cx=size / 2, cy=size / 2,
                       eye=np.zeros(3, np.float32), R=np.eye(3, dtype=np.float32),
                       bg=np.array([0.1, 0.2, 0.3], np.float32))
    mu = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.6, 0.6, n), rng.uniform(1.0, 2.0, n)], 1)
    A = rng.normal(size=(n, 3, 3)) * rng.uniform(0.01, 0.08, size=(n, 1, 1))
    cov = A @ np.transpose(A, (0, 2, 1)) + 1e-5 * np.eye(3)
    op = rng.uniform(0.05, 0.99, n)
    rgb = rng.uniform(0, 1, (n, 3))
    pr = splat.project(mu, cov, cam)
    return cam, pr, op, rgb


@pytest.mark.parametrize("tile", [(4, 4), (8, 8), (16, 16), (8, 16)])
def test_tiled_equals_bruteforce(tile):
    for seed in range(3):
        cam, pr, op, rgb = _random_scene(seed)
        tw, th = tile
        fp = splat.footprint(pr["u"], pr["v"], pr["a"], pr["c"], op, pr["visible"],
                             cam.width, cam.height, tw, th)
        rec = dict(pr)
        rec.update(fp)
        rec["opacity"], rec["rgb"] = op, rgb
        out = splat.render_records(rec, cam, tw, th)
        bf, Tb = splat.composite_bruteforce(rec, rec["visible"], rec["depth"], cam.width, cam.height, cam.bg)
        assert np.array_equal(out["image"], bf)
        assert np.array_equal(out["T"], Tb)


# ---------------------------------------------------------------- binning / sort

def test_sort_invariants_and_python_sorted():
    sc = synth.scene_c1()
    out = frame.render_frame(sc.templates, sc.crowd, sc.camera, np.zeros(1, int))
    keys, vals = out["keys"], out["vals"]
    ref = sorted(range(len(keys)), key=lambda i: (int(keys[i]), i))
    assert np.array_equal(out["sorted_keys"], keys[ref])
    assert np.array_equal(out["sorted_vals"], vals[ref])
    sk = out["sorted_keys"]
    assert np.all(sk[1:] >= sk[:-1])
    rec = out["records"]
    ranges = out["ranges"]
    assert ranges[0, 0] == 0 and ranges[-1, 1] == len(keys)
    assert np.all(ranges[1:, 0] == ranges[:-1, 1])
    ntx = (sc.camera.width + 15) // 16
    tiles = (sk >> np.uint64(31)).astype(np.int64)
    r = rec["rect"][out["sorted_vals"]]
    ty, tx = tiles // ntx, tiles % ntx
    assert np.all((tx >= r[:, 0]) & (tx <= r[:, 2]) & (ty >= r[:, 1]) & (ty <= r[:, 3]))
    np.testing.assert_array_equal(np.bincount(vals, minlength=len(rec["count"])), rec["count"])


def test_fixed_levels_closed_form():
    eye = np.array([0.0, 1.7, -3.0])
    pos = np.array([[0.0, 0.0], [0.0, 10.0 - 3.0], [0.0, 20.0], [0.0, 40.0]])
    lv = frame.fixed_levels(pos, eye, (10.0, 25.0))
    dist = np.sqrt((pos[:, 1] + 3) ** 2 + 1.7 ** 2)
    np.testing.assert_array_equal(lv, np.where(dist < 10, 0, np.where(dist < 25, 1, 2)))
    assert list(lv) == [0, 1, 1, 2]


def test_chunked_walk_equals_the_loop_bit_for_bit():
    """The chunked front-to-back walk (for lists of millions) gives the loop's
    colour, transmittance, fragile flags and counts exactly, with stops, skips
    and clamps inside and across chunk borders."""
    rng = np.random.default_rng(12)
    n = 700
    rec = dict(u=rng.uniform(0, 16, n), v=rng.uniform(0, 16, n), A=rng.uniform(0.02, 0.6, n),
               B=rng.uniform(-0.05, 0.05, n), C=rng.uniform(0.02, 0.6, n),
               opacity=np.where(rng.uniform(size=n) < 0.1, 1.0, rng.uniform(0.002, 0.9, n)),
               rgb=rng.uniform(0, 1.3, (n, 3)))
    gy, gx = np.mgrid[0:16, 0:16]
    px, py = gx.ravel() * 1.0, gy.ravel() * 1.0
    order = rng.permutation(n)
    bg = np.array([0.2, 0.4, 0.6])
    ref = splat._blend_list(px, py, order, rec, bg, 1e-3, 1e-3)
    assert ref[3].min() < ref[3].max() and (ref[1] < 1e-2).any()  # stops and long walks both occur
    for chunk in (1, 7, 64, 4096):
        got = splat._blend_list_chunked(px, py, order, rec, bg, 1e-3, 1e-3, chunk=chunk)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), chunk


def test_alternate_records_widen_the_fragile_band():
    """A second record set widens the fragile bands by its own distance from
    the first: identical records change nothing; an alpha that the two
    records put on opposite sides of 1/255, or a T' they put on opposite
    sides of 1e-4, flags the pixel although the base band alone would not."""
    px = np.array([0.0])
    o = 0.5
    # alpha = (1/255)(1 + 1e-3): outside the 1e-4 band
    r = math.sqrt(-2 * math.log((1 + 1e-3) / (255 * o)))
    rec = _records([0.5 + r], [0.5], [1.0], [o], [[1, 1, 1]])
    base = splat._blend_list_chunked(px, px, [0], rec, np.zeros(3), 1e-4, 1e-4)
    assert not base[2][0] and base[3][0] == 1
    same = splat._blend_list_chunked(px, px, [0], rec, np.zeros(3), 1e-4, 1e-4, sp_alt=dict(rec))
    for a, b in zip(base, same):
        assert np.array_equal(a, b)
    alt = dict(rec, opacity=rec["opacity"] * (1 - 2e-3))  # alpha below 1/255 there
    got = splat._blend_list_chunked(px, px, [0], rec, np.zeros(3), 1e-4, 1e-4, sp_alt=alt)
    assert got[2][0] and np.array_equal(got[0], base[0]) and got[3][0] == 1  # the walk follows rec
    alt = dict(rec, opacity=rec["opacity"] * (1 - 5e-4))  # both above: not flagged
    assert not splat._blend_list_chunked(px, px, [0], rec, np.zeros(3), 1e-4, 1e-4, sp_alt=alt)[2][0]
    # T': three opaque splats of alpha a with (1 - a)^3 = 1e-4 (1 + 1e-3); the
    # alternate's last alpha is a little larger, so its T' falls below 1e-4
    a = 1 - (1e-4 * (1 + 1e-3)) ** (1 / 3)
    rec = _records([0.5] * 3, [0.5] * 3, [1.0] * 3, [a] * 3, [[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    base = splat._blend_list_chunked(px, px, [0, 1, 2], rec, np.zeros(3), 1e-4, 1e-4)
    assert not base[2][0] and base[3][0] == 3
    ops = rec["opacity"].copy()
    ops[2] = 1 - (1 - a) * (1 - 2e-3)
    got = splat._blend_list_chunked(px, px, [0, 1, 2], rec, np.zeros(3), 1e-4, 1e-4,
                                    sp_alt=dict(rec, opacity=ops))
    assert got[2][0] and got[3][0] == 3
    # the first splat's alternate moves T before the third: flagged the same way
    ops = rec["opacity"].copy()
    ops[0] = 1 - (1 - a) * (1 - 2e-3)
    got = splat._blend_list_chunked(px, px, [0, 1, 2], rec, np.zeros(3), 1e-4, 1e-4,
                                    sp_alt=dict(rec, opacity=ops), chunk=1)
    assert got[2][0]


def test_exponent_ulps_widen_the_alpha_band_of_thin_splats():
    """The float32 allowance on the exponent scales with its terms: a thin
    splat whose terms cancel (A = C = 1000, B = -999.9 along the diagonal)
    is flagged at alpha (1 + 2e-5) / 255, a round one at the same alpha is
    not (its terms are about as large as the exponent itself)."""
    px = np.array([0.0])
    o = 0.5
    target = math.log((1 + 2e-5) / (255 * o))  # power giving that alpha
    # thin: power = -0.1 d^2 at dx = dy = d
    d = math.sqrt(-target / 0.1)
    thin = dict(u=np.array([0.5 - d]), v=np.array([0.5 - d]), A=np.array([1000.0]),
                B=np.array([-999.9]), C=np.array([1000.0]), opacity=np.array([o]),
                rgb=np.ones((1, 3)))
    r = math.sqrt(-2 * target)
    round_ = _records([0.5 + r], [0.5], [1.0], [o], [[1, 1, 1]])
    for rec, flagged in [(thin, True), (round_, False)]:
        got = splat._blend_list_chunked(px, px, [0], rec, np.zeros(3), 1e-5, 1e-4, power_ulps=8.0)
        assert got[3][0] == 1  # added: alpha is above 1/255
        assert bool(got[2][0]) == flagged
        assert not splat._blend_list_chunked(px, px, [0], rec, np.zeros(3), 1e-5, 1e-4)[2][0]


def test_float32_footprint_rect():
    """Where the pixel bounds are not near an integer, the float32 rect equals
    the FP64 footprint's rect; a bound whose float32 subtraction rounds onto
    an integer takes the float32 floor; boxes entirely off-screen are culled."""
    rng = np.random.default_rng(13)
    n = 4000
    u, v = rng.uniform(-40, 300, n), rng.uniform(-40, 200, n)
    a, c = rng.uniform(0.3, 400, n), rng.uniform(0.3, 400, n)
    op = rng.uniform(0.01, 1.0, n)
    fp = splat.footprint(u, v, a, c, op, np.ones(n, bool), 256, 160, 16, 16)
    b = fp["bounds"]
    far = np.all(np.abs(b - np.round(b)) > 1e-3, axis=1)
    rect, cnt, vis = splat.footprint_rect_f32(u.astype(np.float32), v.astype(np.float32),
                                              fp["rx"].astype(np.float32), fp["ry"].astype(np.float32),
                                              np.ones(n), 256, 160, 16, 16)
    assert np.array_equal(vis[far], fp["visible"][far])
    ok = far & vis
    assert np.array_equal(rect[ok], fp["rect"][ok]) and np.array_equal(cnt[ok], fp["count"][ok])
    assert ok.sum() > 1000 and (~vis).sum() > 100
    # 2^24 - 0.5 is a tie between two float32 values and rounds to even (2^24)
    u32 = np.array([2.0 ** 24], np.float32)
    r, _, _ = splat.footprint_rect_f32(u32, np.array([1.0], np.float32), np.array([0.5], np.float32),
                                       np.array([0.5], np.float32), np.ones(1), 2 ** 26, 8, 1, 1)
    assert r[0, 0] == 2 ** 24  # the FP64 floor would be 2^24 - 1
    # culled or zero-depth splats get no tiles
    r, cnt, vis = splat.footprint_rect_f32(np.array([-5.0, 40.0], np.float32), np.array([40.0, 40.0], np.float32),
                                           np.array([2.0, 10.0], np.float32), np.array([2.0, 10.0], np.float32),
                                           np.array([1.0, 0.0]), 256, 160, 16, 16)
    assert list(cnt) == [0, 0] and not vis.any()
    r, cnt, vis = splat.footprint_rect_f32(np.array([40.0], np.float32), np.array([40.0], np.float32),
                                           np.array([10.0], np.float32), np.array([10.0], np.float32),
                                           np.array([1.0]), 256, 160, 16, 16)
    assert list(r[0]) == [1, 1, 3, 3] and cnt[0] == 9  # pixels 30..50 -> tiles 1..3


def test_dominant_splat_closed_forms():
    """Splats stacked on one pixel: weights alpha1, alpha2 (1 - alpha1), ...;
    the larger wins; a skipped or stopping splat never wins."""
    px = np.array([0.0])

    def dom(ops):
        rec = _records([0.5] * len(ops), [0.5] * len(ops), [1.0] * len(ops), ops, [[1, 1, 1]] * len(ops))
        return int(splat.dominant_splats(px, px, list(range(len(ops))), rec)[0])

    assert dom([0.3, 0.5]) == 1    # 0.3 against 0.35
    assert dom([0.3, 0.4]) == 0    # 0.3 against 0.28
    assert dom([0.5, 1.0]) == 0    # 0.5 against 0.99 * 0.5 = 0.495
    assert dom([0.002, 0.003]) == -1  # both below 1/255: nothing added
    assert dom([0.5, 1.0, 0.5]) == 0  # 0.5, 0.495, then 0.5 * 0.005 = 0.0025
    assert dom([0.5, 1.0]) == dom([0.5, 1.0, 0.0])  # a zero-opacity splat changes nothing
    # the splat that would take T below 1e-4 is not added, so it cannot win
    assert dom([0.99, 0.99, 0.99]) == 0  # T after two is 1e-4 exactly: the third stops the walk
    assert dom([0.2, 0.2]) == 0  # 0.2 against 0.16


def test_dominant_splat_is_the_largest_single_splat_render():
    """On random scenes the dominant splat of each pixel is the one whose
    colour alone (every other splat black) gives the pixel the most light:
    the weight alpha T read off the compositor's own colour output, one
    render per splat; across chunk sizes the result is the same."""
    rng = np.random.default_rng(21)
    for seed in range(3):
        n = 24
        rec = dict(u=rng.uniform(0, 8, n), v=rng.uniform(0, 8, n), A=rng.uniform(0.05, 1.0, n),
                   B=rng.uniform(-0.05, 0.05, n), C=rng.uniform(0.05, 1.0, n),
                   opacity=rng.uniform(0.05, 0.95, n), rgb=np.zeros((n, 3)))
        gy, gx = np.mgrid[0:8, 0:8]
        px, py = gx.ravel() * 1.0, gy.ravel() * 1.0
        order = rng.permutation(n)
        W = np.zeros((n, px.size))
        for k in range(n):
            r = dict(rec, rgb=np.zeros((n, 3)))
            r["rgb"][k] = 1.0
            C, _, _, _ = splat._blend_list(px, py, order, r, np.zeros(3), 0, 0)
            W[k] = C[0]
        want = np.where(W.max(0) > 0, np.argmax(W, axis=0), -1)
        for chunk in (1, 5, 4096):
            got = splat.dominant_splats(px, py, order, rec, chunk=chunk)
            ok = (got == want) | (np.sort(W, axis=0)[-1] - np.sort(W, axis=0)[-2] < 1e-12)
            assert ok.all(), (seed, chunk)
