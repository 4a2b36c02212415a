"""Pins of the FP64 skinning oracle against things other than itself:
library rotations, an independent subtree-rotation kinematics, and the closed
forms of identity / root-only / single-bone poses."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import skinning
from paper_2501_17792_amd import synth

EPS32 = np.finfo(np.float32).eps


def test_rodrigues_matches_scipy_rotvec():
    rng = np.random.default_rng(0)
    for aa in list(rng.normal(0, 1.0, size=(50, 3))) + [np.array([1e-13, 0, 0]), np.array([0.0, 0, 3.1])]:
        R = skinning.rodrigues(aa)
        ref = Rotation.from_rotvec(aa).as_matrix()
        np.testing.assert_allclose(R, ref, atol=1e-12)


def test_quat_to_rot_matches_scipy():
    rng = np.random.default_rng(1)
    q = rng.normal(size=(100, 4)) * rng.uniform(0.5, 2.0, size=(100, 1))  # not unit
    R = skinning.quat_to_rot(q)
    ref = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], axis=1)).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_canonical_covariance_eigen():
    rng = np.random.default_rng(2)
    s = rng.normal(-4, 0.3, size=(20, 3))
    q = rng.normal(size=(20, 4))
    S = skinning.canonical_covariance(s, q)
    for n in range(20):
        ev = np.sort(np.linalg.eigvalsh(S[n]))
        np.testing.assert_allclose(ev, np.sort(np.exp(2 * s[n])), rtol=1e-10)


def _subtree(parents, j):
    out = {j}
    for c in range(len(parents)):
        if c > j and parents[c] in out:
            out.add(c)
    return out


def _subtree_rotation_pose(points, drive, pose, joints, parents):
    """Independent kinematics: leaves first, rotate every point driven by a
    joint in subtree(j) about the REST position of j by R_j."""
    x = np.array(points, np.float64)
    for j in range(len(parents) - 1, -1, -1):
        sub = _subtree(parents, j)
        sel = np.array([d in sub for d in drive])
        if not sel.any():
            continue
        R = Rotation.from_rotvec(np.asarray(pose[j], np.float64)).as_matrix()
        x[sel] = joints[j] + (x[sel] - joints[j]) @ R.T
    return x


def test_fk_matches_subtree_rotation():
    t = synth.make_template(3, 4096, 0)
    rng = np.random.default_rng(4)
    pose = rng.normal(0, 0.4, size=(24, 3))
    J = t.joints_rest.astype(np.float64)
    B = skinning.bone_matrices(pose, J, t.parents, 0.0, 0.0, 0.0)
    # posed joint positions: B_j applied to the rest joint j
    posed = np.einsum("jik,jk->ji", B[:, :, :3], J) + B[:, :, 3]
    ref = _subtree_rotation_pose(J, np.arange(24), pose, J, t.parents)
    np.testing.assert_allclose(posed, ref, atol=1e-12)
    # a point rigidly attached to each joint
    pts = J + rng.normal(0, 0.1, size=J.shape)
    moved = np.einsum("jik,jk->ji", B[:, :, :3], pts) + B[:, :, 3]
    ref = _subtree_rotation_pose(pts, np.arange(24), pose, J, t.parents)
    np.testing.assert_allclose(moved, ref, atol=1e-12)


def test_identity_pose_returns_template():
    t = synth.make_template(5, 3000, 0)
    mu, cov, L, _ = skinning.skin_instance(t, np.zeros((24, 3)), 0.0, 0.0, 0.0)
    wsum = t.skin_w.astype(np.float64).sum(1)
    np.testing.assert_allclose(wsum, 1.0, atol=4 * EPS32)
    np.testing.assert_allclose(mu, t.mean.astype(np.float64) * wsum[:, None], rtol=0, atol=1e-15)
    cov0 = skinning.canonical_covariance(t.log_scale, t.quat)
    np.testing.assert_allclose(cov, cov0 * wsum[:, None, None] ** 2, rtol=1e-12)


def test_root_only_rotation_is_rigid_about_root():
    t = synth.make_template(6, 2000, 0)
    pose = np.zeros((24, 3))
    pose[0] = (0.3, -0.7, 0.2)
    mu, cov, L, _ = skinning.skin_instance(t, pose, 0.0, 0.0, 0.0)
    R0 = Rotation.from_rotvec(pose[0]).as_matrix()
    J0 = t.joints_rest[0].astype(np.float64)
    wsum = t.skin_w.astype(np.float64).sum(1)
    ref = (t.mean.astype(np.float64) - J0) @ R0.T + J0
    np.testing.assert_allclose(mu, ref * wsum[:, None], atol=1e-12)


def test_single_bone_weight_is_rigid_and_instance_transform():
    t = synth.make_template(7, 64, 0)
    rng = np.random.default_rng(8)
    pose = rng.normal(0, 0.5, size=(24, 3))
    yaw, px, pz = 1.1, 3.0, -2.0
    t.skin_w[:] = 0.0
    t.skin_w[:, 0] = 1.0
    mu, cov, L, B = skinning.skin_instance(t, pose, yaw, px, pz)
    J = t.joints_rest.astype(np.float64)
    world = _subtree_rotation_pose(t.mean, t.skin_idx[:, 0], pose, J, t.parents)
    Ry = Rotation.from_rotvec([0.0, yaw, 0.0]).as_matrix()
    world = world @ Ry.T + np.array([px, 0.0, pz])
    np.testing.assert_allclose(mu, world, atol=1e-12)
    cov0 = skinning.canonical_covariance(t.log_scale, t.quat)
    for n in range(t.n):
        Rn = L[n]
        np.testing.assert_allclose(Rn @ Rn.T, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(cov[n], Rn @ cov0[n] @ Rn.T, rtol=1e-12)


def test_weights_summing_to_one_preserve_translation():
    t = synth.make_template(9, 256, 0)
    w = t.skin_w.astype(np.float64)
    w /= w.sum(1, keepdims=True)
    t.skin_w = w
    shift = np.array([0.5, 0.0, -1.5])
    pose = np.random.default_rng(10).normal(0, 0.3, size=(24, 3))
    mu_a, *_ = skinning.skin_instance(t, pose, 0.4, 0.0, 0.0)
    mu_b, *_ = skinning.skin_instance(t, pose, 0.4, shift[0], shift[2])
    np.testing.assert_allclose(mu_b - mu_a, np.broadcast_to(shift, mu_a.shape), atol=1e-12)


def test_two_different_bones_mixed_weights_with_permuted_slots():
    """Two bones with different rigid transforms (rotations from scipy) and
    mixed weights w, 1 - w stored in permuted slots (the other two slots hold
    zero weight on further bones): the posed mean is the weighted sum of the
    two rigidly moved means, and the posed covariance is the covariance of the
    Gaussian pushed through the blended affine map, checked by the change of
    variables of scipy's normal density (no covariance formula retyped)."""
    from scipy.stats import multivariate_normal

    rng = np.random.default_rng(21)
    n = 48
    Ra = Rotation.from_rotvec(rng.normal(0, 0.8, (n, 3))).as_matrix()
    Rb = Rotation.from_rotvec(rng.normal(0, 0.8, (n, 3))).as_matrix()
    ta, tb = rng.normal(0, 1.0, (n, 3)), rng.normal(0, 1.0, (n, 3))
    w = rng.uniform(0.05, 0.95, n)
    mean = rng.normal(0, 0.5, (n, 3))
    log_scale = rng.normal(-1.5, 0.3, (n, 3))
    quat = rng.normal(0, 1, (n, 4))
    for i in range(n):
        B = np.zeros((24, 3, 4))
        for j in range(24):  # decoy bones on the zero-weight slots
            B[j, :, :3] = Rotation.from_rotvec(rng.normal(0, 1, 3)).as_matrix()
            B[j, :, 3] = rng.normal(0, 3, 3)
        a, b, c, d = rng.choice(24, size=4, replace=False)
        B[a, :, :3], B[a, :, 3] = Ra[i], ta[i]
        B[b, :, :3], B[b, :, 3] = Rb[i], tb[i]
        slots = rng.permutation(4)  # where bone a, bone b and the decoys sit
        idx = np.empty(4, np.int64)
        wt = np.zeros(4)
        idx[slots] = [a, b, c, d]
        wt[slots[0]], wt[slots[1]] = w[i], 1.0 - w[i]
        cov0 = skinning.canonical_covariance(log_scale[i:i + 1], quat[i:i + 1])
        mu, cov, L = skinning.lbs(B, mean[i:i + 1], cov0, idx[None], wt[None])
        ref_mu = w[i] * (Ra[i] @ mean[i] + ta[i]) + (1.0 - w[i]) * (Rb[i] @ mean[i] + tb[i])
        np.testing.assert_allclose(mu[0], ref_mu, atol=1e-12)
        # density of y = A x + t, x ~ N(mean, Sigma): p_x(A^-1 (y - t)) / |det A|
        A = w[i] * Ra[i] + (1.0 - w[i]) * Rb[i]
        t = w[i] * ta[i] + (1.0 - w[i]) * tb[i]
        Rq = Rotation.from_quat(np.roll(quat[i], -1)).as_matrix()  # scipy takes (x, y, z, w)
        sig = Rq @ np.diag(np.exp(2.0 * log_scale[i])) @ Rq.T
        ys = ref_mu + rng.normal(0, 0.3, (5, 3))
        xs = np.linalg.solve(A, (ys - t).T).T
        ref_pdf = multivariate_normal(mean[i], sig).pdf(xs) / abs(np.linalg.det(A))
        got_pdf = multivariate_normal(mu[0], cov[0]).pdf(ys)
        np.testing.assert_allclose(got_pdf, ref_pdf, rtol=1e-9)
