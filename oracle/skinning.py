"""FP64 forward kinematics and linear blend skinning (oracle).

CrowdSplat §2 (Fig. 2, stage 2): every character is a posed copy of a shared
canonical template; linear blend skinning moves the template's Gaussians.
Characters of one template share every attribute except the pose (§2, the
paragraph on shared template attributes).

Conventions (readings where the paper is silent):
* joint rotations are axis-angle vectors turned into matrices by Rodrigues'
  formula; the chain is G_0 = [R_0 | J_0], G_j = G_parent [R_j | J_j - J_parent];
* the skinning matrix of joint j is A_j = G_j [I | -J_j], placed in the world by
  the instance transform W = [R_y(yaw) | (px, 0, pz)];
* each Gaussian blends 4 bone matrices with its stored (not renormalised)
  weights: M = sum_k w_k B_{b_k}; the mean maps as mu' = M [mu; 1] and the
  covariance as Sigma' = L Sigma L^T with L the linear part of M.
"""
from __future__ import annotations

import numpy as np


def skew(v: np.ndarray) -> np.ndarray:
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def rodrigues(aa: np.ndarray) -> np.ndarray:
    """Rotation matrix of an axis-angle vector (first order below 1e-12 rad)."""
    aa = np.asarray(aa, np.float64)
    theta = float(np.linalg.norm(aa))
    if theta < 1e-12:
        return np.eye(3) + skew(aa)
    K = skew(aa / theta)
    return np.eye(3) + np.sin(theta) * K + (1.0 - np.cos(theta)) * (K @ K)


def rot_y(yaw: float) -> np.ndarray:
    c, s = np.cos(yaw), np.sin(yaw)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def global_transforms(pose, joints_rest, parents) -> np.ndarray:
    """G_j as 4x4 matrices [24,4,4]: rotations composed down the tree."""
    pose = np.asarray(pose, np.float64)
    J = np.asarray(joints_rest, np.float64)
    n = J.shape[0]
    G = np.zeros((n, 4, 4))
    for j in range(n):
        local = np.eye(4)
        local[:3, :3] = rodrigues(pose[j])
        p = int(parents[j])
        if p < 0:
            local[:3, 3] = J[j]
            G[j] = local
        else:
            local[:3, 3] = J[j] - J[p]
            G[j] = G[p] @ local
    return G


def skinning_matrices(pose, joints_rest, parents) -> np.ndarray:
    """A_j = G_j [I | -J_j] as [24,3,4]."""
    G = global_transforms(pose, joints_rest, parents)
    J = np.asarray(joints_rest, np.float64)
    A = np.zeros((J.shape[0], 3, 4))
    for j in range(J.shape[0]):
        back = np.eye(4)
        back[:3, 3] = -J[j]
        A[j] = (G[j] @ back)[:3]
    return A


def instance_transform(yaw: float, px: float, pz: float) -> np.ndarray:
    W = np.eye(4)
    W[:3, :3] = rot_y(float(yaw))
    W[:3, 3] = (float(px), 0.0, float(pz))
    return W


def bone_matrices(pose, joints_rest, parents, yaw, px, pz) -> np.ndarray:
    """B_j = W A_j, the world-space skinning matrices of one instance [24,3,4]."""
    A = skinning_matrices(pose, joints_rest, parents)
    W = instance_transform(yaw, px, pz)
    B = np.zeros_like(A)
    for j in range(A.shape[0]):
        A4 = np.vstack([A[j], [0.0, 0.0, 0.0, 1.0]])
        B[j] = (W @ A4)[:3]
    return B


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [N,3,3] of quaternions (w, x, y, z), normalised first."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def canonical_covariance(log_scale, quat) -> np.ndarray:
    """Sigma = R(q) diag(exp(2 s)) R(q)^T, per Gaussian [N,3,3] (3DGS)."""
    R = quat_to_rot(quat)
    S2 = np.exp(2.0 * np.asarray(log_scale, np.float64))
    return np.einsum("nij,nj,nkj->nik", R, S2, R)


def blend_matrices(B, skin_idx, skin_w) -> np.ndarray:
    """M = sum_k w_k B[idx_k], per Gaussian [N,3,4]."""
    idx = np.asarray(skin_idx).astype(np.int64)
    w = np.asarray(skin_w, np.float64)
    return np.einsum("nk,nkij->nij", w, np.asarray(B, np.float64)[idx])


def lbs(B, mean, cov, skin_idx, skin_w):
    """Posed means [N,3], posed covariances [N,3,3] and the blended linear
    parts L [N,3,3] of one instance."""
    M = blend_matrices(B, skin_idx, skin_w)
    L = M[:, :, :3]
    mu = np.einsum("nij,nj->ni", L, np.asarray(mean, np.float64)) + M[:, :, 3]
    cov_p = np.einsum("nij,njk,nlk->nil", L, cov, L)
    return mu, cov_p, L


def skin_instance(template, pose, yaw, px, pz, n: int | None = None, mean=None):
    """Skin the first ``n`` Gaussians of ``template`` for one instance;
    ``mean`` [n, 3] replaces the canonical means (pose-dependent offsets
    added before skinning)."""
    n = template.n if n is None else n
    B = bone_matrices(pose, template.joints_rest, template.parents, yaw, px, pz)
    cov = canonical_covariance(template.log_scale[:n], template.quat[:n])
    m = template.mean[:n] if mean is None else mean
    mu, cov_p, L = lbs(B, m, cov, template.skin_idx[:n], template.skin_w[:n])
    return mu, cov_p, L, B
