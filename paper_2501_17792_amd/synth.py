"""Seeded synthetic inputs for the crowd-splatting hot path.

The paper's own data (reconstructed avatar templates, AMASS motions, the grid
crowd of CrowdSplat §2 and §3) is not available, so every workload is drawn
here from fixed seeds with the shapes and distributions of the five
workloads below:

* ``c1``  plain method, one 2,048-Gaussian SH0 template, one instance, 256x256;
* ``c2``  14 templates x 100k Gaussians (SH3), 500 instances, 1920x1080,
          fixed 3-level LoD;
* ``c3``  the same templates, 3,500 instances on an 80x80 m plane, 300-frame
          keyframed animation;
* ``c4``  C3's scene with 5 LoD levels (learned LoD);
* ``c5``  one 100k template at 512x512 seen from 64 cameras (differentiable fit).

This module is shared by the oracle's tests and by the GPU path's callers. It
holds none of the method's arithmetic: no forward kinematics, skinning,
projection, sorting or compositing. It only draws random numbers and lays
them out (the skeleton's rest joints, capsule samples, skin weights from
point-to-bone distances, an importance order for the LoD prefixes, crowd
placements, keyframed poses and camera frames).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

N_JOINTS = 24
SH_C0 = 0.28209479177387814  # 1 / (2 sqrt(pi)): the degree-0 real SH constant

#: A project-defined 24-joint humanoid tree (parents[j] < j, pelvis root).
JOINT_NAMES = [
    "pelvis", "spine1", "spine2", "spine3", "neck", "head",
    "l_hip", "l_knee", "l_ankle", "l_foot",
    "r_hip", "r_knee", "r_ankle", "r_foot",
    "l_collar", "l_shoulder", "l_elbow", "l_wrist", "l_hand",
    "r_collar", "r_shoulder", "r_elbow", "r_wrist", "r_hand",
]
PARENTS = np.array([-1, 0, 1, 2, 3, 4,
                    0, 6, 7, 8,
                    0, 10, 11, 12,
                    3, 14, 15, 16, 17,
                    3, 19, 20, 21, 22], dtype=np.int32)

# Unit rest directions (T-pose) of the bone parent(j) -> j, world y up.
_REST_DIRS = {
    1: (0, 1, 0), 2: (0, 1, 0), 3: (0, 1, 0), 4: (0, 1, 0), 5: (0, 1, 0),
    6: (0.6, -0.8, 0), 7: (0, -1, 0), 8: (0, -1, 0), 9: (0, -0.6, 0.8),
    10: (-0.6, -0.8, 0), 11: (0, -1, 0), 12: (0, -1, 0), 13: (0, -0.6, 0.8),
    14: (0.8, 0.6, 0), 15: (1, 0, 0), 16: (1, 0, 0), 17: (1, 0, 0), 18: (1, 0, 0),
    19: (-0.8, 0.6, 0), 20: (-1, 0, 0), 21: (-1, 0, 0), 22: (-1, 0, 0), 23: (-1, 0, 0),
}

CAPSULE_RADIUS = 0.06
SKIN_TEMPERATURE = 0.05


@dataclasses.dataclass
class Template:
    """One canonical Gaussian avatar template, stored in importance order.

    Level ``l`` of the LoD is the prefix ``[0, level_count[l])``.
    """
    mean: np.ndarray        # f32 [N,3]
    log_scale: np.ndarray   # f32 [N,3]
    quat: np.ndarray        # f32 [N,4]  (w, x, y, z), not necessarily unit
    opacity: np.ndarray     # f32 [N]    in (0, 1)
    sh: np.ndarray          # f32 [N,(D+1)^2,3]
    skin_idx: np.ndarray    # u8  [N,4]  driving joint of each of the 4 bones
    skin_w: np.ndarray      # f32 [N,4]  not renormalised
    joints_rest: np.ndarray  # f32 [24,3]
    parents: np.ndarray     # i32 [24]
    sh_degree: int
    level_count: np.ndarray  # i32 [L], non-increasing, [0] == N

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def subset(self, n: int) -> "Template":
        """The first ``n`` Gaussians (an importance prefix) as a template."""
        return dataclasses.replace(
            self, mean=self.mean[:n].copy(), log_scale=self.log_scale[:n].copy(),
            quat=self.quat[:n].copy(), opacity=self.opacity[:n].copy(),
            sh=self.sh[:n].copy(), skin_idx=self.skin_idx[:n].copy(),
            skin_w=self.skin_w[:n].copy(),
            level_count=np.array([n], dtype=np.int32))


@dataclasses.dataclass
class Camera:
    """Pinhole camera, world y up; camera frame x right, y down, z forward."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    eye: np.ndarray      # f32 [3]
    R: np.ndarray        # f32 [3,3] world -> camera, rows (right, down, forward)
    near: float = 0.2
    bg: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3, np.float32))


@dataclasses.dataclass
class Crowd:
    tid: np.ndarray      # i32 [n]
    yaw: np.ndarray      # f32 [n]
    pos: np.ndarray      # f32 [n,2]  (px, pz) on the ground plane y = 0
    pose: np.ndarray     # f32 [n,24,3] axis-angle per joint

    @property
    def n(self) -> int:
        return int(self.tid.shape[0])


# ----------------------------------------------------------------------------
# skeleton and template
# ----------------------------------------------------------------------------

def rest_joints(rng: np.random.Generator) -> np.ndarray:
    """Rest joint positions: each child at parent + U(0.1, 0.5) m along its
    fixed rest direction; the pelvis at the origin (before the ground shift)."""
    lengths = rng.uniform(0.1, 0.5, size=N_JOINTS)
    joints = np.zeros((N_JOINTS, 3), np.float64)
    for j in range(1, N_JOINTS):
        d = np.asarray(_REST_DIRS[j], np.float64)
        d = d / np.linalg.norm(d)
        joints[j] = joints[PARENTS[j]] + lengths[j] * d
    return joints


def _bones(joints: np.ndarray):
    """The 23 bones (segments parent(j) -> j); each is driven by its parent joint."""
    child = np.arange(1, N_JOINTS)
    return joints[PARENTS[child]], joints[child], PARENTS[child].astype(np.int64)


def _orthonormal_pair(axis: np.ndarray):
    a = axis / np.linalg.norm(axis)
    helper = np.array([1.0, 0, 0]) if abs(a[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(a, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    return a, e1, e2


def sample_capsules(rng: np.random.Generator, joints: np.ndarray, n: int,
                    radius: float = CAPSULE_RADIUS) -> np.ndarray:
    """n points uniform on the union of bone capsules (bone chosen with
    probability proportional to the capsule's surface area)."""
    a, b, _ = _bones(joints)
    length = np.linalg.norm(b - a, axis=1)
    area = 2 * np.pi * radius * length + 4 * np.pi * radius ** 2
    bone = rng.choice(len(length), size=n, p=area / area.sum())
    on_cyl = rng.uniform(size=n) < (2 * np.pi * radius * length[bone]) / area[bone]
    t = rng.uniform(size=n)
    phi = rng.uniform(0, 2 * np.pi, size=n)
    sph = rng.normal(size=(n, 3))
    sph /= np.linalg.norm(sph, axis=1, keepdims=True)
    pts = np.empty((n, 3), np.float64)
    for k in range(len(length)):
        sel = np.nonzero(bone == k)[0]
        if sel.size == 0:
            continue
        ax, e1, e2 = _orthonormal_pair(b[k] - a[k])
        cyl = (a[k] + t[sel, None] * (b[k] - a[k])
               + radius * (np.cos(phi[sel])[:, None] * e1 + np.sin(phi[sel])[:, None] * e2))
        up = (sph[sel] @ ax) >= 0
        cap = np.where(up[:, None], b[k], a[k]) + radius * sph[sel]
        pts[sel] = np.where(on_cyl[sel, None], cyl, cap)
    return pts


def skin_weights(points: np.ndarray, joints: np.ndarray,
                 temperature: float = SKIN_TEMPERATURE):
    """Softmax over -distance/temperature to the 4 nearest bones.

    Returns (driving joint u8 [N,4], weight f32 [N,4]); weights are stored as
    FP32 and not renormalised afterwards.
    """
    a, b, drive = _bones(joints)
    ab = b - a
    rel = points[:, None, :] - a[None, :, :]
    t = np.clip((rel * ab[None]).sum(-1) / (ab * ab).sum(-1)[None], 0.0, 1.0)
    dist = np.linalg.norm(rel - t[..., None] * ab[None], axis=-1)
    nearest = np.argsort(dist, axis=1, kind="stable")[:, :4]
    d4 = np.take_along_axis(dist, nearest, axis=1)
    logits = -d4 / temperature
    logits -= logits.max(axis=1, keepdims=True)
    w = np.exp(logits)
    w /= w.sum(axis=1, keepdims=True)
    return drive[nearest].astype(np.uint8), w.astype(np.float32)


def make_template(seed: int, n: int, sh_degree: int,
                  level_fractions: Sequence[float] = (1.0,)) -> Template:
    """A synthetic avatar template drawn from ``seed``.

    Means on bone capsules (radius 0.06 m); log-scales ~ N(-4, 0.3); uniform
    random unit quaternions (w, x, y, z); opacity = sigmoid(N(1, 1));
    RGB ~ U(0, 1) stored as the SH DC term; higher SH bands ~ N(0, 0.05^2).
    The Gaussians are permuted into descending importance
    opacity * (sx sy sz)^(2/3) (ties by index) so that every LoD level is a prefix.
    """
    rng = np.random.default_rng(seed)
    joints = rest_joints(rng)
    mean = sample_capsules(rng, joints, n)
    log_scale = rng.normal(-4.0, 0.3, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(1.0, 1.0, size=n)))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    n_coef = (sh_degree + 1) ** 2
    sh = np.zeros((n, n_coef, 3), np.float64)
    sh[:, 0, :] = (rgb - 0.5) / SH_C0
    if n_coef > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(n, n_coef - 1, 3))
    skin_idx, skin_w = skin_weights(mean, joints)
    # ground the template: min y over the means is 0
    shift = mean[:, 1].min()
    mean[:, 1] -= shift
    joints = joints.copy()
    joints[:, 1] -= shift
    importance = opacity * np.exp((2.0 / 3.0) * log_scale.sum(axis=1))
    order = np.argsort(-importance, kind="stable")
    level_count = np.array([int(round(n * f)) for f in level_fractions], np.int32)
    return Template(
        mean=mean[order].astype(np.float32),
        log_scale=log_scale[order].astype(np.float32),
        quat=q[order].astype(np.float32),
        opacity=opacity[order].astype(np.float32),
        sh=sh[order].astype(np.float32),
        skin_idx=skin_idx[order],
        skin_w=skin_w[order],
        joints_rest=joints.astype(np.float32),
        parents=PARENTS.copy(),
        sh_degree=sh_degree,
        level_count=level_count,
    )


# ----------------------------------------------------------------------------
# cameras and crowds
# ----------------------------------------------------------------------------

def look_at(eye, target, width: int, height: int, fov_y_deg: float = 60.0,
            near: float = 0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at ``eye`` looking at ``target``; vertical field of view."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    focal = height / (2.0 * math.tan(math.radians(fov_y_deg) / 2.0))
    return Camera(width=width, height=height, fx=focal, fy=focal,
                  cx=width / 2.0, cy=height / 2.0,
                  eye=eye.astype(np.float32),
                  R=np.stack([r, d, f]).astype(np.float32), near=near,
                  bg=np.asarray(bg, np.float32))


def make_crowd(seed: int, n: int, n_templates: int, extent: float,
               pose_sigma: float) -> Crowd:
    rng = np.random.default_rng(seed)
    tid = rng.integers(0, n_templates, size=n).astype(np.int32)
    yaw = rng.uniform(0.0, 2 * np.pi, size=n).astype(np.float32)
    pos = rng.uniform(0.0, extent, size=(n, 2)).astype(np.float32)
    pose = rng.normal(0.0, pose_sigma, size=(n, N_JOINTS, 3)).astype(np.float32)
    return Crowd(tid=tid, yaw=yaw, pos=pos, pose=pose)


def keyframe_poses(seed: int, n: int, n_frames: int, every: int,
                   sigma: float) -> np.ndarray:
    """Per-frame poses f32 [n_frames, n, 24, 3]: a keyframe every ``every``
    frames (pose ~ N(0, sigma)), componentwise linear interpolation between
    keyframes (a 30 Hz playback of seeded keyframes)."""
    rng = np.random.default_rng(seed)
    n_keys = n_frames // every + 2
    keys = rng.normal(0.0, sigma, size=(n_keys, n, N_JOINTS, 3))
    out = np.empty((n_frames, n, N_JOINTS, 3), np.float32)
    for f in range(n_frames):
        k, r = divmod(f, every)
        a = r / every
        out[f] = ((1.0 - a) * keys[k] + a * keys[k + 1]).astype(np.float32)
    return out


def sphere_cameras(seed: int, count: int, center, radius: float, width: int,
                   height: int) -> List[Camera]:
    """Cameras uniform on a sphere about ``center`` looking at it, rejecting
    views with |forward . y| >= 0.99."""
    rng = np.random.default_rng(seed)
    cams = []
    center = np.asarray(center, np.float64)
    while len(cams) < count:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if abs(d[1]) >= 0.99:
            continue
        cams.append(look_at(center + radius * d, center, width, height))
    return cams


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    name: str
    templates: List[Template]
    crowd: Crowd
    camera: Camera
    tile: tuple = (16, 16)
    lod_thresholds: Optional[Sequence[float]] = None  # fixed-distance LoD
    frame_poses: Optional[np.ndarray] = None          # [F, n, 24, 3]


C2_LEVELS = (1.0, 0.25, 0.0625)
C4_LEVELS = (1.0, 0.5, 0.25, 0.125, 0.0625)


def scene_c1() -> Scene:
    """Plain method: 1 template (2,048 Gaussians, SH0, seed 0) x 1 instance,
    256x256, pose ~ N(0, 0.2), camera 3 m away at mid-height."""
    t = make_template(0, 2048, 0)
    rng = np.random.default_rng(1)
    pose = rng.normal(0.0, 0.2, size=(1, N_JOINTS, 3)).astype(np.float32)
    crowd = Crowd(tid=np.zeros(1, np.int32), yaw=np.zeros(1, np.float32),
                  pos=np.zeros((1, 2), np.float32), pose=pose)
    h = 0.5 * float(t.mean[:, 1].max())
    cam = look_at((0.0, h, -3.0), (0.0, h, 0.0), 256, 256)
    return Scene("c1", [t], crowd, cam)


def c2_templates(n_gauss: int = 100_000, levels=C2_LEVELS, count: int = 14):
    return [make_template(t, n_gauss, 3, levels) for t in range(count)]


def scene_c2(templates=None, n_gauss: int = 100_000) -> Scene:
    """14 templates x 100k Gaussians (SH3), 500 instances on a 50x50 m plane,
    fixed 3-level LoD (100/25/6.25 %) at 10 m and 25 m, 1920x1080."""
    templates = templates or c2_templates(n_gauss)
    crowd = make_crowd(100, 500, len(templates), 50.0, 0.3)
    cam = look_at((25.0, 1.7, -3.0), (25.0, 1.0, 25.0), 1920, 1080)
    return Scene("c2", templates, crowd, cam, lod_thresholds=(10.0, 25.0))


def scene_c3(templates=None, n_frames: int = 300, n_gauss: int = 100_000,
             n_inst: int = 3500) -> Scene:
    """3,500 instances on an 80x80 m plane, same templates and LoD as C2,
    300-frame animation from keyframes every 15 frames, 1920x1080."""
    templates = templates or c2_templates(n_gauss)
    crowd = make_crowd(200, n_inst, len(templates), 80.0, 0.3)
    frames = keyframe_poses(300, n_inst, n_frames, 15, 0.3) if n_frames else None
    if frames is not None:
        crowd.pose = frames[0].copy()
    cam = look_at((40.0, 1.7, -3.0), (40.0, 1.0, 40.0), 1920, 1080)
    return Scene("c3", templates, crowd, cam, lod_thresholds=(10.0, 25.0),
                 frame_poses=frames)


def scene_c5(n_gauss: int = 100_000, width: int = 512):
    """One template (seed 500, SH3) at the origin, 64 cameras on a 3 m sphere
    about its bounding-box centre (seed 501)."""
    t = make_template(500, n_gauss, 3)
    center = 0.5 * (t.mean.min(axis=0) + t.mean.max(axis=0))
    cams = sphere_cameras(501, 64, center, 3.0, width, width)
    crowd = Crowd(tid=np.zeros(1, np.int32), yaw=np.zeros(1, np.float32),
                  pos=np.zeros((1, 2), np.float32),
                  pose=np.zeros((1, N_JOINTS, 3), np.float32))
    return t, crowd, cams


def perturb_template(t: Template, seed: int = 502, pos_sigma: float = 0.01,
                     rgb_sigma: float = 0.1) -> Template:
    """The fit's starting point: positions + N(0, pos_sigma) m, colours +
    N(0, rgb_sigma) (added to the DC band as eps / SH_C0)."""
    rng = np.random.default_rng(seed)
    out = dataclasses.replace(t, mean=t.mean.copy(), sh=t.sh.copy())
    out.mean += rng.normal(0.0, pos_sigma, size=t.mean.shape).astype(np.float32)
    out.sh[:, 0, :] += (rng.normal(0.0, rgb_sigma, size=(t.n, 3)) / SH_C0).astype(np.float32)
    return out


# ----------------------------------------------------------------------------
# the paper's own crowd set-up (§2 last paragraph, §3 Tab. 1 and Tab. 2)
# ----------------------------------------------------------------------------

#: Gaussians per character in the paper's three template resolutions (§2, §3).
PAPER_SIZES = (202_738, 12_661, 3_176)
#: characters per cell of Tab. 1 / Tab. 2
PAPER_CHARS = (1, 100, 400, 1_000, 5_000)
#: the cells Tab. 2 fills: (Gaussians, animated) -> character counts
TAB2_CELLS = {
    (202_738, False): (1, 100, 400), (202_738, True): (1, 100),
    (12_661, False): PAPER_CHARS, (12_661, True): PAPER_CHARS,
    (3_176, False): PAPER_CHARS, (3_176, True): PAPER_CHARS,
}
#: the cells Tab. 1 fills: Gaussians -> character counts
TAB1_CELLS = {202_738: (1, 100), 12_661: PAPER_CHARS, 3_176: PAPER_CHARS}
GRID_SPACING = 1.5   # metres between neighbouring grid cells
N_CLIPS = 15         # looping motion clips driving the crowd (§2: 15 motion sequences)
CLIP_FRAMES = 60     # frames per loop (2 s at 30 Hz)


def make_template_counts(seed: int, level_counts: Sequence[int], sh_degree: int = 3) -> Template:
    """A template whose LoD levels hold exactly ``level_counts`` Gaussians
    (importance prefixes of one template of ``level_counts[0]`` Gaussians)."""
    n = int(level_counts[0])
    t = make_template(seed, n, sh_degree)
    t.level_count = np.asarray(level_counts, np.int32)
    return t


def grid_crowd(seed: int, n: int, n_templates: int, spacing: float = GRID_SPACING) -> Crowd:
    """``n`` characters on a square-ish grid (columns = ceil(sqrt(n)), rows
    filled front to back), each with a random template and yaw; the first row
    is at z = 0 and the grid is centred on x = 0. Poses are zero (rest pose);
    animated crowds take theirs from ``clip_poses``."""
    rng = np.random.default_rng(seed)
    cols = max(1, int(math.ceil(math.sqrt(n))))
    k = np.arange(n)
    row, col = k // cols, k % cols
    x = (col - 0.5 * (cols - 1)) * spacing
    z = row * spacing
    tid = rng.integers(0, n_templates, size=n).astype(np.int32)
    yaw = rng.uniform(0.0, 2 * np.pi, size=n).astype(np.float32)
    pos = np.stack([x, z], axis=1).astype(np.float32)
    return Crowd(tid=tid, yaw=yaw, pos=pos, pose=np.zeros((n, N_JOINTS, 3), np.float32))


def looping_clips(seed: int, n_clips: int = N_CLIPS, frames: int = CLIP_FRAMES,
                  sigma: float = 0.3) -> np.ndarray:
    """``n_clips`` seeded looping motions, f32 [n_clips, frames, 24, 3]: every
    joint angle is a sum of two sinusoids (the loop's fundamental and its
    second harmonic) with random amplitudes ~ |N(0, sigma)| and phases, so a
    clip returns to its first pose after ``frames`` frames."""
    rng = np.random.default_rng(seed)
    a1 = np.abs(rng.normal(0.0, sigma, size=(n_clips, 1, N_JOINTS, 3)))
    a2 = np.abs(rng.normal(0.0, 0.5 * sigma, size=(n_clips, 1, N_JOINTS, 3)))
    p1 = rng.uniform(0.0, 2 * np.pi, size=(n_clips, 1, N_JOINTS, 3))
    p2 = rng.uniform(0.0, 2 * np.pi, size=(n_clips, 1, N_JOINTS, 3))
    t = (2 * np.pi * np.arange(frames) / frames)[None, :, None, None]
    return (a1 * np.sin(t + p1) + a2 * np.sin(2 * t + p2)).astype(np.float32)


def clip_assignment(seed: int, n: int, n_clips: int = N_CLIPS, frames: int = CLIP_FRAMES):
    """Each character's clip and its phase offset (in frames)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, n_clips, size=n).astype(np.int64),
            rng.integers(0, frames, size=n).astype(np.int64))


def clip_poses(clips: np.ndarray, clip_of: np.ndarray, phase: np.ndarray, frame: int) -> np.ndarray:
    """The crowd's poses at ``frame`` (f32 [n, 24, 3]): character i plays clip
    clip_of[i] from frame phase[i], looping."""
    f = (frame + phase) % clips.shape[1]
    return np.ascontiguousarray(clips[clip_of, f])


def paper_camera(width: int, height: int, first_row_z: float = 0.0) -> Camera:
    """Static camera three metres in front of the crowd's first row (§2), at
    eye height, looking down the grid."""
    return look_at((0.0, 1.7, first_row_z - 3.0), (0.0, 1.0, first_row_z + 25.0), width, height)


def scene_tab2(n_gauss: int, n_chars: int, animated: bool, width: int = 1280, height: int = 720,
               template: Optional[Template] = None, frames: int = CLIP_FRAMES) -> Scene:
    """One cell of Tab. 1 / Tab. 2: ``n_chars`` duplicates of one SH3 template
    of ``n_gauss`` Gaussians (seed 600 + its size index) on the grid, static
    camera 3 m from the first row, 1280x720. Animated cells carry
    ``frames`` frames of looping clips (``frame_poses``); static cells keep the
    rest pose."""
    if template is None:
        k = PAPER_SIZES.index(n_gauss) if n_gauss in PAPER_SIZES else 3
        template = make_template(600 + k, n_gauss, 3)
    crowd = grid_crowd(700 + n_chars, n_chars, 1)
    poses = None
    if animated:
        clips = looping_clips(800)
        clip_of, phase = clip_assignment(801 + n_chars, n_chars)
        poses = np.stack([clip_poses(clips, clip_of, phase, f) for f in range(frames)])
        crowd.pose = poses[0].copy()
    cam = paper_camera(width, height)
    return Scene(f"tab2_{n_gauss}x{n_chars}_{'anim' if animated else 'static'}", [template], crowd, cam,
                 frame_poses=poses)


def scene_paper_lod(n_chars: int = 3500, n_templates: int = 14, width: int = 1920, height: int = 1080,
                    templates=None, frames: int = CLIP_FRAMES, sh_degree: int = 3) -> Scene:
    """The paper's LoD set-up (§2 last paragraph): 3,500 characters from 14
    templates on the grid, camera 3 m from the first row, 15 looping motions,
    three levels of 202,738 / 12,661 / 3,176 Gaussians (importance prefixes)
    chosen at 5 m and 10 m."""
    if templates is None:
        templates = [make_template_counts(900 + t, PAPER_SIZES, sh_degree) for t in range(n_templates)]
    crowd = grid_crowd(1000, n_chars, len(templates))
    clips = looping_clips(1001)
    clip_of, phase = clip_assignment(1002, n_chars)
    poses = np.stack([clip_poses(clips, clip_of, phase, f) for f in range(frames)]) if frames else None
    if poses is not None:
        crowd.pose = poses[0].copy()
    cam = paper_camera(width, height)
    return Scene("paper_lod", templates, crowd, cam, lod_thresholds=(5.0, 10.0), frame_poses=poses)


# ----------------------------------------------------------------------------
# pose-dependent offset network (synthetic weights; §2's GaussianAvatar stage)
# ----------------------------------------------------------------------------

def pose_net_weights(seed: int = 1100, offset_scale: float = 0.01) -> dict:
    """Synthetic weights of the 112 -> 64 -> 64 -> 3 offset network
    (float32): He-scaled hidden layers with small random biases, and an
    output layer scaled so that offsets are about ``offset_scale`` metres."""
    rng = np.random.default_rng(seed)
    return dict(w1=rng.normal(0.0, math.sqrt(2.0 / 112), (64, 112)).astype(np.float32),
                b1=rng.normal(0.0, 0.1, 64).astype(np.float32),
                w2=rng.normal(0.0, math.sqrt(2.0 / 64), (64, 64)).astype(np.float32),
                b2=rng.normal(0.0, 0.1, 64).astype(np.float32),
                w3=rng.normal(0.0, offset_scale / 8.0, (3, 64)).astype(np.float32),
                b3=rng.normal(0.0, 0.1 * offset_scale, 3).astype(np.float32))


def pose_embeddings(seed: int, n: int) -> np.ndarray:
    """Per-Gaussian embeddings [n, 32] ~ N(0, 1) (float32) of one template."""
    return np.random.default_rng(seed).normal(0.0, 1.0, (n, 32)).astype(np.float32)
