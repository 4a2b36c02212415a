"""ctypes binding of libcrowdsplat.so (the C ABI in include/crowdsplat.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels. torch supplies device memory (tensors) and the stream. If the
library has not been built, importing the binding raises; there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrowdsplat.so")

CS_OK = 0
CS_ERR_INVALID, CS_ERR_OOM, CS_ERR_DEVICE, CS_ERR_CAPACITY, CS_ERR_STATE, CS_ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6
CS_MEM_HOST, CS_MEM_DEVICE = 0, 1
CS_SKIN_FULL, CS_SKIN_MEANS_ONLY = 0, 1
CS_LAUNCH_BATCHED, CS_LAUNCH_PER_INSTANCE = 0, 1
CS_SORT_TILE_BUCKET, CS_SORT_ONESWEEP, CS_SORT_REDUCE_SCAN = 0, 1, 2
CS_NOALLOC_MAX_PAIRS = 1 << 20
CS_SORT_RANKS_CHECKED, CS_SORT_RANKS_BALLOT = 0, 1
CS_LOD_FULL, CS_LOD_FIXED, CS_LOD_LEARNED, CS_LOD_CONSTANT, CS_LOD_BUDGET = 0, 1, 2, 3, 4
CS_LOD_BUDGET_VISIBLE = 5
CS_MLP_NPARAM, CS_MLP_NBF16 = 7312, 7168
#: offsets of the layers inside cs_mlp.params (out-major weights)
MLP_OFF = dict(w1=(0, (64, 32)), b1=(2048, (64,)), w2=(2112, (64, 64)), b2=(6208, (64,)),
               w3=(6272, (16, 64)), b3=(7296, (16,)))
CS_MAX_LEVELS = 8

BUF = dict(BONES=1, LEVEL=2, OFFSET=3, SKIN_MU=4, SKIN_COV=5, SKIN_COV2=6, RECORD=7, RECT=8,
           COUNT=9, PAIR_OFF=10, KEYS=11, VALS=12, SKEYS=13, SVALS=14, RANGES=15, FEATURES=16,
           PRED=17, VIEWS=18, JOINTS=19, OFFSETS=20, VISIBLE=21)

#: every symbol include/crowdsplat.h declares
EXPORTS = ["cs_create", "cs_destroy", "cs_last_error", "cs_version", "cs_upload_templates",
           "cs_select_lod", "cs_skin_instances", "cs_render_frame", "cs_render_backward",
           "cs_reserve", "cs_frame_capture", "cs_frame_launch", "cs_frame_poll", "cs_debug_copy",
           "cs_sort_pairs", "cs_stage_times", "cs_lod_features", "cs_mlp_predict", "cs_mlp_sync",
           "cs_mlp_train_step", "cs_render_views", "cs_view_psnr", "cs_update_template", "cs_fit_loss",
           "cs_adam", "cs_materialise_instances", "cs_memory_report",
           "cs_frame_capture_render", "cs_set_pose_ring", "cs_upload_pose_net", "cs_sort_pairs_noalloc", "cs_copy"]
STAGES = ["lod", "fk", "skin", "project", "scan", "emit", "sort", "ranges", "blend", "segsort", "offsets"]


class CsOptions(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("skin_mode", ctypes.c_int32), ("launch_mode", ctypes.c_int32),
                ("fuse_skin_project", ctypes.c_int32), ("profile_stages", ctypes.c_int32),
                ("max_splats", ctypes.c_int64), ("max_pairs", ctypes.c_int64),
                ("sort_algo", ctypes.c_int32), ("sort_ranks", ctypes.c_int32),
                ("count_blend", ctypes.c_int32), ("bin_blocks", ctypes.c_int32), ("sort_blocks", ctypes.c_int32),
                ("blend_split", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class CsTemplateDesc(ctypes.Structure):
    _fields_ = [("n_gauss", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("level_count", ctypes.c_void_p), ("mean", ctypes.c_void_p),
                ("log_scale", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("skin_idx", ctypes.c_void_p), ("skin_w", ctypes.c_void_p),
                ("joints_rest", ctypes.c_void_p), ("parents", ctypes.c_void_p)]


class CsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("eye", ctypes.c_float * 3), ("R", ctypes.c_float * 9),
                ("near_plane", ctypes.c_float), ("bg", ctypes.c_float * 3)]


class CsLodParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n_thresholds", ctypes.c_int32),
                ("thresholds", ctypes.c_float * 7), ("level", ctypes.c_int32),
                ("psnr_min", ctypes.c_float), ("margin", ctypes.c_float), ("mlp", ctypes.c_void_p)]


class CsMlp(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_float * 32), ("inv_sd", ctypes.c_float * 32),
                ("pca_mean", ctypes.c_float * 72), ("pca_basis", ctypes.c_float * (8 * 72)),
                ("params", ctypes.c_float * CS_MLP_NPARAM), ("w_bf16", ctypes.c_uint16 * CS_MLP_NBF16)]


class CsFrameStats(ctypes.Structure):
    _fields_ = [("n_splats", ctypes.c_int64), ("n_visible", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("overflow", ctypes.c_int32),
                ("n_instances", ctypes.c_int32), ("level_hist", ctypes.c_int32 * CS_MAX_LEVELS),
                ("sort_fallbacks", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("blend_evals", ctypes.c_int64), ("blend_eval_slots", ctypes.c_int64),
                ("blend_done_slots", ctypes.c_int64), ("blend_adds", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 1)]


CS_PNET_EMBED, CS_PNET_POSE, CS_PNET_HIDDEN = 32, 80, 64


class CsPoseNet(ctypes.Structure):
    _fields_ = [("w1", (ctypes.c_float * (CS_PNET_EMBED + CS_PNET_POSE)) * CS_PNET_HIDDEN),
                ("b1", ctypes.c_float * CS_PNET_HIDDEN),
                ("w2", (ctypes.c_float * CS_PNET_HIDDEN) * CS_PNET_HIDDEN),
                ("b2", ctypes.c_float * CS_PNET_HIDDEN),
                ("w3", (ctypes.c_float * CS_PNET_HIDDEN) * 3), ("b3", ctypes.c_float * 3),
                ("reserved", ctypes.c_int32)]


class CsMemoryStats(ctypes.Structure):
    _fields_ = [("templates", ctypes.c_int64), ("instance_copies", ctypes.c_int64),
                ("per_instance", ctypes.c_int64), ("per_splat", ctypes.c_int64),
                ("per_pair", ctypes.c_int64), ("workspace", ctypes.c_int64), ("total", ctypes.c_int64),
                ("peak", ctypes.c_int64), ("cap_instances", ctypes.c_int64), ("cap_splats", ctypes.c_int64),
                ("cap_pairs", ctypes.c_int64), ("n_copies", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 4)]


class CsTemplateGrads(ctypes.Structure):
    _fields_ = [("template_id", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


INSTANCE_DTYPE = np.dtype([("tid", "<i4"), ("yaw", "<f4"), ("px", "<f4"), ("pz", "<f4")])


class CrowdSplatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"crowdsplat error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2501_17792_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "cs_create": (i32, [i32, P, ctypes.POINTER(CsOptions), ctypes.POINTER(P)]),
        "cs_destroy": (None, [P]),
        "cs_last_error": (ctypes.c_char_p, [P]),
        "cs_version": (ctypes.c_char_p, []),
        "cs_upload_templates": (i32, [P, ctypes.POINTER(CsTemplateDesc), i32, i32]),
        "cs_select_lod": (i32, [P, i32, P, P, ctypes.POINTER(CsCamera), ctypes.POINTER(CsLodParams), P]),
        "cs_skin_instances": (i32, [P, i32, P, P]),
        "cs_render_frame": (i32, [P, ctypes.POINTER(CsCamera), P, ctypes.POINTER(CsFrameStats)]),
        "cs_render_backward": (i32, [P, P, ctypes.POINTER(CsTemplateGrads)]),
        "cs_reserve": (i32, [P, i64, i64, i64]),
        "cs_frame_capture": (i32, [P, i32, P, P, ctypes.POINTER(CsCamera), ctypes.POINTER(CsLodParams), P]),
        "cs_frame_launch": (i32, [P]),
        "cs_frame_capture_render": (i32, [P, ctypes.POINTER(CsCamera), P]),
        "cs_set_pose_ring": (i32, [P, P, i32, i32, i64]),
        "cs_upload_pose_net": (i32, [P, ctypes.POINTER(CsPoseNet), P]),
        "cs_frame_poll": (i32, [P, ctypes.POINTER(CsFrameStats)]),
        "cs_debug_copy": (i32, [P, i32, P, i64, i64]),
        "cs_sort_pairs": (i32, [P, P, P, i64, i32]),
        "cs_sort_pairs_noalloc": (i32, [P, P, P, i64, i32]),
        "cs_copy": (i32, [P, P, P, i64]),
        "cs_materialise_instances": (i32, [P, i32, P]),
        "cs_memory_report": (i32, [P, ctypes.POINTER(CsMemoryStats)]),
        "cs_stage_times": (i32, [P, ctypes.POINTER(ctypes.c_float), i32]),
        "cs_lod_features": (i32, [P, i32, P, P, ctypes.POINTER(CsCamera), P, P]),
        "cs_mlp_predict": (i32, [P, P, P, i32, P]),
        "cs_mlp_sync": (i32, [P, P]),
        "cs_mlp_train_step": (i32, [P, P, P, P, P, P, i32, i32, ctypes.c_float, P]),
        "cs_render_views": (i32, [P, ctypes.POINTER(CsCamera), P, i64, ctypes.POINTER(i64)]),
        "cs_view_psnr": (i32, [P, P, P, P]),
        "cs_update_template": (i32, [P, i32, ctypes.POINTER(CsTemplateDesc), i32]),
        "cs_fit_loss": (i32, [P, P, P, i32, i32, ctypes.c_float, P, P]),
        "cs_adam": (i32, [P, P, P, P, P, i64, i32, ctypes.c_float]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def camera_struct(cam) -> CsCamera:
    c = CsCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.eye[:] = [float(v) for v in np.asarray(cam.eye, np.float32)]
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).ravel()]
    c.near_plane = float(cam.near)
    c.bg[:] = [float(v) for v in np.asarray(cam.bg, np.float32)]
    return c


def lod_struct(mode: int, thresholds: Sequence[float] = (), psnr_min: float = 40.0,
               margin: float = 1.0, mlp_ptr: int = 0, level: int = 0) -> CsLodParams:
    p = CsLodParams()
    p.mode = mode
    p.level = level
    p.n_thresholds = len(thresholds)
    for k, t in enumerate(thresholds):
        p.thresholds[k] = float(t)
    p.psnr_min = psnr_min
    p.margin = margin
    p.mlp = mlp_ptr or None
    return p


def instance_bytes(crowd) -> np.ndarray:
    a = np.zeros(crowd.n, INSTANCE_DTYPE)
    a["tid"] = crowd.tid
    a["yaw"] = crowd.yaw
    a["px"] = crowd.pos[:, 0]
    a["pz"] = crowd.pos[:, 1]
    return a


class Renderer:
    """One library context on one device and stream."""

    def __init__(self, device: int = 0, stream=None, tile=(16, 16), skin_mode=CS_SKIN_FULL,
                 launch_mode=CS_LAUNCH_BATCHED, fuse=False, max_splats=0, max_pairs=0,
                 profile=False, sort_algo=CS_SORT_TILE_BUCKET, sort_ranks=CS_SORT_RANKS_CHECKED,
                 count_blend=False, blocks=(0, 0), blend_split=0):
        """``blocks``: (bin_blocks, sort_blocks) of cs_options (0: defaults);
        ``blend_split``: workgroups compositing one binning tile (0: one)."""
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        opt = CsOptions()
        opt.tile_w, opt.tile_h = tile
        opt.skin_mode, opt.launch_mode, opt.fuse_skin_project = skin_mode, launch_mode, int(fuse)
        opt.profile_stages = int(profile)
        opt.sort_algo = sort_algo
        opt.sort_ranks = sort_ranks
        opt.count_blend = int(count_blend)
        opt.bin_blocks, opt.sort_blocks = (int(b) for b in blocks)
        opt.blend_split = int(blend_split)
        opt.max_splats, opt.max_pairs = max_splats, max_pairs
        self.tile = tuple(tile)
        ctx = ctypes.c_void_p()
        self._check(self.lib.cs_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(opt), ctypes.byref(ctx)), None)
        self.ctx = ctx
        self._keep = []
        self.templates = None

    # ------------------------------------------------------------------ util
    def _check(self, status: int, ctx=None):
        if status != CS_OK:
            c = ctx if ctx is not None else getattr(self, "ctx", None)
            msg = self.lib.cs_last_error(c).decode() if c else "(no context)"
            raise CrowdSplatError(status, msg)

    def _hold(self, *tensors):
        """Device tensors the library reads asynchronously on the context's
        stream: the caching allocator must not hand their memory to a later
        allocation before that stream's work up to here has run."""
        for t in tensors:
            if t.is_cuda:
                t.record_stream(self.stream)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.cs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def to_device(self, arr: np.ndarray):
        t = self.torch.from_numpy(np.ascontiguousarray(arr).view(np.uint8).reshape(-1).copy())
        return t.to(self.device)

    # ------------------------------------------------------------------ calls
    def upload_templates(self, templates, mem=CS_MEM_HOST):
        descs = (CsTemplateDesc * len(templates))()
        keep = []
        for d, t in zip(descs, templates):
            arrs = dict(level_count=np.ascontiguousarray(t.level_count, np.int32),
                        mean=np.ascontiguousarray(t.mean, np.float32),
                        log_scale=np.ascontiguousarray(t.log_scale, np.float32),
                        quat=np.ascontiguousarray(t.quat, np.float32),
                        opacity=np.ascontiguousarray(t.opacity, np.float32),
                        sh=np.ascontiguousarray(t.sh, np.float32),
                        skin_idx=np.ascontiguousarray(t.skin_idx, np.uint8),
                        skin_w=np.ascontiguousarray(t.skin_w, np.float32),
                        joints_rest=np.ascontiguousarray(t.joints_rest, np.float32),
                        parents=np.ascontiguousarray(t.parents, np.int32))
            keep.append(arrs)
            d.n_gauss, d.sh_degree, d.n_levels = t.n, t.sh_degree, len(t.level_count)
            for k, a in arrs.items():
                setattr(d, k, a.ctypes.data)
        self._check(self.lib.cs_upload_templates(self.ctx, descs, len(templates), mem))
        self.templates = templates

    def set_crowd(self, crowd):
        """Device copies of the instance table and poses (kept alive here)."""
        self.inst_dev = self.to_device(instance_bytes(crowd))
        self.pose_dev = self.torch.from_numpy(np.ascontiguousarray(crowd.pose, np.float32)).to(self.device)
        self.n_inst = crowd.n

    def select_lod(self, cam, mode=CS_LOD_FIXED, thresholds=(10.0, 25.0), level_out=None,
                   psnr_min=40.0, margin=1.0, mlp_ptr=0, level=0):
        c = camera_struct(cam)
        p = lod_struct(mode, thresholds, psnr_min, margin, mlp_ptr, level)
        self._check(self.lib.cs_select_lod(self.ctx, self.n_inst, self.inst_dev.data_ptr(),
                                           self.pose_dev.data_ptr(), ctypes.byref(c), ctypes.byref(p),
                                           level_out.data_ptr() if level_out is not None else None))

    def skin(self):
        self._check(self.lib.cs_skin_instances(self.ctx, self.n_inst, self.inst_dev.data_ptr(),
                                               self.pose_dev.data_ptr()))

    def render(self, cam, image=None, stats: bool = False):
        torch = self.torch
        if image is None:
            image = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=self.device)
        c = camera_struct(cam)
        st = CsFrameStats()
        self._check(self.lib.cs_render_frame(self.ctx, ctypes.byref(c), image.data_ptr(),
                                             ctypes.byref(st) if stats else None))
        self.last_stats = st if stats else None
        self.last_camera = cam
        return image

    def frame(self, cam, mode=CS_LOD_FIXED, thresholds=(10.0, 25.0), image=None, stats=False):
        self.select_lod(cam, mode, thresholds)
        self.skin()
        return self.render(cam, image, stats)

    def reserve(self, max_instances=0, max_splats=0, max_pairs=0):
        self._check(self.lib.cs_reserve(self.ctx, max_instances, max_splats, max_pairs))

    def capture(self, cam, image, mode=CS_LOD_FIXED, thresholds=(10.0, 25.0), mlp_ptr=0,
                psnr_min=40.0, margin=1.0):
        """Capture select_lod -> skin -> render for fixed pointers into a graph."""
        c = camera_struct(cam)
        p = lod_struct(mode, thresholds, psnr_min, margin, mlp_ptr)
        self._keep = [c, p]
        self._check(self.lib.cs_frame_capture(self.ctx, self.n_inst, self.inst_dev.data_ptr(),
                                              self.pose_dev.data_ptr(), ctypes.byref(c),
                                              ctypes.byref(p), image.data_ptr()))

    def upload_pose_net(self, net, embeds):
        """The pose-dependent offset network (dict w1 [64,112], b1, w2 [64,64],
        b2, w3 [3,64], b3; float32) and one [n, 32] embedding array per
        uploaded template; ``net=None`` removes it."""
        if net is None:
            self._check(self.lib.cs_upload_pose_net(self.ctx, None, None))
            return
        n = CsPoseNet()
        for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
            a = np.ascontiguousarray(net[k], np.float32)
            ctypes.memmove(ctypes.addressof(getattr(n, k)), a.ctypes.data, a.nbytes)
        keep = [np.ascontiguousarray(e, np.float32) for e in embeds]
        ptrs = (ctypes.c_void_p * len(keep))(*[e.ctypes.data for e in keep])
        self._check(self.lib.cs_upload_pose_net(self.ctx, ctypes.byref(n), ptrs))

    def set_pose_ring(self, ring, first: int = 0):
        """Poses of every replay of the next captured frame come from ``ring``
        (tensor [n_frames, n_inst, 24, 3] f32, on the device or pinned on the
        host); None removes it."""
        if ring is None:
            self._check(self.lib.cs_set_pose_ring(self.ctx, None, 0, 0, 0))
            self.pose_ring = None
            return
        assert ring.dtype == self.torch.float32 and ring.is_contiguous() and ring.dim() == 4
        self._check(self.lib.cs_set_pose_ring(self.ctx, ring.data_ptr(), ring.shape[0], ring.shape[1], first))
        self.pose_ring = ring  # the library reads it at every replay

    def capture_render(self, cam, image):
        """Capture rendering alone over the resident skinned crowd (static crowd)."""
        c = camera_struct(cam)
        self._keep = [c]
        self._check(self.lib.cs_frame_capture_render(self.ctx, ctypes.byref(c), image.data_ptr()))

    def launch(self):
        self._check(self.lib.cs_frame_launch(self.ctx))

    def poll(self) -> CsFrameStats:
        st = CsFrameStats()
        self._check(self.lib.cs_frame_poll(self.ctx, ctypes.byref(st)))
        return st

    def materialise(self, enable: bool = True):
        """Give every instance of the current crowd its own copy of its
        template's attributes (the unshared layout), or return to sharing."""
        self._check(self.lib.cs_materialise_instances(self.ctx, self.n_inst if enable else 0,
                                                      self.inst_dev.data_ptr() if enable else None))

    def memory(self) -> dict:
        """Device bytes this context holds, by category (cs_memory_report)."""
        m = CsMemoryStats()
        self._check(self.lib.cs_memory_report(self.ctx, ctypes.byref(m)))
        return {name: int(getattr(m, name)) for name, _ in CsMemoryStats._fields_ if name != "reserved"}

    def debug(self, name: str, dtype, count: int, offset: int = 0) -> np.ndarray:
        out = np.empty(count, dtype)
        self._check(self.lib.cs_debug_copy(self.ctx, BUF[name], out.ctypes.data,
                                           offset * out.itemsize, out.nbytes))
        return out

    def stage_times(self) -> dict:
        ms = (ctypes.c_float * len(STAGES))()
        self._check(self.lib.cs_stage_times(self.ctx, ms, len(STAGES)))
        return {name: float(ms[k]) for k, name in enumerate(STAGES) if ms[k] >= 0}

    # ------------------------------------------------------------ learned LoD
    def lod_features(self, cam, net, feat=None):
        torch = self.torch
        if feat is None:
            feat = torch.empty((self.n_inst, 32), dtype=torch.float32, device=self.device)
        c = camera_struct(cam)
        self._check(self.lib.cs_lod_features(self.ctx, self.n_inst, self.inst_dev.data_ptr(),
                                             self.pose_dev.data_ptr(), ctypes.byref(c), net.data_ptr(),
                                             feat.data_ptr()))
        return feat

    def mlp_predict(self, net, feat):
        pred = self.torch.empty((feat.shape[0], 16), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.cs_mlp_predict(self.ctx, net.data_ptr(), feat.data_ptr(), feat.shape[0],
                                            pred.data_ptr()))
        return pred

    def mlp_sync(self, net):
        self._check(self.lib.cs_mlp_sync(self.ctx, net.data_ptr()))

    def mlp_train_step(self, net, m, v, feat, target, step, lr=1e-3, loss=None):
        self._check(self.lib.cs_mlp_train_step(self.ctx, net.data_ptr(), m.data_ptr(), v.data_ptr(),
                                               feat.data_ptr(), target.data_ptr(), feat.shape[0], step,
                                               lr, loss.data_ptr() if loss is not None else None))

    def render_views(self, cam, atlas=None):
        """Render each instance alone into its window; returns (atlas, views [n,6])."""
        torch = self.torch
        c = camera_struct(cam)
        need = ctypes.c_int64(0)
        if atlas is None:
            atlas = torch.empty(1, dtype=torch.float32, device=self.device)
        st = self.lib.cs_render_views(self.ctx, ctypes.byref(c), atlas.data_ptr(), atlas.numel(),
                                      ctypes.byref(need))
        if st == CS_ERR_CAPACITY and need.value > atlas.numel():
            atlas = torch.empty(max(need.value, 1), dtype=torch.float32, device=self.device)
            st = self.lib.cs_render_views(self.ctx, ctypes.byref(c), atlas.data_ptr(), atlas.numel(),
                                          ctypes.byref(need))
        self._check(st)
        views = self.debug("VIEWS", np.int64, 6 * self.n_inst).reshape(self.n_inst, 6)
        return atlas, views

    def view_psnr(self, atlas_ref, atlas):
        out = self.torch.empty(self.n_inst, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.cs_view_psnr(self.ctx, atlas_ref.data_ptr(), atlas.data_ptr(), out.data_ptr()))
        return out

    # ------------------------------------------------------------ backward / fit
    def render_backward(self, dimg, tid: int = 0):
        """Template gradients of sum(dimg * last image): dict of device tensors."""
        torch = self.torch
        t = self.templates[tid]
        K = (t.sh_degree + 1) ** 2
        out = dict(mean=torch.empty((t.n, 3), device=self.device), log_scale=torch.empty((t.n, 3), device=self.device),
                   quat=torch.empty((t.n, 4), device=self.device), opacity_logit=torch.empty(t.n, device=self.device),
                   sh=torch.empty((t.n, K, 3), device=self.device))
        g = CsTemplateGrads()
        g.template_id = tid
        for k, v in out.items():
            setattr(g, k, v.data_ptr())
        dimg_c = dimg.contiguous()
        self._check(self.lib.cs_render_backward(self.ctx, dimg_c.data_ptr(), ctypes.byref(g)))
        self._hold(dimg_c)
        return out

    def update_template(self, tid, mean, log_scale, quat, opacity, sh, skin_idx, skin_w, opacity_is_logit=True):
        d = CsTemplateDesc()
        t = self.templates[tid]
        d.n_gauss, d.sh_degree, d.n_levels = t.n, t.sh_degree, len(t.level_count)
        held = []
        for k, v in dict(mean=mean, log_scale=log_scale, quat=quat, opacity=opacity, sh=sh, skin_idx=skin_idx,
                         skin_w=skin_w).items():
            vc = v.contiguous()
            held.append(vc)
            setattr(d, k, vc.data_ptr())
        self._check(self.lib.cs_update_template(self.ctx, tid, ctypes.byref(d), int(opacity_is_logit)))
        self._hold(*held)

    def fit_loss(self, x, y, lam=0.2, want_grad=True):
        torch = self.torch
        loss = torch.empty(1, device=self.device)
        dx = torch.empty_like(x) if want_grad else None
        self._check(self.lib.cs_fit_loss(self.ctx, x.data_ptr(), y.data_ptr(), x.shape[2], x.shape[1], lam,
                                          loss.data_ptr(), dx.data_ptr() if dx is not None else None))
        return loss, dx

    def adam(self, p, g, m, v, step, lr):
        self._check(self.lib.cs_adam(self.ctx, p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(),
                                     step, lr))

    def sort_pairs(self, keys, vals, key_bits: int):
        self._check(self.lib.cs_sort_pairs(self.ctx, keys.data_ptr(), vals.data_ptr(),
                                           keys.numel(), key_bits))

    def copy(self, dst, src, nbytes=None):
        """Device copy with the library's copy kernel (bandwidth reference)."""
        nb = src.numel() * src.element_size() if nbytes is None else nbytes
        assert dst.numel() * dst.element_size() >= nb
        self._hold(dst, src)
        self._check(self.lib.cs_copy(self.ctx, dst.data_ptr(), src.data_ptr(), nb))

    def sort_pairs_noalloc(self, keys, vals, key_bits: int, n=None):
        """The same sort with the library's fixed per-device scratch
        (asynchronous on the context's stream; n <= CS_NOALLOC_MAX_PAIRS)."""
        self._hold(keys, vals)
        self._check(self.lib.cs_sort_pairs_noalloc(self.ctx, keys.data_ptr(), vals.data_ptr(),
                                                   keys.numel() if n is None else n, key_bits))
