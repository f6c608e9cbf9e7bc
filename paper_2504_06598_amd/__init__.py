"""Python binding of libsrt: stochastic ray tracing of transparent 3D Gaussians
on AMD MI355X (gfx950).

Argument marshalling only: every step runs in the HIP kernels of libsrt.so,
reached through its C ABI (include/srt.h). PyTorch provides device memory and
the current stream. The functions carry the C entry points' names.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import COUNTER_NAMES, SRT_NUM_COUNTERS, SrtError

__all__ = ["DeviceScene", "Bvh", "BatchPlan", "srt_build_bvh", "srt_refit_bvh",
           "srt_trace_forward",
           "srt_trace_backward", "srt_camera_rays", "srt_trace_pathmix", "srt_batch_plan_create",
           "TraceFn", "render", "counters_dict", "new_counters", "COUNTER_NAMES"]


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libsrt takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libsrt takes contiguous tensors")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _f32(x, device):
    return torch.as_tensor(x, dtype=torch.float32, device=device).contiguous()


class DeviceScene:
    """Raw Gaussian parameters on the device (FP32, contiguous)."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree):
        self.means = means
        self.log_scales = log_scales
        self.quats = quats
        self.opacity_logits = opacity_logits
        self.sh = sh
        self.sh_degree = int(sh_degree)

    @classmethod
    def from_host(cls, scene, device="cuda"):
        """From any object with NumPy fields means, log_scales, quats,
        opacity_logits, sh and sh_degree."""
        return cls(_f32(scene.means, device), _f32(scene.log_scales, device),
                   _f32(scene.quats, device), _f32(scene.opacity_logits, device),
                   _f32(scene.sh, device), scene.sh_degree)

    @property
    def num_gaussians(self):
        return int(self.means.shape[0])

    def c_struct(self):
        return _lib.SrtScene(self.num_gaussians, self.sh_degree, _ptr(self.means),
                             _ptr(self.log_scales), _ptr(self.quats),
                             _ptr(self.opacity_logits), _ptr(self.sh))


class Bvh:
    """Owning wrapper of an srt_bvh handle; keeps its scene (whose SH buffer the
    handle reads) alive."""

    def __init__(self, handle, scene):
        self.handle = handle
        self.scene = scene
        # held by the object: module globals may already be gone when a
        # handle is collected at interpreter exit
        self._destroy = _lib.load().srt_destroy_bvh
        self._sync = torch.cuda.synchronize

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                self._sync()
            except Exception:
                pass
            self._destroy(self.handle)
            self.handle = None

    def info(self):
        inf = _lib.SrtBvhInfo()
        _lib.check("srt_bvh_get_info", _lib.load().srt_bvh_get_info(self.handle, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _lib.SrtBvhInfo._fields_}

    def records(self):
        G = self.scene.num_gaussians
        dev = self.scene.means.device
        out = dict(mu=torch.empty((G, 3), device=dev), M=torch.empty((G, 9), device=dev),
                   opacity=torch.empty(G, device=dev), box_lo=torch.empty((G, 3), device=dev),
                   box_hi=torch.empty((G, 3), device=dev))
        _lib.check("srt_bvh_records", _lib.load().srt_bvh_records(
            self.handle, _ptr(out["mu"]), _ptr(out["M"]), _ptr(out["opacity"]),
            _ptr(out["box_lo"]), _ptr(out["box_hi"]), _stream()))
        return out

    def nodes(self):
        inf = self.info()
        W = inf["width"]
        dev = self.scene.means.device
        raw = torch.empty((inf["num_nodes"], 8 * W), dtype=torch.int32, device=dev)
        order = torch.empty(max(1, self.scene.num_gaussians), dtype=torch.int32, device=dev)
        _lib.check("srt_bvh_nodes", _lib.load().srt_bvh_nodes(self.handle, _ptr(raw), _ptr(order),
                                                              _stream()))
        return raw, order[: self.scene.num_gaussians]


DEFAULT_SIZE_SPLIT = 0


def srt_set_memory_limit(nbytes: int) -> None:
    """Cap the device bytes the library holds for BVH handles and build
    temporaries (0: no cap); a build beyond it raises SrtError (OOM)."""
    _lib.check("srt_set_memory_limit", _lib.load().srt_set_memory_limit(int(nbytes)))


def srt_memory_stats() -> dict:
    """Device bytes the library holds in use and keeps for reuse."""
    a, b = C.c_int64(), C.c_int64()
    _lib.check("srt_memory_stats", _lib.load().srt_memory_stats(C.byref(a), C.byref(b)))
    return {"in_use": a.value, "cached": b.value}


def srt_build_bvh(scene: DeviceScene, width: int = 4, leaf_size: int = 4,
                  size_split: int = DEFAULT_SIZE_SPLIT) -> Bvh:
    lib = _lib.load()
    sc = scene.c_struct()
    opts = _lib.SrtBuildOpts(int(width), int(leaf_size), int(size_split))
    h = C.c_void_p()
    _lib.check("srt_build_bvh", lib.srt_build_bvh(C.byref(sc), C.byref(opts), _stream(),
                                                  C.byref(h)))
    return Bvh(h.value, scene)


def srt_refit_bvh(bvh: Bvh, scene: DeviceScene) -> Bvh:
    """Refit `bvh` in place to `scene` (the same Gaussians with new parameter
    values): records and boxes are recomputed, the topology is kept."""
    sc = scene.c_struct()
    _lib.check("srt_refit_bvh", _lib.load().srt_refit_bvh(bvh.handle, C.byref(sc), _stream()))
    bvh.scene = scene
    return bvh


def new_counters(device="cuda"):
    return torch.zeros(SRT_NUM_COUNTERS, dtype=torch.int64, device=device)


def counters_dict(c):
    v = c.tolist()
    return {n: int(x) for n, x in zip(COUNTER_NAMES, v)}


ESTIMATORS = {"plain": 0, "rb": 1}
RNGS = {"philox": 0, "hash": 1}
WALKS = {"auto": 0, "lane": 1, "wave": 2}


def _opts(seed, spp, n_per_traversal, sample_offset, bg, any_hit, stack_limit, depth_mode=0,
          depth_axis=(0.0, 0.0, 0.0), image_width=0, persistent=False, refill_threshold=0,
          estimator="plain", rng="philox", walk="auto"):
    o = _lib.SrtTraceOpts()
    if walk not in WALKS:
        raise ValueError(f"walk must be one of {sorted(WALKS)}")
    o.walk = WALKS[walk]
    if estimator not in ESTIMATORS:
        raise ValueError(f"estimator must be one of {sorted(ESTIMATORS)}")
    if rng not in RNGS:
        raise ValueError(f"rng must be one of {sorted(RNGS)}")
    o.estimator = ESTIMATORS[estimator]
    o.rng = RNGS[rng]
    o.image_width = int(image_width)
    o.persistent = 1 if persistent else 0
    o.refill_threshold = int(refill_threshold)
    o.depth_mode = int(depth_mode)
    for i in range(3):
        o.depth_axis[i] = float(depth_axis[i])
    o.seed = int(seed)
    o.spp = int(spp)
    o.n_per_traversal = int(n_per_traversal)
    o.sample_offset = int(sample_offset)
    for i in range(3):
        o.bg[i] = float(bg[i])
    o.any_hit = 1 if any_hit else 0
    o.stack_limit = int(stack_limit)
    return o


def srt_trace_forward(bvh: Bvh, origins, dirs, *, tmin=None, tmax=None, ignore_gid=None,
                      ray_ids=None, sample_ids=None, purpose=0, seed=0, spp=1,
                      n_per_traversal=1, sample_offset=0, bg=(0.0, 0.0, 0.0), any_hit=False,
                      stack_limit=0, depth_mode=0, depth_axis=(0.0, 0.0, 0.0), image_width=0,
                      persistent=False, refill_threshold=0, rng="philox", walk="auto",
                      want_rgb=True, want_hits=True, counters=None, out=None, workspace=None):
    """Trace rays (device tensors [R,3]); returns dict(rgb [R,3], hit_gid [R,spp],
    hit_t [R,spp]). image_width > 0 declares the rays a row-major image of that
    width (traced in 8x8 tiles); persistent=True runs work-stealing waves
    (refilled once refill_threshold lanes are idle); walk="wave" makes the 64 rays
    of a tile walk the BVH together ("auto": wherever supported, "lane": one
    walk per ray). None of these changes results."""
    lib = _lib.load()
    R = int(origins.shape[0])
    dev = origins.device
    rays = _lib.SrtRays(R, _ptr(origins), _ptr(dirs), _ptr(tmin), _ptr(tmax), _ptr(ignore_gid),
                        _ptr(ray_ids), _ptr(sample_ids), int(purpose))
    opts = _opts(seed, spp, n_per_traversal, sample_offset, bg, any_hit, stack_limit, depth_mode,
                 depth_axis, image_width, persistent, refill_threshold, rng=rng, walk=walk)
    res = dict(out or {})
    if want_rgb and "rgb" not in res:
        res["rgb"] = torch.empty((R, 3), dtype=torch.float32, device=dev)
    if want_hits and "hit_gid" not in res:
        res["hit_gid"] = torch.empty((R, spp), dtype=torch.int32, device=dev)
        res["hit_t"] = torch.empty((R, spp), dtype=torch.float32, device=dev)
    need = lib.srt_trace_workspace_size(bvh.handle, R)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _lib.check("srt_trace_forward", lib.srt_trace_forward(
        bvh.handle, C.byref(rays), C.byref(opts), _ptr(res.get("rgb")), _ptr(res.get("hit_gid")),
        _ptr(res.get("hit_t")), _ptr(counters), _ptr(workspace), need, _stream()))
    return res


def srt_trace_forward_noalloc(bvh: Bvh, origins, dirs, out, *, tmin=None, tmax=None,
                              ignore_gid=None, ray_ids=None, sample_ids=None, purpose=0, seed=0,
                              spp=1, n_per_traversal=1, sample_offset=0, bg=(0.0, 0.0, 0.0),
                              any_hit=False, stack_limit=0, depth_mode=0,
                              depth_axis=(0.0, 0.0, 0.0), image_width=0, persistent=False,
                              refill_threshold=0, walk="auto", counters=None):
    """srt_trace_forward with the library's static per-device scratch: no
    workspace and no allocation (the caller passes the outputs in `out`:
    rgb [R,3] and/or hit_gid, hit_t [R,spp]). Calls that overlap on one GPU
    race on its scratch."""
    lib = _lib.load()
    R = int(origins.shape[0])
    rays = _lib.SrtRays(R, _ptr(origins), _ptr(dirs), _ptr(tmin), _ptr(tmax), _ptr(ignore_gid),
                        _ptr(ray_ids), _ptr(sample_ids), int(purpose))
    opts = _opts(seed, spp, n_per_traversal, sample_offset, bg, any_hit, stack_limit, depth_mode,
                 depth_axis, image_width, persistent, refill_threshold, walk=walk)
    _lib.check("srt_trace_forward_noalloc", lib.srt_trace_forward_noalloc(
        bvh.handle, C.byref(rays), C.byref(opts), _ptr(out.get("rgb")), _ptr(out.get("hit_gid")),
        _ptr(out.get("hit_t")), _ptr(counters), _stream()))
    return out


def srt_trace_backward(bvh: Bvh, origins, dirs, grad_rgb, *, hit_gid=None, hit_t=None,
                       tmin=None, tmax=None, ignore_gid=None, ray_ids=None, sample_ids=None,
                       purpose=0, seed=0, spp=1, n_per_traversal=1, sample_offset=0,
                       bg=(0.0, 0.0, 0.0), depth_mode=0, depth_axis=(0.0, 0.0, 0.0),
                       image_width=0, estimator="plain", rng="philox", walk="auto",
                       stack_limit=0, grads=None, counters=None, workspace=None):
    """Accumulate gradients of sum(grad_rgb * E[rgb]) into `grads` (a dict of
    tensors shaped like the scene's; zeros are allocated when absent).
    estimator: "plain" (per-sample score terms) or "rb" (each term averaged
    over its own acceptance number; no larger variance). walk: as in
    srt_trace_forward (wave-shared walks for image launches by default)."""
    lib = _lib.load()
    sc = bvh.scene
    R = int(origins.shape[0])
    dev = origins.device
    if grads is None:
        grads = {k: torch.zeros_like(getattr(sc, k)) for k in
                 ("means", "log_scales", "quats", "opacity_logits", "sh")}
    rays = _lib.SrtRays(R, _ptr(origins), _ptr(dirs), _ptr(tmin), _ptr(tmax), _ptr(ignore_gid),
                        _ptr(ray_ids), _ptr(sample_ids), int(purpose))
    opts = _opts(seed, spp, n_per_traversal, sample_offset, bg, False, stack_limit, depth_mode,
                 depth_axis, image_width, estimator=estimator, rng=rng, walk=walk)
    need = lib.srt_backward_workspace_size(bvh.handle, R)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    scs = sc.c_struct()
    _lib.check("srt_trace_backward", lib.srt_trace_backward(
        bvh.handle, C.byref(scs), C.byref(rays), C.byref(opts), _ptr(grad_rgb), _ptr(hit_gid),
        _ptr(hit_t), _ptr(grads["means"]), _ptr(grads["log_scales"]), _ptr(grads["quats"]),
        _ptr(grads["opacity_logits"]), _ptr(grads["sh"]), _ptr(counters), _ptr(workspace), need,
        _stream()))
    return grads


class TraceFn(torch.autograd.Function):
    """rgb = E-estimate of the pixel colours of `origins`/`dirs` through the
    Gaussians (means, log_scales, quats, opacity_logits, sh). The forward
    builds the BVH from the current parameters and saves each sample's
    (id, depth); the backward re-traverses and returns the estimator's
    gradients for the five parameter tensors."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, origins, dirs, cfg):
        scene = DeviceScene(means.detach().contiguous(), log_scales.detach().contiguous(),
                            quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                            sh.detach().contiguous(), cfg["sh_degree"])
        bvh = cfg.get("bvh")
        if bvh is not None:  # a handle kept across optimisation steps: refit it
            srt_refit_bvh(bvh, scene)
        else:
            bvh = srt_build_bvh(scene, cfg.get("width", 4), cfg.get("leaf_size", 4))
        res = srt_trace_forward(bvh, origins, dirs, seed=cfg.get("seed", 0), spp=cfg["spp"],
                                n_per_traversal=cfg.get("n_per_traversal", 1),
                                sample_offset=cfg.get("sample_offset", 0),
                                bg=cfg.get("bg", (0.0, 0.0, 0.0)),
                                image_width=cfg.get("image_width", 0),
                                rng=cfg.get("rng", "philox"))
        ctx.bvh = bvh
        ctx.cfg = cfg
        ctx.save_for_backward(origins, dirs, res["hit_gid"], res["hit_t"])
        return res["rgb"]

    @staticmethod
    def backward(ctx, grad_rgb):
        origins, dirs, hit_gid, hit_t = ctx.saved_tensors
        cfg = ctx.cfg
        g = srt_trace_backward(ctx.bvh, origins, dirs, grad_rgb.contiguous(), hit_gid=hit_gid,
                               hit_t=hit_t, seed=cfg.get("seed", 0), spp=cfg["spp"],
                               n_per_traversal=cfg.get("n_per_traversal", 1),
                               sample_offset=cfg.get("sample_offset", 0),
                               bg=cfg.get("bg", (0.0, 0.0, 0.0)),
                               image_width=cfg.get("image_width", 0),
                               estimator=cfg.get("estimator", "plain"),
                               rng=cfg.get("rng", "philox"))
        return (g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], None, None,
                None)


def render(means, log_scales, quats, opacity_logits, sh, origins, dirs, **cfg):
    """Differentiable stochastic render (see TraceFn); cfg keys: sh_degree, spp,
    n_per_traversal, seed, sample_offset, bg, width, leaf_size, image_width,
    estimator ("plain" or "rb", see srt_trace_backward), and bvh (a handle of
    the same Gaussians to refit instead of building a new one)."""
    return TraceFn.apply(means, log_scales, quats, opacity_logits, sh, origins, dirs, cfg)


def _camera(cam):
    c = _lib.SrtCamera()
    for name in ("eye", "forward", "right", "up"):
        v = getattr(cam, name)
        arr = getattr(c, name)
        for i in range(3):
            arr[i] = float(v[i])
    c.tan_half = float(cam.tan_half)
    c.width = int(cam.width)
    c.height = int(cam.height)
    jit = getattr(cam, "jitter", (0.0, 0.0))
    c.jitter[0] = float(jit[0])
    c.jitter[1] = float(jit[1])
    return c


def srt_camera_rays(cam, device="cuda"):
    """Canonical pinhole rays of a camera (origins, dirs) [H*W,3]."""
    lib = _lib.load()
    R = int(cam.width) * int(cam.height)
    o = torch.empty((R, 3), dtype=torch.float32, device=device)
    d = torch.empty((R, 3), dtype=torch.float32, device=device)
    c = _camera(cam)
    _lib.check("srt_camera_rays", lib.srt_camera_rays(C.byref(c), _ptr(o), _ptr(d), _stream()))
    return o, d


def srt_trace_pathmix(bvh: Bvh, cam, *, ray_id_base=0, seed=0, spp=1, n_per_traversal=1,
                      sample_offset=0, bg=(0.0, 0.0, 0.0), light=(5.0, 5.0, 5.0), plane_y=-2.5,
                      tmin_secondary=1e-4, stack_limit=0, persistent=False, refill_threshold=0,
                      rng="philox", walk="auto", want_hits=True, counters=None, workspace=None,
                      out=None, stages=0):
    """Path-tracer mix of one camera; returns dict(rgb [, cam_gid, cam_t,
    shadow_vis, mirror_gid]). walk applies to the camera rays. stages: 0 for
    the whole mix, else a mask of PATHMIX_CAMERA/SHADOW/MIRROR/COMPOSE (run
    in order on the same workspace, they give the whole mix)."""
    lib = _lib.load()
    dev = bvh.scene.means.device
    R = int(cam.width) * int(cam.height)
    c = _camera(cam)
    opts = _opts(seed, spp, n_per_traversal, sample_offset, bg, False, stack_limit,
                 persistent=persistent, refill_threshold=refill_threshold, rng=rng, walk=walk)
    pm = _lib.SrtPathmixOpts()
    for i in range(3):
        pm.light[i] = float(light[i])
    pm.plane_y = float(plane_y)
    pm.tmin_secondary = float(tmin_secondary)
    pm.stages = int(stages)
    res = dict(out or {})
    if "rgb" not in res:
        res["rgb"] = torch.empty((R, 3), dtype=torch.float32, device=dev)
    if want_hits and "cam_gid" not in res:
        res["cam_gid"] = torch.empty((R, spp), dtype=torch.int32, device=dev)
        res["cam_t"] = torch.empty((R, spp), dtype=torch.float32, device=dev)
        res["shadow_vis"] = torch.empty((R, spp), dtype=torch.uint8, device=dev)
        res["mirror_gid"] = torch.empty((R, spp), dtype=torch.int32, device=dev)
    need = lib.srt_pathmix_workspace_size(bvh.handle, C.byref(c), int(spp))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _lib.check("srt_trace_pathmix", lib.srt_trace_pathmix(
        bvh.handle, C.byref(c), int(ray_id_base), C.byref(opts), C.byref(pm), _ptr(res["rgb"]),
        _ptr(res.get("cam_gid")), _ptr(res.get("cam_t")), _ptr(res.get("shadow_vis")),
        _ptr(res.get("mirror_gid")), _ptr(counters), _ptr(workspace), need, _stream()))
    return res


PATHMIX_CAMERA, PATHMIX_SHADOW, PATHMIX_MIRROR, PATHMIX_COMPOSE = 1, 2, 4, 8


class BatchPlan:
    """Owning wrapper of an srt_batch_plan (see srt_batch_plan_create)."""

    def __init__(self, handle, bvh, keep):
        self.handle = handle
        self.bvh = bvh
        self._keep = keep  # host/device objects the plan refers to
        self._destroy = _lib.load().srt_batch_plan_destroy
        self._sync = torch.cuda.synchronize
        rows, samples, items = C.c_int64(), C.c_int64(), C.c_int64()
        _lib.check("srt_batch_plan_info", _lib.load().srt_batch_plan_info(
            handle, C.byref(rows), C.byref(samples), C.byref(items)))
        self.rows, self.samples, self.items = rows.value, samples.value, items.value

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                self._sync()
            except Exception:
                pass
            self._destroy(self.handle)
            self.handle = None

    def execute(self, rgb=None, hit_gid=None, counters=None, eager=False):
        dev = self.bvh.scene.means.device
        if rgb is None:
            rgb = torch.empty((self.rows, 3), dtype=torch.float32, device=dev)
        lib = _lib.load()
        fn = lib.srt_batch_plan_execute_eager if eager else lib.srt_batch_plan_execute
        _lib.check("srt_batch_plan_execute", fn(self.handle, _ptr(rgb), _ptr(hit_gid),
                                                 _ptr(counters), _stream()))
        return rgb


def srt_batch_plan_create(bvh: Bvh, cameras, spp, *, extra_origins=None, extra_dirs=None,
                          extra_tmin=None, extra_tmax=None, extra_ray_ids=None, extra_purpose=4,
                          extra_spp=1, ray_id_base=0, seed=0, n_per_traversal=4,
                          sample_offset=0, bg=(0.0, 0.0, 0.0), stack_limit=0, persistent=True,
                          refill_threshold=16, waves_per_cu=8, depth_mode=0,
                          depth_axis=(0.0, 0.0, 0.0), rng="philox", walk="auto",
                          lds_stack=0) -> BatchPlan:
    """Plan of the batched forward (views with their spp, plus extra rays).
    walk: "auto"/"wave" trace the views' 8x8 tiles as wave-shared walks,
    "lane" one lane per pixel; extra rays always walk one lane per ray."""
    lib = _lib.load()
    nv = len(cameras)
    cams = (_lib.SrtCamera * max(nv, 1))(*[_camera(c) for c in cameras])
    spp_arr = (C.c_int32 * max(nv, 1))(*[int(x) for x in spp])
    n_extra = 0 if extra_origins is None else int(extra_origins.shape[0])
    extra = _lib.SrtRays(n_extra, _ptr(extra_origins), _ptr(extra_dirs), _ptr(extra_tmin),
                         _ptr(extra_tmax), None, _ptr(extra_ray_ids), None, int(extra_purpose))
    batch = _lib.SrtBatch(nv, C.cast(cams, C.c_void_p), C.cast(spp_arr, C.c_void_p), extra,
                          int(extra_spp) if n_extra else 0, int(ray_id_base))
    opts = _opts(seed, 1, n_per_traversal, sample_offset, bg, False, stack_limit, depth_mode,
                 depth_axis, rng=rng, walk=walk)
    tun = _lib.SrtTuning(1 if persistent else 0, int(refill_threshold), int(waves_per_cu),
                         int(lds_stack))
    h = C.c_void_p()
    _lib.check("srt_batch_plan_create", lib.srt_batch_plan_create(
        bvh.handle, C.byref(batch), C.byref(opts), C.byref(tun), _stream(), C.byref(h)))
    return BatchPlan(h.value, bvh, (extra_origins, extra_dirs, extra_tmin, extra_tmax,
                                    extra_ray_ids))
