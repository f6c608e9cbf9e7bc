"""FP64 CPU oracle for stochastic ray tracing of transparent 3D Gaussians.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the GPU library. The arithmetic
lives in ``srt_oracle.c`` (plain C, FP64, brute force over every Gaussian);
this module builds it with gcc and marshals NumPy arrays through ctypes.

What it computes, per the paper (Sun et al., "Stochastic Ray Tracing of
Transparent 3D Gaussians"):
  * ``records``            eqn "gaussian": whitening matrix M = S^-1 R^T,
                           opacity sigmoid(logit) (canonical FP32 record).
  * ``trace``              eqns "rr", "cloest", "multisample": the nearest
                           accepted hit per sample, Philox-keyed acceptance.
  * ``composite``          eqn "accumulated": exact sorted compositing.
  * ``composite_grad``     derivative of eqn "accumulated".
  * ``estimator_grad``     the unbiased per-sample gradient estimator on the
                           same random realisation as ``trace``.
  * ``pathmix``            camera + shadow + mirror rays (Sec. 1, Sec. 5).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = f"{_LIB}.tmp{os.getpid()}"  # concurrent test workers each write their own
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(path: str) -> str:
    """The oracle compiled with AddressSanitizer and UndefinedBehaviorSanitizer
    (abort on the first report), for running its tests with gcc's libasan
    preloaded and SRT_ORACLE_LIB pointing here."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-ffp-contract=off", "-fno-fast-math", "-Wall",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", path, _SRC, "-lm"])
    return path


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("SRT_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        _lib = C.CDLL(path)
        _lib.srto_accept_u.restype = C.c_double
        _lib.srto_candidates.restype = C.c_int64
        _lib.srto_isect_one.restype = C.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, np.float32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, np.float64)


def _u32(a):
    return None if a is None else np.ascontiguousarray(a, np.uint32)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, np.int32)


def default_threads() -> int:
    """OpenMP threads: SRT_ORACLE_THREADS, else OMP_NUM_THREADS, else up to 16."""
    v = os.environ.get("SRT_ORACLE_THREADS") or os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else min(16, os.cpu_count() or 1)


# ---------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters [n,4] under one key [2] -> [n,4] uint32."""
    lib = _load()
    ctr = _u32(np.atleast_2d(ctr))
    key = _u32(key)
    out = np.zeros_like(ctr)
    lib.srto_philox_many(C.c_int64(ctr.shape[0]), _p(ctr), _p(key), _p(out))
    return out


def accept_u(seed, ray_id, sample, gid, purpose=0) -> float:
    return _load().srto_accept_u(C.c_uint64(seed), C.c_uint32(ray_id), C.c_uint32(sample),
                                 C.c_uint32(gid), C.c_uint32(purpose))


class Records:
    """Canonical Gaussian records: mu [G,3], M [G,9] (row-major), op [G]."""

    def __init__(self, scene, round_f32: bool = True):
        lib = _load()
        self.scene = scene
        G = scene.num_gaussians
        self.mu = np.zeros((G, 3), np.float64)
        self.M = np.zeros((G, 9), np.float64)
        self.op = np.zeros(G, np.float64)
        self._means = _f32(scene.means)
        self._ls = _f32(scene.log_scales)
        self._q = _f32(scene.quats)
        self._lg = _f32(scene.opacity_logits)
        self._sh = _f32(scene.sh)
        lib.srto_records(C.c_int64(G), _p(self._means), _p(self._ls), _p(self._q),
                         _p(self._lg), C.c_int(1 if round_f32 else 0),
                         _p(self.mu), _p(self.M), _p(self.op))

    @property
    def G(self):
        return self.mu.shape[0]

    @property
    def deg(self):
        return self.scene.sh_degree


def quat_to_rot(q):
    out = np.zeros(9, np.float64)
    _load().srto_quat_to_rot(_p(_f64(q)), _p(out))
    return out.reshape(3, 3)


def sh_basis(deg, dirs):
    """Real SH basis [n,(deg+1)^2] at directions [n,3]."""
    lib = _load()
    dirs = _f64(np.atleast_2d(dirs))
    K = (deg + 1) ** 2
    out = np.zeros((dirs.shape[0], 16), np.float64)
    for i in range(dirs.shape[0]):
        lib.srto_sh_basis(C.c_int(deg), _p(dirs[i]), out[i].ctypes.data_as(C.c_void_p))
    return out[:, :K]


def isect_one(rec: Records, g, o, d, tmin=0.0, tmax=np.inf):
    """(valid, t, q, alpha) of one ray against Gaussian g."""
    out = np.zeros(3, np.float64)
    o = _f32(o)
    d = _f32(d)
    v = _load().srto_isect_one(_p(np.ascontiguousarray(rec.mu[g])),
                               _p(np.ascontiguousarray(rec.M[g])), C.c_double(rec.op[g]),
                               _p(o), _p(d), C.c_double(tmin), C.c_double(tmax), _p(out))
    return bool(v), out[0], out[1], out[2]


def _axis(depth_axis):
    return _f64(np.asarray(depth_axis, np.float64).reshape(3))


def candidates(rec: Records, o, d, tmin=0.0, tmax=np.inf, ignore_gid=-1, cap=1 << 16,
               depth_mode=0, depth_axis=(0.0, 0.0, 0.0)):
    """Valid candidates of one ray, sorted by (FP32 depth, id). depth_mode:
    0 = the mean of the 1D Gaussian along the ray (Sec. 3.1); 1 = the centre
    projected onto depth_axis (Sec. 4.1; a zero axis means the ray's own
    direction). The same keyword applies to every function below that
    collects candidates."""
    lib = _load()
    t = np.zeros(cap)
    q = np.zeros(cap)
    a = np.zeros(cap)
    t32 = np.zeros(cap, np.float32)
    g = np.zeros(cap, np.int32)
    n = lib.srto_candidates(C.c_int64(rec.G), _p(rec.mu), _p(rec.M), _p(rec.op), _p(_f32(o)),
                            _p(_f32(d)), C.c_double(tmin), C.c_double(tmax),
                            C.c_int32(ignore_gid), C.c_int(depth_mode), _p(_axis(depth_axis)),
                            C.c_int64(cap), _p(t), _p(q), _p(a),
                            _p(t32), _p(g))
    n = min(n, cap)
    return dict(t=t[:n], q=q[:n], alpha=a[:n], t32=t32[:n], gid=g[:n])


class Rays:
    def __init__(self, o, d, tmin=None, tmax=None, ignore_gid=None, ray_id=None,
                 sample_base=None):
        self.o = _f32(o)
        self.d = _f32(d)
        self.tmin = _f32(tmin)
        self.tmax = _f32(tmax)
        self.ignore_gid = _i32(ignore_gid)
        self.ray_id = _u32(ray_id)
        self.sample_base = _u32(sample_base)

    @property
    def count(self):
        return self.o.shape[0]


def trace(rec: Records, rays: Rays, spp=1, seed=0, purpose=0, any_hit=False,
          bg=(0.0, 0.0, 0.0), u_override=None, threads=None, depth_mode=0,
          depth_axis=(0.0, 0.0, 0.0)):
    """Nearest accepted hit per sample (brute force, FP64)."""
    lib = _load()
    R = rays.count
    rgb = np.zeros((R, 3))
    gid = np.zeros((R, spp), np.int32)
    t = np.zeros((R, spp), np.float32)
    flags = np.zeros((R, spp), np.uint8)
    margin = np.zeros((R, spp))
    bg = _f64(bg)
    uo = _f64(u_override)
    lib.srto_trace(C.c_int64(rec.G), _p(rec.mu), _p(rec.M), _p(rec.op), C.c_int(rec.deg),
                   _p(rec._sh), C.c_int64(R), _p(rays.o), _p(rays.d), _p(rays.tmin),
                   _p(rays.tmax), _p(rays.ignore_gid), _p(rays.ray_id), _p(rays.sample_base),
                   C.c_int32(spp), C.c_uint64(seed), C.c_uint32(purpose),
                   C.c_int(1 if any_hit else 0), _p(bg), _p(uo), C.c_int(depth_mode),
                   _p(_axis(depth_axis)), _p(rgb), _p(gid), _p(t),
                   _p(flags), _p(margin), C.c_int(threads or default_threads()))
    return dict(rgb=rgb, hit_gid=gid, hit_t=t, flags=flags, margin=margin)


def composite(rec: Records, rays: Rays, bg=(0.0, 0.0, 0.0), threads=None, depth_mode=0,
              depth_axis=(0.0, 0.0, 0.0)):
    """Exact sorted front-to-back composite L [R,3], single-sample variance,
    final transmittance and candidate count."""
    lib = _load()
    R = rays.count
    L = np.zeros((R, 3))
    var = np.zeros((R, 3))
    T = np.zeros(R)
    n = np.zeros(R, np.int32)
    lib.srto_composite(C.c_int64(rec.G), _p(rec.mu), _p(rec.M), _p(rec.op), C.c_int(rec.deg),
                       _p(rec._sh), C.c_int64(R), _p(rays.o), _p(rays.d), _p(rays.tmin),
                       _p(rays.tmax), _p(rays.ignore_gid), _p(_f64(bg)), C.c_int(depth_mode),
                       _p(_axis(depth_axis)), _p(L), _p(var),
                       _p(T), _p(n), C.c_int(threads or default_threads()))
    return dict(L=L, var=var, T_end=T, n_cand=n)


def _grad_bufs(rec):
    G = rec.G
    K = (rec.deg + 1) ** 2
    return dict(means=np.zeros((G, 3)), log_scales=np.zeros((G, 3)),
                quats=np.zeros((G, 4)), opacity_logits=np.zeros(G),
                sh=np.zeros((G, K, 3)))


def composite_grad(rec: Records, rays: Rays, dL, bg=(0.0, 0.0, 0.0), threads=None,
                   depth_mode=0, depth_axis=(0.0, 0.0, 0.0)):
    """Gradient of sum_i <dL_i, L_i> (exact composite) w.r.t. raw parameters."""
    lib = _load()
    g = _grad_bufs(rec)
    lib.srto_composite_grad(C.c_int64(rec.G), _p(rec.mu), _p(rec.M), _p(rec.op),
                            C.c_int(rec.deg), _p(rec._sh), _p(rec._ls), _p(rec._q),
                            _p(rec._lg), C.c_int64(rays.count), _p(rays.o), _p(rays.d),
                            _p(rays.tmin), _p(rays.tmax), _p(rays.ignore_gid), _p(_f64(bg)),
                            C.c_int(depth_mode), _p(_axis(depth_axis)),
                            _p(_f64(dL)), _p(g["means"]), _p(g["log_scales"]),
                            _p(g["quats"]), _p(g["opacity_logits"]), _p(g["sh"]),
                            C.c_int(threads or default_threads()))
    return g


def estimator_grad(rec: Records, rays: Rays, dL, spp=1, seed=0, purpose=0,
                   bg=(0.0, 0.0, 0.0), threads=None, estimator="plain", depth_mode=0,
                   depth_axis=(0.0, 0.0, 0.0)):
    """The stochastic gradient estimator on the realisation ``trace`` draws;
    estimator="rb" averages each candidate's term over its own acceptance
    number (see srto_estimator_grad_rb)."""
    lib = _load()
    g = _grad_bufs(rec)
    if estimator not in ("plain", "rb"):
        raise ValueError(estimator)
    fn = lib.srto_estimator_grad if estimator == "plain" else lib.srto_estimator_grad_rb
    fn(C.c_int64(rec.G), _p(rec.mu), _p(rec.M), _p(rec.op),
                            C.c_int(rec.deg), _p(rec._sh), _p(rec._ls), _p(rec._q),
                            _p(rec._lg), C.c_int64(rays.count), _p(rays.o), _p(rays.d),
                            _p(rays.tmin), _p(rays.tmax), _p(rays.ignore_gid),
                            _p(rays.ray_id), _p(rays.sample_base), C.c_int32(spp),
                            C.c_uint64(seed), C.c_uint32(purpose), _p(_f64(bg)),
                            C.c_int(depth_mode), _p(_axis(depth_axis)),
                            _p(_f64(dL)), _p(g["means"]), _p(g["log_scales"]),
                            _p(g["quats"]), _p(g["opacity_logits"]), _p(g["sh"]),
                            C.c_int(threads or default_threads()))
    return g


def pathmix(rec: Records, o, d, ray_id=None, spp=1, seed=0, light=(5.0, 5.0, 5.0),
            plane_y=-2.5, bg=(0.0, 0.0, 0.0), threads=None, u_override=None):
    """Camera rays with shadow and mirror secondaries (see srt_oracle.c).
    u_override [G]: replaces every acceptance number of Gaussian g by
    u_override[g] (tests inject binary outcomes)."""
    lib = _load()
    o = _f32(o)
    d = _f32(d)
    R = o.shape[0]
    rgb = np.zeros((R, 3))
    cg = np.zeros((R, spp), np.int32)
    ct = np.zeros((R, spp), np.float32)
    vis = np.zeros((R, spp), np.uint8)
    mg = np.zeros((R, spp), np.int32)
    fl = np.zeros((R, spp), np.uint8)
    lib.srto_pathmix(C.c_int64(rec.G), _p(rec.mu), _p(rec.M), _p(rec.op), C.c_int(rec.deg),
                     _p(rec._sh), C.c_int64(R), _p(o), _p(d), _p(_u32(ray_id)),
                     C.c_int32(spp), C.c_uint64(seed), _p(_f32(light)),
                     C.c_float(plane_y), _p(_f64(bg)), _p(_f64(u_override)), _p(rgb), _p(cg),
                     _p(ct), _p(vis),
                     _p(mg), _p(fl), C.c_int(threads or default_threads()))
    return dict(rgb=rgb, cam_gid=cg, cam_t=ct, shadow_vis=vis, mirror_gid=mg, flags=fl)


def exact_loss(rec_fn, scene, rays: Rays, target, bg=(0.0, 0.0, 0.0)):
    """L2 loss sum |L - target|^2 of the exact composite (for finite differences)."""
    L = composite(rec_fn(scene), rays, bg)["L"]
    return float(((L - target) ** 2).sum())
