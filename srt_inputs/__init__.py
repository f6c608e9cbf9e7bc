"""Seeded synthetic inputs for the stochastic Gaussian ray tracer.

This module is shared by the GPU library's tests and benchmark and by the
CPU oracle's tests. It holds no arithmetic of the method itself (no
intersection, no opacity, no acceptance, no shading): only the random
scene parameters, camera descriptions and the canonical FP32 camera-ray
construction that both sides consume bit for bit.

Scenes follow the paper's parameterisation of a 3D Gaussian (mean, per-axis
scale, rotation, opacity and a view-dependent colour; Sec. 3.1, eqn
"gaussian"). The raw parameters are stored the way a training pipeline
keeps them: log-scales, an unnormalised (w, x, y, z) quaternion, an opacity
logit and real spherical-harmonic coefficients.

The five workloads are synthetic stand-ins for the paper's reconstructed
assets (Sec. 5), sized to overlap its range of 0.09M-7.63M Gaussians.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

F32 = np.float32
# Value of the degree-0 real spherical harmonic, used only to store a DC
# colour as an SH coefficient such that the rendered colour equals it.
SH_C0 = 0.28209479177387814


@dataclasses.dataclass
class Scene:
    means: np.ndarray           # [G,3] f32
    log_scales: np.ndarray      # [G,3] f32
    quats: np.ndarray           # [G,4] f32, (w, x, y, z), not normalised
    opacity_logits: np.ndarray  # [G]   f32
    sh: np.ndarray              # [G,(deg+1)^2,3] f32
    sh_degree: int

    @property
    def num_gaussians(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)

    def copy(self) -> "Scene":
        return self.subset(np.arange(self.num_gaussians))


def _logit(o):
    o = np.asarray(o, np.float64)
    return np.log(o / (1.0 - o)).astype(F32)


def _random_quats(rng, n):
    # A normalised 4D standard normal is uniform on SO(3); stored as drawn.
    return rng.standard_normal((n, 4)).astype(F32)


def _unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _sh_coeffs(rng, n, degree, dc_rgb, band_sigma):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3), np.float64)
    sh[:, 0, :] = (dc_rgb - 0.5) / SH_C0
    if k > 1 and band_sigma > 0:
        sh[:, 1:, :] = rng.normal(0.0, band_sigma, (n, k - 1, 3))
    return sh.astype(F32)


def scene_uniform_cube(seed: int, n: int = 1000, degree: int = 0) -> Scene:
    """Tiny scene: means U[-1,1]^3, scales log-U[0.01,0.05], opacity U(0.05,0.99)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3)).astype(F32)
    log_scales = rng.uniform(math.log(0.01), math.log(0.05), (n, 3)).astype(F32)
    quats = _random_quats(rng, n)
    op = rng.uniform(0.05, 0.99, n)
    dc = rng.uniform(0.0, 1.0, (n, 3))
    sh = _sh_coeffs(rng, n, degree, dc, 0.1 if degree > 0 else 0.0)
    return Scene(means, log_scales, quats, _logit(op), sh, degree)


def scene_shell(seed: int, n: int = 200_000, degree: int = 3,
                scale_range=(0.002, 0.02), radial_sigma=0.02) -> Scene:
    """Object-like scene: means on the unit sphere with N(0, sigma) radial noise,
    opacity Beta(0.5, 0.5) clipped to [0.01, 0.99], DC U[0,1], bands N(0, 0.1)."""
    rng = np.random.default_rng(seed)
    u = _unit_vectors(rng, n)
    r = 1.0 + rng.normal(0.0, radial_sigma, (n, 1))
    means = (u * r).astype(F32)
    log_scales = rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]),
                             (n, 3)).astype(F32)
    quats = _random_quats(rng, n)
    op = np.clip(rng.beta(0.5, 0.5, n), 0.01, 0.99)
    dc = rng.uniform(0.0, 1.0, (n, 3))
    sh = _sh_coeffs(rng, n, degree, dc, 0.1)
    return Scene(means, log_scales, quats, _logit(op), sh, degree)


def scene_four_shells(seed: int, n: int = 1_000_000, degree: int = 3) -> Scene:
    """Path-tracer scene: four shells of radius 0.5/1/1.5/2 with n/4 Gaussians
    each exactly on the shell, scales and opacity as the tiny scene, SH as the
    object-like scene."""
    rng = np.random.default_rng(seed)
    per = n // 4
    radii = np.repeat(np.array([0.5, 1.0, 1.5, 2.0]), per)
    radii = np.concatenate([radii, np.full(n - radii.size, 2.0)])
    means = (_unit_vectors(rng, n) * radii[:, None]).astype(F32)
    log_scales = rng.uniform(math.log(0.01), math.log(0.05), (n, 3)).astype(F32)
    quats = _random_quats(rng, n)
    op = rng.uniform(0.05, 0.99, n)
    dc = rng.uniform(0.0, 1.0, (n, 3))
    sh = _sh_coeffs(rng, n, degree, dc, 0.1)
    return Scene(means, log_scales, quats, _logit(op), sh, degree)


def scene_batched(seed: int, n_small: int = 3_000_000, n_large: int = 300_000,
                  degree: int = 3) -> Scene:
    """Batched workload scene: the object-like scene plus large diffuse
    Gaussians (scales log-U[0.05,0.2], DC colour only) on the same shell."""
    small = scene_shell(seed, n_small, degree)
    rng = np.random.default_rng(seed + 1000)
    u = _unit_vectors(rng, n_large)
    r = 1.0 + rng.normal(0.0, 0.02, (n_large, 1))
    means = (u * r).astype(F32)
    log_scales = rng.uniform(math.log(0.05), math.log(0.2), (n_large, 3)).astype(F32)
    quats = _random_quats(rng, n_large)
    op = np.clip(rng.beta(0.5, 0.5, n_large), 0.01, 0.99)
    dc = rng.uniform(0.0, 1.0, (n_large, 3))
    sh = _sh_coeffs(rng, n_large, degree, dc, 0.0)
    return Scene(np.concatenate([small.means, means]),
                 np.concatenate([small.log_scales, log_scales]),
                 np.concatenate([small.quats, quats]),
                 np.concatenate([small.opacity_logits, _logit(op)]),
                 np.concatenate([small.sh, sh]), degree)


def perturbed(scene: Scene, seed: int, mean_sigma=0.01, logit_sigma=0.2) -> Scene:
    """The differentiation target's scene: means + N(0, 0.01), logits + N(0, 0.2)."""
    rng = np.random.default_rng(seed)
    s = scene.copy()
    s.means = (s.means + rng.normal(0.0, mean_sigma, s.means.shape)).astype(F32)
    s.opacity_logits = (s.opacity_logits
                        + rng.normal(0.0, logit_sigma, s.opacity_logits.shape)).astype(F32)
    return s


# ----------------------------------------------------------------------------
# Cameras and rays
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Camera:
    """Pinhole camera. The orthonormal basis is formed here in FP32 and handed
    to both sides as data, so neither side re-derives it."""
    eye: np.ndarray      # [3] f32
    forward: np.ndarray  # [3] f32
    right: np.ndarray    # [3] f32
    up: np.ndarray       # [3] f32
    tan_half: np.float32
    width: int
    height: int
    # sub-pixel offset from the pixel centre, in pixels ([-0.5, 0.5); a
    # frame's perturbation of its camera rays)
    jitter: tuple = (0.0, 0.0)

    def as_array(self) -> np.ndarray:
        """Packed FP32 record [eye3, forward3, right3, up3, tan_half, 0, 0, 0]."""
        a = np.zeros(16, F32)
        a[0:3], a[3:6], a[6:9], a[9:12] = self.eye, self.forward, self.right, self.up
        a[12] = self.tan_half
        return a


def _normalize32(v):
    v = np.asarray(v, F32)
    n = np.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
    return (v / n).astype(F32)


def _cross32(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]], F32)


def look_at(eye, target, width, height, vfov_deg=60.0, up=(0.0, 1.0, 0.0)) -> Camera:
    eye = np.asarray(eye, F32)
    f = _normalize32(np.asarray(target, F32) - eye)
    upv = np.asarray(up, F32)
    if abs(float(np.dot(f.astype(np.float64), upv.astype(np.float64)))) > 0.999:
        upv = np.array([0.0, 0.0, 1.0], F32)
    r = _normalize32(_cross32(f, upv))
    u = _cross32(r, f)
    tan_half = F32(math.tan(math.radians(vfov_deg) * 0.5))
    return Camera(eye, f, r, u, tan_half, int(width), int(height))


def camera_rays(cam: Camera):
    """Canonical FP32 pinhole rays, one per pixel centre, row 0 at the top.

    Every operation is a single correctly rounded FP32 operation in the order
    written (no fused multiply-add), so a device generator that performs the
    same operations in the same order reproduces these bits exactly:
        px = ((x + 0.5) + jx) / W;  sx = ((px * 2) - 1) * tan_half * aspect
        py = ((y + 0.5) + jy) / H;  sy = (1 - (py * 2)) * tan_half
    ((jx, jy) = cam.jitter, (0, 0) by default: the pixel centres.)
        v  = (f + sx * r) + sy * u;  d = v / sqrt((vx*vx + vy*vy) + vz*vz)
    Returns (origins [H*W,3], dirs [H*W,3]) as f32, pixel index y*W + x.
    """
    W, H = cam.width, cam.height
    x = np.arange(W, dtype=F32)
    y = np.arange(H, dtype=F32)
    aspect = F32(W) / F32(H)
    jx, jy = F32(cam.jitter[0]), F32(cam.jitter[1])
    px = ((x + F32(0.5)) + jx) / F32(W)
    sx = ((px * F32(2.0)) - F32(1.0)) * cam.tan_half * aspect
    py = ((y + F32(0.5)) + jy) / F32(H)
    sy = (F32(1.0) - (py * F32(2.0))) * cam.tan_half
    SX = np.broadcast_to(sx[None, :], (H, W))
    SY = np.broadcast_to(sy[:, None], (H, W))
    d = np.empty((H, W, 3), F32)
    for i in range(3):
        d[..., i] = (cam.forward[i] + SX * cam.right[i]) + SY * cam.up[i]
    n = np.sqrt((d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2])
    d = d / n[..., None]
    o = np.ascontiguousarray(np.broadcast_to(cam.eye, (H * W, 3)), dtype=F32)
    return o, np.ascontiguousarray(d.reshape(H * W, 3), dtype=F32)


def sobol2(n: int) -> np.ndarray:
    """The first n points of the two-dimensional Sobol sequence (Sobol 1967;
    no scrambling), as [n,2] f64 in [0,1): dimension 1 is the base-2 van der
    Corput sequence, dimension 2 uses the direction numbers of the primitive
    polynomial x + 1 (m_1 = 1, m_k = 2 m_{k-1} xor m_{k-1}). Point i is the
    xor of the direction numbers of the set bits of i's Gray code."""
    bits = 32
    v1 = [1 << (bits - 1 - k) for k in range(bits)]
    m, v2 = 1, []
    for k in range(bits):
        if k > 0:
            m = (2 * m) ^ m
        v2.append(m << (bits - 1 - k))
    out = np.zeros((n, 2))
    for i in range(n):
        g = i ^ (i >> 1)
        x = y = 0
        k = 0
        while g:
            if g & 1:
                x ^= v1[k]
                y ^= v2[k]
            g >>= 1
            k += 1
        out[i] = (x / 2.0 ** bits, y / 2.0 ** bits)
    return out


def jittered(cam: Camera, frame: int) -> Camera:
    """The camera of frame `frame`: its rays perturbed by Sobol point `frame`
    (offset from the pixel centre), the frame-dependent camera ray generation
    of Sec. 4.2."""
    p = sobol2(frame + 1)[frame]
    return dataclasses.replace(cam, jitter=(float(F32(p[0] - 0.5)), float(F32(p[1] - 0.5))))


def ring_cameras(n_views, radius, width, height, vfov_deg=60.0):
    """Views on a horizontal ring, azimuth 2*pi*k/n, view 0 at (0, 0, radius)."""
    cams = []
    for k in range(n_views):
        a = 2.0 * math.pi * k / n_views
        eye = (radius * math.sin(a), 0.0, radius * math.cos(a))
        cams.append(look_at(eye, (0.0, 0.0, 0.0), width, height, vfov_deg))
    return cams


def fibonacci_cameras(n_views, radius, width, height, vfov_deg=60.0):
    """Views on a Fibonacci sphere of the given radius, all looking at the origin."""
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for k in range(n_views):
        y = 1.0 - 2.0 * (k + 0.5) / n_views
        r = math.sqrt(max(0.0, 1.0 - y * y))
        a = golden * k
        eye = (radius * r * math.cos(a), radius * y, radius * r * math.sin(a))
        cams.append(look_at(eye, (0.0, 0.0, 0.0), width, height, vfov_deg))
    return cams


def incoherent_rays(seed: int, n: int, lo, hi):
    """Origins uniform in the box [lo, hi], directions uniform on the sphere."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), (n, 3)).astype(F32)
    d = _unit_vectors(rng, n).astype(F32)
    return o, d


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

PHILOX_SEED = 0
LIGHT_POS = (5.0, 5.0, 5.0)
PLANE_Y = -2.5
SECONDARY_TMIN = 1e-4


def workload(idx: int, small: bool = False):
    """Scene and camera description of workload `idx` (1..5).

    `small=True` shrinks scenes and images for CPU-side tests while keeping
    each generator's distribution.
    """
    if idx == 1:
        scene = scene_uniform_cube(1, 1000, 0)
        cams = [look_at((0, 0, 3), (0, 0, 0), 64, 64)]
        return dict(scene=scene, cameras=cams, spp=[1], n_per_traversal=1)
    if idx == 2:
        scene = scene_shell(2, 20_000 if small else 200_000, 3)
        w = 96 if small else 800
        return dict(scene=scene, cameras=[look_at((0, 0, 3), (0, 0, 0), w, w)],
                    spp=[4], n_per_traversal=4)
    if idx == 3:
        scene = scene_four_shells(3, 40_000 if small else 1_000_000, 3)
        w, h = (96, 54) if small else (1920, 1080)
        return dict(scene=scene, cameras=[look_at((0, 0, 4), (0, 0, 0), w, h)],
                    spp=[16], n_per_traversal=4, light=LIGHT_POS, plane_y=PLANE_Y)
    if idx == 4:
        scene = scene_uniform_cube(1, 1000, 0)
        w = 64 if small else 800
        target = perturbed(scene, 104)
        return dict(scene=scene, target_scene=target,
                    cameras=ring_cameras(8, 3.0, w, w), spp=[4] * 8, n_per_traversal=4)
    if idx == 5:
        scene = (scene_batched(5, 30_000, 3_000, 3) if small
                 else scene_batched(5, 3_000_000, 300_000, 3))
        nv, w = (8, 64) if small else (64, 512)
        cams = fibonacci_cameras(nv, 3.0, w, w)
        rng = np.random.default_rng(105)
        spp = [int(x) for x in 2 ** rng.integers(0, 7, nv)]
        lo = scene.means.min(0)
        hi = scene.means.max(0)
        n_inc = 40_000 if small else 4_000_000
        o, d = incoherent_rays(106, n_inc, lo, hi)
        return dict(scene=scene, cameras=cams, spp=spp, n_per_traversal=4,
                    incoherent=(o, d))
    raise ValueError(idx)
