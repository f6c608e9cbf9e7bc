"""Pins of the FP64 oracle against facts fixed outside it: published known
answers, closed forms, library routines, brute-force enumeration, exact
probabilities and the paper's worked example. CPU only."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.special
from scipy.spatial.transform import Rotation
from scipy.stats import binomtest, chisquare

import oracle
import srt_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _scene(means, log_scales, quats, logits, sh=None, deg=0):
    G = len(means)
    if sh is None:
        sh = np.zeros((G, (deg + 1) ** 2, 3), F32)
    return si.Scene(np.asarray(means, F32).reshape(G, 3),
                    np.asarray(log_scales, F32).reshape(G, 3),
                    np.asarray(quats, F32).reshape(G, 4),
                    np.asarray(logits, F32).reshape(G), np.asarray(sh, F32), deg)


def _logit(o):
    return math.log(o / (1 - o))


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(np.array([v[0:4]], np.uint32), np.array(v[4:6], np.uint32))
        assert [int(x) for x in out[0]] == v[6:10]


def test_philox_bijective_and_uniform():
    n = 1 << 16
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 2] = 12345
    out = oracle.philox4x32_10(ctr, np.array([7, 9], np.uint32))
    # a bijection of the counter: no two outputs collide
    as_bytes = out.view(np.dtype((np.void, 16))).ravel()
    assert np.unique(as_bytes).size == n
    # the top byte of every word is uniform
    top = (out >> 24).ravel()
    assert chisquare(np.bincount(top, minlength=256)).pvalue > 1e-4


def test_acceptance_number_layout():
    # u = (word[sample mod 4] >> 8) * 2^-24 of counter (ray, sample/4, gid, purpose)
    seed = 0x1234_0000_0000_0005
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    for sample in range(8):
        w = oracle.philox4x32_10(np.array([[77, sample // 4, 901, 3]], np.uint32), key)[0]
        expect = float(int(w[sample % 4]) >> 8) / 2 ** 24
        assert oracle.accept_u(seed, 77, sample, 901, 3) == expect


# --------------------------------------------------------------------------
# Gaussian records (eqn "gaussian")
# --------------------------------------------------------------------------
def test_rotation_matches_library():
    rng = np.random.default_rng(0)
    for _ in range(50):
        q = rng.standard_normal(4)
        R = oracle.quat_to_rot(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scalar-last
        np.testing.assert_allclose(R, ref, atol=1e-13)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-13
    # 90 degrees about +z maps +x to +y
    s = math.sqrt(0.5)
    np.testing.assert_allclose(oracle.quat_to_rot([s, 0, 0, s]) @ [1, 0, 0], [0, 1, 0],
                               atol=1e-15)


def test_records_whiten_the_covariance():
    sc = si.scene_uniform_cube(3, 64, 0)
    rec = oracle.Records(sc, round_f32=False)
    for g in range(64):
        q = sc.quats[g].astype(np.float64)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        S = np.diag(np.exp(sc.log_scales[g].astype(np.float64)))
        Sigma = R @ S @ S @ R.T
        M = rec.M[g].reshape(3, 3)
        np.testing.assert_allclose(M @ Sigma @ M.T, np.eye(3), atol=1e-10)
        np.testing.assert_allclose(M.T @ M, np.linalg.inv(Sigma), rtol=1e-9)
        assert abs(rec.op[g] - 1 / (1 + math.exp(-float(sc.opacity_logits[g])))) < 1e-15
    r32 = oracle.Records(sc, round_f32=True)
    assert np.array_equal(r32.M, r32.M.astype(F32).astype(np.float64))
    assert np.array_equal(r32.M.astype(F32), rec.M.astype(F32))


# --------------------------------------------------------------------------
# Spherical harmonics
# --------------------------------------------------------------------------
def _real_sh_scipy(l, m, d):
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)  # Condon-Shortley phase
    if m > 0:
        return math.sqrt(2) * Y.real
    if m < 0:
        return math.sqrt(2) * Y.imag
    return Y.real


def test_sh_basis_matches_library():
    rng = np.random.default_rng(1)
    dirs = rng.standard_normal((40, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    Y = oracle.sh_basis(3, dirs)
    for i, d in enumerate(dirs):
        for l in range(4):
            for m in range(-l, l + 1):
                assert abs(Y[i, l * l + l + m] - _real_sh_scipy(l, m, d)) < 1e-12


def test_sh_addition_theorem_and_orthonormality():
    rng = np.random.default_rng(2)
    dirs = rng.standard_normal((2000, 3))
    Y = oracle.sh_basis(3, dirs)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-12)
    # Gauss-Legendre x uniform-phi quadrature is exact for these polynomials
    xs, ws = np.polynomial.legendre.leggauss(12)
    phis = np.arange(24) * 2 * math.pi / 24
    pts, wts = [], []
    for z, w in zip(xs, ws):
        r = math.sqrt(1 - z * z)
        for p in phis:
            pts.append((r * math.cos(p), r * math.sin(p), z))
            wts.append(w * 2 * math.pi / 24)
    Yq = oracle.sh_basis(3, np.array(pts))
    gram = (Yq * np.array(wts)[:, None]).T @ Yq
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


# --------------------------------------------------------------------------
# Intersection: closed forms (Sec. 3.1, eqn "cuboid")
# --------------------------------------------------------------------------
def test_single_gaussian_closed_form():
    sig = np.array([0.2, 0.1, 0.05])
    op = 0.7
    sc = _scene([[0, 0, 0]], np.log(sig), [[1, 0, 0, 0]], [_logit(op)])
    rec = oracle.Records(sc, round_f32=False)
    op = 1.0 / (1.0 + math.exp(-float(sc.opacity_logits[0])))  # of the stored FP32 logit
    sig = np.exp(sc.log_scales[0].astype(np.float64))
    Z = 3.0
    for bx, by in [(0.0, 0.0), (0.1, 0.05), (-0.3, 0.1), (0.5, 0.0), (0.56, 0.01)]:
        o = np.array([bx, by, -Z], F32)
        valid, t, q, a = oracle.isect_one(rec, 0, o, [0, 0, 1])
        bx32, by32 = float(o[0]), float(o[1])
        q_ref = bx32 ** 2 / sig[0] ** 2 + by32 ** 2 / sig[1] ** 2
        assert abs(t - Z) < 1e-12
        assert abs(q - q_ref) < 1e-9 * max(1, q_ref)
        assert abs(a - op * math.exp(-q_ref / 2)) < 1e-12
        assert valid == (q_ref <= 8.0)


def test_single_gaussian_rotation_invariance():
    rng = np.random.default_rng(4)
    for _ in range(20):
        sig = np.exp(rng.uniform(np.log(0.05), np.log(0.3), 3))
        Rq = Rotation.random(random_state=rng)
        xyzw = Rq.as_quat()
        quat = [xyzw[3], xyzw[0], xyzw[1], xyzw[2]]
        mu = rng.uniform(-1, 1, 3)
        # a ray expressed in the Gaussian's frame, then rotated into the world
        o_loc = np.array([rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), -4.0])
        d_loc = np.array([0.0, 0.0, 1.0])
        R = Rq.as_matrix()
        o = (mu + R @ o_loc).astype(F32)
        d = (R @ d_loc).astype(F32)
        sc = _scene([mu], np.log(sig), [quat], [0.0])
        rec = oracle.Records(sc, round_f32=False)
        valid, t, q, a = oracle.isect_one(rec, 0, o, d)
        # closed form in the local frame, from the FP32 ray and parameters stored
        q32 = sc.quats[0].astype(np.float64)
        Rt = Rotation.from_quat([q32[1], q32[2], q32[3], q32[0]]).as_matrix().T
        sig = np.exp(sc.log_scales[0].astype(np.float64))
        ol = Rt @ (o.astype(np.float64) - np.asarray(sc.means[0], np.float64))
        dl = Rt @ d.astype(np.float64)
        A = ol / sig
        B = dl / sig
        t_ref = -A @ B / (B @ B)
        q_ref = np.sum((A + t_ref * B) ** 2)
        assert abs(t - t_ref) < 1e-9
        assert abs(q - q_ref) < 1e-8 * max(1, q_ref)
        # the ideal (unrounded) ray: depth 4, q from the lateral offset
        assert abs(t - 4.0) < 1e-5
        assert abs(q - (o_loc[0] ** 2 / sig[0] ** 2 + o_loc[1] ** 2 / sig[1] ** 2)) < 1e-3


def test_range_and_ellipsoid_cull():
    sc = _scene([[0, 0, 0]], np.log([0.1, 0.1, 0.1]), [[1, 0, 0, 0]], [0.0])
    rec = oracle.Records(sc, round_f32=False)
    d = [0, 0, 1]
    # behind the origin (t < 0) is culled, as is t outside (tmin, tmax)
    assert not oracle.isect_one(rec, 0, [0, 0, 1], d)[0]
    assert oracle.isect_one(rec, 0, [0, 0, -1], d)[0]
    assert not oracle.isect_one(rec, 0, [0, 0, -1], d, tmin=1.0)[0]
    assert not oracle.isect_one(rec, 0, [0, 0, -1], d, tmax=1.0)[0]
    assert oracle.isect_one(rec, 0, [0, 0, -1], d, tmin=0.999, tmax=1.001)[0]
    # the boundary of the 2 sqrt 2 ellipsoid: q = 8 exactly is inside
    b = 0.25  # q = 6.25
    assert oracle.isect_one(rec, 0, [b, 0, -1], d)[0]
    assert not oracle.isect_one(rec, 0, [0.3, 0, -1], d)[0]  # q = 9


# --------------------------------------------------------------------------
# Stochastic selection (eqns "rr", "cloest", "multisample"; Fig. 2)
# --------------------------------------------------------------------------
def _line_scene(depths, ops, deg=0):
    n = len(depths)
    means = [[0.0, 0.0, float(z)] for z in depths]
    sh = np.zeros((n, 1, 3), F32)
    sh[:, 0, 0] = (np.arange(n) / n - 0.5) / si.SH_C0
    return _scene(means, np.log(np.full((n, 3), 0.05)), [[1, 0, 0, 0]] * n,
                  [_logit(o) for o in ops], sh, deg)


def test_fig2_closest_opaque_whatever_the_visit_order():
    line = [l for l in open(os.path.join(GOLDEN, "fig2_binary_opacities.txt"))
            if l.strip() and not l.startswith("#")][0]
    bits_s, res_s = line.split(";")
    bits = [int(b) for b in bits_s.split()]
    expect = int(res_s) - 1
    depths = [1.0, 1.5, 2.0, 2.5, 3.0, 3.5]
    for perm in itertools.permutations(range(6)):
        # storage slot k holds the intersection perm[k]; the oracle visits slots in order
        sc = _line_scene([depths[p] for p in perm], [0.5] * 6)
        rec = oracle.Records(sc)
        u = np.array([0.0 if bits[p] else 0.9 for p in perm])  # u < alpha <=> opaque
        rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]])
        r = oracle.trace(rec, rays, spp=1, u_override=u, threads=1)
        assert perm[r["hit_gid"][0, 0]] == expect


def test_two_gaussian_probabilities():
    a1, a2 = 0.3, 0.6
    sc = _line_scene([1.0, 2.0], [a1, a2])
    rec = oracle.Records(sc, round_f32=False)
    a1, a2 = rec.op
    n = 1 << 16
    rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]], ray_id=[42])
    r = oracle.trace(rec, rays, spp=n, seed=11)
    g = r["hit_gid"][0]
    assert binomtest(int((g == 0).sum()), n, a1).pvalue > 1e-4
    assert binomtest(int((g == 1).sum()), n, (1 - a1) * a2).pvalue > 1e-4
    assert binomtest(int((g == -1).sum()), n, (1 - a1) * (1 - a2)).pvalue > 1e-4
    # the result is a deterministic function of (seed, ray, sample)
    r2 = oracle.trace(rec, rays, spp=n, seed=11)
    assert np.array_equal(r2["hit_gid"], r["hit_gid"])


def test_brute_force_selection_by_hand():
    """Nearest accepted = lexicographic min of (FP32 depth, id) over accepted
    valid candidates, recomputed here from per-candidate probes."""
    sc = si.scene_uniform_cube(7, 60, 0)
    sc.log_scales[:] = np.log(0.3)  # big Gaussians: many candidates per ray
    rec = oracle.Records(sc)
    rng = np.random.default_rng(3)
    o = np.tile(np.array([0, 0, 3], F32), (16, 1))
    d = rng.standard_normal((16, 3))
    d[:, 2] = -4
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)
    spp = 6
    r = oracle.trace(rec, oracle.Rays(o, d), spp=spp, seed=5)
    n_hits = 0
    for i in range(16):
        probes = [oracle.isect_one(rec, g, o[i], d[i]) for g in range(60)]
        for s in range(spp):
            best = None
            for g, (valid, t, q, a) in enumerate(probes):
                if valid and oracle.accept_u(5, i, s, g, 0) < a:
                    key = (np.float32(t), g)
                    best = key if best is None or key < best else best
            assert r["hit_gid"][i, s] == (-1 if best is None else best[1])
            n_hits += best is not None
    assert n_hits > 20


def test_ties_break_by_id():
    # duplicate Gaussians: equal depth keys, the smaller id wins when both accept
    sc = _line_scene([2.0, 2.0, 2.0], [0.9, 0.9, 0.9])
    rec = oracle.Records(sc)
    r = oracle.trace(rec, oracle.Rays([[0, 0, 0]], [[0, 0, 1]]), spp=1,
                     u_override=np.array([0.95, 0.1, 0.1]))
    assert r["hit_gid"][0, 0] == 1


def test_flags_mark_threshold_flips():
    sc = _line_scene([1.0, 2.0], [0.5, 0.5])
    rec = oracle.Records(sc)
    a = rec.op[0]
    rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]])
    r = oracle.trace(rec, rays, u_override=np.array([a - 5e-7, 0.9]))
    assert r["flags"][0, 0] & 1 and r["hit_gid"][0, 0] == 0
    r = oracle.trace(rec, rays, u_override=np.array([a - 5e-6, 0.9]))
    assert r["flags"][0, 0] == 0
    # behind the result, a near-flip does not matter
    r = oracle.trace(rec, rays, u_override=np.array([0.0, a - 1e-9]))
    assert r["flags"][0, 0] == 0


def _offsets_near_q8():
    """FP32 ray offsets (bx, by) with q = bx^2 + by^2 (FP64) just inside and
    just outside the ellipsoid boundary q = 8 (within 1e-9 relative), and one
    clearly inside. With M = I and the ray (bx, by, -3) + t (0, 0, 1) the 1D
    mean is t* = 3 and q = bx^2 + by^2 exactly as the oracle evaluates it."""
    bx = (F32(1.9) + F32(2.0 ** -23) * np.arange(400000, dtype=np.float64)).astype(F32)
    by0 = np.sqrt(8.0 - bx.astype(np.float64) ** 2).astype(F32)
    found = {}
    for by in (by0, np.nextafter(by0, F32(3)), np.nextafter(by0, F32(0))):
        q = bx.astype(np.float64) * bx + by.astype(np.float64) * by
        for name, sel in (("in", (q < 8) & (q > 8 - 4e-9)), ("out", (q > 8) & (q < 8 + 4e-9)),
                          ("far_in", (q < 8 - 1e-6) & (q > 8 - 1e-5))):
            if name not in found and sel.any():
                i = int(np.argmax(sel))
                found[name] = (bx[i], by[i], q[i])
    return found


def test_flags_mark_the_ellipsoid_boundary():
    """A candidate whose q lies within 1e-9 (relative) of s^2 = 8 (eqn
    "cuboid") may be valid on one side and not on the other once the GPU
    rounds differently: an accepted one is flagged FLAG_GEO (2) on either
    side; a clearly inside one and a rejected borderline one are not."""
    sc = _scene([[0.0, 0.0, 0.0]], [[0.0, 0.0, 0.0]], [[1, 0, 0, 0]], [_logit(0.9)])
    rec = oracle.Records(sc)
    assert np.array_equal(rec.M[0], np.eye(3).ravel()) and np.all(rec.mu[0] == 0)
    off = _offsets_near_q8()
    d = [[0.0, 0.0, 1.0]]
    for name, (bx, by, q) in off.items():
        rays = oracle.Rays([[bx, by, -3.0]], d)
        valid, t, qq, a = oracle.isect_one(rec, 0, [bx, by, -3.0], d[0])
        assert qq == q and t == 3.0 and valid == (q <= 8.0), (name, qq, q)
        r = oracle.trace(rec, rays, u_override=np.array([0.0]))
        assert r["hit_gid"][0, 0] == (0 if q <= 8.0 else -1), name
        assert bool(r["flags"][0, 0] & 2) == (name != "far_in"), (name, r["flags"])
        # rejected (u >= alpha): nothing to flip
        r = oracle.trace(rec, rays, u_override=np.array([0.999]))
        assert r["hit_gid"][0, 0] == -1 and r["flags"][0, 0] == 0, name


def test_flags_mark_keys_one_ulp_apart():
    """Two accepted candidates whose FP32 depth keys are adjacent floats may
    swap order under another FP64 evaluation order of t*: flagged FLAG_GEO.
    Two ulps apart, equal keys (ties go by id, exactly) or a rejected
    neighbour: not flagged. With M = I and the ray along the z axis through
    the centres, t* = mu_z exactly."""
    z0 = F32(2.0)
    cases = {"one_ulp": np.nextafter(z0, F32(3)), "two_ulps": np.nextafter(
        np.nextafter(z0, F32(3)), F32(3)), "equal": z0}
    rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]])
    for name, z1 in cases.items():
        sc = _scene([[0, 0, z0], [0, 0, z1]], np.zeros((2, 3)), [[1, 0, 0, 0]] * 2,
                    [_logit(0.5)] * 2)
        rec = oracle.Records(sc)
        c = oracle.candidates(rec, [0, 0, 0], [0, 0, 1])
        assert c["t32"].tolist() == [z0, z1] and c["t"].tolist() == [float(z0), float(z1)]
        r = oracle.trace(rec, rays, u_override=np.array([0.0, 0.0]))
        assert r["hit_gid"][0, 0] == 0
        assert bool(r["flags"][0, 0] & 2) == (name == "one_ulp"), (name, r["flags"])
        r = oracle.trace(rec, rays, u_override=np.array([0.0, 0.999]))
        assert r["hit_gid"][0, 0] == 0 and r["flags"][0, 0] == 0, name


# --------------------------------------------------------------------------
# Exact compositing (eqn "accumulated") and convergence of the estimator
# --------------------------------------------------------------------------
def test_composite_closed_form_two_gaussians():
    a1, a2 = 0.3, 0.6
    sc = _line_scene([1.0, 2.0], [a1, a2])
    rec = oracle.Records(sc, round_f32=False)
    a1, a2 = rec.op  # sigmoid of the stored FP32 logits
    bg = np.array([0.2, 0.4, 0.6])
    c = np.array([[0.0, 0.5, 0.5], [0.5, 0.5, 0.5]])
    c[:, 0] = np.arange(2) / 2
    rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]])
    out = oracle.composite(rec, rays, bg)
    L = a1 * c[0] + (1 - a1) * a2 * c[1] + (1 - a1) * (1 - a2) * bg
    np.testing.assert_allclose(out["L"][0], L, atol=1e-12)
    assert abs(out["T_end"][0] - (1 - a1) * (1 - a2)) < 1e-12
    E2 = a1 * c[0] ** 2 + (1 - a1) * a2 * c[1] ** 2 + (1 - a1) * (1 - a2) * bg ** 2
    np.testing.assert_allclose(out["var"][0], E2 - L ** 2, atol=1e-12)


def _busy_rays(rec, n, seed):
    """Rays of the tiny scene's camera that cross several Gaussians."""
    cam = si.look_at((0, 0, 3), (0, 0, 0), 64, 64)
    o, d = si.camera_rays(cam)
    nc = oracle.composite(rec, oracle.Rays(o, d))["n_cand"]
    idx = np.argsort(-nc, kind="stable")[:n]
    return o[idx], d[idx], idx


def test_estimator_converges_to_exact_composite():
    sc = si.workload(1)["scene"]
    rec = oracle.Records(sc)
    o, d, idx = _busy_rays(rec, 32, 0)
    rays = oracle.Rays(o, d, ray_id=idx)
    K = 1 << 14
    ex = oracle.composite(rec, rays)
    r = oracle.trace(rec, rays, spp=K, seed=9)
    se = np.sqrt(np.maximum(ex["var"], 1e-30) / K)
    assert np.all(np.abs(r["rgb"] - ex["L"]) <= 5 * se + 1e-12)
    # the accepted index follows {T_k alpha_k}, the remainder is the miss
    for i in range(4):
        cands = oracle.candidates(rec, o[i], d[i])
        a = cands["alpha"]
        T = np.concatenate([[1.0], np.cumprod(1 - a)])
        p = np.concatenate([T[:-1] * a, [T[-1]]])
        pos = {g: k for k, g in enumerate(cands["gid"])}
        hist = np.zeros(len(p))
        for g in r["hit_gid"][i]:
            hist[pos[g] if g >= 0 else len(p) - 1] += 1
        keep = p * K >= 5
        exp_ = np.concatenate([p[keep], [p[~keep].sum()]]) * K
        obs = np.concatenate([hist[keep], [hist[~keep].sum()]])
        if exp_[-1] < 5:
            exp_, obs = exp_[:-1], obs[:-1]
            obs[-1] += hist[~keep].sum()
            exp_[-1] += p[~keep].sum() * K
        assert chisquare(obs, exp_).pvalue > 1e-4


# --------------------------------------------------------------------------
# Gradients
# --------------------------------------------------------------------------
def _grad_scene():
    rng = np.random.default_rng(21)
    n = 12
    means = rng.uniform(-0.25, 0.25, (n, 3))
    means[:, 2] = rng.uniform(-0.5, 0.5, n)
    ls = np.log(rng.uniform(0.12, 0.3, (n, 3)))
    quats = rng.standard_normal((n, 4))
    logits = rng.uniform(-1.5, 1.5, n)
    sh = rng.normal(0, 0.3, (n, 4, 3))
    return _scene(means, ls, quats, logits, sh, 1)


def _grad_rays():
    cam = si.look_at((0.1, 0.05, 3), (0, 0, 0), 12, 12, vfov_deg=20)
    return si.camera_rays(cam)


def _loss(scene, o, d, target, bg):
    rec = oracle.Records(scene, round_f32=False)
    L = oracle.composite(rec, oracle.Rays(o, d), bg)["L"]
    return float(((L - target) ** 2).sum()), L


def _orders(scene, o, d):
    rec = oracle.Records(scene, round_f32=False)
    return [tuple(oracle.candidates(rec, o[i], d[i])["gid"]) for i in range(o.shape[0])]


def test_exact_gradient_matches_finite_differences():
    """Central differences of the exact L2 loss. The composite jumps where two
    depths swap or a Gaussian crosses the ellipsoid boundary, so rays whose
    sorted candidate list differs between theta+eps and theta-eps are left
    out of both sides."""
    sc = _grad_scene()
    o, d = _grad_rays()
    bg = np.array([0.1, 0.2, 0.3])
    rng = np.random.default_rng(5)
    target = rng.uniform(0, 1, (o.shape[0], 3))
    _, L = _loss(sc, o, d, target, bg)
    rec = oracle.Records(sc, round_f32=False)
    dL_full = 2 * (L - target)
    base = _orders(sc, o, d)
    checked = masked = 0
    for name, eps in [("means", 1e-4), ("log_scales", 1e-4), ("quats", 1e-4),
                      ("opacity_logits", 1e-4), ("sh", 1e-3)]:
        arr = getattr(sc, name)
        flat = arr.reshape(-1)
        for j in range(flat.size):
            orig = flat[j]
            plus, minus = F32(orig + eps), F32(orig - eps)
            flat[j] = plus
            Lp = _loss(sc, o, d, target, bg)[1]
            op_ = _orders(sc, o, d) if name != "sh" else base
            flat[j] = minus
            Lm = _loss(sc, o, d, target, bg)[1]
            om_ = _orders(sc, o, d) if name != "sh" else base
            flat[j] = orig
            keep = np.array([a == b == c for a, b, c in zip(op_, om_, base)])
            masked += int((~keep).sum())
            lp = (((Lp - target) ** 2).sum(1) * keep).sum()
            lm = (((Lm - target) ** 2).sum(1) * keep).sum()
            fd = (lp - lm) / (float(plus) - float(minus))
            g = oracle.composite_grad(rec, oracle.Rays(o, d), dL_full * keep[:, None], bg)
            an = g[name].reshape(-1)[j]
            assert abs(fd - an) <= 1e-4 * max(1.0, abs(an)) + 1e-6, (name, j, fd, an)
            checked += 1
    assert checked > 150
    assert masked < checked  # the mask is the exception


def test_estimator_gradient_is_unbiased():
    sc = _grad_scene()
    o, d = _grad_rays()
    bg = np.array([0.1, 0.2, 0.3])
    rng = np.random.default_rng(6)
    dL = rng.normal(0, 1, (o.shape[0], 3))
    rec = oracle.Records(sc)
    rays = oracle.Rays(o, d)
    exact = oracle.composite_grad(rec, rays, dL, bg)
    runs = [oracle.estimator_grad(rec, rays, dL, spp=64, seed=s, bg=bg) for s in range(40)]
    for name in exact:
        est = np.stack([r[name] for r in runs])
        m, se = est.mean(0), est.std(0, ddof=1) / math.sqrt(len(runs))
        z = np.abs(m - exact[name]) / np.maximum(se, 1e-12)
        tol = 5 * se + 1e-3 * np.abs(exact[name]) + 1e-9
        assert np.all(np.abs(m - exact[name]) <= tol), (name, float(z.max()))


def test_estimator_gradient_single_sample_by_hand():
    """One ray, one sample: the estimator's alpha-weights and colour gradient
    recomputed from the sorted candidates and the Philox numbers."""
    sc = _line_scene([1.0, 1.5, 2.0, 2.5], [0.4, 0.5, 0.6, 0.7])
    sc.sh = np.zeros((4, 1, 3), F32)
    sc.sh[:, 0, :] = ((np.array([0.1, 0.3, 0.5, 0.9]) - 0.5) / si.SH_C0)[:, None]
    rec = oracle.Records(sc, round_f32=False)
    rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]], ray_id=[3])
    dL = np.array([[1.0, -0.5, 0.25]])
    bg = np.array([0.0, 0.0, 0.0])
    for seed in range(8):
        g = oracle.estimator_grad(rec, rays, dL, spp=1, seed=seed, bg=bg)
        c = 0.5 + sc.sh[:, 0, :].astype(np.float64) * oracle.sh_basis(0, [[0, 0, 1]])[0, 0]
        us = [oracle.accept_u(seed, 3, 0, k, 0) for k in range(4)]
        a = next((k for k in range(4) if us[k] < rec.op[k]), None)
        X = c[a] if a is not None else bg
        for k in range(4 if a is None else a):
            s_alpha = dL[0] @ (c[k] - X) / (1 - rec.op[k])
            # d alpha / d logit = alpha (1 - sigmoid) with q = 0 on the axis
            expect = s_alpha * rec.op[k] * (1 - rec.op[k])
            assert abs(g["opacity_logits"][k] - expect) < 1e-12
        if a is not None:
            np.testing.assert_allclose(g["sh"][a, 0], dL[0] * si.SH_C0, atol=1e-12)
            for k in range(a + 1, 4):
                assert g["opacity_logits"][k] == 0.0


def test_rb_estimator_single_sample_by_hand():
    """The Rao-Blackwellised estimator on one ray and one sample: front
    candidates get <dL, c_k - c_a> (no 1 / (1 - alpha_k)), the first accepted
    a gets <dL, c_a - c_a2> with a2 the next accepted behind it (bg if none),
    the colour gradient stays on a."""
    sc = _line_scene([1.0, 1.5, 2.0, 2.5], [0.4, 0.5, 0.6, 0.7])
    sc.sh = np.zeros((4, 1, 3), F32)
    sc.sh[:, 0, :] = ((np.array([0.1, 0.3, 0.5, 0.9]) - 0.5) / si.SH_C0)[:, None]
    rec = oracle.Records(sc, round_f32=False)
    rays = oracle.Rays([[0, 0, 0]], [[0, 0, 1]], ray_id=[3])
    dL = np.array([[1.0, -0.5, 0.25]])
    bg = np.array([0.05, 0.1, 0.2])
    c = 0.5 + sc.sh[:, 0, :].astype(np.float64) * oracle.sh_basis(0, [[0, 0, 1]])[0, 0]
    seen = set()
    for seed in range(16):
        g = oracle.estimator_grad(rec, rays, dL, spp=1, seed=seed, bg=bg, estimator="rb")
        us = [oracle.accept_u(seed, 3, 0, k, 0) for k in range(4)]
        acc = [k for k in range(4) if us[k] < rec.op[k]]
        a = acc[0] if acc else None
        a2 = acc[1] if len(acc) > 1 else None
        seen.add((a, a2))
        X = c[a] if a is not None else bg
        X2 = c[a2] if a2 is not None else bg
        for k in range(4):
            if a is None or k < a:
                s_alpha = dL[0] @ (c[k] - X)
            elif k == a:
                s_alpha = dL[0] @ (X - X2)
            else:
                s_alpha = 0.0
            expect = s_alpha * rec.op[k] * (1 - rec.op[k])  # d alpha / d logit on the axis
            assert abs(g["opacity_logits"][k] - expect) < 1e-12, (seed, k)
        if a is not None:
            np.testing.assert_allclose(g["sh"][a, 0], dL[0] * si.SH_C0, atol=1e-12)
    assert len(seen) >= 4  # several different (a, a2) realisations were covered


def test_rb_estimator_is_exact_on_single_candidate_rays():
    """With one candidate per ray the averaged term is <dL, c - bg> whatever
    the sample draws, i.e. the exact gradient of the composite for every
    parameter that reaches alpha."""
    means = [[x, y, 0.0] for x in (-0.6, 0.0, 0.6) for y in (-0.6, 0.0, 0.6)]
    n = len(means)
    rng = np.random.default_rng(8)
    sc = _scene(means, np.log(rng.uniform(0.03, 0.08, (n, 3))), rng.standard_normal((n, 4)),
                rng.uniform(-1.5, 1.5, n), rng.normal(0, 0.3, (n, 4, 3)), 1)
    rec = oracle.Records(sc)
    cam = si.look_at((0.05, 0.02, 3), (0, 0, 0), 24, 24, vfov_deg=35)
    o, d = si.camera_rays(cam)
    rays = oracle.Rays(o, d)
    assert oracle.composite(rec, rays)["n_cand"].max() == 1
    assert (oracle.composite(rec, rays)["n_cand"] == 1).sum() > 20
    bg = np.array([0.3, 0.2, 0.1])
    dL = rng.normal(0, 1, (len(o), 3))
    exact = oracle.composite_grad(rec, rays, dL, bg)
    for seed in (0, 1):
        g = oracle.estimator_grad(rec, rays, dL, spp=3, seed=seed, bg=bg, estimator="rb")
        for name in ("means", "log_scales", "quats", "opacity_logits"):
            np.testing.assert_allclose(g[name], exact[name], rtol=1e-9,
                                       atol=1e-12 * max(1.0, np.abs(exact[name]).max()))


def test_rb_estimator_unbiased_with_lower_variance():
    sc = _grad_scene()
    o, d = _grad_rays()
    bg = np.array([0.1, 0.2, 0.3])
    rng = np.random.default_rng(6)
    dL = rng.normal(0, 1, (o.shape[0], 3))
    rec = oracle.Records(sc)
    rays = oracle.Rays(o, d)
    exact = oracle.composite_grad(rec, rays, dL, bg)
    runs = {e: [oracle.estimator_grad(rec, rays, dL, spp=8, seed=s, bg=bg, estimator=e)
                for s in range(60)] for e in ("plain", "rb")}
    var = {}
    for e, rs in runs.items():
        var[e] = 0.0
        for name in ("means", "log_scales", "quats", "opacity_logits"):
            est = np.stack([r[name] for r in rs])
            m, se = est.mean(0), est.std(0, ddof=1) / math.sqrt(len(rs))
            tol = 5 * se + 1e-3 * np.abs(exact[name]) + 1e-9
            assert np.all(np.abs(m - exact[name]) <= tol), (e, name)
            var[e] += float(est.var(0, ddof=1).sum())
    assert var["rb"] < 0.7 * var["plain"], var


# --------------------------------------------------------------------------
# Path-tracer mix
# --------------------------------------------------------------------------
def test_pathmix_empty_scene_is_the_lit_mirror_plane():
    sc = _line_scene([100.0], [0.5])
    sc.means[:] = 1000.0  # nothing in view
    rec = oracle.Records(sc)
    cam = si.look_at((0, 0, 4), (0, 0, 0), 16, 12)
    o, d = si.camera_rays(cam)
    bg = np.array([0.05, 0.1, 0.2])
    r = oracle.pathmix(rec, o, d, spp=2, bg=bg)
    for i in range(o.shape[0]):
        dy = float(d[i, 1])
        if dy < 0:
            t = F32(F32(-2.5) - o[i, 1]) / d[i, 1]
            P = (o[i] + (t * d[i]).astype(F32)).astype(F32)
            P[1] = F32(-2.5)
            v = (np.array([5, 5, 5], F32) - P).astype(F32)
            ln = np.sqrt(F32(F32(v[0] * v[0]) + F32(v[1] * v[1])) + F32(v[2] * v[2]))
            ly = float(F32(v[1] / ln))
            np.testing.assert_allclose(r["rgb"][i], 0.5 * max(0.0, ly) + 0.5 * bg, atol=1e-12)
            assert np.all(r["shadow_vis"][i] == 1) and np.all(r["mirror_gid"][i] == -1)
        else:
            np.testing.assert_allclose(r["rgb"][i], bg, atol=0)
            assert np.all(r["shadow_vis"][i] == 255)


def test_pathmix_shadow_occlusion_probability():
    # one Gaussian between every plane point near the image centre and the light
    op = 0.4
    sc = _scene([[2.5, 2.5, 2.5]], np.log([3.0, 3.0, 3.0]), [[1, 0, 0, 0]], [_logit(op)])
    rec = oracle.Records(sc)
    o = np.array([[0, 0, 0]], F32)
    d = (np.array([[0.0, -1.0, 0.01]]) / np.linalg.norm([0, -1, 0.01])).astype(F32)
    n = 1 << 14
    r = oracle.pathmix(rec, o, d, spp=n, seed=4)
    assert np.all(r["cam_gid"] == -1)
    occl = int((r["shadow_vis"][0] == 0).sum())
    # the shadow ray the plane point spawns, built with the same FP32 steps
    t = F32(F32(-2.5) - o[0, 1]) / d[0, 1]
    P = (o[0] + (t * d[0]).astype(F32)).astype(F32)
    P[1] = F32(-2.5)
    v = (np.array([5, 5, 5], F32) - P).astype(F32)
    ln = np.sqrt(F32(F32(v[0] * v[0]) + F32(v[1] * v[1])) + F32(v[2] * v[2]))
    cand = oracle.candidates(rec, P, (v / ln).astype(F32), tmin=float(F32(1e-4)), tmax=float(ln))
    assert cand["gid"].tolist() == [0]
    assert binomtest(occl, n, float(cand["alpha"][0])).pvalue > 1e-4


def _sh_colour_scipy(coef, direction):
    """max(0, 0.5 + sum_lm k_lm Y_lm(d)) per channel with scipy's harmonics."""
    dv = np.asarray(direction, np.float64)
    dv = dv / np.linalg.norm(dv)
    K = coef.shape[0]
    deg = int(round(math.sqrt(K))) - 1
    Y = np.array([_real_sh_scipy(l, m, dv) for l in range(deg + 1) for m in range(-l, l + 1)])
    return np.maximum(0.0, 0.5 + Y @ coef.astype(np.float64))


def _fp32_shading_point(o, d, t):
    """P = o + (t * d), per component in FP32 (the secondary-ray construction)."""
    return np.array([F32(F32(o[i]) + F32(F32(t) * F32(d[i]))) for i in range(3)], F32)


def _fp32_light_dir(P, light=(5.0, 5.0, 5.0)):
    v = (np.asarray(light, F32) - P).astype(F32)
    ln = np.sqrt(F32(F32(F32(v[0] * v[0]) + F32(v[1] * v[1])) + F32(v[2] * v[2])))
    return (v / ln).astype(F32), F32(ln)


def test_pathmix_gaussian_hit_colour_and_self_shadow():
    """A camera sample that accepts Gaussian A is shaded c_A (0.3 + 0.7 V),
    c_A its SH colour along the camera ray and V the visibility of the light
    (Sec. 1 / Sec. 5 secondary rays). The shadow ray starts inside A, where
    A is a valid candidate of it, yet it must never report A (its spawning
    Gaussian): with the occluder B switched off, V = 1. With B accepted,
    V = 0."""
    rng = np.random.default_rng(17)
    sh = rng.normal(0, 0.4, (3, 16, 3)).astype(F32)
    o = np.array([-0.05, 0.0, 4.0], F32)
    d = np.array([0.0, 0.0, -1.0], F32)
    # A near the camera ray at depth 2; B straddles the shadow ray 1.0 further on
    P_est = np.array([-0.05, 0.0, 2.0])
    l_est = np.array([5.0, 5.0, 5.0]) - P_est
    l_est /= np.linalg.norm(l_est)
    B = P_est + 1.0 * l_est
    C = [5.0, -40.0, 5.0]  # far away, never a candidate
    sc = _scene([[0.0, 0.0, 2.0], B, C], np.log(np.full((3, 3), 0.1)), [[1, 0, 0, 0]] * 3,
                [_logit(0.8)] * 3, sh, deg=3)
    rec = oracle.Records(sc)
    for V, uB in ((1, 1.0), (0, 0.0)):
        u = np.array([0.0, uB, 1.0])
        r = oracle.pathmix(rec, o[None], d[None], spp=1, u_override=u)
        assert r["cam_gid"][0, 0] == 0 and r["mirror_gid"][0, 0] == -2
        assert r["shadow_vis"][0, 0] == V
        cA = _sh_colour_scipy(sh[0], d)
        np.testing.assert_allclose(r["rgb"][0], cA * (0.3 + 0.7 * V), rtol=1e-12, atol=1e-12)
    # the precondition that makes the check bite: A is a valid candidate of
    # the shadow ray it spawns, and B lies on it
    P = _fp32_shading_point(o, d, r["cam_t"][0, 0])
    l, ln = _fp32_light_dir(P)
    cand = oracle.candidates(rec, P, l, tmin=float(F32(1e-4)), tmax=float(ln))
    assert set(cand["gid"].tolist()) == {0, 1}, cand


def test_pathmix_mirror_hit_colour():
    """A camera ray that reaches the ground plane y = -2.5 spawns a mirror ray
    along (dx, -dy, dz); the plane point is shaded 0.5 V max(0, l_y) + 0.5 c,
    c the SH colour of the mirror ray's accepted Gaussian seen along the
    reflected direction (not the camera's)."""
    rng = np.random.default_rng(18)
    sh = rng.normal(0, 0.4, (2, 16, 3)).astype(F32)
    o = np.array([0.0, 0.0, 4.0], F32)
    d = (np.array([0.0, -1.0, -0.5]) / math.sqrt(1.25)).astype(F32)
    tp = F32(F32(F32(-2.5) - o[1]) / d[1])
    P = _fp32_shading_point(o, d, tp)
    P[1] = F32(-2.5)
    md = np.array([d[0], -d[1], d[2]], F32)
    Cg = P.astype(np.float64) + 2.0 * md
    sc = _scene([Cg, [5.0, -40.0, 5.0]], np.log(np.full((2, 3), 0.1)), [[1, 0, 0, 0]] * 2,
                [_logit(0.8)] * 2, sh, deg=3)
    rec = oracle.Records(sc)
    bg = np.array([0.05, 0.1, 0.2])
    for uC, hit in ((0.0, True), (1.0, False)):
        r = oracle.pathmix(rec, o[None], d[None], spp=1, bg=bg, u_override=np.array([uC, 1.0]))
        assert r["cam_gid"][0, 0] == -1 and r["shadow_vis"][0, 0] == 1
        assert r["mirror_gid"][0, 0] == (0 if hit else -1)
        l, _ = _fp32_light_dir(P)
        Lm = _sh_colour_scipy(sh[0], md) if hit else bg
        expect = 0.5 * max(0.0, float(l[1])) + 0.5 * Lm
        np.testing.assert_allclose(r["rgb"][0], expect, rtol=1e-12, atol=1e-12)
    # the reflected direction matters: the camera direction would give another colour
    assert np.abs(_sh_colour_scipy(sh[0], md) - _sh_colour_scipy(sh[0], d)).max() > 0.05


# --------------------------------------------------------------------------
# Centre depth (Sec. 4.1)
# --------------------------------------------------------------------------
def test_center_depth_orders_by_projected_centre():
    """Two Gaussians whose 1D means and projected centres order differently:
    an elongated, tilted front Gaussian whose mean along the ray lies behind a
    round one, while its centre projects in front of it."""
    s = math.sqrt(0.5)
    q_tilt = [math.cos(math.pi / 8), 0.0, math.sin(math.pi / 8), 0.0]  # 45 deg about y
    sc = _scene([[0.3, 0.0, 1.9], [0.0, 0.0, 2.0]], np.log([[0.6, 0.05, 0.05], [0.1, 0.1, 0.1]]),
                [q_tilt, [1, 0, 0, 0]], [_logit(0.9), _logit(0.9)])
    rec = oracle.Records(sc, round_f32=False)
    o, d = [0, 0, 0], [0, 0, 1]
    c_mean = oracle.candidates(rec, o, d)
    assert list(c_mean["gid"]) == [1, 0], c_mean
    c_ctr = oracle.candidates(rec, o, d, depth_mode=1)
    assert list(c_ctr["gid"]) == [0, 1]
    np.testing.assert_allclose(c_ctr["t"], [np.float32(1.9), 2.0], rtol=1e-7)
    # alpha stays at the 1D peak: identical in both modes
    np.testing.assert_allclose(sorted(c_ctr["alpha"]), sorted(c_mean["alpha"]), rtol=1e-15)
    # with a viewing axis, the depth is the centre's depth along it converted
    # to the ray parameter
    axis = np.array([0.0, 0.6, 0.8])
    d2 = np.array([0.0, 0.05, 1.0], np.float32)
    c_ax = oracle.candidates(rec, o, d2, depth_mode=1, depth_axis=axis)
    for g, t in zip(c_ax["gid"], c_ax["t"]):
        mu = rec.mu[g]
        assert abs(t - (mu @ axis) / (d2.astype(np.float64) @ axis)) < 1e-12
