"""GPU parity of the forward path against the FP64 oracle, through the C ABI.

Accepted ids must match the oracle bit for bit on every sample it does not
flag (|alpha - u| < 1e-6 or a geometric tie); pixel colours within 1e-4."""
import numpy as np
import pytest
import torch

import oracle
import srt_inputs as si
from _parity import (check_bvh_structure, compare_ids, compare_rgb, device_scene, say,
                     tiny_scene, to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srt():
    import paper_2504_06598_amd as srt
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    srt._lib.load()
    return srt


def _cuda(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _trace(srt, bvh, o, d, **kw):
    res = srt.srt_trace_forward(bvh, _cuda(o), _cuda(d), **kw)
    torch.cuda.synchronize()
    return {k: to_np(v) for k, v in res.items()}


def _ulps(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


# --------------------------------------------------------------------------
def test_records_match_oracle(srt):
    say("records: tiny cube scene, 1000 Gaussians")
    sc = si.workload(1)["scene"]
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    r = {k: to_np(v) for k, v in bvh.records().items()}
    ora = oracle.Records(sc)
    dM = _ulps(r["M"], ora.M.astype(np.float32))
    dop = _ulps(r["opacity"], ora.op.astype(np.float32))
    assert dM.max() <= 1 and (dM == 0).mean() > 0.999
    assert dop.max() <= 1 and (dop == 0).mean() > 0.999
    assert np.array_equal(r["mu"], sc.means)
    # each box contains the exact box of its record's k-sigma ellipsoid
    M = r["M"].astype(np.float64).reshape(-1, 3, 3)
    Minv = np.linalg.inv(M)
    h = np.sqrt(8.0 * (Minv ** 2).sum(2))
    mu = r["mu"].astype(np.float64)
    assert np.all(r["box_lo"] <= mu - h) and np.all(r["box_hi"] >= mu + h)
    assert np.all(r["box_hi"] - r["box_lo"] <= 2 * h * (1 + 1e-5) + 1e-6)


@pytest.mark.parametrize("W,L", [(2, 1), (4, 4), (8, 8), (4, 1), (8, 3)])
def test_bvh_structure(srt, W, L):
    say(f"bvh structure W={W} L={L}")
    sc = si.scene_shell(9, 5000, 0)
    bvh = srt.srt_build_bvh(device_scene(sc), W, L)
    check_bvh_structure(bvh, W, L, 5000)


def test_camera_rays_bit_exact(srt):
    cams = [si.look_at((0, 0, 3), (0, 0, 0), 64, 64),
            si.look_at((0.3, -1.0, 2.5), (0.1, 0, 0), 97, 41, vfov_deg=45.0),
            *si.ring_cameras(3, 3.0, 33, 17), *si.fibonacci_cameras(4, 3.0, 20, 20)]
    for cam in cams:
        say(f"camera rays {cam.width}x{cam.height}")
        o, d = srt.srt_camera_rays(cam)
        ho, hd = si.camera_rays(cam)
        assert np.array_equal(to_np(o).view(np.uint32), ho.view(np.uint32))
        assert np.array_equal(to_np(d).view(np.uint32), hd.view(np.uint32))


def test_forward_parity_tiny_workload(srt):
    say("forward parity: 1000 Gaussians, 64x64, 1 spp, N=1")
    w = si.workload(1)
    sc, cam = w["scene"], w["cameras"][0]
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    g = _trace(srt, bvh, o, d, seed=0, spp=1, n_per_traversal=1)
    ora = oracle.trace(oracle.Records(sc), oracle.Rays(o, d), spp=1, seed=0)
    nf = compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"])
    same = (g["hit_gid"] == ora["hit_gid"]) & (ora["hit_gid"] >= 0)
    assert same.sum() > 500 and (ora["hit_gid"] < 0).sum() > 500
    assert _ulps(g["hit_t"][same], ora["hit_t"][same]).max() <= 1
    err = compare_rgb(g["rgb"], ora["rgb"], ora["flags"])
    say(f"  flagged {nf}, colour err {err:.2e}")


@pytest.mark.parametrize("N,spp", [(1, 8), (2, 8), (4, 8), (8, 8), (4, 6), (8, 3)])
def test_multisample_matches_oracle(srt, N, spp):
    say(f"multi-sample N={N} spp={spp}")
    sc = tiny_scene(11, 1500, (0.02, 0.08), deg=2)
    cam = si.look_at((0.2, 0.3, 3), (0, 0, 0), 40, 30)
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    g = _trace(srt, bvh, o, d, seed=123456789012345, spp=spp, n_per_traversal=N,
               sample_offset=5, bg=(0.1, 0.2, 0.3))
    ora = oracle.trace(oracle.Records(sc), oracle.Rays(o, d, sample_base=np.full(len(o), 5)),
                       spp=spp, seed=123456789012345, bg=(0.1, 0.2, 0.3))
    compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"])
    compare_rgb(g["rgb"], ora["rgb"], ora["flags"])
    if N > 1:
        g1 = _trace(srt, bvh, o, d, seed=123456789012345, spp=spp, n_per_traversal=1,
                    sample_offset=5, bg=(0.1, 0.2, 0.3))
        assert np.array_equal(g1["hit_gid"], g["hit_gid"]), "N per traversal changes results"


def test_width_and_leaf_size_invariance(srt):
    sc = tiny_scene(12, 3000, (0.01, 0.06))
    cam = si.look_at((0, 0.5, 2.8), (0, 0, 0), 48, 48)
    o, d = si.camera_rays(cam)
    ref = None
    dsc = device_scene(sc)
    for W in (2, 4, 8):
        for L in (1, 2, 4, 8):
            say(f"invariance W={W} L={L}")
            bvh = srt.srt_build_bvh(dsc, W, L)
            g = _trace(srt, bvh, o, d, seed=3, spp=4, n_per_traversal=4)
            if ref is None:
                ref = g["hit_gid"]
                ora = oracle.trace(oracle.Records(sc), oracle.Rays(o, d), spp=4, seed=3)
                compare_ids(ref, ora["hit_gid"], ora["flags"])
            else:
                assert np.array_equal(g["hit_gid"], ref), (W, L)


def test_deep_stack_fallback_is_exact(srt, tmp_path):
    say("deep-stack fallback: stack limit 1 and 2")
    sc = tiny_scene(13, 2000, (0.03, 0.1))
    cam = si.look_at((0, 0, 3), (0, 0, 0), 32, 32)
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(sc), 2, 1)
    base = _trace(srt, bvh, o, d, seed=1, spp=2, n_per_traversal=2)
    for lim in (1, 2):
        cnt = srt.new_counters()
        g = _trace(srt, bvh, o, d, seed=1, spp=2, n_per_traversal=2, stack_limit=lim,
                   counters=cnt)
        c = srt.counters_dict(cnt)
        assert c["deep"] > 0 and c["lost"] == 0
        assert c["ray_samples"] == len(o) * 2  # a rerun ray is counted once
        assert np.array_equal(g["hit_gid"], base["hit_gid"])
        np.testing.assert_array_equal(g["rgb"], base["rgb"])


def test_coincident_duplicates_tie_by_id(srt):
    say("coincident duplicates: 300 copies, W=2 L=1")
    base = tiny_scene(14, 1, (0.2, 0.2))
    n = 300
    sc = si.Scene(np.repeat(base.means, n, 0), np.repeat(base.log_scales, n, 0),
                  np.repeat(base.quats, n, 0), np.full(n, -1.0, np.float32),
                  np.repeat(base.sh, n, 0), 0)
    mu = base.means[0]
    o = np.tile((mu + np.array([0, 0, 3])).astype(np.float32), (64, 1))
    rng = np.random.default_rng(0)
    d = np.tile(np.array([0, 0, -1], np.float32), (64, 1))
    d[:, :2] += rng.normal(0, 0.02, (64, 2)).astype(np.float32)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    bvh = srt.srt_build_bvh(device_scene(sc), 2, 1)
    g = _trace(srt, bvh, o, d, seed=2, spp=4, n_per_traversal=4)
    ora = oracle.trace(oracle.Records(sc), oracle.Rays(o, d), spp=4, seed=2)
    compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"])
    # equal depth keys: the smallest accepted id wins
    assert (g["hit_gid"] >= 0).mean() > 0.9


def test_ray_fields_and_any_hit(srt):
    say("ray fields: tmin/tmax/ignore/ray ids/sample ids/purpose; any-hit")
    sc = tiny_scene(15, 2000, (0.02, 0.06), deg=1)
    rng = np.random.default_rng(5)
    R = 3000
    o = rng.uniform(-1.2, 1.2, (R, 3)).astype(np.float32)
    d = rng.normal(0, 1, (R, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tmin = rng.uniform(0, 0.3, R).astype(np.float32)
    tmax = rng.uniform(0.5, 3.0, R).astype(np.float32)
    tmax[:20] = tmin[:20] * 0.5  # empty ranges
    ign = rng.integers(-1, 2000, R).astype(np.int32)
    rid = rng.integers(0, 2 ** 32, R, dtype=np.uint64).astype(np.uint32)
    sid = rng.integers(0, 1000, R).astype(np.uint32)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    rec = oracle.Records(sc)
    for purpose, any_hit in [(4, False), (2, True)]:
        g = _trace(srt, bvh, o, d, tmin=_cuda(tmin), tmax=_cuda(tmax), ignore_gid=_cuda(ign),
                   ray_ids=_cuda(rid), sample_ids=_cuda(sid), purpose=purpose, seed=77, spp=1,
                   n_per_traversal=1, any_hit=any_hit)
        ora = oracle.trace(rec, oracle.Rays(o, d, tmin, tmax, ign, rid, sid), spp=1, seed=77,
                           purpose=purpose, any_hit=any_hit)
        if any_hit:
            occl_g = g["hit_gid"] >= 0
            occl_o = ora["hit_gid"] >= 0
            bad = (occl_g != occl_o) & (ora["flags"] == 0)
            assert not bad.any()
            assert occl_o.sum() > 50
            vis = 1.0 - occl_g[:, 0].astype(np.float32)
            np.testing.assert_array_equal(g["rgb"][:, 0], vis)
            # whatever id the GPU reports is an accepted valid candidate
            for i in np.nonzero(occl_g[:, 0])[0][:100]:
                gid = int(g["hit_gid"][i, 0])
                ok, t, q, a = oracle.isect_one(rec, gid, o[i], d[i], tmin[i], tmax[i])
                assert ok and gid != ign[i]
                assert oracle.accept_u(77, int(rid[i]), int(sid[i]), gid, purpose) < a
        else:
            compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"])
            compare_rgb(g["rgb"], ora["rgb"], ora["flags"])
            assert np.all(g["hit_gid"][:20] == -1)


def test_edge_cases(srt):
    say("edge cases: no rays, no Gaussians, one Gaussian, one leaf")
    sc = tiny_scene(16, 500)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    z = np.zeros((0, 3), np.float32)
    g = _trace(srt, bvh, z, z, spp=2)
    assert g["rgb"].shape == (0, 3)
    cam = si.look_at((0, 0, 3), (0, 0, 0), 16, 16)
    o, d = si.camera_rays(cam)
    for n in (0, 1, 3):
        say(f"  scene of {n} Gaussians")
        s = sc.subset(np.arange(n))
        s.log_scales[:] = np.log(0.5)
        b = srt.srt_build_bvh(device_scene(s), 4, 4)
        g = _trace(srt, b, o, d, seed=4, spp=3, n_per_traversal=1, bg=(0.25, 0.5, 0.75))
        if n == 0:
            assert np.all(g["hit_gid"] == -1)
            np.testing.assert_allclose(g["rgb"], np.tile([0.25, 0.5, 0.75], (256, 1)))
        else:
            ora = oracle.trace(oracle.Records(s), oracle.Rays(o, d), spp=3, seed=4,
                               bg=(0.25, 0.5, 0.75))
            compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"], max_flag_frac=0.01)
            compare_rgb(g["rgb"], ora["rgb"], ora["flags"])


def test_error_codes(srt):
    sc = tiny_scene(17, 100)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    o = torch.zeros((10, 3), device="cuda")
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_forward(bvh, o, o, n_per_traversal=3)
    assert e.value.code == 1
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_forward(bvh, o, o, any_hit=True, n_per_traversal=4, spp=4)
    assert e.value.code == 1
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    lib = srt._lib.load()
    import ctypes as C
    rays = srt._lib.SrtRays(10, o.data_ptr(), o.data_ptr(), None, None, None, None, None, 0)
    opts = srt._opts(0, 1, 1, 0, (0, 0, 0), False, 0)
    assert lib.srt_trace_forward(bvh.handle, C.byref(rays), C.byref(opts), None, None, None,
                                 None, ws.data_ptr(), 16, None) == 5
    with pytest.raises(srt.SrtError):
        srt.srt_build_bvh(device_scene(sc), 3, 4)


def test_counters(srt):
    sc = tiny_scene(18, 2000)
    cam = si.look_at((0, 0, 3), (0, 0, 0), 32, 32)
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    cnt = srt.new_counters()
    _trace(srt, bvh, o, d, spp=4, n_per_traversal=2, counters=cnt)
    c = srt.counters_dict(cnt)
    assert c["traversals"] == 1024 * 2
    assert c["ray_samples"] == 1024 * 4
    assert c["nodes"] >= c["traversals"]
    assert c["prims"] >= c["candidates"] > 0
    assert c["philox"] > 0 and c["deep"] == 0 and c["lost"] == 0


@pytest.mark.parametrize("axis", ["camera", "ray"])
def test_center_depth_matches_oracle(srt, axis):
    """Centre depth (Sec. 4.1): order and range-test by the centre projected
    onto the camera axis (or each ray's direction), alpha at the 1D peak."""
    say(f"centre depth, axis = {axis}")
    sc = tiny_scene(41, 2500, (0.02, 0.12), deg=1)
    cam = si.look_at((0.4, 0.3, 2.7), (0, 0, 0), 48, 40)
    o, d = si.camera_rays(cam)
    ax = tuple(float(x) for x in cam.forward) if axis == "camera" else (0.0, 0.0, 0.0)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    g = _trace(srt, bvh, o, d, seed=8, spp=8, n_per_traversal=4, depth_mode=1, depth_axis=ax)
    ora = oracle.trace(oracle.Records(sc), oracle.Rays(o, d), spp=8, seed=8, depth_mode=1,
                       depth_axis=ax)
    compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"])
    compare_rgb(g["rgb"], ora["rgb"], ora["flags"])
    same = (g["hit_gid"] == ora["hit_gid"]) & (ora["hit_gid"] >= 0)
    assert _ulps(g["hit_t"][same], ora["hit_t"][same]).max() <= 1
    # the centre depth changes results compared with the mean depth
    g0 = _trace(srt, bvh, o, d, seed=8, spp=8, n_per_traversal=4)
    assert (g0["hit_gid"] != g["hit_gid"]).mean() > 0.01


@pytest.mark.parametrize("axis,inside,walk", [("camera", False, "lane"),
                                               ("camera", False, "wave"),
                                               ("ray", False, "wave"),
                                               ("camera", True, "lane"),
                                               ("camera", True, "wave"),
                                               ("ray", True, "lane")])
def test_center_depth_with_tmin_matches_oracle(srt, axis, inside, walk):
    """Centre depth with tmin > 0: a Gaussian whose centre depth lies past
    tmin but which the ray crosses before tmin is still a candidate, so boxes
    that the ray leaves before tmin (but not before tmin minus the depth
    slack) must be walked. Rays start at random tmin in [0, 1.5], and (inside)
    from a camera in the middle of the cloud."""
    say(f"centre depth with tmin: axis {axis}, camera inside {inside}, {walk} walks")
    sc = tiny_scene(43, 3000, (0.02, 0.12), deg=1)
    if inside:
        cam = si.look_at((0.05, -0.1, 0.0), (0.3, 0.2, -1.0), 40, 32, vfov_deg=80.0)
    else:
        cam = si.look_at((0.3, 0.2, 2.2), (0, 0, 0), 40, 32, vfov_deg=75.0)
    o, d = si.camera_rays(cam)
    R = len(o)
    rng = np.random.default_rng(44)
    tmin = rng.uniform(0.0, 1.5 if inside else 3.0, R).astype(np.float32)
    if inside:
        tmin[::3] = 0.0
    ax = tuple(float(x) for x in cam.forward) if axis == "camera" else (0.0, 0.0, 0.0)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    g = _trace(srt, bvh, o, d, seed=9, spp=8, n_per_traversal=4, depth_mode=1, depth_axis=ax,
               tmin=_cuda(tmin), image_width=cam.width, walk=walk)
    rays = oracle.Rays(o, d, tmin, None, None)
    ora = oracle.trace(oracle.Records(sc), rays, spp=8, seed=9, depth_mode=1, depth_axis=ax)
    compare_ids(g["hit_gid"], ora["hit_gid"], ora["flags"])
    compare_rgb(g["rgb"], ora["rgb"], ora["flags"])
    hit = ora["hit_gid"] >= 0
    assert hit.mean() > 0.2
    if axis == "camera":
        # the case the test is about occurs: accepted Gaussians whose exact
        # k-sigma box the ray leaves before tmin
        rec = oracle.Records(sc)
        Minv = np.linalg.inv(rec.M.reshape(-1, 3, 3))
        h = np.sqrt(8.0 * (Minv ** 2).sum(2))
        r_idx, s_idx = np.nonzero(hit)
        gg = ora["hit_gid"][r_idx, s_idx]
        inv = 1.0 / d[r_idx].astype(np.float64)
        a = (rec.mu[gg] - h[gg] - o[r_idx]) * inv
        b = (rec.mu[gg] + h[gg] - o[r_idx]) * inv
        t_exit = np.maximum(a, b).min(1)
        assert (t_exit < tmin[r_idx]).sum() > 0


@pytest.mark.parametrize("w,h", [(13, 9), (40, 24), (1, 5), (8, 8)])
def test_image_tiles_change_nothing(srt, w, h):
    say(f"tiled image launch {w}x{h}")
    sc = tiny_scene(19, 2500, (0.02, 0.08))
    cam = si.look_at((0.2, 0.1, 2.9), (0, 0, 0), w, h)
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    for lim in (0, 1):  # the on-chip stack, and the deep-stack rerun of every ray
        base = _trace(srt, bvh, o, d, seed=5, spp=4, n_per_traversal=4, stack_limit=lim)
        cnt = srt.new_counters()
        tiled = _trace(srt, bvh, o, d, seed=5, spp=4, n_per_traversal=4, stack_limit=lim,
                       image_width=w, counters=cnt)
        for k in ("hit_gid", "hit_t", "rgb"):
            np.testing.assert_array_equal(tiled[k], base[k])
        c = srt.counters_dict(cnt)
        assert c["ray_samples"] == w * h * 4 and c["lost"] == 0
    if (w, h) == (13, 9):
        ora = oracle.trace(oracle.Records(sc), oracle.Rays(o, d), spp=4, seed=5)
        compare_ids(tiled["hit_gid"], ora["hit_gid"], ora["flags"])


def test_image_width_errors(srt):
    sc = tiny_scene(20, 100)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    o = torch.zeros((10, 3), device="cuda")
    for bad in (3, -1):
        with pytest.raises(srt.SrtError) as e:
            srt.srt_trace_forward(bvh, o, o, image_width=bad)
        assert e.value.code == 1
        with pytest.raises(srt.SrtError) as e:
            srt.srt_trace_backward(bvh, o, o, torch.ones((10, 3), device="cuda"),
                                   image_width=bad)
        assert e.value.code == 1


@pytest.mark.parametrize("N,spp,any_hit,thr", [(4, 8, False, 16), (1, 3, False, 1),
                                               (8, 8, False, 64), (2, 6, False, 0),
                                               (1, 1, True, 16)])
def test_persistent_equals_plain(srt, N, spp, any_hit, thr):
    say(f"persistent waves vs one lane per ray: N={N} spp={spp} any_hit={any_hit} thr={thr}")
    sc = tiny_scene(21, 3000, (0.02, 0.08))
    cam = si.look_at((0.1, 0.3, 2.8), (0, 0, 0), 37, 29)
    o, d = si.camera_rays(cam)
    R = len(o)
    rng = np.random.default_rng(5)
    tmin = rng.uniform(0.0, 1.5, R).astype(np.float32)
    tmax = (tmin + rng.uniform(-0.2, 4.0, R)).astype(np.float32)  # some rays empty
    ign = rng.integers(-1, 3000, R).astype(np.int32)
    kw = dict(seed=11, spp=spp, n_per_traversal=N, any_hit=any_hit, bg=(0.2, 0.1, 0.7),
              tmin=_cuda(tmin), tmax=_cuda(tmax), ignore_gid=_cuda(ign), sample_offset=7)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    for lim, iw in ((0, 0), (1, 0), (0, cam.width)):
        base = _trace(srt, bvh, o, d, stack_limit=lim, image_width=iw, **kw)
        cnt = srt.new_counters()
        pers = _trace(srt, bvh, o, d, stack_limit=lim, image_width=iw, persistent=True,
                      refill_threshold=thr, counters=cnt, **kw)
        for k in ("hit_gid", "hit_t", "rgb"):
            np.testing.assert_array_equal(pers[k], base[k], err_msg=f"{k} lim={lim} iw={iw}")
        c = srt.counters_dict(cnt)
        assert c["lost"] == 0
        assert c["ray_samples"] == int((tmax > tmin).sum()) * spp
        if lim:
            assert c["deep"] > 0


def test_persistent_pathmix_equals_plain(srt):
    say("path-tracer mix: persistent waves and wave-shared walks change nothing")
    w = si.workload(3, small=True)
    cam = w["cameras"][0]
    bvh = srt.srt_build_bvh(device_scene(w["scene"]), 4, 2)
    outs = []
    for pers, walk in ((False, "lane"), (True, "lane"), (False, "wave"), (False, "auto")):
        res = srt.srt_trace_pathmix(bvh, cam, seed=2, spp=8, n_per_traversal=4,
                                    light=si.LIGHT_POS, plane_y=si.PLANE_Y,
                                    tmin_secondary=si.SECONDARY_TMIN, persistent=pers, walk=walk)
        torch.cuda.synchronize()
        outs.append({k: to_np(v) for k, v in res.items()})
    for o in outs[1:]:
        for k in outs[0]:
            np.testing.assert_array_equal(o[k], outs[0][k], err_msg=k)


def test_persistent_option_errors(srt):
    sc = tiny_scene(22, 100)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    o = torch.zeros((10, 3), device="cuda")
    for kw in (dict(persistent=True, refill_threshold=65),
               dict(persistent=True, refill_threshold=-1)):
        with pytest.raises(srt.SrtError) as e:
            srt.srt_trace_forward(bvh, o, o, **kw)
        assert e.value.code == 1
    opts = srt._opts(0, 1, 1, 0, (0, 0, 0), False, 0)
    opts.persistent = 2
    import ctypes as C
    lib = srt._lib.load()
    rays = srt._lib.SrtRays(10, o.data_ptr(), o.data_ptr(), None, None, None, None, None, 0)
    ws = torch.empty(lib.srt_trace_workspace_size(bvh.handle, 10), dtype=torch.uint8,
                     device="cuda")
    assert lib.srt_trace_forward(bvh.handle, C.byref(rays), C.byref(opts), None, None, None,
                                 None, ws.data_ptr(), ws.numel(), None) == 1


def test_camera_jitter_bit_exact(srt):
    cam = si.look_at((0.3, 0.1, 3), (0, 0, 0), 33, 21)
    for frame in (1, 6, 99):
        jc = si.jittered(cam, frame)
        o, d = srt.srt_camera_rays(jc)
        ho, hd = si.camera_rays(jc)
        assert np.array_equal(to_np(d), hd) and np.array_equal(to_np(o), ho)


def test_hash_rng_accepts_with_probability_alpha(srt):
    """One Gaussian on the axis of parallel rays (q = 0 on the axis, so alpha
    is its opacity): the share of samples that accept it, over many rays and
    samples, is alpha within the binomial spread plus the hash's FP32
    resolution."""
    from scipy.stats import binom
    for op in (0.2, 0.55, 0.9):
        sc = si.Scene(np.zeros((1, 3), np.float32), np.full((1, 3), np.log(0.3), np.float32),
                      np.array([[1, 0, 0, 0]], np.float32),
                      np.array([np.log(op / (1 - op))], np.float32),
                      np.zeros((1, 1, 3), np.float32), 0)
        bvh = srt.srt_build_bvh(device_scene(sc), 4, 1)
        n = 4096
        rng = np.random.default_rng(3)
        o = np.zeros((n, 3), np.float32)
        o[:, :2] = rng.uniform(-1e-3, 1e-3, (n, 2))
        o[:, 2] = -3.0
        d = np.tile(np.array([[0, 0, 1]], np.float32), (n, 1))
        res = _trace(srt, bvh, o, d, spp=8, n_per_traversal=8, rng="hash")
        hits = int((res["hit_gid"] >= 0).sum())
        total = res["hit_gid"].size
        alpha = float(oracle.Records(sc).op[0])
        lo, hi = binom.ppf([1e-6, 1 - 1e-6], total, alpha)
        slack = total / 128.0  # the FP32 hash resolves about 1/256
        assert lo - slack <= hits <= hi + slack, (op, hits / total, alpha)


def test_hash_rng_converges_to_the_exact_composite(srt):
    """Frames of Sobol-jittered camera rays with hash acceptance: the frame
    average of each pixel approaches the average of the exact composites of
    the same jittered rays (the oracle), within the sample noise and the
    hash's FP32 resolution."""
    say("hash RNG: 96 jittered frames of a 24x24 view")
    sc = tiny_scene(23, 600, (0.04, 0.12))
    cam = si.look_at((0.1, 0.2, 3), (0, 0, 0), 24, 24)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    rec = oracle.Records(sc)
    F = 96
    acc = np.zeros((24 * 24, 3))
    exact = np.zeros((24 * 24, 3))
    var = np.zeros((24 * 24, 3))
    for f in range(F):
        jc = si.jittered(cam, f + 1)
        o, d = si.camera_rays(jc)
        res = _trace(srt, bvh, o, d, spp=1, rng="hash", want_hits=False)
        acc += res["rgb"]
        ex = oracle.composite(rec, oracle.Rays(o, d))
        exact += ex["L"]
        var += ex["var"]
    acc /= F
    exact /= F
    se = np.sqrt(var / F / F)
    err = np.abs(acc - exact)
    assert np.mean(err <= 5 * se + 0.02) > 0.995, float((err / (se + 1e-3)).max())
    # and the average error is at the level of the noise
    assert err.mean() < 3 * se.mean() + 0.005


def test_hash_rng_unsupported_combinations(srt):
    sc = tiny_scene(24, 100)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    o = torch.zeros((10, 3), device="cuda")
    d = torch.tensor([[0.0, 0.0, 1.0]] * 10, device="cuda")
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_forward(bvh, o, d, rng="hash", persistent=True)
    assert e.value.code == 4
    g = torch.ones((10, 3), device="cuda")
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_backward(bvh, o, d, g, rng="hash")  # recompute needs numbers
    assert e.value.code == 4
    fw = srt.srt_trace_forward(bvh, o, d, rng="hash", spp=2, n_per_traversal=2)
    srt.srt_trace_backward(bvh, o, d, g, hit_gid=fw["hit_gid"], hit_t=fw["hit_t"], spp=2,
                           n_per_traversal=2, rng="hash")  # stored results: fine
    with pytest.raises(srt.SrtError) as e:
        srt.srt_batch_plan_create(bvh, [si.look_at((0, 0, 3), (0, 0, 0), 8, 8)], [1],
                                  rng="hash")
    assert e.value.code == 4
    opts = srt._opts(0, 1, 1, 0, (0, 0, 0), False, 0)
    opts.rng = 2
    import ctypes as C
    lib = srt._lib.load()
    rays = srt._lib.SrtRays(10, o.data_ptr(), d.data_ptr(), None, None, None, None, None, 0)
    ws = torch.empty(lib.srt_trace_workspace_size(bvh.handle, 10), dtype=torch.uint8,
                     device="cuda")
    assert lib.srt_trace_forward(bvh.handle, C.byref(rays), C.byref(opts), None, None, None,
                                 None, ws.data_ptr(), ws.numel(), None) == 1


@pytest.mark.parametrize("W,L,N,spp,mode,lim,image,any_hit", [
    (4, 2, 4, 8, 0, 0, True, False), (2, 1, 1, 3, 0, 0, True, False),
    (8, 4, 8, 8, 0, 0, True, False), (4, 4, 2, 6, 1, 0, True, False),
    (4, 2, 4, 8, 0, 5, True, False), (8, 1, 4, 4, 1, 2, True, False),
    (4, 2, 4, 8, 0, 0, False, False), (4, 2, 1, 1, 0, 0, False, True),
    (4, 2, 1, 3, 0, 3, True, True), (2, 4, 1, 2, 1, 0, False, True),
    (4, 2, 4, 16, 0, 0, True, False), (4, 2, 4, 13, 1, 0, True, False),
    (2, 4, 4, 7, 0, 3, True, False), (8, 2, 2, 8, 0, 0, True, False),
    (4, 2, 8, 16, 0, 0, True, False), (4, 2, 8, 16, 1, 0, True, False),
    (4, 2, 8, 13, 0, 0, True, False)])
def test_wave_walk_equals_lane_walk(srt, W, L, N, spp, mode, lim, image, any_hit):
    """The 64 rays of a tile (or 64 consecutive rays) walking the BVH together
    reach, per ray, the same candidates as the ray's own walk: outputs equal
    bit for bit, with ragged tiles, empty rays, ignored ids and (lim > 0)
    groups whose shared stack overflows into the deep pass. Images whose rays
    need 2 or 4 passes put each pass of a pixel on its own lane (8x4 or 4x4
    pixels per wave; colours summed in sample order across the lanes), also
    with a partial last pass. Any-hit rays: the same visibility; the reported
    id is some accepted candidate, which may differ with the visiting
    order."""
    say(f"wave-shared walk vs lane walk: W={W} L={L} N={N} spp={spp} depth mode {mode} "
        f"stack limit {lim} image {image} any-hit {any_hit}")
    sc = tiny_scene(23, 3000, (0.02, 0.08))
    cam = si.look_at((0.1, 0.3, 2.8), (0, 0, 0), 37, 29)
    o, d = si.camera_rays(cam)
    R = len(o)
    rng = np.random.default_rng(9)
    tmin = rng.uniform(0.0, 1.5, R).astype(np.float32)
    tmax = (tmin + rng.uniform(-0.2, 4.0, R)).astype(np.float32)
    tmax[::7] = np.inf
    ign = rng.integers(-1, 3000, R).astype(np.int32)
    kw = dict(seed=13, spp=spp, n_per_traversal=N, bg=(0.2, 0.1, 0.7), tmin=_cuda(tmin),
              tmax=_cuda(tmax), ignore_gid=_cuda(ign), sample_offset=3, depth_mode=mode,
              image_width=cam.width if image else 0, stack_limit=lim, any_hit=any_hit)
    bvh = srt.srt_build_bvh(device_scene(sc), W, L)
    lane = _trace(srt, bvh, o, d, walk="lane", **kw)
    cnt = srt.new_counters()
    wave = _trace(srt, bvh, o, d, walk="wave", counters=cnt, **kw)
    if any_hit:
        np.testing.assert_array_equal(wave["rgb"], lane["rgb"])
        np.testing.assert_array_equal(wave["hit_gid"] >= 0, lane["hit_gid"] >= 0)
        hit = wave["hit_gid"] >= 0
        t = wave["hit_t"]
        assert np.all(hit == np.isfinite(t))
        lo = np.repeat(tmin[:, None], spp, 1)
        hi = np.repeat(tmax[:, None], spp, 1)
        assert np.all((t[hit] > lo[hit]) & (t[hit] < hi[hit]))
        assert np.all(wave["hit_gid"][hit] != np.repeat(ign[:, None], spp, 1)[hit])
        # each reported id is a valid candidate of the ray that its sample's
        # own number accepts (u < alpha), whichever accepted one the walk met
        rec = oracle.Records(sc)
        for r_, k_ in np.argwhere(hit)[:: max(1, int(hit.sum()) // 200)]:
            gid = int(wave["hit_gid"][r_, k_])
            cands = oracle.candidates(rec, o[r_], d[r_], tmin=float(tmin[r_]),
                                      tmax=float(tmax[r_]), ignore_gid=int(ign[r_]),
                                      depth_mode=mode)
            pos = np.nonzero(cands["gid"] == gid)[0]
            assert len(pos) == 1, (r_, k_, gid)
            u = oracle.accept_u(13, r_, 3 + k_, gid)
            assert u < cands["alpha"][pos[0]] + 1e-9, (r_, k_, gid, u)
    else:
        for k in ("hit_gid", "hit_t", "rgb"):
            np.testing.assert_array_equal(wave[k], lane[k], err_msg=k)
    c = srt.counters_dict(cnt)
    assert c["lost"] == 0
    assert c["ray_samples"] == int((tmax > tmin).sum()) * spp
    if lim:
        assert c["deep"] > 0
    if not any_hit and not lim and (W, L) == (4, 2):
        rays = oracle.Rays(o, d, tmin, tmax, ign, sample_base=np.full(R, 3, np.uint32))
        ora = oracle.trace(oracle.Records(sc), rays, spp=spp, seed=13, bg=(0.2, 0.1, 0.7),
                           depth_mode=mode)
        compare_ids(wave["hit_gid"], ora["hit_gid"], ora["flags"])
        compare_rgb(wave["rgb"], ora["rgb"], ora["flags"])


def test_wave_walk_on_the_four_shell_scene(srt):
    """Camera tiles of the path-tracer scene (small variant): the wave-shared
    walk equals the lane walk. (Its per-ray node and Gaussian counts differ:
    the tile visits children in one lane's near-to-far order, so the other
    lanes' depth cuts shrink at other times.)"""
    say("wave-shared walk on the four-shell scene, 160x96, 8 spp")
    w = si.workload(3, small=True)
    cam = si.look_at((0.0, 0.0, 4.0), (0, 0, 0), 160, 96)
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(w["scene"]), 4, 2)
    res, cnts = {}, {}
    for walk in ("lane", "wave"):
        cnt = srt.new_counters()
        res[walk] = _trace(srt, bvh, o, d, seed=4, spp=8, n_per_traversal=4,
                           image_width=cam.width, walk=walk, counters=cnt)
        cnts[walk] = srt.counters_dict(cnt)
    for k in ("hit_gid", "hit_t", "rgb"):
        np.testing.assert_array_equal(res["wave"][k], res["lane"][k], err_msg=k)
    say(f"counters lane {cnts['lane']} wave {cnts['wave']}")
    for k in ("traversals", "ray_samples"):
        assert cnts["wave"][k] == cnts["lane"][k]


def test_walk_option_errors(srt):
    sc = tiny_scene(24, 100)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    o = torch.zeros((16, 3), device="cuda")
    d = torch.tensor([[0.0, 0.0, 1.0]] * 16, device="cuda")
    for kw in (dict(image_width=4, persistent=True), dict(persistent=True),
               dict(image_width=4, rng="hash")):
        with pytest.raises(srt.SrtError) as e:
            srt.srt_trace_forward(bvh, o, d, walk="wave", **kw)
        assert e.value.code == 4, kw
    with pytest.raises(ValueError):
        srt.srt_trace_forward(bvh, o, d, walk="tile")
    opts = srt._opts(0, 1, 1, 0, (0, 0, 0), False, 0)
    opts.walk = 3
    import ctypes as C
    lib = srt._lib.load()
    rays = srt._lib.SrtRays(16, o.data_ptr(), d.data_ptr(), None, None, None, None, None, 0)
    ws = torch.empty(lib.srt_trace_workspace_size(bvh.handle, 16), dtype=torch.uint8,
                     device="cuda")
    assert lib.srt_trace_forward(bvh.handle, C.byref(rays), C.byref(opts), None, None, None,
                                 None, ws.data_ptr(), ws.numel(), None) == 1
