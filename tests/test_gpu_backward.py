"""GPU backward against the oracle: element-wise on the same random
realisation, and in expectation against the FP64 gradient of the exact
composite (which the CPU suite pins to finite differences)."""
import math

import numpy as np
import pytest
import torch

import oracle
import srt_inputs as si
from _parity import device_scene, say, tiny_scene, to_np

pytestmark = pytest.mark.gpu

NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def srt():
    import paper_2504_06598_amd as srt
    assert torch.cuda.is_available()
    srt._lib.load()
    return srt


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _scene():
    sc = tiny_scene(31, 800, (0.03, 0.1), deg=1)
    return sc


def _close(g, o, name, rel=2e-4):
    g = np.asarray(g, np.float64)
    scale = max(np.abs(o).max(), 1e-12)
    err = np.abs(g - o)
    tol = rel * scale + 2e-3 * np.abs(o)
    assert np.all(err <= tol), (name, float((err / scale).max()), float(scale))


@pytest.mark.parametrize("N,deg,est", [(1, 1, "plain"), (4, 1, "plain"), (4, 3, "plain"),
                                       (2, 0, "plain"), (1, 1, "rb"), (4, 3, "rb"),
                                       (8, 0, "rb")])
def test_backward_matches_oracle_same_realisation(srt, N, deg, est):
    say(f"backward vs oracle estimator, N={N}, SH degree {deg}, estimator {est}")
    sc = tiny_scene(31 + deg, 800, (0.03, 0.1), deg=deg)
    cam = si.look_at((0.1, 0.2, 3), (0, 0, 0), 40, 40)
    o, d = si.camera_rays(cam)
    spp, seed = 4, 1234
    bg = (0.1, 0.3, 0.2)
    rec = oracle.Records(sc)
    ora_f = oracle.trace(rec, oracle.Rays(o, d), spp=spp, seed=seed, bg=bg)
    rng = np.random.default_rng(7)
    dL = rng.normal(0, 1, (len(o), 3))
    dL[(ora_f["flags"] != 0).any(1)] = 0.0  # leave out rays whose realisation is ambiguous
    dsc = device_scene(sc)
    bvh = srt.srt_build_bvh(dsc, 4, 2)
    oc, dc = _cu(o), _cu(d)
    fw = srt.srt_trace_forward(bvh, oc, dc, seed=seed, spp=spp, n_per_traversal=N, bg=bg)
    dLc = _cu(dL.astype(np.float32))
    cnt = srt.new_counters()
    g = srt.srt_trace_backward(bvh, oc, dc, dLc, hit_gid=fw["hit_gid"], hit_t=fw["hit_t"],
                               seed=seed, spp=spp, n_per_traversal=N, bg=bg, counters=cnt,
                               estimator=est)
    torch.cuda.synchronize()
    ora = oracle.estimator_grad(rec, oracle.Rays(o, d), dL.astype(np.float32).astype(np.float64),
                                spp=spp, seed=seed, bg=bg, estimator=est)
    for name in NAMES:
        _close(to_np(g[name]).reshape(ora[name].shape), ora[name], name)
    c = srt.counters_dict(cnt)
    assert c["lost"] == 0 and c["candidates"] > 0
    # recomputing the forward inside the backward gives the same gradients
    g2 = srt.srt_trace_backward(bvh, oc, dc, dLc, seed=seed, spp=spp, n_per_traversal=N, bg=bg,
                                estimator=est)
    torch.cuda.synchronize()
    for name in NAMES:
        a, b = to_np(g[name]), to_np(g2[name])
        assert np.abs(a - b).max() <= 1e-5 * max(np.abs(a).max(), 1e-12), name
    # walking the rays as 8x8 tiles of the 40x40 image changes only the order
    # of the FP32 sums
    g3 = srt.srt_trace_backward(bvh, oc, dc, dLc, hit_gid=fw["hit_gid"], hit_t=fw["hit_t"],
                                seed=seed, spp=spp, n_per_traversal=N, bg=bg, image_width=40,
                                estimator=est)
    torch.cuda.synchronize()
    for name in NAMES:
        a, b = to_np(g[name]), to_np(g3[name])
        assert np.abs(a - b).max() <= 1e-5 * max(np.abs(a).max(), 1e-12), name


def test_autograd_function(srt):
    say("torch.autograd.Function: loss = sum(G * rgb)")
    sc = _scene()
    cam = si.look_at((0, 0, 3), (0, 0, 0), 24, 24)
    o, d = si.camera_rays(cam)
    params = [_cu(getattr(sc, n)).requires_grad_(True) for n in NAMES]
    Gw = _cu(np.random.default_rng(3).normal(0, 1, (len(o), 3)).astype(np.float32))
    rgb = srt.render(*params, _cu(o), _cu(d), sh_degree=sc.sh_degree, spp=4, n_per_traversal=4,
                     seed=9)
    (rgb * Gw).sum().backward()
    ora = oracle.estimator_grad(oracle.Records(sc), oracle.Rays(o, d),
                                to_np(Gw).astype(np.float64), spp=4, seed=9)
    ora_f = oracle.trace(oracle.Records(sc), oracle.Rays(o, d), spp=4, seed=9)
    assert (ora_f["flags"] == 0).all(), "pick a seed without flagged samples"
    for p, name in zip(params, NAMES):
        _close(to_np(p.grad).reshape(ora[name].shape), ora[name], name)


def test_estimator_is_unbiased_for_the_exact_gradient(srt):
    """Differentiation recipe in miniature: the tiny cube scene, L2 loss against
    the exact composite of a perturbed scene, gradient on Gaussians 0..499; the
    GPU estimator's mean over independent seeds must match the FP64 exact
    gradient within 5 standard errors, and central differences (eps 1e-3) of
    the exact loss on a few parameters."""
    say("unbiasedness: 2 views 48x48, 4 spp, 48 seeds")
    w = si.workload(4, small=True)
    sc = w["scene"]
    target_sc = w["target_scene"]
    cams = si.ring_cameras(2, 3.0, 48, 48)
    rays = [si.camera_rays(c) for c in cams]
    o = np.concatenate([r[0] for r in rays])
    d = np.concatenate([r[1] for r in rays])
    rec = oracle.Records(sc)
    L = oracle.composite(rec, oracle.Rays(o, d))["L"]
    Y = oracle.composite(oracle.Records(target_sc), oracle.Rays(o, d))["L"]
    dL = 2.0 * (L - Y)
    exact = oracle.composite_grad(rec, oracle.Rays(o, d), dL)
    dsc = device_scene(sc)
    bvh = srt.srt_build_bvh(dsc, 4, 4)
    oc, dc, dLc = _cu(o), _cu(d), _cu(dL.astype(np.float32))
    K = 48
    runs = {n: [] for n in NAMES}
    for k in range(K):
        fw = srt.srt_trace_forward(bvh, oc, dc, seed=1000 + k, spp=4, n_per_traversal=4,
                                   want_rgb=False)
        g = srt.srt_trace_backward(bvh, oc, dc, dLc, hit_gid=fw["hit_gid"], hit_t=fw["hit_t"],
                                   seed=1000 + k, spp=4, n_per_traversal=4)
        for n in NAMES:
            runs[n].append(to_np(g[n]).reshape(exact[n].shape)[:500])
    torch.cuda.synchronize()
    for n in NAMES:
        est = np.stack(runs[n]).astype(np.float64)
        m = est.mean(0)
        se = est.std(0, ddof=1) / math.sqrt(K)
        ex = exact[n][:500]
        # aggregate bias test: sum (mean - exact)^2 against its expectation
        # sum se^2 under no bias (chi-square-like, 6 standard deviations)
        S = float(((m - ex) ** 2).sum())
        E = float((se ** 2).sum())
        V = float(2 * (se ** 4).sum())
        assert S <= E + 6 * math.sqrt(V) + 1e-6 * float((ex ** 2).sum()) + 1e-18, (n, S, E, V)
        # entry-wise: rare events make single-entry standard errors unreliable,
        # so at most 1% of the entries may sit beyond 5 of them
        tol = 5 * se + 2e-3 * np.abs(ex) + 1e-6 * max(np.abs(ex).max(), 1e-12)
        bad = np.abs(m - ex) > tol
        assert bad.mean() < 1e-2, (n, int(bad.sum()), bad.size)
    # central differences (eps 1e-3) of the exact loss, on parameters whose
    # perturbation changes no ray's sorted candidate list (the exact composite
    # jumps where depths swap or a Gaussian crosses its ellipsoid boundary)
    def loss_and_lists(scene):
        r = oracle.Records(scene)
        Lx = oracle.composite(r, oracle.Rays(o, d))["L"]
        lists = [tuple(oracle.candidates(r, o[i], d[i])["gid"]) for i in range(len(o))]
        return float(((Lx - Y) ** 2).sum()), lists

    _, base_lists = loss_and_lists(sc)
    for n in ("means", "opacity_logits", "log_scales"):
        est = np.stack(runs[n]).astype(np.float64)
        mean_g = est.mean(0).reshape(-1)
        se_g = (est.std(0, ddof=1) / math.sqrt(K)).reshape(-1)
        flat = getattr(sc, n).reshape(-1)
        checked = 0
        for j in np.argsort(-np.abs(exact[n][:500].reshape(-1)))[:12]:
            orig = flat[j]
            flat[j] = np.float32(orig + 1e-3)
            lp, lists_p = loss_and_lists(sc)
            flat[j] = np.float32(orig - 1e-3)
            lm, lists_m = loss_and_lists(sc)
            flat[j] = orig
            if lists_p != base_lists or lists_m != base_lists:
                continue
            fd = (lp - lm) / (float(np.float32(orig + 1e-3)) - float(np.float32(orig - 1e-3)))
            assert abs(mean_g[j] - fd) <= 5 * se_g[j] + 0.05 * abs(fd) + 1e-6, (n, j, mean_g[j], fd)
            checked += 1
            if checked == 3:
                break
        assert checked >= 1, n


@pytest.mark.parametrize("inside,walk", [(False, "lane"), (True, "lane"), (True, "wave")])
def test_backward_center_depth_matches_oracle(srt, inside, walk):
    """Centre depth (Sec. 4.1) in the backward; inside: a camera in the middle
    of the cloud with rays starting at random tmin, so Gaussians whose centre
    depth lies past tmin are crossed before it (their boxes must still be
    re-traversed)."""
    say(f"backward with centre depth vs oracle estimator, camera inside {inside}, {walk} walks")
    sc = tiny_scene(51, 800 if not inside else 2000, (0.03, 0.1), deg=1)
    if inside:
        cam = si.look_at((0.05, -0.1, 0.0), (0.3, 0.2, -1.0), 32, 32, vfov_deg=80.0)
    else:
        cam = si.look_at((0.1, 0.2, 3), (0, 0, 0), 32, 32)
    o, d = si.camera_rays(cam)
    tmin = None
    if inside:
        tmin = np.random.default_rng(52).uniform(0.0, 1.5, len(o)).astype(np.float32)
        tmin[::3] = 0.0
    ax = tuple(float(x) for x in cam.forward)
    rec = oracle.Records(sc)
    rays = oracle.Rays(o, d, tmin)
    ora_f = oracle.trace(rec, rays, spp=4, seed=5, depth_mode=1, depth_axis=ax)
    dL = np.random.default_rng(8).normal(0, 1, (len(o), 3))
    dL[(ora_f["flags"] != 0).any(1)] = 0.0
    ora = oracle.estimator_grad(rec, rays, dL.astype(np.float32).astype(np.float64),
                                spp=4, seed=5, depth_mode=1, depth_axis=ax)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    oc, dc = _cu(o), _cu(d)
    tc = None if tmin is None else _cu(tmin)
    fw = srt.srt_trace_forward(bvh, oc, dc, seed=5, spp=4, n_per_traversal=4, depth_mode=1,
                               depth_axis=ax, tmin=tc)
    g = srt.srt_trace_backward(bvh, oc, dc, _cu(dL.astype(np.float32)), hit_gid=fw["hit_gid"],
                               hit_t=fw["hit_t"], seed=5, spp=4, n_per_traversal=4,
                               depth_mode=1, depth_axis=ax, tmin=tc, walk=walk,
                               image_width=cam.width)
    torch.cuda.synchronize()
    for name in NAMES:
        _close(to_np(g[name]).reshape(ora[name].shape), ora[name], name)


def test_rb_estimator_has_lower_variance_on_gpu(srt):
    """Both estimators on the same 24 seeds of the tiny cube scene (GPU):
    their means agree within the noise and the Rao-Blackwellised one has the
    smaller spread for the parameters that reach alpha."""
    say("RB vs plain estimator variance over 24 seeds")
    sc = _scene()
    cam = si.look_at((0, 0.2, 3), (0, 0, 0), 48, 48)
    o, d = si.camera_rays(cam)
    oc, dc = _cu(o), _cu(d)
    dsc = device_scene(sc)
    bvh = srt.srt_build_bvh(dsc, 4, 2)
    rng = np.random.default_rng(4)
    dLc = _cu(rng.normal(0, 1, (len(o), 3)).astype(np.float32))
    runs = {}
    for est in ("plain", "rb"):
        rs = []
        for seed in range(24):
            fw = srt.srt_trace_forward(bvh, oc, dc, seed=seed, spp=4, n_per_traversal=4)
            g = srt.srt_trace_backward(bvh, oc, dc, dLc, hit_gid=fw["hit_gid"],
                                       hit_t=fw["hit_t"], seed=seed, spp=4, n_per_traversal=4,
                                       estimator=est)
            rs.append({k: to_np(v).astype(np.float64) for k, v in g.items()})
        torch.cuda.synchronize()
        runs[est] = rs
    var = {}
    for est, rs in runs.items():
        var[est] = 0.0
        for name in ("means", "log_scales", "quats", "opacity_logits"):
            var[est] += float(np.stack([r[name] for r in rs]).var(0, ddof=1).sum())
    for name in ("means", "opacity_logits"):
        a = np.stack([r[name] for r in runs["plain"]])
        b = np.stack([r[name] for r in runs["rb"]])
        se = np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
        assert np.mean(np.abs(a.mean(0) - b.mean(0)) <= 4 * se + 1e-9) > 0.97, name
    say(f"variance sum: plain {var['plain']:.4e}, rb {var['rb']:.4e}")
    assert var["rb"] < 0.8 * var["plain"], var


@pytest.mark.parametrize("N,est,mode,stored,lim", [(4, "plain", 0, True, 0), (4, "rb", 0, True, 0),
                                                   (1, "plain", 1, False, 0),
                                                   (8, "rb", 0, False, 2),
                                                   (2, "plain", 0, True, 1)])
def test_wave_walk_backward_equals_lane_walk(srt, N, est, mode, stored, lim):
    """Re-traversing each 8x8 tile as one wave-shared walk reaches, per ray,
    the same candidates as the lane walk: gradients equal up to the order of
    the FP32 sums, with ragged tiles, empty rays, ignored ids, results
    recomputed in the backward (stored=False) and stacks pushed into global
    memory (lim > 0)."""
    say(f"backward wave walk vs lane walk: N={N} {est} depth mode {mode} stored={stored} "
        f"lds stack {lim or 'default'}")
    sc = tiny_scene(61, 2500, (0.02, 0.08), deg=2)
    cam = si.look_at((0.1, 0.2, 2.9), (0, 0, 0), 37, 29)
    o, d = si.camera_rays(cam)
    R = len(o)
    rng = np.random.default_rng(12)
    tmin = rng.uniform(0.0, 1.0, R).astype(np.float32)
    tmax = (tmin + rng.uniform(-0.2, 4.0, R)).astype(np.float32)
    tmax[::5] = np.inf
    ign = rng.integers(-1, 2500, R).astype(np.int32)
    dLc = _cu(rng.normal(0, 1, (R, 3)).astype(np.float32))
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 2)
    oc, dc = _cu(o), _cu(d)
    kw = dict(seed=21, spp=8, n_per_traversal=N, bg=(0.2, 0.1, 0.3), tmin=_cu(tmin),
              tmax=_cu(tmax), ignore_gid=_cu(ign), depth_mode=mode, estimator=est,
              image_width=cam.width, stack_limit=lim)
    if stored:
        fw = srt.srt_trace_forward(bvh, oc, dc, seed=21, spp=8, n_per_traversal=N,
                                   tmin=kw["tmin"], tmax=kw["tmax"], ignore_gid=kw["ignore_gid"],
                                   depth_mode=mode)
        kw.update(hit_gid=fw["hit_gid"], hit_t=fw["hit_t"])
    out, cnts = {}, {}
    for walk in ("lane", "wave"):
        cnt = srt.new_counters()
        out[walk] = srt.srt_trace_backward(bvh, oc, dc, dLc, walk=walk, counters=cnt, **kw)
        torch.cuda.synchronize()
        cnts[walk] = srt.counters_dict(cnt)
    for name in NAMES:
        a, b = to_np(out["lane"][name]), to_np(out["wave"][name])
        assert np.abs(a - b).max() <= 2e-5 * max(np.abs(a).max(), 1e-12), name
    for k in ("ray_samples", "traversals", "lost"):
        assert cnts["wave"][k] == cnts["lane"][k], (k, cnts)
    assert cnts["wave"]["lost"] == 0
    if (N, est, stored) == (4, "plain", True):
        rays = oracle.Rays(o, d, tmin, tmax, ign)
        ora_f = oracle.trace(oracle.Records(sc), rays, spp=8, seed=21, bg=kw["bg"])
        dL = to_np(dLc).astype(np.float64)
        dL[(ora_f["flags"] != 0).any(1)] = 0.0
        g = srt.srt_trace_backward(bvh, oc, dc, _cu(dL.astype(np.float32)), walk="wave", **kw)
        torch.cuda.synchronize()
        ora = oracle.estimator_grad(oracle.Records(sc), rays, dL, spp=8, seed=21, bg=kw["bg"])
        for name in NAMES:
            _close(to_np(g[name]).reshape(ora[name].shape), ora[name], name)


def test_backward_walk_option_errors(srt):
    sc = tiny_scene(62, 100)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    o = torch.zeros((16, 3), device="cuda")
    d = torch.tensor([[0.0, 0.0, 1.0]] * 16, device="cuda")
    g = torch.ones((16, 3), device="cuda")
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_backward(bvh, o, d, g, walk="wave")
    assert e.value.code == 4
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_backward(bvh, o, d, g, stack_limit=-1)
    assert e.value.code == 1
