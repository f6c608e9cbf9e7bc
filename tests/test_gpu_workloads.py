"""GPU parity at the workloads' real sizes, on pixels the oracle resolves one
by one, plus the path-tracer mix (camera, shadow and mirror rays)."""
import numpy as np
import pytest
import torch

import oracle
import srt_inputs as si
from _parity import compare_ids, compare_rgb, device_scene, say, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srt():
    import paper_2504_06598_amd as srt
    assert torch.cuda.is_available()
    srt._lib.load()
    return srt


def _pick(n_total, k, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=k, replace=False))


def _pathmix_check(srt, sc, cam, spp, N, pixels, seed=0, width=4, leaf=4):
    bvh = srt.srt_build_bvh(device_scene(sc), width, leaf)
    cnt = srt.new_counters()
    res = srt.srt_trace_pathmix(bvh, cam, seed=seed, spp=spp, n_per_traversal=N,
                                light=si.LIGHT_POS, plane_y=si.PLANE_Y,
                                tmin_secondary=si.SECONDARY_TMIN, counters=cnt)
    torch.cuda.synchronize()
    g = {k: to_np(v) for k, v in res.items()}
    o, d = si.camera_rays(cam)
    ora = oracle.pathmix(oracle.Records(sc), o[pixels], d[pixels], ray_id=pixels, spp=spp,
                         seed=seed, light=si.LIGHT_POS, plane_y=si.PLANE_Y)
    fl = ora["flags"]
    compare_ids(g["cam_gid"][pixels], ora["cam_gid"], fl, max_flag_frac=5e-3, what="camera")
    compare_ids(g["shadow_vis"][pixels], ora["shadow_vis"], fl, max_flag_frac=5e-3,
                what="shadow visibility")
    compare_ids(g["mirror_gid"][pixels], ora["mirror_gid"], fl, max_flag_frac=5e-3,
                what="mirror")
    compare_rgb(g["rgb"][pixels], ora["rgb"], fl)
    c = srt.counters_dict(cnt)
    n_sec = int((g["shadow_vis"] != 255).sum() + (g["mirror_gid"] != -2).sum())
    assert c["ray_samples"] == g["cam_gid"].size + n_sec
    return g, ora, c


def test_pathmix_small(srt):
    say("path-tracer mix: 40k Gaussians on four shells, 96x54, 4 spp, N=4")
    w = si.workload(3, small=True)
    cam = w["cameras"][0]
    R = cam.width * cam.height
    g, ora, c = _pathmix_check(srt, w["scene"], cam, 4, 4, np.arange(R))
    assert (ora["mirror_gid"] >= -1).any() and (ora["shadow_vis"] == 0).any()
    assert (ora["cam_gid"] >= 0).mean() > 0.2


@pytest.mark.parametrize("width,leaf", [(2, 2), (8, 4), (4, 8)])
def test_pathmix_widths_and_leaf_sizes(srt, width, leaf):
    """The shadow-group queue at each width: width 4 queues up to 7 records
    per lane and step, so leaves of 8 are taken in two parts; widths 2 and 8
    queue up to 4 over their own stack depths."""
    say(f"path-tracer mix: 40k Gaussians, 96x54, 4 spp, N=4, width {width}, leaf {leaf}")
    w = si.workload(3, small=True)
    cam = w["cameras"][0]
    R = cam.width * cam.height
    g, ora, c = _pathmix_check(srt, w["scene"], cam, 4, 4, np.arange(R), seed=7, width=width,
                               leaf=leaf)
    assert (ora["shadow_vis"] == 0).any() and c["lost"] == 0


def test_object_scene_full_size_sampled(srt):
    say("object-like scene: 200k Gaussians, 800x800, 4 spp, N=4 (400 sampled pixels)")
    w = si.workload(2)
    sc, cam = w["scene"], w["cameras"][0]
    o, d = si.camera_rays(cam)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    res = srt.srt_trace_forward(bvh, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(),
                                seed=0, spp=4, n_per_traversal=4)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    allpx = np.arange(len(o))
    central = allpx[((allpx % 800 - 400) ** 2 + (allpx // 800 - 400) ** 2) < 250 ** 2]
    px = np.unique(np.concatenate([rng.choice(len(o), 200, replace=False),
                                   rng.choice(central, 200, replace=False)]))
    ora = oracle.trace(oracle.Records(sc), oracle.Rays(o[px], d[px], ray_id=px), spp=4, seed=0)
    g_gid = to_np(res["hit_gid"])[px]
    compare_ids(g_gid, ora["hit_gid"], ora["flags"], max_flag_frac=5e-3)
    compare_rgb(to_np(res["rgb"])[px], ora["rgb"], ora["flags"])
    assert (ora["hit_gid"] >= 0).sum() > 300


def test_path_tracer_full_size_sampled(srt):
    say("path-tracer mix: 1M Gaussians, 1920x1080, 16 spp, N=4 (48 sampled pixels)")
    w = si.workload(3)
    cam = w["cameras"][0]
    R = cam.width * cam.height
    # pixels on the shells, on the plane and in the background
    rows = np.array([100, 300, 540, 700, 900, 1050])
    cols = np.array([200, 600, 900, 960, 1100, 1500, 1700, 1900])
    px = (rows[:, None] * cam.width + cols[None, :]).ravel()
    g, ora, c = _pathmix_check(srt, w["scene"], cam, 16, 4, px)
    assert c["ray_samples"] > R * 16


@pytest.mark.parametrize("spp,N", [(80, 8), (64, 8), (12, 4), (5, 1)])
def test_pathmix_many_samples_per_pixel(srt, spp, N):
    """Shadow rays of a pixel are resolved per group of identical rays: with
    spp dividing 64 (groups found by lane shuffles), with other spp up to 64
    (one thread per pixel), and per sample above 64."""
    say(f"path-tracer mix: {spp} spp, N={N}, 24x14")
    w = si.workload(3, small=True)
    cam = si.look_at((0, 0, 4), (0, 0, 0), 24, 14)
    _pathmix_check(srt, w["scene"], cam, spp, N, np.arange(24 * 14))


@pytest.mark.parametrize("limit", [1, 3])
def test_pathmix_deep_stack_is_exact(srt, limit):
    """A shadow-ray group whose stack overflows reruns each of its samples in
    the deep pass (limit 3: some groups finish on chip, others overflow)."""
    say(f"path-tracer mix through the deep-stack pass (stack limit {limit})")
    w = si.workload(3, small=True)
    cam = si.look_at((0.3, -0.2, 4), (0, 0, 0), 48, 27)
    bvh = srt.srt_build_bvh(device_scene(w["scene"]), 4, 2)
    out = []
    for lim in (0, limit):
        cnt = srt.new_counters()
        res = srt.srt_trace_pathmix(bvh, cam, seed=3, spp=8, n_per_traversal=4, sample_offset=5,
                                    light=si.LIGHT_POS, plane_y=si.PLANE_Y,
                                    tmin_secondary=si.SECONDARY_TMIN, stack_limit=lim,
                                    counters=cnt)
        torch.cuda.synchronize()
        out.append(({k: to_np(v) for k, v in res.items()}, srt.counters_dict(cnt)))
    (a, ca), (b, cb) = out
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    assert cb["deep"] > 0 and cb["lost"] == 0 and ca["deep"] == 0


def test_pathmix_stages_run_alone_equal_the_whole_mix(srt):
    """The mix's stages (camera, shadow, mirror, compose) run as separate
    calls on one workspace give the whole mix's outputs bit for bit."""
    say("path-tracer mix stage by stage")
    w = si.workload(3, small=True)
    cam = si.look_at((0.2, -0.1, 4), (0, 0, 0), 40, 24)
    bvh = srt.srt_build_bvh(device_scene(w["scene"]), 4, 2)
    kw = dict(seed=6, spp=16, n_per_traversal=8, light=si.LIGHT_POS, plane_y=si.PLANE_Y,
              tmin_secondary=si.SECONDARY_TMIN)
    whole = srt.srt_trace_pathmix(bvh, cam, **kw)
    import ctypes as C
    lib = srt._lib.load()
    ws = torch.empty(lib.srt_pathmix_workspace_size(bvh.handle, C.byref(srt._camera(cam)), 16),
                     dtype=torch.uint8, device="cuda")
    R = cam.width * cam.height
    out = dict(rgb=torch.full((R, 3), -1.0, device="cuda"),
               cam_gid=torch.full((R, 16), -9, dtype=torch.int32, device="cuda"),
               cam_t=torch.zeros((R, 16), device="cuda"),
               shadow_vis=torch.zeros((R, 16), dtype=torch.uint8, device="cuda"),
               mirror_gid=torch.full((R, 16), -9, dtype=torch.int32, device="cuda"))
    for st in (srt.PATHMIX_CAMERA, srt.PATHMIX_SHADOW, srt.PATHMIX_MIRROR, srt.PATHMIX_COMPOSE):
        srt.srt_trace_pathmix(bvh, cam, out=out, workspace=ws, stages=st, **kw)
    torch.cuda.synchronize()
    for k in whole:
        np.testing.assert_array_equal(to_np(out[k]), to_np(whole[k]), err_msg=k)
    with pytest.raises(srt.SrtError) as e:
        srt.srt_trace_pathmix(bvh, cam, out=out, workspace=ws, stages=16, **kw)
    assert e.value.code == 1
