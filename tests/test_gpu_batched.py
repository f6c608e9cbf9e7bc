"""The batched forward (plain and persistent work-stealing kernels, graph
launched) against srt_trace_forward on the same rays and against the oracle."""
import json

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


@pytest.fixture(scope="module")
def setup(srt):
    w = si.workload(5, small=True)
    sc = w["scene"]
    # one view whose size is not a multiple of the 8x8 tile
    cams = w["cameras"][:6] + [si.look_at((0.5, 2.5, 1.5), (0, 0, 0), 37, 29)]
    spp = w["spp"][:6] + [3]
    eo, ed = w["incoherent"]
    eo, ed = eo[:20000], ed[:20000]
    dsc = device_scene(sc)
    bvh = srt.srt_build_bvh(dsc, 4, 4)
    return dict(sc=sc, cams=cams, spp=spp, eo=eo, ed=ed, dsc=dsc, bvh=bvh,
                eoc=torch.from_numpy(eo).cuda(), edc=torch.from_numpy(ed).cuda())


def _plan(srt, s, bvh=None, **kw):
    return srt.srt_batch_plan_create(bvh or s["bvh"], s["cams"], s["spp"],
                                     extra_origins=s["eoc"], extra_dirs=s["edc"], extra_spp=2,
                                     seed=21, n_per_traversal=4, **kw)


def _run(plan, eager=False):
    hits = torch.empty(plan.samples, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(8, dtype=torch.int64, device="cuda")
    rgb = plan.execute(hit_gid=hits, counters=cnt, eager=eager)
    torch.cuda.synchronize()
    return to_np(rgb), to_np(hits), to_np(cnt)


def _reference(srt, s):
    """Per-row results through srt_trace_forward on explicit rays."""
    rgbs, hits = [], []
    row = 0
    for cam, spp in zip(s["cams"], s["spp"]):
        o, d = srt.srt_camera_rays(cam)
        R = o.shape[0]
        rid = torch.arange(row, row + R, dtype=torch.int64, device="cuda").to(torch.int32)
        r = srt.srt_trace_forward(s["bvh"], o, d, ray_ids=rid, seed=21, spp=spp,
                                  n_per_traversal=4)
        rgbs.append(to_np(r["rgb"]))
        hits.append(to_np(r["hit_gid"]).reshape(-1))
        row += R
    R = s["eoc"].shape[0]
    rid = torch.arange(row, row + R, dtype=torch.int64, device="cuda").to(torch.int32)
    r = srt.srt_trace_forward(s["bvh"], s["eoc"], s["edc"], ray_ids=rid, purpose=4, seed=21,
                              spp=2, n_per_traversal=4)
    rgbs.append(to_np(r["rgb"]))
    hits.append(to_np(r["hit_gid"]).reshape(-1))
    torch.cuda.synchronize()
    return np.concatenate(rgbs), np.concatenate(hits)


@pytest.mark.parametrize("walk", ["wave", "lane"])
def test_plain_and_persistent_match_trace_forward(srt, setup, walk):
    s = setup
    say(f"batched: plain vs persistent vs srt_trace_forward, {walk} walks for the views")
    ref_rgb, ref_hits = _reference(srt, s)
    for persistent, thr, wpc in [(False, 16, 8), (True, 16, 8), (True, 1, 2), (True, 64, 16),
                                 (True, 40, 5)]:
        say(f"  persistent={persistent} threshold={thr} waves/CU={wpc}")
        plan = _plan(srt, s, persistent=persistent, refill_threshold=thr, waves_per_cu=wpc,
                     walk=walk)
        rgb, hits, cnt = _run(plan)
        assert np.array_equal(hits, ref_hits)
        np.testing.assert_allclose(rgb, ref_rgb, atol=2e-6, rtol=1e-5)
        assert cnt[6] == plan.samples and cnt[7] == 0
        del plan


def test_batched_matches_oracle_on_sampled_rows(srt, setup):
    s = setup
    say("batched vs oracle on 300 sampled rows")
    plan = _plan(srt, s, persistent=True)
    rgb, hits, _ = _run(plan)
    rows_o, rows_d, rid, spp_of, first = [], [], [], [], []
    row = 0
    sample = 0
    for cam, spp in zip(s["cams"], s["spp"]):
        o, d = si.camera_rays(cam)
        rows_o.append(o); rows_d.append(d)
        rid.append(np.arange(row, row + len(o))); spp_of.append(np.full(len(o), spp))
        first.append(sample + np.arange(len(o)) * spp)
        row += len(o); sample += len(o) * spp
    rows_o.append(s["eo"]); rows_d.append(s["ed"])
    rid.append(np.arange(row, row + len(s["eo"]))); spp_of.append(np.full(len(s["eo"]), 2))
    first.append(sample + np.arange(len(s["eo"])) * 2)
    O, D, RID = np.concatenate(rows_o), np.concatenate(rows_d), np.concatenate(rid)
    SPP, FIRST = np.concatenate(spp_of), np.concatenate(first)
    rng = np.random.default_rng(4)
    rec = oracle.Records(s["sc"])
    n_cam = row
    for lo, hi, purpose in [(0, n_cam, 0), (n_cam, len(O), 4)]:
        pick = np.sort(rng.choice(np.arange(lo, hi), 150, replace=False))
        for spp in np.unique(SPP[pick]):
            sel = pick[SPP[pick] == spp]
            ora = oracle.trace(rec, oracle.Rays(O[sel], D[sel], ray_id=RID[sel]), spp=int(spp),
                               seed=21, purpose=purpose)
            g = np.stack([hits[FIRST[i]:FIRST[i] + spp] for i in sel])
            compare_ids(g, ora["hit_gid"], ora["flags"], max_flag_frac=0.01)
            compare_rgb(rgb[sel], ora["rgb"], ora["flags"])


def test_graph_replays_equal_eager(srt, setup):
    s = setup
    say("graph replays vs eager, with eager work in between")
    plan = _plan(srt, s, persistent=True)
    e_rgb, e_hits, _ = _run(plan, eager=True)
    rgb_buf = torch.empty((plan.rows, 3), device="cuda")
    hit_buf = torch.empty(plan.samples, dtype=torch.int32, device="cuda")
    for rep in range(4):
        rgb_buf.fill_(123.0)
        hit_buf.fill_(-7)
        plan.execute(rgb=rgb_buf, hit_gid=hit_buf)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(hit_buf), e_hits), rep
        np.testing.assert_allclose(to_np(rgb_buf), e_rgb, atol=2e-6, rtol=1e-5)
        # unrelated eager work between replays
        _ = srt.srt_trace_forward(s["bvh"], s["eoc"], s["edc"], spp=1)
        torch.cuda.synchronize()


def test_graph_recaptured_for_new_output_pointers(srt, setup):
    """A call with other output pointers re-captures the plan's graph: every
    buffer it is given, in turn and back again, receives the eager result,
    and the buffers it is no longer given stay untouched."""
    s = setup
    say("graph re-capture when the output pointers change")
    plan = _plan(srt, s, persistent=True)
    e_rgb, e_hits, _ = _run(plan, eager=True)
    bufs = [(torch.empty((plan.rows, 3), device="cuda"),
             torch.empty(plan.samples, dtype=torch.int32, device="cuda")) for _ in range(3)]
    cnt = srt.new_counters()
    for i in (0, 1, 2, 1, 0):
        for r, h in bufs:
            r.fill_(55.0)
            h.fill_(-9)
        rgb, hit = bufs[i]
        # the counters pointer alternates too (None, then a buffer)
        plan.execute(rgb=rgb, hit_gid=hit, counters=cnt if i % 2 else None)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(hit), e_hits), i
        np.testing.assert_allclose(to_np(rgb), e_rgb, atol=2e-6, rtol=1e-5)
        for j, (r, h) in enumerate(bufs):
            if j != i:
                assert (to_np(h) == -9).all() and (to_np(r) == 55.0).all(), (i, j)
    c = srt.counters_dict(cnt)
    assert c["ray_samples"] == 2 * plan.samples and c["lost"] == 0


def test_deep_stack_and_widths(srt, setup):
    s = setup
    say("batched deep-stack fallback and BVH widths")
    base = _plan(srt, s, persistent=True)
    _, ref_hits, _ = _run(base)
    for lim in (1, 3):
        for persistent in (False, True):
            for walk in ("wave", "lane"):
                plan = _plan(srt, s, persistent=persistent, stack_limit=lim, walk=walk)
                _, hits, cnt = _run(plan)
                assert np.array_equal(hits, ref_hits)
                assert cnt[5] > 0 and cnt[7] == 0
                assert cnt[6] == plan.samples  # rerun rays and items are counted once
    for W, L in [(2, 1), (8, 8), (8, 2)]:
        bvh = srt.srt_build_bvh(s["dsc"], W, L)
        plan = _plan(srt, s, bvh=bvh, persistent=True)
        _, hits, cnt = _run(plan)
        assert np.array_equal(hits, ref_hits), (W, L)
    # the lane kernel's stacks with 1 or 2 entries per lane in LDS: every
    # deeper entry goes to the lanes' global-memory part, none to the deep pass
    for lds in (1, 2):
        for walk in ("wave", "lane"):
            plan = _plan(srt, s, persistent=True, walk=walk, lds_stack=lds)
            _, hits, cnt = _run(plan)
            assert np.array_equal(hits, ref_hits), (lds, walk)
            assert cnt[5] == 0 and cnt[7] == 0 and cnt[6] == plan.samples
    for bad in (-1, 25):
        with pytest.raises(srt.SrtError) as e:
            _plan(srt, s, persistent=True, lds_stack=bad)
        assert e.value.code == 1
    for n in (3, 32):
        with pytest.raises(srt.SrtError) as e:
            srt.srt_batch_plan_create(s["bvh"], s["cams"], s["spp"], n_per_traversal=n)
        assert e.value.code == 1


def test_autotuner_guards_and_picks(srt, setup, tmp_path):
    from paper_2504_06598_amd.autotune import autotune
    s = setup
    say("autotuner on the small batched workload")
    res = autotune(s["dsc"], s["cams"][:3], s["spp"][:3], extra_origins=s["eoc"][:5000],
                   extra_dirs=s["edc"][:5000], extra_spp=2, seed=21, widths=(2, 4),
                   leaves=(1, 4), thresholds=(16, 48), waves=(4, 8), reps=1,
                   cache_path=str(tmp_path / "tune.json"))
    assert res["rejected"] == 0
    assert res["persistent"] is not None and res["plain"] is not None
    assert len(res["table"]) == 2 * 2 * (1 + 2 * 2)
    again = autotune(s["dsc"], s["cams"][:3], s["spp"][:3], extra_origins=s["eoc"][:5000],
                     extra_dirs=s["edc"][:5000], extra_spp=2, seed=21, widths=(2, 4),
                     leaves=(1, 4), thresholds=(16, 48), waves=(4, 8), reps=1,
                     cache_path=str(tmp_path / "tune.json"))
    assert again == json.loads(json.dumps(res))


@pytest.mark.parametrize("N,mode", [(2, 1), (8, 0), (1, 0)])
def test_wave_and_lane_walks_agree(srt, setup, N, mode):
    """The views' tiles on wave-shared walks (plain: one wave per tile;
    persistent: (tile, pass) groups after the extra rays) give the same hit
    ids as lane walks, for other N and the centre depth mode, and colours up
    to the order of the FP32 sums."""
    s = setup
    say(f"batched wave vs lane walks, N={N}, depth mode {mode}")
    out = {}
    for persistent in (False, True):
        for walk in ("lane", "wave"):
            plan = srt.srt_batch_plan_create(s["bvh"], s["cams"], s["spp"],
                                             extra_origins=s["eoc"], extra_dirs=s["edc"],
                                             extra_spp=2, seed=5, n_per_traversal=N,
                                             depth_mode=mode, persistent=persistent, walk=walk)
            rgb, hits, cnt = _run(plan)
            assert cnt[6] == plan.samples and cnt[7] == 0
            out[(persistent, walk)] = (rgb, hits)
            del plan
    ref_rgb, ref_hits = out[(False, "lane")]
    for k, (rgb, hits) in out.items():
        assert np.array_equal(hits, ref_hits), k
        np.testing.assert_allclose(rgb, ref_rgb, atol=2e-6, rtol=1e-5, err_msg=str(k))


def test_sixteen_samples_per_traversal(srt, setup):
    """N = 16 (views on wave-shared walks take passes of 16 samples, lane
    walks passes of 8): the same hit ids as N = 4, with extra rays of 20
    samples (three lane passes of 8, 8 and 4), views whose spp are not
    multiples of 16, and the deep-stack pass (stack limit 1) for both
    pass sizes."""
    s = setup
    say("batched N=16 vs N=4")
    kw = dict(extra_origins=s["eoc"][:5000], extra_dirs=s["edc"][:5000], extra_spp=20, seed=8)
    ref = srt.srt_batch_plan_create(s["bvh"], s["cams"], s["spp"], n_per_traversal=4,
                                    persistent=False, walk="lane", **kw)
    ref_rgb, ref_hits, _ = _run(ref)
    del ref
    for persistent in (False, True):
        for walk in ("wave", "lane"):
            for lim in (0, 1):
                plan = srt.srt_batch_plan_create(s["bvh"], s["cams"], s["spp"],
                                                 n_per_traversal=16, persistent=persistent,
                                                 walk=walk, stack_limit=lim, **kw)
                rgb, hits, cnt = _run(plan)
                key = (persistent, walk, lim)
                assert cnt[6] == plan.samples and cnt[7] == 0, key
                if lim:
                    assert cnt[5] > 0, key
                assert np.array_equal(hits, ref_hits), key
                np.testing.assert_allclose(rgb, ref_rgb, atol=2e-6, rtol=1e-5, err_msg=str(key))
                del plan

