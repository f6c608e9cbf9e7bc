"""Benchmark of the stochastic Gaussian ray tracer on one MI355X.

A step is one pass of the hot path over one batch of synthetic input:
  1. canonical records + BVH build of a 1M-Gaussian scene (four shells),
  2. forward: the path-tracer mix at 1920x1080, 16 spp, N = 8 samples per
     traversal (two passes per pixel): camera rays, one any-hit shadow ray per
     shading point and a mirror ray per ground-plane point;
  3. forward + backward of an L2 loss on 8 views of 800x800 at 4 spp on a
     ring of radius 3 against targets rendered (once, before timing) from the
     scene with perturbed means and opacity logits.
The metric counts ray-samples resolved per second (forward camera samples and
secondary rays, plus backward ray-samples whose gradient is accumulated),
from the library's own device counters.

Beside the step, the batched workload (3.3M Gaussians; 64 views of 512x512
with samples per pixel drawn per view from {1,...,64}; 4M incoherent rays)
runs as one graph launch with the persistent work-stealing kernel and with
the plain one-lane-per-ray kernel, each at the configuration the autotuner
picks on a subsample, and both Mrays/s are reported.

After the timed region the dominant kernel (the camera-ray traversal of the
same workload) is launched alone, timed with HIP events on its stream, and
its algorithmic bytes per launch (node, record, SH and ray traffic counted
by the kernel) give the roofline figure. The CPU baseline is the FP64
oracle on a bounded pixel sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mrays/s fwd+bwd at 1M Gaussians, 1 GPU; fraction of HBM roofline; persistent vs plain"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--width", type=int, default=4)
    p.add_argument("--leaf", type=int, default=2)
    p.add_argument("--n-per-traversal", type=int, default=8)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--overlap", action=argparse.BooleanOptionalAction, default=True,
                   help="run the ring views' forward + backward on a second stream")
    p.add_argument("--cpu-pixels", type=int, default=192)
    p.add_argument("--roofline-launches", type=int, default=5)
    p.add_argument("--no-batched", action="store_true",
                   help="skip the persistent-vs-plain measurement on the batched workload")
    p.add_argument("--batched-reps", type=int, default=3)
    p.add_argument("--profile-kernel", action="store_true",
                   help="only launch the dominant kernel (camera-ray traversal) 3 times and "
                        "a 256 MiB elementwise copy (for calibrating HBM counters), then exit")
    return p.parse_args()


def node_bytes(W):
    return 32 * W


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is "
                          "described in DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2504_06598_amd as srt
    import srt_inputs as si

    torch.cuda.set_device(0)
    dev = "cuda:0"
    w = si.workload(3)
    sc_host, cam = w["scene"], w["cameras"][0]
    spp, N = w["spp"][0], args.n_per_traversal
    scene = srt.DeviceScene.from_host(sc_host, dev)
    R = cam.width * cam.height
    stream = torch.cuda.current_stream()
    print(f"# workload: {sc_host.num_gaussians} Gaussians, {cam.width}x{cam.height}, "
          f"{spp} spp, N={N}, W={args.width}, L={args.leaf}", file=sys.stderr, flush=True)

    if args.profile_kernel:
        profile_kernel(args, srt, si, torch, scene, cam, spp, N, dev)
        return

    # persistent buffers, allocated once (the step itself allocates nothing
    # beyond the BVH handle it builds)
    out = dict(rgb=torch.empty((R, 3), device=dev))
    probe = srt.srt_build_bvh(scene, args.width, args.leaf)
    import ctypes as C
    need = srt._lib.load().srt_pathmix_workspace_size(probe.handle, C.byref(srt._camera(cam)),
                                                      spp)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    del probe
    counters = srt.new_counters(dev)

    # differentiation recipe: 8 ring views, 4 spp, L2 loss against a perturbed-scene target
    views = si.ring_cameras(8, 3.0, 800, 800)
    vo, vd = zip(*[srt.srt_camera_rays(v, dev) for v in views])
    vo, vd = torch.cat(vo).contiguous(), torch.cat(vd).contiguous()
    Rb = vo.shape[0]
    bspp = 4
    tgt_host = si.perturbed(sc_host, 104)
    tgt_bvh = srt.srt_build_bvh(srt.DeviceScene.from_host(tgt_host, dev), args.width, args.leaf)
    target = srt.srt_trace_forward(tgt_bvh, vo, vd, seed=77, spp=64, n_per_traversal=8,
                                   want_hits=False)["rgb"]
    torch.cuda.synchronize()
    del tgt_bvh
    bout = dict(rgb=torch.empty((Rb, 3), device=dev),
                hit_gid=torch.empty((Rb, bspp), dtype=torch.int32, device=dev),
                hit_t=torch.empty((Rb, bspp), device=dev))
    grads = {k: torch.zeros_like(getattr(scene, k)) for k in
             ("means", "log_scales", "quats", "opacity_logits", "sh")}
    fws = None
    bws = None
    bw_counters = srt.new_counters(dev)

    # the path-tracer mix and the ring views' forward + backward only share the
    # (read-only) BVH: with --overlap they run on two streams of default
    # priority, so each one's tail of long walks overlaps the other's work
    side = torch.cuda.Stream(device=dev) if args.overlap else None

    def step(k, cnt, bcnt):
        nonlocal fws, bws
        main = torch.cuda.current_stream()
        bvh = srt.srt_build_bvh(scene, args.width, args.leaf)  # synchronises
        if fws is None:
            L = srt._lib.load()
            fws = torch.empty(L.srt_trace_workspace_size(bvh.handle, Rb), dtype=torch.uint8,
                              device=dev)
            bws = torch.empty(L.srt_backward_workspace_size(bvh.handle, Rb), dtype=torch.uint8,
                              device=dev)
        if side is not None:
            side.wait_stream(main)
        with torch.cuda.stream(side if side is not None else main):
            srt.srt_trace_forward(bvh, vo, vd, seed=si.PHILOX_SEED, spp=bspp,
                                  n_per_traversal=bspp, sample_offset=k * bspp,
                                  image_width=views[0].width, counters=cnt, out=bout,
                                  workspace=fws)
            grad_rgb = (bout["rgb"] - target) * (2.0 / Rb)
            for g in grads.values():
                g.zero_()
            srt.srt_trace_backward(bvh, vo, vd, grad_rgb, hit_gid=bout["hit_gid"],
                                   hit_t=bout["hit_t"], seed=si.PHILOX_SEED, spp=bspp,
                                   n_per_traversal=bspp, sample_offset=k * bspp,
                                   image_width=views[0].width, grads=grads, counters=bcnt,
                                   workspace=bws)
        srt.srt_trace_pathmix(bvh, cam, seed=si.PHILOX_SEED, spp=spp, n_per_traversal=N,
                              sample_offset=k * spp, light=si.LIGHT_POS, plane_y=si.PLANE_Y,
                              tmin_secondary=si.SECONDARY_TMIN, want_hits=False,
                              counters=cnt, workspace=ws, out=out)
        if side is not None:
            main.wait_stream(side)
        return bvh

    for k in range(args.warmup):
        step(k, None, None)
        print(f"# warmup step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    keep = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        keep.append(step(args.warmup + k, None, None))
        if len(keep) > 1:
            keep.pop(0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    keep.clear()
    # the same steps again with the library's counters (deterministic: same
    # seeds and sample offsets), to count the ray-samples the timed steps did
    counters.zero_()
    bw_counters.zero_()
    for k in range(args.steps):
        keep.append(step(args.warmup + k, counters, bw_counters))
        if len(keep) > 1:
            keep.pop(0)
    torch.cuda.synchronize()
    keep.clear()
    c = srt.counters_dict(counters)
    cb = srt.counters_dict(bw_counters)
    ms = (t1 - t0) * 1000.0 / args.steps
    fwd_rs = c["ray_samples"] / args.steps
    bwd_rs = cb["ray_samples"] / args.steps
    ray_samples = fwd_rs + bwd_rs
    value = ray_samples / (ms * 1e-3) / 1e6
    print(f"# timed {args.steps} steps: {ms:.2f} ms/step, {fwd_rs / 1e6:.1f} M forward + "
          f"{bwd_rs / 1e6:.1f} M backward ray-samples per step", file=sys.stderr, flush=True)
    assert c["lost"] == 0 and cb["lost"] == 0

    # ---- roofline of the dominant kernel: the camera-ray traversal ----
    bvh = srt.srt_build_bvh(scene, args.width, args.leaf)
    o, d = srt.srt_camera_rays(cam, dev)
    rc = srt.new_counters(dev)
    trace_out = dict(rgb=torch.empty((R, 3), device=dev))
    tws = torch.empty(srt._lib.load().srt_trace_workspace_size(bvh.handle, R),
                      dtype=torch.uint8, device=dev)

    def cam_trace(cnt):
        srt.srt_trace_forward(bvh, o, d, seed=si.PHILOX_SEED, spp=spp, n_per_traversal=N,
                              image_width=cam.width, want_hits=False, counters=cnt,
                              out=trace_out, workspace=tws)

    cam_trace(rc)
    torch.cuda.synchronize()
    kc = srt.counters_dict(rc)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.roofline_launches)]
    for i in range(args.roofline_launches):
        ev[2 * i].record(stream)
        cam_trace(None)
        ev[2 * i + 1].record(stream)
    torch.cuda.synchronize()
    launch_ms = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.roofline_launches)]
    avg_ms = sum(launch_ms) / len(launch_ms)
    sh_bytes = 3 * 4 * (sc_host.sh_degree + 1) ** 2
    # hits shaded: at most one SH gather per sample; counted as every sample
    bytes_per_launch = (kc["nodes"] * node_bytes(args.width) + kc["prims"] * 64 +
                        kc["ray_samples"] * sh_bytes + R * (24 + 12))
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.width, args.leaf),
            "kernel": f"k_trace_wave<W={args.width},N={N}> camera rays (wave-shared walks of image tiles)",
            "kernel_ms": round(avg_ms, 3),
            "bytes_per_launch": int(bytes_per_launch),
            "per_ray_sample": {"nodes": round(kc["nodes"] / kc["ray_samples"] * N, 2),
                               "prims": round(kc["prims"] / kc["ray_samples"] * N, 2),
                               "candidates": round(kc["candidates"] / kc["ray_samples"] * N, 2)}}
    print(f"# dominant kernel {avg_ms:.3f} ms/launch, {bytes_per_launch / 1e9:.3f} GB "
          f"algorithmic -> {achieved:.0f} GB/s", file=sys.stderr, flush=True)

    # ---- the two backward estimators on the ring views: time per launch and
    # the variance of the alpha-side gradients over fresh samples ----
    est_cmp = compare_estimators(args, srt, si, torch, bvh, vo, vd, target, bout, grads, fws,
                                 bws, bspp, stream)
    print(f"# backward estimators: {est_cmp}", file=sys.stderr, flush=True)

    # ---- BVH build vs refit at 1M (a refit replaces the build inside an
    # optimisation loop; both synchronise) ----
    def timed(fn, reps=3):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return min(ts)

    bvh_times = {"build_ms": round(timed(lambda: srt.srt_build_bvh(scene, args.width,
                                                                   args.leaf)), 3),
                 "refit_ms": round(timed(lambda: srt.srt_refit_bvh(bvh, scene)), 3)}
    print(f"# BVH at 1M: build {bvh_times['build_ms']} ms, refit {bvh_times['refit_ms']} ms",
          file=sys.stderr, flush=True)

    # ---- CPU baseline: the oracle on a bounded pixel sample ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rec = oracle.Records(sc_host)
        ho, hd = si.camera_rays(cam)
        rng = np.random.default_rng(0)
        px = np.sort(rng.choice(R, args.cpu_pixels, replace=False))
        threads = oracle.default_threads()
        tc0 = time.perf_counter()
        r = oracle.pathmix(rec, ho[px], hd[px], ray_id=px, spp=spp, seed=si.PHILOX_SEED,
                           light=si.LIGHT_POS, plane_y=si.PLANE_Y, threads=threads)
        tc1 = time.perf_counter()
        n_rs = (r["cam_gid"].size + int((r["shadow_vis"] != 255).sum()) +
                int((r["mirror_gid"] != -2).sum()))
        cpu = {"value": round(n_rs / (tc1 - tc0) / 1e6, 6), "unit": "Mrays/s",
               "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_pixels} random pixels of the same path-tracer mix at "
                         f"{spp} spp ({n_rs} ray-samples, brute force over all "
                         f"{sc_host.num_gaussians} Gaussians, {tc1 - tc0:.1f} s)"}
        print(f"# cpu oracle: {cpu['value']} Mrays/s on {threads} threads", file=sys.stderr,
              flush=True)

    # ---- persistent vs plain on the batched workload ----
    batched = None
    if not args.no_batched:
        del bvh, tws, trace_out, o, d
        del ws, out, bout, grads, fws, bws, target, vo, vd
        torch.cuda.empty_cache()
        batched = bench_batched(args, srt, si, torch, dev)

    line = {"metric": METRIC, "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "1M Gaussians on 4 shells, SH degree 3; forward: path-tracer "
                                   "mix 1920x1080, 16 spp, shadow + mirror rays; forward + "
                                   "backward: L2 loss on 8 ring views 800x800, 4 spp; step "
                                   "includes the BVH build",
                       "gaussians": sc_host.num_gaussians, "width": args.width,
                       "leaf_size": args.leaf, "n_per_traversal": N,
                       "streams": 2 if args.overlap else 1,
                       "forward_ray_samples_per_step": int(fwd_rs),
                       "backward_ray_samples_per_step": int(bwd_rs)},
            "roofline": roof, "cpu_baseline": cpu, "persistent_vs_plain": batched,
            "bvh": bvh_times, "backward_estimators": est_cmp}
    print(json.dumps(line), flush=True)


def compare_estimators(args, srt, si, torch, bvh, vo, vd, target, bout, grads, fws, bws, bspp,
                       stream, seeds=6):
    """Plain and Rao-Blackwellised backward on the same forward realisations
    (sample offsets 1000 + k*spp): best launch time of each and the summed
    variance, over the realisations, of the gradients of means, log-scales,
    quaternions and opacity logits."""
    names = ("means", "log_scales", "quats", "opacity_logits")
    Rb = vo.shape[0]
    width = int(round((Rb // 8) ** 0.5))
    res = {}
    for est in ("plain", "rb"):
        per, ms = [], []
        for k in range(seeds):
            srt.srt_trace_forward(bvh, vo, vd, seed=si.PHILOX_SEED, spp=bspp,
                                  n_per_traversal=bspp, sample_offset=1000 + k * bspp,
                                  image_width=width, out=bout, workspace=fws)
            grad_rgb = (bout["rgb"] - target) * (2.0 / Rb)
            for g in grads.values():
                g.zero_()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            srt.srt_trace_backward(bvh, vo, vd, grad_rgb, hit_gid=bout["hit_gid"],
                                   hit_t=bout["hit_t"], seed=si.PHILOX_SEED, spp=bspp,
                                   n_per_traversal=bspp, sample_offset=1000 + k * bspp,
                                   image_width=width, estimator=est, grads=grads, workspace=bws)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            per.append(torch.cat([grads[n].flatten() for n in names]).double())
        var = float(torch.stack(per).var(0).sum())
        res[est] = (min(ms), var)
        del per
    (pm, pv), (rm, rv) = res["plain"], res["rb"]
    return {"plain_ms": round(pm, 3), "rb_ms": round(rm, 3),
            "variance_ratio": round(rv / pv, 4) if pv > 0 else None,
            "variance_time_ratio": round(rv * rm / (pv * pm), 4) if pv > 0 else None,
            "realisations": seeds}


def measured_traffic(width, leaf, root=ROOT):
    """HBM bytes per launch of the camera-ray kernel, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs recorded under profiles/ (scaled by the same
    counters read on a copy of known size); None when the kernel's sources or
    the tree shape differ from those that were measured."""
    import hashlib
    path = os.path.join(root, "profiles", "k_trace_wave_camera_1M_pmc.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha1()
        for f in rec["sources"]:
            h.update(open(os.path.join(root, f), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    if h.hexdigest() != rec["sources_sha1"] or (width, leaf) != (rec["width"], rec["leaf_size"]):
        return None
    return int(rec["hbm_bytes_per_launch"])


def profile_kernel(args, srt, si, torch, scene, cam, spp, N, dev):
    bvh = srt.srt_build_bvh(scene, args.width, args.leaf)
    o, d = srt.srt_camera_rays(cam, dev)
    R = o.shape[0]
    out = dict(rgb=torch.empty((R, 3), device=dev))
    tws = torch.empty(srt._lib.load().srt_trace_workspace_size(bvh.handle, R),
                      dtype=torch.uint8, device=dev)
    for i in range(3):
        srt.srt_trace_forward(bvh, o, d, seed=si.PHILOX_SEED, spp=spp, n_per_traversal=N,
                              image_width=cam.width, want_hits=False, out=out, workspace=tws)
        torch.cuda.synchronize()
        print(f"# dominant kernel launch {i} done", file=sys.stderr, flush=True)
    x = torch.ones(64 << 20, device=dev)  # 256 MiB read, 256 MiB written
    y = torch.empty_like(x)
    for _ in range(3):
        torch.add(x, 0.0, out=y)
    torch.cuda.synchronize()
    print("# calibration copy: 268435456 bytes read and written per launch", file=sys.stderr,
          flush=True)


def bench_batched(args, srt, si, torch, dev):
    """Persistent vs plain on the batched scene. The full workload (64 views of
    512x512 and 4M incoherent rays) takes tens of seconds per launch (every
    ray crosses thousands of overlapping large Gaussians), so the bench runs
    the same scene and views at 1/16 of the pixels (128x128, the same spp per
    view) with 1/16 of the incoherent rays; the autotuner picks its
    configuration on 8 of those views and 1/8 of those rays."""
    from paper_2504_06598_amd.autotune import autotune
    t0 = time.perf_counter()
    w = si.workload(5)
    sc = srt.DeviceScene.from_host(w["scene"], dev)
    cams = si.fibonacci_cameras(len(w["cameras"]), 3.0, 128, 128)
    spp = w["spp"]
    n_inc = w["incoherent"][0].shape[0] // 16
    eo, ed = (torch.from_numpy(x[:n_inc]).to(dev) for x in w["incoherent"])
    print(f"# batched workload: {sc.num_gaussians} Gaussians, {len(cams)} views 128x128, "
          f"{n_inc} incoherent rays (generated in {time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    sub = slice(0, None, 8)
    tune = autotune(sc, cams[sub], spp[sub], extra_origins=eo[: n_inc // 8],
                    extra_dirs=ed[: n_inc // 8], extra_spp=1, seed=si.PHILOX_SEED,
                    widths=(4, 8), leaves=(2, 4), splits=(0, 4), thresholds=(16, 32, 48),
                    waves=(4, 8), reps=1, use_cache=False, cache_path=None,
                    log=lambda r: print("# tune", r, file=sys.stderr, flush=True))
    print(f"# autotuner: persistent {tune['persistent']}, plain {tune['plain']}, rejected "
          f"{tune['rejected']}", file=sys.stderr, flush=True)
    res = {}
    for kind in ("plain", "persistent"):
        cfg = tune[kind]
        bvh = srt.srt_build_bvh(sc, cfg["width"], cfg["leaf_size"], cfg["size_split"])
        plan = srt.srt_batch_plan_create(bvh, cams, spp, extra_origins=eo, extra_dirs=ed,
                                         extra_spp=1, seed=si.PHILOX_SEED, n_per_traversal=4,
                                         persistent=cfg["persistent"],
                                         refill_threshold=cfg["refill_threshold"],
                                         waves_per_cu=cfg["waves_per_cu"])
        rgb = torch.empty((plan.rows, 3), device=dev)
        cnt = srt.new_counters(dev)
        plan.execute(rgb=rgb, counters=cnt)
        torch.cuda.synchronize()
        c = srt.counters_dict(cnt)
        assert c["ray_samples"] == plan.samples and c["lost"] == 0
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(args.batched_reps):
            plan.execute(rgb=rgb, counters=cnt)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.batched_reps
        res[kind] = {"mrays_per_s": round(plan.samples / (ms * 1e-3) / 1e6, 2),
                     "ms_per_launch": round(ms, 3), "width": cfg["width"],
                     "leaf_size": cfg["leaf_size"], "size_split": cfg["size_split"],
                     "refill_threshold": cfg["refill_threshold"],
                     "waves_per_cu": cfg["waves_per_cu"]}
        print(f"# batched {kind}: {ms:.2f} ms per launch, {res[kind]['mrays_per_s']} Mrays/s",
              file=sys.stderr, flush=True)
        res["ray_samples_per_launch"] = int(plan.samples)
        del plan, bvh
    res["speedup"] = round(res["persistent"]["mrays_per_s"] / res["plain"]["mrays_per_s"], 3)
    res["workload"] = ("3.3M Gaussians (3M object-like + 300k large diffuse); 64 views on a "
                       "Fibonacci sphere at 128x128 (1/16 of 512x512), spp per view from "
                       "{1,...,64}; 250k incoherent rays (1/16 of 4M); N=4; one graph launch")
    return res


if __name__ == "__main__":
    main()
