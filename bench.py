"""Benchmark of the stochastic Gaussian ray tracer on one MI355X.

A step is one pass of the hot path over one batch of synthetic input:
  1. canonical records + BVH build of a 1M-Gaussian scene (four shells),
  2. forward: the path-tracer mix at 1920x1080, 16 spp, N = 8 samples per
     traversal (two passes per pixel): camera rays, one any-hit shadow ray per
     shading point and a mirror ray per ground-plane point,
  3. forward + backward of an L2 loss on 8 views of 800x800 at 4 spp on a
     ring of radius 3 against targets rendered (once, before timing) from the
     scene with perturbed means and opacity logits.
The metric counts ray-samples resolved per second (forward camera samples and
secondary rays, plus backward ray-samples whose gradient is accumulated),
from the library's own device counters; the forward and backward rates are
also reported on their own.

After the timed region each major kernel of the step (camera rays, shadow
rays, ring-view forward, backward) is launched alone in the step's
configuration and timed with HIP events on its stream; its algorithmic bytes
per launch (nodes, Gaussian records, SH rows and ray I/O, counted by the
kernel) over its time give the roofline figure of the one that takes longest.
Measured HBM traffic and L2 hit rates come from the rocprofv3 counter runs
summarised under profiles/ (reported while the kernel sources are unchanged).

Beside the step: the multi-sample speed-up on the object-like scene (N = 1
vs N = 4 samples per traversal), the two backward estimators, BVH build and
refit, and the batched workload (3.3M Gaussians; 64 views with samples per
pixel drawn per view from {1,...,64}; 4M incoherent rays) as one graph
launch with the persistent work-stealing kernel and with the plain one, each
at the configuration the autotuner picks on a subsample. The CPU baseline is
the FP64 oracle on a bounded sample of the same workloads.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --profile-kernels          (launches for rocprofv3)
       python bench.py --summarize-profiles DIR...  (tables from its CSVs)
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
    p.add_argument("--leaf", type=int, default=4)
    p.add_argument("--n-per-traversal", type=int, default=8)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--overlap", action=argparse.BooleanOptionalAction, default=True,
                   help="run the ring views' forward + backward on a second stream")
    p.add_argument("--cpu-pixels", type=int, default=512)
    p.add_argument("--cpu-grad-rays", type=int, default=4096)
    p.add_argument("--kernel-launches", type=int, default=5)
    p.add_argument("--no-batched", action="store_true",
                   help="skip the persistent-vs-plain measurement on the batched workload")
    p.add_argument("--batched-scale", type=int, default=1,
                   help="run the batched workload at 1/k of its pixels and incoherent rays")
    p.add_argument("--batched-reps", type=int, default=1)
    p.add_argument("--batched-only", action="store_true",
                   help="run only the persistent-vs-plain measurement and print its record")
    p.add_argument("--batched-config", metavar="W,L,THRESHOLD,WAVES,N",
                   help="skip the autotuner: both kinds at this tree (size split 4) and N "
                        "samples per traversal, the persistent one at this refill threshold "
                        "and workgroups per CU")
    p.add_argument("--no-multisample", action="store_true",
                   help="skip the N = 1 vs N = 4 comparison on the object-like scene")
    p.add_argument("--profile-kernels", action="store_true",
                   help="launch each major kernel of the step 3 times and a 256 MiB "
                        "elementwise copy (HBM counter calibration), then exit")
    p.add_argument("--summarize-profiles", nargs="+", metavar="DIR",
                   help="summarise rocprofv3 CSV output of --profile-kernels runs and exit")
    p.add_argument("--write-profile-json", metavar="PATH",
                   help="with --summarize-profiles: write the per-kernel counter record")
    return p.parse_args()


def node_bytes(W):
    return 32 * W


def ev_time(torch, fn, reps):
    """Average ms of `reps` launches of fn, HIP events on the current stream
    (the stream the library launches on)."""
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in evs) / reps


class Step:
    """The benchmark's scene, buffers and the step's library calls."""

    def __init__(self, args, srt, si, torch, dev):
        self.args, self.srt, self.si, self.torch, self.dev = args, srt, si, torch, dev
        import ctypes as C
        w = si.workload(3)
        self.sc_host, self.cam = w["scene"], w["cameras"][0]
        self.spp, self.N = w["spp"][0], args.n_per_traversal
        self.scene = srt.DeviceScene.from_host(self.sc_host, dev)
        self.R = self.cam.width * self.cam.height
        L = srt._lib.load()
        self.out = dict(rgb=torch.empty((self.R, 3), device=dev))
        probe = srt.srt_build_bvh(self.scene, args.width, args.leaf)
        self.ws = torch.empty(L.srt_pathmix_workspace_size(probe.handle,
                                                           C.byref(srt._camera(self.cam)),
                                                           self.spp),
                              dtype=torch.uint8, device=dev)
        # differentiation recipe: 8 ring views, 4 spp, L2 loss against a
        # perturbed-scene target
        self.views = si.ring_cameras(8, 3.0, 800, 800)
        vo, vd = zip(*[srt.srt_camera_rays(v, dev) for v in self.views])
        self.vo, self.vd = torch.cat(vo).contiguous(), torch.cat(vd).contiguous()
        self.Rb = self.vo.shape[0]
        self.bspp = 4
        tgt_host = si.perturbed(self.sc_host, 104)
        tgt_bvh = srt.srt_build_bvh(srt.DeviceScene.from_host(tgt_host, dev), args.width,
                                    args.leaf)
        self.target = srt.srt_trace_forward(tgt_bvh, self.vo, self.vd, seed=77, spp=64,
                                            n_per_traversal=8, want_hits=False)["rgb"]
        torch.cuda.synchronize()
        del tgt_bvh
        self.bout = dict(rgb=torch.empty((self.Rb, 3), device=dev),
                         hit_gid=torch.empty((self.Rb, self.bspp), dtype=torch.int32, device=dev),
                         hit_t=torch.empty((self.Rb, self.bspp), device=dev))
        self.grads = {k: torch.zeros_like(getattr(self.scene, k)) for k in
                      ("means", "log_scales", "quats", "opacity_logits", "sh")}
        self.fws = torch.empty(L.srt_trace_workspace_size(probe.handle, self.Rb),
                               dtype=torch.uint8, device=dev)
        self.bws = torch.empty(L.srt_backward_workspace_size(probe.handle, self.Rb),
                               dtype=torch.uint8, device=dev)
        del probe
        # the path-tracer mix and the ring views' forward + backward only share
        # the (read-only) BVH: with --overlap they run on two streams of
        # default priority, so each one's tail of long walks overlaps the
        # other's work
        self.side = torch.cuda.Stream(device=dev) if args.overlap else None

    def build(self):
        return self.srt.srt_build_bvh(self.scene, self.args.width, self.args.leaf)

    def camera_trace(self, bvh, k, cnt=None):
        """The mix's camera-ray launch on its own (the same kernel and outputs:
        per-sample ids and depths, no colour)."""
        srt, torch = self.srt, self.torch
        if not hasattr(self, "co"):
            self.co, self.cd = srt.srt_camera_rays(self.cam, self.dev)
            self.cam_out = dict(
                hit_gid=torch.empty((self.R, self.spp), dtype=torch.int32, device=self.dev),
                hit_t=torch.empty((self.R, self.spp), device=self.dev))
            self.tws = torch.empty(srt._lib.load().srt_trace_workspace_size(bvh.handle, self.R),
                                   dtype=torch.uint8, device=self.dev)
        srt.srt_trace_forward(bvh, self.co, self.cd, seed=self.si.PHILOX_SEED, spp=self.spp,
                              n_per_traversal=self.N, sample_offset=k * self.spp,
                              image_width=self.cam.width, want_rgb=False, counters=cnt,
                              out=self.cam_out, workspace=self.tws)

    def pathmix(self, bvh, k, cnt=None, stages=0):
        si = self.si
        self.srt.srt_trace_pathmix(bvh, self.cam, seed=si.PHILOX_SEED, spp=self.spp,
                                   n_per_traversal=self.N, sample_offset=k * self.spp,
                                   light=si.LIGHT_POS, plane_y=si.PLANE_Y,
                                   tmin_secondary=si.SECONDARY_TMIN, want_hits=False,
                                   counters=cnt, workspace=self.ws, out=self.out, stages=stages)

    def ring_forward(self, bvh, k, cnt=None):
        self.srt.srt_trace_forward(bvh, self.vo, self.vd, seed=self.si.PHILOX_SEED,
                                   spp=self.bspp, n_per_traversal=self.bspp,
                                   sample_offset=k * self.bspp, image_width=self.views[0].width,
                                   counters=cnt, out=self.bout, workspace=self.fws)

    def ring_backward(self, bvh, k, cnt=None, estimator="plain"):
        grad_rgb = (self.bout["rgb"] - self.target) * (2.0 / self.Rb)
        for g in self.grads.values():
            g.zero_()
        self.srt.srt_trace_backward(bvh, self.vo, self.vd, grad_rgb, hit_gid=self.bout["hit_gid"],
                                    hit_t=self.bout["hit_t"], seed=self.si.PHILOX_SEED,
                                    spp=self.bspp, n_per_traversal=self.bspp,
                                    sample_offset=k * self.bspp,
                                    image_width=self.views[0].width, grads=self.grads,
                                    counters=cnt, workspace=self.bws, estimator=estimator)

    def step(self, k, cnt=None, bcnt=None):
        torch = self.torch
        main = torch.cuda.current_stream()
        bvh = self.build()  # synchronises
        if self.side is not None:
            self.side.wait_stream(main)
        with torch.cuda.stream(self.side if self.side is not None else main):
            self.ring_forward(bvh, k, cnt)
            self.ring_backward(bvh, k, bcnt)
        self.pathmix(bvh, k, cnt)
        if self.side is not None:
            main.wait_stream(self.side)
        return bvh


def kernel_specs(st, bvh, k=0):
    """The step's major kernels as separate launches in the step's
    configuration: name -> (kernel label, setup, launch(counters), bytes(counters))."""
    W, N, spp, R = st.args.width, st.N, st.spp, st.R
    sh_row = 3 * 4 * (st.sc_host.sh_degree + 1) ** 2

    def graph_bytes(c):
        return c["nodes"] * node_bytes(W) + c["prims"] * 64

    return {
        "camera": (f"k_trace_wave<{W}, {N}> camera rays (wave-shared walks of 8x4-pixel tiles, "
                   f"two lanes per pixel)",
                   lambda: None,
                   lambda c: st.camera_trace(bvh, k, c),
                   # nodes, records; per sample its (id, depth) written; per pixel its ray
                   lambda c: graph_bytes(c) + c["ray_samples"] * 8 + R * 24),
        "shadow": ("k_shadow_queue<" + str(W) + "> shadow-ray groups (work-stealing waves, "
                   "records tested from a wave-wide queue)",
                   lambda: st.pathmix(bvh, k, None, stages=st.srt.PATHMIX_CAMERA),
                   lambda c: st.pathmix(bvh, k, c, stages=st.srt.PATHMIX_SHADOW),
                   # nodes, records; per group its entry (12 B) and ray (40 B); per
                   # sample its visibility written (4 B)
                   lambda c: graph_bytes(c) + c["traversals"] * 52 + c["ray_samples"] * 4),
        "ring_forward": (f"k_trace_wave<{W}, 4> ring views (wave-shared walks of 8x8 tiles)",
                         lambda: None,
                         lambda c: st.ring_forward(bvh, k, c),
                         # + one SH row per sample, ray 24 B and colour 12 B per pixel,
                         # (id, depth) 8 B per sample
                         lambda c: graph_bytes(c) + c["ray_samples"] * (sh_row + 8) +
                         st.Rb * 36),
        "backward": (f"k_backward<{W}, 4> ring views (wave-shared re-traversal, plain estimator)",
                     lambda: st.ring_forward(bvh, k, None),
                     lambda c: st.ring_backward(bvh, k, c),
                     # + a record and an SH row per candidate in front of a result,
                     # ray, upstream gradient and the stored (id, depth) per sample
                     lambda c: graph_bytes(c) + c["candidates"] * sh_row +
                     st.Rb * 36 + c["ray_samples"] * 8),
    }


def measure_kernels(st, bvh, launches, profiles):
    """Per kernel: average launch time (HIP events), counters and algorithmic
    bytes of one launch, and the counter record from profiles/ if current."""
    srt, torch = st.srt, st.torch
    res = {}
    for name, (label, setup, launch, nbytes) in kernel_specs(st, bvh).items():
        setup()
        cnt = srt.new_counters(st.dev)
        launch(cnt)
        torch.cuda.synchronize()
        c = srt.counters_dict(cnt)
        launch(None)
        ms = ev_time(torch, lambda: launch(None), launches)
        b = nbytes(c)
        trav = max(c["traversals"], 1)
        e = {"kernel": label, "ms": round(ms, 3), "algorithmic_bytes": int(b),
             "algorithmic_gbs": round(b / (ms * 1e-3) / 1e9, 1),
             "traversals": c["traversals"], "ray_samples": c["ray_samples"],
             "per_traversal": {"nodes": round(c["nodes"] / trav, 2),
                               "records": round(c["prims"] / trav, 2),
                               "candidates": round(c["candidates"] / trav, 2)}}
        p = (profiles or {}).get(name)
        if p:
            e["hbm_bytes"] = int(p["hbm_bytes_per_launch"])
            e["hbm_gbs"] = round(p["hbm_bytes_per_launch"] / (ms * 1e-3) / 1e9, 2)
            e["hbm_frac"] = round(e["hbm_gbs"] / HBM_PEAK_GBS, 5)
            for k in ("l2_hit_rate", "valu_insts", "salu_insts", "valu_busy", "salu_busy",
                      "valu_lanes_active"):
                if k in p:
                    e[k] = p[k]
        res[name] = e
        print(f"# kernel {name}: {ms:.3f} ms, {b / 1e9:.2f} GB algorithmic, "
              f"{e['per_traversal']}", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is "
                          "described in DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2504_06598_amd as srt
    import srt_inputs as si

    torch.cuda.set_device(0)
    dev = "cuda:0"
    if args.batched_only:
        print(json.dumps({"persistent_vs_plain": bench_batched(args, srt, si, torch, dev)}))
        return
    st = Step(args, srt, si, torch, dev)
    print(f"# workload: {st.sc_host.num_gaussians} Gaussians, {st.cam.width}x{st.cam.height}, "
          f"{st.spp} spp, N={st.N}, W={args.width}, L={args.leaf}", file=sys.stderr, flush=True)

    if args.profile_kernels:
        profile_kernels(st)
        return

    for k in range(args.warmup):
        st.step(k)
        print(f"# warmup step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    keep = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        keep.append(st.step(args.warmup + k))
        if len(keep) > 1:
            keep.pop(0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    keep.clear()
    # the same steps again with the library's counters (deterministic: same
    # seeds and sample offsets), to count the ray-samples the timed steps did
    counters = srt.new_counters(dev)
    bw_counters = srt.new_counters(dev)
    for k in range(args.steps):
        keep.append(st.step(args.warmup + k, counters, bw_counters))
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

    # ---- forward and backward on their own (one stream; same work) ----
    bvh = st.build()
    fwd_ms = ev_time(torch, lambda: (st.pathmix(bvh, 0), st.ring_forward(bvh, 0)), 3)
    bwd_ms = ev_time(torch, lambda: st.ring_backward(bvh, 0), 3)
    split = {"forward_mrays_per_s": round(fwd_rs / (fwd_ms * 1e-3) / 1e6, 2),
             "forward_ms": round(fwd_ms, 3),
             "backward_mrays_per_s": round(bwd_rs / (bwd_ms * 1e-3) / 1e6, 2),
             "backward_ms": round(bwd_ms, 3)}
    print(f"# forward alone {fwd_ms:.2f} ms, backward alone {bwd_ms:.2f} ms", file=sys.stderr,
          flush=True)

    # ---- the step's major kernels, each launched alone ----
    profiles = measured_profiles(args.width, args.leaf)
    kern = measure_kernels(st, bvh, args.kernel_launches, profiles)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    achieved = d["algorithmic_bytes"] / (d["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": d.get("hbm_bytes"),
            "kernel": d["kernel"], "kernel_ms": d["ms"],
            "achieved_is": "algorithmic bytes per launch (nodes x 32W + Gaussian records tested "
                           "x 64 + SH rows + ray I/O, from the kernel's own counters) / launch "
                           "time; not measured HBM traffic",
            "algorithmic_bytes_per_launch": d["algorithmic_bytes"],
            "per_traversal": d["per_traversal"]}
    for k in ("hbm_gbs", "hbm_frac", "l2_hit_rate", "valu_busy", "valu_lanes_active"):
        if k in d:
            roof[k] = d[k]
    print(f"# dominant kernel: {dom} ({d['ms']:.3f} ms)", file=sys.stderr, flush=True)

    # ---- the two backward estimators on the ring views ----
    est_cmp = compare_estimators(st, bvh)
    print(f"# backward estimators: {est_cmp}", file=sys.stderr, flush=True)

    # ---- BVH build vs refit at 1M ----
    def timed(fn, reps=3):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return min(ts)

    bvh_times = {"build_ms": round(timed(st.build), 3),
                 "refit_ms": round(timed(lambda: srt.srt_refit_bvh(bvh, st.scene)), 3)}
    print(f"# BVH at 1M: build {bvh_times['build_ms']} ms, refit {bvh_times['refit_ms']} ms",
          file=sys.stderr, flush=True)

    # ---- CPU baseline: the oracle on bounded samples ----
    cpu = None if args.no_cpu_baseline else cpu_baseline(args, st)

    del bvh
    st_keep = {"sh_degree": st.sc_host.sh_degree, "G": st.sc_host.num_gaussians}
    del st
    torch.cuda.empty_cache()

    # ---- N samples per traversal on the object-like scene ----
    multi = None if args.no_multisample else multisample(args, srt, si, torch, dev)

    # ---- persistent vs plain on the batched workload ----
    batched = None if args.no_batched else bench_batched(args, srt, si, torch, dev)

    line = {"metric": METRIC, "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "1M Gaussians on 4 shells, SH degree 3; forward: path-tracer "
                                   "mix 1920x1080, 16 spp, shadow + mirror rays; forward + "
                                   "backward: L2 loss on 8 ring views 800x800, 4 spp; step "
                                   "includes the BVH build",
                       "gaussians": st_keep["G"], "width": args.width,
                       "leaf_size": args.leaf, "n_per_traversal": args.n_per_traversal,
                       "streams": 2 if args.overlap else 1,
                       "precision": "FP64 candidate test (t*, q, alpha, u < alpha); FP32 "
                                    "traversal, shading and gradient accumulation",
                       "forward_ray_samples_per_step": int(fwd_rs),
                       "backward_ray_samples_per_step": int(bwd_rs)},
            "forward_backward": split, "roofline": roof, "kernels": kern,
            "cpu_baseline": cpu, "persistent_vs_plain": batched, "multisample": multi,
            "bvh": bvh_times, "backward_estimators": est_cmp, "paper_context": PAPER_CONTEXT}
    print(json.dumps(line), flush=True)


# The paper's own timings with their hardware, for context: full samples of
# its production path tracer on its assets (each sample traces the camera ray
# and its secondary rays; no rays/s, no backward), offline-timing and
# multi-sample tables and the interactive comparison.
PAPER_CONTEXT = {
    "hardware": "NVIDIA GeForce RTX 3090 (hardware ray tracing, Vulkan); AMD Ryzen 9 5950X, "
                "16 cores (Embree)",
    "unit": "M path samples/s (pixels x spp / s)",
    "room_1.59M_1200x800_1024spp": {"gpu_s": 9.43, "gpu_rate": 104.2, "cpu_s": 508.62,
                                    "cpu_rate": 1.93},
    "drjohnson_3.41M_1200x800_1024spp": {"gpu_s": 13.41, "gpu_rate": 73.3, "cpu_s": 759.40,
                                         "cpu_rate": 1.29},
    "room_1200x800_1024spp_8_per_traversal": {"gpu_s": 4.51, "gpu_rate": 218.0,
                                              "cpu_s": 103.05, "cpu_rate": 9.5},
    "room_1.28M_1557x1038_per_spp_frame": {"gpu_ms": 12.2, "gpu_rate": 132.0},
    "note": "context only: another GPU with ray-tracing units, another workload and unit",
}


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(args, st):
    """The FP64 oracle (brute force over every Gaussian, OpenMP) on a random
    pixel sample of the path-tracer mix, and its exact gradient (sorted
    composite, eqn "accumulated" differentiated) on a random ray sample of
    the ring views."""
    import numpy as np

    import oracle
    si = st.si
    rec = oracle.Records(st.sc_host)
    ho, hd = si.camera_rays(st.cam)
    rng = np.random.default_rng(0)
    px = np.sort(rng.choice(st.R, args.cpu_pixels, replace=False))
    threads = oracle.default_threads()
    tc0 = time.perf_counter()
    r = oracle.pathmix(rec, ho[px], hd[px], ray_id=px, spp=st.spp, seed=si.PHILOX_SEED,
                       light=si.LIGHT_POS, plane_y=si.PLANE_Y, threads=threads)
    tc1 = time.perf_counter()
    n_rs = (r["cam_gid"].size + int((r["shadow_vis"] != 255).sum()) +
            int((r["mirror_gid"] != -2).sum()))
    vo = st.vo.cpu().numpy()
    vd = st.vd.cpu().numpy()
    gi = np.sort(rng.choice(len(vo), args.cpu_grad_rays, replace=False))
    dL = rng.normal(0, 1, (len(gi), 3))
    tg0 = time.perf_counter()
    oracle.composite_grad(rec, oracle.Rays(vo[gi], vd[gi]), dL, threads=threads)
    tg1 = time.perf_counter()
    cpu = {"value": round(n_rs / (tc1 - tc0) / 1e6, 6), "unit": "Mrays/s",
           "cores": threads, "kind": "oracle",
           "sample": f"{args.cpu_pixels} random pixels of the same path-tracer mix at "
                     f"{st.spp} spp ({n_rs} ray-samples, brute force over all "
                     f"{st.sc_host.num_gaussians} Gaussians, {tc1 - tc0:.1f} s)",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "exact_gradient": {"rays_per_s": round(len(gi) / (tg1 - tg0), 2),
                              "sample": f"{len(gi)} random rays of the 8 ring views "
                                        f"(exact sorted composite and its gradient, "
                                        f"{tg1 - tg0:.1f} s)"}}
    print(f"# cpu oracle: {cpu['value']} Mrays/s, exact gradient "
          f"{cpu['exact_gradient']['rays_per_s']} rays/s on {threads} threads", file=sys.stderr,
          flush=True)
    return cpu


def multisample(args, srt, si, torch, dev):
    """Forward of the object-like scene (200k Gaussians, 800x800, 4 spp) with
    N = 1 and N = 4 samples per traversal (identical results)."""
    w = si.workload(2)
    sc = srt.DeviceScene.from_host(w["scene"], dev)
    cam = w["cameras"][0]
    o, d = srt.srt_camera_rays(cam, dev)
    bvh = srt.srt_build_bvh(sc, args.width, args.leaf)
    R = o.shape[0]
    out = dict(rgb=torch.empty((R, 3), device=dev))
    ws = torch.empty(srt._lib.load().srt_trace_workspace_size(bvh.handle, R), dtype=torch.uint8,
                     device=dev)
    res = {}
    for n in (1, 4):
        def launch():
            srt.srt_trace_forward(bvh, o, d, seed=si.PHILOX_SEED, spp=4, n_per_traversal=n,
                                  image_width=cam.width, want_hits=False, out=out, workspace=ws)
        launch()
        res[f"n{n}_ms"] = round(ev_time(torch, launch, 5), 3)
    res["speedup"] = round(res["n1_ms"] / res["n4_ms"], 3)
    res["workload"] = "200k Gaussians (object-like shell), 800x800, 4 spp, image launch"
    print(f"# multisample: {res}", file=sys.stderr, flush=True)
    return res


def compare_estimators(st, bvh, seeds=6):
    """Plain and Rao-Blackwellised backward on the same forward realisations
    (sample offsets 1000 + k*spp): average launch time of each and the summed
    variance, over the realisations, of the gradients of means, log-scales,
    quaternions and opacity logits."""
    torch = st.torch
    names = ("means", "log_scales", "quats", "opacity_logits")
    res = {}
    for est in ("plain", "rb"):
        per, ms = [], []
        for k in range(seeds):
            st.ring_forward(bvh, 250 + k)
            ms.append(ev_time(torch, lambda: st.ring_backward(bvh, 250 + k, estimator=est), 1))
            per.append(torch.cat([st.grads[n].flatten() for n in names]).double())
        var = float(torch.stack(per).var(0).sum())
        res[est] = (min(ms), var)
        del per
    (pm, pv), (rm, rv) = res["plain"], res["rb"]
    return {"plain_ms": round(pm, 3), "rb_ms": round(rm, 3),
            "variance_ratio": round(rv / pv, 4) if pv > 0 else None,
            "variance_time_ratio": round(rv * rm / (pv * pm), 4) if pv > 0 else None,
            "realisations": seeds}


PROFILE_JSON = "kernels_1M_pmc.json"
PROFILE_SOURCES = ["include/srt.h", "paper_2504_06598_amd/csrc/srt_device.hpp",
                   "paper_2504_06598_amd/csrc/srt_walk.hpp",
                   "paper_2504_06598_amd/csrc/srt_internal.hpp",
                   "paper_2504_06598_amd/csrc/trace.hip", "paper_2504_06598_amd/csrc/backward.hip",
                   "paper_2504_06598_amd/csrc/build.hip"]


def sources_sha1(files, root=ROOT):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        h.update(open(os.path.join(root, f), "rb").read())
    return h.hexdigest()


def measured_profiles(width, leaf, root=ROOT):
    """Per-kernel counter figures (HBM bytes per launch from FETCH_SIZE and
    WRITE_SIZE scaled by a copy of known size, L2 hit rate, instruction
    counts) recorded under profiles/ by --summarize-profiles; None when the
    kernel sources or the tree shape differ from those that were measured."""
    path = os.path.join(root, "profiles", PROFILE_JSON)
    try:
        rec = json.load(open(path))
        h = sources_sha1(rec["sources"], root)
    except (OSError, ValueError, KeyError):
        return None
    if h != rec["sources_sha1"] or (width, leaf) != (rec["width"], rec["leaf_size"]):
        return None
    return rec["kernels"]


def profile_kernels(st):
    """For rocprofv3: each major kernel of the step launched 3 times in the
    step's configuration (after its inputs are made), then a 256 MiB
    elementwise copy whose counters calibrate FETCH_SIZE / WRITE_SIZE."""
    torch = st.torch
    bvh = st.build()
    specs = kernel_specs(st, bvh)
    for _, (_, setup, _, _) in specs.items():
        setup()
    torch.cuda.synchronize()
    for name, (label, _, launch, _) in specs.items():
        for i in range(3):
            launch(None)
            torch.cuda.synchronize()
        print(f"# {name}: {label}, 3 launches done", file=sys.stderr, flush=True)
    x = torch.ones(64 << 20, device=st.dev)  # 256 MiB read, 256 MiB written
    y = torch.empty_like(x)
    for _ in range(3):
        torch.add(x, 0.0, out=y)
    torch.cuda.synchronize()
    print("# calibration copy: 268435456 bytes read and written per launch", file=sys.stderr,
          flush=True)


# kernel-name patterns of the --profile-kernels launches (the last 3 matching
# dispatches of each are the measured ones)
PROFILE_PATTERNS = {"camera": ("k_trace_wave<4, 8,",), "shadow": ("k_shadow_queue",),
                    "ring_forward": ("k_trace_wave<4, 4,",), "backward": ("k_backward",),
                    "calibration": ("CUDAFunctorOnSelf_add",)}


def _csv_rows(dirs, suffix):
    import csv
    import glob
    rows = []
    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
            with open(f) as fh:
                rows.extend(csv.DictReader(fh))
    return rows


def _match(name, pats):
    return any(p in name for p in pats)


def summarize_profiles(args):
    """Per-kernel tables from rocprofv3 output directories of --profile-kernels
    runs: kernel-trace durations and per-dispatch counters (FETCH_SIZE,
    WRITE_SIZE, TCC_HIT_sum, TCC_MISS_sum, SQ_* instruction counts)."""
    dirs = args.summarize_profiles
    trace = _csv_rows(dirs, "kernel_trace.csv")
    out = {}
    for name, pats in PROFILE_PATTERNS.items():
        ds = [r for r in trace if _match(r.get("Kernel_Name", ""), pats)][-3:]
        if ds:
            durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in ds]
            out.setdefault(name, {})["ms"] = [round(x, 3) for x in durs]
            out[name]["kernel_name"] = ds[0]["Kernel_Name"]
    counters = {}
    for r in _csv_rows(dirs, "counter_collection.csv"):
        name = next((n for n, p in PROFILE_PATTERNS.items() if _match(r.get("Kernel_Name", ""), p)),
                    None)
        if name is None:
            continue
        key = (name, int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))))
        counters.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    per = {}
    for (name, disp), cv in sorted(counters.items()):
        per.setdefault(name, []).append(cv)
    cal = per.get("calibration", [])
    fetch_f = write_f = None
    if cal:
        f = [c["FETCH_SIZE"] for c in cal if "FETCH_SIZE" in c][-1:]
        w = [c["WRITE_SIZE"] for c in cal if "WRITE_SIZE" in c][-1:]
        fetch_f = 262144.0 / f[0] if f else None
        write_f = 262144.0 / w[0] if w else None
    rec = {}
    for name, lst in per.items():
        if name == "calibration":
            continue
        lst = lst[-6:]
        avg = {}
        for k in {k for c in lst for k in c}:
            vals = [c[k] for c in lst if k in c][-3:]
            avg[k] = sum(vals) / len(vals)
        e = {"counters": {k: round(v, 1) for k, v in sorted(avg.items())}}
        if "FETCH_SIZE" in avg and "WRITE_SIZE" in avg and fetch_f and write_f:
            e["hbm_bytes_per_launch"] = int(1024 * (avg["FETCH_SIZE"] * fetch_f +
                                                    avg["WRITE_SIZE"] * write_f))
        if "TCC_HIT_sum" in avg and "TCC_MISS_sum" in avg:
            tot = avg["TCC_HIT_sum"] + avg["TCC_MISS_sum"]
            e["l2_hit_rate"] = round(avg["TCC_HIT_sum"] / tot, 4) if tot else None
        for k, kk in (("SQ_INSTS_VALU", "valu_insts"), ("SQ_INSTS_SALU", "salu_insts")):
            if k in avg:
                e[kk] = int(avg[k])
        # derived metrics in percent: time the vector / scalar ALUs are busy,
        # lanes active per vector instruction
        for k, kk in (("VALUBusy", "valu_busy"), ("SALUBusy", "salu_busy"),
                      ("VALUUtilization", "valu_lanes_active")):
            if k in avg:
                e[kk] = round(avg[k], 1)
        if name in out:
            e["ms"] = out[name]["ms"]
            e["kernel_name"] = out[name]["kernel_name"]
        rec[name] = e
    for name, e in out.items():
        rec.setdefault(name, e)
    print(json.dumps({"fetch_factor": fetch_f, "write_factor": write_f, "kernels": rec}, indent=1))
    if args.write_profile_json:
        full = {"sources": PROFILE_SOURCES, "sources_sha1": sources_sha1(PROFILE_SOURCES),
                "width": args.width, "leaf_size": args.leaf, "fetch_factor": fetch_f,
                "write_factor": write_f,
                "kernels": {k: v for k, v in rec.items() if "hbm_bytes_per_launch" in v}}
        with open(args.write_profile_json, "w") as fh:
            json.dump(full, fh, indent=1)


# samples per traversal of the batched launch's sweep: in this scene's fog of
# large Gaussians a traversal tests ~10k records whatever its N, so larger N
# means fewer traversals of views with many spp (camera items at full size:
# 3.5 s at N = 4, 2.1 s at N = 8); the best configuration of each kind is also
# timed at N = 16
BATCH_N = 8


def bench_batched(args, srt, si, torch, dev):
    """Persistent vs plain on the batched scene: 64 views of 512x512 with
    their spp and 4M incoherent rays in one graph launch (with
    --batched-scale k: 1/k of the pixels, views of 512/sqrt(k) pixels a side
    with the same spp, and 1/k of the incoherent rays). The autotuner sweeps
    width {2,4,8} x leaf size {1,2,4,8} (size split 4: Gaussians more than 16x
    apart in size in subtrees of their own, 2x faster than none on this scene)
    x refill threshold {16,32} x workgroups per CU {8,12} (each persistent
    grid capped at what its kernel keeps resident) at N = 8 samples per
    traversal, then the best of each kind at N = 16, on a subsample that keeps
    the workload's
    coherence and mix: every 8th view in order of spp, at full resolution, and
    the incoherent rays in the same proportion to the camera samples; each
    kind then runs the workload at its pick, one warm-up launch and
    --batched-reps timed launches."""
    import numpy as np

    from paper_2504_06598_amd.autotune import autotune
    t0 = time.perf_counter()
    w = si.workload(5)
    sc = srt.DeviceScene.from_host(w["scene"], dev)
    k = args.batched_scale
    side = int(round(512 / k ** 0.5))
    cams = si.fibonacci_cameras(len(w["cameras"]), 3.0, side, side)
    spp = w["spp"]
    n_all = w["incoherent"][0].shape[0]
    n_inc = n_all // k
    eo, ed = (torch.from_numpy(x[:n_inc]).to(dev) for x in w["incoherent"])
    del w
    print(f"# batched workload: {sc.num_gaussians} Gaussians, {len(cams)} views {side}x{side}, "
          f"{n_inc} incoherent rays (generated in {time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    # every 8th view in order of spp: the tuning launch keeps the workload's
    # spp mix and so its passes per sample (a pass of N samples costs about
    # the same whatever its number of active samples)
    order = np.argsort(np.asarray(spp), kind="stable")
    sub = sorted(int(i) for i in order[4::8])
    full_cams = si.fibonacci_cameras(len(cams), 3.0, 512, 512)
    tcams = [full_cams[i] for i in sub]
    tspp = [spp[i] for i in sub]
    n_t = max(1, int(round(n_all * sum(tspp) / sum(spp))))
    t1 = time.perf_counter()
    if args.batched_config:
        W, L, thr, wpc, n = (int(x) for x in args.batched_config.split(","))
        base = {"width": W, "leaf_size": L, "size_split": 4, "refill_threshold": thr,
                "waves_per_cu": wpc, "n_per_traversal": n}
        tune = {"persistent": dict(base, persistent=True),
                "plain": dict(base, persistent=False), "table": []}
    else:
        tune = autotune(sc, tcams, tspp, extra_origins=eo[:n_t], extra_dirs=ed[:n_t],
                        extra_spp=1, seed=si.PHILOX_SEED, n_per_traversal=BATCH_N,
                        widths=(2, 4, 8), leaves=(1, 2, 4, 8),
                        splits=(4,), thresholds=(16, 32), waves=(8, 12), reps=1,
                        more_n=(16,), use_cache=False, cache_path=None,
                        log=lambda r: print("# tune", r, file=sys.stderr, flush=True))
        print(f"# autotuner ({time.perf_counter() - t1:.1f} s): persistent "
              f"{tune['persistent']}, plain {tune['plain']}, rejected {tune['rejected']}",
              file=sys.stderr, flush=True)
    res = {}
    for kind in ("plain", "persistent"):
        cfg = tune[kind]
        bvh = srt.srt_build_bvh(sc, cfg["width"], cfg["leaf_size"], cfg["size_split"])
        plan = srt.srt_batch_plan_create(bvh, cams, spp, extra_origins=eo, extra_dirs=ed,
                                         extra_spp=1, seed=si.PHILOX_SEED,
                                         n_per_traversal=cfg["n_per_traversal"],
                                         persistent=cfg["persistent"],
                                         refill_threshold=cfg["refill_threshold"],
                                         waves_per_cu=cfg["waves_per_cu"])
        rgb = torch.empty((plan.rows, 3), device=dev)
        cnt = srt.new_counters(dev)
        plan.execute(rgb=rgb, counters=cnt)
        torch.cuda.synchronize()
        c = srt.counters_dict(cnt)
        assert c["ray_samples"] == plan.samples and c["lost"] == 0
        print(f"# batched {kind}: warm-up launch done", file=sys.stderr, flush=True)
        ms = ev_time(torch, lambda: plan.execute(rgb=rgb), args.batched_reps)
        tr = max(c["traversals"], 1)
        res[kind] = {"mrays_per_s": round(plan.samples / (ms * 1e-3) / 1e6, 2),
                     "ms_per_launch": round(ms, 3), "width": cfg["width"],
                     "leaf_size": cfg["leaf_size"], "size_split": cfg["size_split"],
                     "refill_threshold": cfg["refill_threshold"],
                     "waves_per_cu": cfg["waves_per_cu"],
                     "n_per_traversal": cfg["n_per_traversal"],
                     "per_traversal": {"nodes": round(c["nodes"] / tr, 1),
                                       "records": round(c["prims"] / tr, 1),
                                       "candidates": round(c["candidates"] / tr, 1),
                                       "philox": round(c["philox"] / tr, 1)}}
        print(f"# batched {kind}: {ms:.2f} ms per launch, {res[kind]['mrays_per_s']} Mrays/s",
              file=sys.stderr, flush=True)
        res["ray_samples_per_launch"] = int(plan.samples)
        del plan, bvh, rgb
    res["speedup"] = round(res["persistent"]["mrays_per_s"] / res["plain"]["mrays_per_s"], 3)
    scale = "full size" if k == 1 else f"1/{k} of the pixels and incoherent rays"
    res["workload"] = (f"3.3M Gaussians (3M object-like + 300k large diffuse); 64 views on a "
                       f"Fibonacci sphere at {side}x{side}, spp per view from {{1,...,64}}; "
                       f"{n_inc} incoherent rays; one graph launch ({scale}); samples per "
                       f"traversal tuned from {{{BATCH_N}, 16}} per kind")
    res["autotune_configs"] = len(tune["table"])
    return res


if __name__ == "__main__":
    main()
