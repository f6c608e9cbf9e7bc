"""Shared helpers of the GPU parity tests: device scenes, oracle runs and the
comparison rules (ids bit-exact outside flagged samples, colour within 1e-4)."""
import sys

import numpy as np

import oracle
import srt_inputs as si

COLOUR_ATOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_scene(scene):
    import paper_2504_06598_amd as srt
    return srt.DeviceScene.from_host(scene)


def to_np(t):
    return t.detach().cpu().numpy()


def compare_ids(gpu_gid, ora_gid, flags, max_flag_frac=1e-3, what="hit ids"):
    """Ids must match bit for bit on every sample the oracle did not flag."""
    gpu_gid = np.asarray(gpu_gid)
    ora_gid = np.asarray(ora_gid)
    flagged = np.asarray(flags) != 0
    bad = (gpu_gid != ora_gid) & ~flagged
    n_bad = int(bad.sum())
    assert n_bad == 0, (f"{what}: {n_bad} of {bad.size} unflagged samples differ; first at "
                        f"{np.argwhere(bad)[:5].tolist()}: gpu {gpu_gid[bad][:5]} oracle "
                        f"{ora_gid[bad][:5]}")
    frac = flagged.mean() if flagged.size else 0.0
    assert frac <= max_flag_frac, f"{what}: {frac:.2e} of samples flagged"
    return int(flagged.sum())


def compare_rgb(gpu_rgb, ora_rgb, flags, atol=COLOUR_ATOL):
    """Pixels holding a flagged sample may legitimately differ; all others must
    agree within atol."""
    flagged_px = (np.asarray(flags) != 0).reshape(len(gpu_rgb), -1).any(1)
    err = np.abs(np.asarray(gpu_rgb, np.float64) - np.asarray(ora_rgb))[~flagged_px]
    worst = float(err.max()) if err.size else 0.0
    assert worst <= atol, f"colour error {worst:.3e} > {atol}"
    return worst


def tiny_scene(seed, n, scale=(0.01, 0.05), deg=0):
    sc = si.scene_uniform_cube(seed, n, deg)
    lo, hi = np.log(scale[0]), np.log(scale[1])
    rng = np.random.default_rng(seed + 77)
    sc.log_scales = rng.uniform(lo, hi, sc.log_scales.shape).astype(np.float32)
    return sc
