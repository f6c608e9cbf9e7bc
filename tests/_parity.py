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


def _parse_nodes(raw, W):
    f = raw.view(np.float32)
    lo = f[:, 0:3 * W].reshape(-1, 3, W)
    hi = f[:, 3 * W:6 * W].reshape(-1, 3, W)
    child = raw[:, 6 * W:7 * W]
    return lo, hi, child


def check_bvh_structure(bvh, W, L, G):
    """Every Gaussian in exactly one leaf of at most L, every slot box holds
    its child's boxes (or its Gaussians' boxes), no node reached twice."""
    info = bvh.info()
    raw, order = bvh.nodes()
    raw, order = to_np(raw), to_np(order)
    recs = {k: to_np(v) for k, v in bvh.records().items()}
    lo, hi, child = _parse_nodes(raw, W)
    assert sorted(order.tolist()) == list(range(G))
    seen = np.zeros(G, np.int32)
    stack = [(0, 1)]
    max_depth = 0
    visited = 0
    while stack:
        n, depth = stack.pop()
        visited += 1
        assert visited <= info["num_nodes"], "node reached twice"
        assert 0 <= n < info["num_nodes"]
        max_depth = max(max_depth, depth)
        for c in range(W):
            ref = int(child[n, c])
            if ref == 0x7FFFFFFF:
                assert lo[n, 0, c] > hi[n, 0, c]
                continue
            if ref >= 0:
                # the slot box contains every box of the child node
                sub = child[ref] != 0x7FFFFFFF
                assert np.all(lo[n, :, c][:, None] <= lo[ref][:, sub])
                assert np.all(hi[n, :, c][:, None] >= hi[ref][:, sub])
                stack.append((ref, depth + 1))
            else:
                v = ~ref & 0xFFFFFFFF
                first, count = v >> 3, (v & 7) + 1
                assert count <= L
                for p in range(first, first + count):
                    seen[p] += 1
                    g = order[p]
                    assert np.all(lo[n, :, c] <= recs["box_lo"][g])
                    assert np.all(hi[n, :, c] >= recs["box_hi"][g])
    assert np.all(seen == 1), "every Gaussian in exactly one leaf"
    assert visited == info["num_nodes"]
    assert max_depth <= info["depth"]
