"""srt_trace_forward_noalloc (the forward with the library's static per-device
scratch instead of a caller workspace) against srt_trace_forward, through the
C ABI: equal outputs on consecutive calls, the second one smaller (the
scratch keeps the previous call's contents), including the deep-stack pass
that uses the scratch's global stacks; a size beyond the scratch is refused
before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

import srt_inputs as si
from _parity import device_scene, say, tiny_scene, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srt():
    import paper_2504_06598_amd as srt
    assert torch.cuda.is_available()
    srt._lib.load()
    return srt


def _outputs(R, spp):
    return dict(rgb=torch.full((R, 3), -7.0, device="cuda"),
                hit_gid=torch.full((R, spp), -7, dtype=torch.int32, device="cuda"),
                hit_t=torch.full((R, spp), -7.0, device="cuda"))


def _call_noalloc(srt, bvh, o, d, out, cnt, **kw):
    lib = srt._lib.load()
    R = int(o.shape[0])
    rays = srt._lib.SrtRays(R, o.data_ptr(), d.data_ptr(), None, None, None, None, None, 0)
    opts = srt._opts(kw.get("seed", 0), kw["spp"], kw["n_per_traversal"], 0, (0.1, 0.2, 0.3),
                     kw.get("any_hit", False), kw.get("stack_limit", 0), 0, (0.0, 0.0, 0.0),
                     kw.get("image_width", 0), False, 0)
    st = lib.srt_trace_forward_noalloc(bvh.handle, C.byref(rays), C.byref(opts),
                                       out["rgb"].data_ptr(), out["hit_gid"].data_ptr(),
                                       out["hit_t"].data_ptr(), cnt.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
    assert st == 0, lib.srt_status_str(st)


@pytest.mark.parametrize("image,lim,any_hit", [(True, 0, False), (False, 0, False),
                                               (True, 2, False), (False, 0, True)])
def test_noalloc_equals_forward_on_consecutive_calls(srt, image, lim, any_hit):
    w = si.workload(3, small=True)
    bvh = srt.srt_build_bvh(device_scene(w["scene"]), 4, 2)
    for k, (wd, ht) in enumerate([(96, 54), (40, 24)]):
        say(f"no-alloc forward, call {k}: {wd}x{ht}, image {image}, stack limit {lim}, "
            f"any-hit {any_hit}")
        cam = si.look_at((0.2, 0.1, 4.0), (0, 0, 0), wd, ht)
        o, d = srt.srt_camera_rays(cam)
        R = wd * ht
        spp, N = (3, 1) if any_hit else (16, 8)
        kw = dict(seed=5 + k, spp=spp, n_per_traversal=N, stack_limit=lim, any_hit=any_hit,
                  image_width=wd if image else 0)
        ref_cnt = srt.new_counters()
        ref = srt.srt_trace_forward(bvh, o, d, bg=(0.1, 0.2, 0.3), counters=ref_cnt, **kw)
        out = _outputs(R, spp)
        cnt = srt.new_counters()
        _call_noalloc(srt, bvh, o, d, out, cnt, **kw)
        torch.cuda.synchronize()
        for key in ("rgb", "hit_gid", "hit_t"):
            np.testing.assert_array_equal(to_np(out[key]), to_np(ref[key]), err_msg=key)
        c, rc = srt.counters_dict(cnt), srt.counters_dict(ref_cnt)
        assert c == rc
        assert c["lost"] == 0 and (c["deep"] > 0) == (lim > 0)


def test_noalloc_refuses_sizes_beyond_its_scratch(srt):
    lib = srt._lib.load()
    sc = tiny_scene(5, 200)
    bvh = srt.srt_build_bvh(device_scene(sc), 4, 4)
    limit = int(srt._lib.NOALLOC_SCRATCH_BYTES)
    R = 1
    while lib.srt_trace_workspace_size(bvh.handle, R) <= limit:
        R *= 2
    assert R >= 1 << 20
    say(f"no-alloc forward refuses {R} rays ({lib.srt_trace_workspace_size(bvh.handle, R)} B "
        f"of scratch > {limit} B)")
    o = torch.zeros((4, 3), device="cuda")
    rays = srt._lib.SrtRays(R, o.data_ptr(), o.data_ptr(), None, None, None, None, None, 0)
    opts = srt._opts(0, 1, 1, 0, (0.0, 0.0, 0.0), False, 0)
    # validation fails on the host before any launch, so the short arrays are never read
    st = lib.srt_trace_forward_noalloc(bvh.handle, C.byref(rays), C.byref(opts), None, None,
                                       None, None, None)
    assert st == 5
