"""Host-side logic of bench.py: the per-kernel counter record is reported only
for the kernel sources and tree shape it was measured on, and the profile
summariser reads rocprofv3's CSV layout."""
import csv
import hashlib
import json
import os
import types

import bench


def _setup(tmp_path, width=4, leaf=2):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    (tmp_path / "profiles").mkdir()
    rec = {"sources": ["k.hip"], "sources_sha1": hashlib.sha1(b"kernel v1").hexdigest(),
           "width": width, "leaf_size": leaf,
           "kernels": {"shadow": {"hbm_bytes_per_launch": 1234, "l2_hit_rate": 0.9}}}
    (tmp_path / "profiles" / bench.PROFILE_JSON).write_text(json.dumps(rec))
    return src


def test_profiles_reported_for_the_measured_kernels(tmp_path):
    _setup(tmp_path)
    p = bench.measured_profiles(4, 2, root=str(tmp_path))
    assert p["shadow"]["hbm_bytes_per_launch"] == 1234


def test_profiles_null_after_a_source_change(tmp_path):
    src = _setup(tmp_path)
    src.write_bytes(b"kernel v2")
    assert bench.measured_profiles(4, 2, root=str(tmp_path)) is None


def test_profiles_null_for_another_tree_shape_or_no_record(tmp_path):
    _setup(tmp_path)
    assert bench.measured_profiles(4, 4, root=str(tmp_path)) is None
    os.remove(tmp_path / "profiles" / bench.PROFILE_JSON)
    assert bench.measured_profiles(4, 2, root=str(tmp_path)) is None


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_summariser_scales_counters_by_the_calibration_copy(tmp_path, capsys):
    d = tmp_path / "pmc"
    d.mkdir()
    rows = []
    disp = 0
    copy = "at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<float> >"
    for name, fetch, write, hit, miss in [("void k_shadow_queue<4, false, 0>(...)", 100.0,
                                           50.0, 90.0, 10.0)] * 3 + \
                                          [(copy, 131072.0, 262144.0, 1.0, 1.0)]:
        disp += 1
        for cn, cv in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write), ("TCC_HIT_sum", hit),
                       ("TCC_MISS_sum", miss), ("VALUBusy", 95.26), ("VALUUtilization", 39.4)):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": cn,
                         "Counter_Value": cv})
    _write_csv(d / "run_counter_collection.csv", rows)
    trace = [{"Kernel_Name": "void k_shadow_queue<4, false, 0>(...)", "Start_Timestamp": 0,
              "End_Timestamp": 2_000_000}]
    _write_csv(d / "run_kernel_trace.csv", trace)
    out = tmp_path / "rec.json"
    args = types.SimpleNamespace(summarize_profiles=[str(d)], write_profile_json=str(out),
                                 width=4, leaf=2)
    bench.summarize_profiles(args)
    rec = json.load(open(out))
    k = rec["kernels"]["shadow"]
    # FETCH_SIZE x 2 (the copy reads 256 MiB, reported as 128 MiB), WRITE_SIZE x 1
    assert k["hbm_bytes_per_launch"] == 1024 * (100 * 2 + 50)
    assert abs(k["l2_hit_rate"] - 0.9) < 1e-9
    assert k["valu_busy"] == 95.3  # percent, rounded to 0.1
    assert k["valu_lanes_active"] == 39.4
    assert k["ms"] == [2.0]
    assert rec["sources_sha1"] == bench.sources_sha1(bench.PROFILE_SOURCES)
