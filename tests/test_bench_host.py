"""Host-side logic of bench.py: the HBM traffic figure is reported only for
the kernel sources and tree shape it was measured on."""
import hashlib
import json
import os

import bench


def _setup(tmp_path, width=4, leaf=2):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    (tmp_path / "profiles").mkdir()
    rec = {"sources": ["k.hip"], "sources_sha1": hashlib.sha1(b"kernel v1").hexdigest(),
           "width": width, "leaf_size": leaf, "hbm_bytes_per_launch": 1234}
    (tmp_path / "profiles" / "k_trace_wave_camera_1M_pmc.json").write_text(json.dumps(rec))
    return src


def test_traffic_reported_for_the_measured_kernel(tmp_path):
    _setup(tmp_path)
    assert bench.measured_traffic(4, 2, root=str(tmp_path)) == 1234


def test_traffic_null_after_a_source_change(tmp_path):
    src = _setup(tmp_path)
    src.write_bytes(b"kernel v2")
    assert bench.measured_traffic(4, 2, root=str(tmp_path)) is None


def test_traffic_null_for_another_tree_shape_or_no_record(tmp_path):
    _setup(tmp_path)
    assert bench.measured_traffic(4, 4, root=str(tmp_path)) is None
    os.remove(tmp_path / "profiles" / "k_trace_wave_camera_1M_pmc.json")
    assert bench.measured_traffic(4, 2, root=str(tmp_path)) is None
