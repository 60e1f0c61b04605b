"""Host-side checks of the benchmark's bookkeeping (no GPU): the recorded HBM
traffic is reported only for the sources it was measured on, and the
algorithmic counts follow their stated formulas."""
import json
import os
import shutil

import bench


def _fake_root(tmp_path, kernel_src, host_src, rec):
    csrc = tmp_path / "paper_2008_05858_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k_table.hip").write_bytes(kernel_src)
    (csrc / "api.cpp").write_bytes(host_src)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "render_table_c1_batch4_hbm_traffic.md").write_text(
        "# traffic\n\n```json\n" + json.dumps(rec) + "\n```\n")
    return str(tmp_path)


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    import hashlib
    k, h = b"kernel source", b"host source"
    rec = {"hbm_bytes_per_launch": 123.0,
           "kernel_source_sha256": hashlib.sha256(k).hexdigest(),
           "host_source_sha256": hashlib.sha256(h).hexdigest()}
    root = _fake_root(tmp_path, k, h, rec)
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic() == 123.0
    # a kernel edit, or a change of the host code that orders the work list,
    # voids the record
    (tmp_path / "paper_2008_05858_amd" / "csrc" / "k_table.hip").write_bytes(k + b" ")
    assert bench.measured_traffic() is None
    (tmp_path / "paper_2008_05858_amd" / "csrc" / "k_table.hip").write_bytes(k)
    (tmp_path / "paper_2008_05858_amd" / "csrc" / "api.cpp").write_bytes(h + b" ")
    assert bench.measured_traffic() is None


def test_traffic_missing_or_malformed_record(tmp_path, monkeypatch):
    root = _fake_root(tmp_path, b"k", b"h", {"hbm_bytes_per_launch": 1.0})
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic() is None  # no source hashes recorded
    shutil.rmtree(os.path.join(root, "profiles"))
    assert bench.measured_traffic() is None  # no record at all


def test_table_flop_count_formula():
    """One straight trace fully on a 100-px detector: x from 10 to 90 px
    (80 px of x-span = 320 slot columns x 2 rows x 4 layers = 2560 deposit
    cells), 1000 samples, 32 x 32-cell tables at 4 cells per pixel (9 x 9
    taps): 32 x 1000 + 2 x 81 x 2560 flop."""
    import numpy as np
    from workloads import Psf, Scene, Trace
    tr = Trace(0, 0, 0, 500.0, 501.0, 1000, [50.0, 40.0], [20.0], 1.0, 0)
    psf = Psf(kind="table", gx=1, gy=1, kw=32, kh=32, os=4,
              tables=np.full((1, 1, 32, 32), 1.0 / 1024, np.float32))
    sc = Scene("flops", 100, 40, [tr], psf, [np.ones(1000, np.float32)], "f32")
    assert bench.table_flops_frame(sc) == 32.0 * 1000 + 2.0 * 81 * 2560
