"""Host-side checks of the benchmark: the one-GPU contract and the
algorithmic work count behind the roofline figure."""
import json
import os
import subprocess
import sys

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_crossing_count_matches_traced_rays(orc):
    """bench.crossings (chord (|u_x| + |u_y|) / D cells per ray) against the
    oracle's Siddon traces: the cells each ray crosses with positive length."""
    sys.path.insert(0, ROOT)
    import bench
    geom = synth.ScanGeometry(n_phases=1, L=32, n_views=12, n_bins=48)
    G = orc.Geometry(geom)
    traced = 0
    for v in range(geom.n_views):
        for b in range(geom.n_bins):
            pix, ln = orc.trace_ray(G, 0, v, b)
            traced += int((ln > 0).sum())
    est = bench.crossings(geom)
    assert abs(est - traced) <= 0.01 * traced, (est, traced)


def test_traffic_figure_only_for_the_profiled_source(tmp_path, monkeypatch):
    """The bench line's HBM traffic comes from the stored counter summary only
    while it was taken on the benchmark's workload and the kernel's sources
    hash to the value recorded with it; any change
    to them (a comment included) makes it null until the counters are taken
    again."""
    sys.path.insert(0, ROOT)
    import bench
    files = bench.KERNEL_SOURCES["project"]
    for f in files:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("project") is None   # no summary stored
    (tmp_path / "profiles").mkdir()
    rec = {"project": {"source_hash": bench.source_hash(files), "bytes_per_launch": 1.25e8}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_for("project") is None   # taken on no named workload
    rec["project"]["workload"] = "another workload"
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_for("project") is None   # taken on another workload
    rec["project"]["workload"] = bench.WORKLOAD_KEY
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_for("project") == 1.25e8
    assert bench.traffic_for("regularize") is None   # no record for this kernel
    with open(tmp_path / files[0], "a") as fh:
        fh.write("// edited\n")
    assert bench.traffic_for("project") is None
