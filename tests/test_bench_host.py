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
    """bench.crossings (|dc| + |dr| + 1 cells per ray, from the chord) against
    the oracle's Siddon traces: the cells each ray crosses with positive length."""
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
