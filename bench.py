#!/usr/bin/env python
"""Benchmark of the TNLM 4DCT reconstruction hot path on one MI355X.

Workload (one "step"): the 256x256 paper-size slice in its three dose cases,
each a full solve -- FBP of all phases' views, then 50 outer iterations of
(3 CGLS steps -> patch weights over a 15x15 window of phases i+-1 with 7x7
patches -> one Gauss-Jacobi sweep -> positivity):
    a: 360 views/phase, I0 = 2e4     b: 60 views/phase, I0 = 1e6
    c: 60 views/phase, I0 = 2e4      (10 phases, 512 bins, fan-beam arc)
Inputs are seeded synthetic phantoms (nested ellipses, moving tumour,
analytic line integrals, Poisson noise) resident in HBM before timing.

Metric: phase-pixel*iterations per second = sum over slices of N*L^2*K / wall
seconds, plus wall seconds per 10-phase slice. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
OPS_PER_CROSSING = 8                       # projector: ops per ray-pixel crossing (matrix entry)
OPS_PER_PAIR = 10                          # regulariser: ops per (pixel, candidate) pair


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def crossings(geom) -> float:
    """Number of nonzeros of P (ray-pixel crossings) over all phases, from the
    chord of each ray through the image square: |dc| + |dr| + 1 cells per ray."""
    src, u = geom.rays()
    S = geom.fov_mm
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.stack([(-S / 2 - src[..., 0]) / u[..., 0], (S / 2 - src[..., 0]) / u[..., 0]])
        ty = np.stack([(-S / 2 - src[..., 1]) / u[..., 1], (S / 2 - src[..., 1]) / u[..., 1]])
    chord = np.maximum(np.minimum(tx.max(0), ty.max(0)) - np.maximum(tx.min(0), ty.min(0)), 0.0)
    n = np.where(chord > 0, chord * (np.abs(u[..., 0]) + np.abs(u[..., 1])) / geom.pixel_mm + 1.0, 0.0)
    return float(n.sum())


def pairs(case) -> float:
    """(pixel, candidate) pairs of one regulariser sweep: both neighbours, window truncated to the image."""
    L, R = case.geom.L, case.window // 2
    per_axis = sum(min(x + R, L - 1) - max(x - R, 0) + 1 for x in range(L))
    return 2.0 * case.geom.n_phases * per_axis * per_axis


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "backproject": ["paper_1009_1351_amd/csrc/proj.hip"],
    "project": ["paper_1009_1351_amd/csrc/proj.hip"],
    "regularize": ["paper_1009_1351_amd/csrc/tnlm_reg.hip"],
}


def traffic_for(kernel: str, launches_per_step: float):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p)).get(kernel)
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(case_fn):
    """The FP64 oracle on the host cores: one outer iteration of dose case c
    (10 phases, 256^2, 60 views x 512 bins) from its FBP start."""
    import oracle
    oracle.build()
    case = case_fn("C2c")
    G = oracle.Geometry(case.geom)
    y = np.asarray(case.y, np.float32).astype(np.float64)
    w = np.asarray(case.w, np.float32).astype(np.float64)
    f0 = oracle.fbp(G, y)
    prm = oracle.case_params(case)
    t0 = time.perf_counter()
    oracle.step(G, prm, y, w, f0)
    dt = time.perf_counter() - t0
    units = case.geom.n_phases * case.geom.L ** 2
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    threads = min(threads, len(os.sched_getaffinity(0)))
    return {"value": units / dt, "unit": "phase-pixel*iters/s", "cores": threads, "kind": "oracle",
            "sample": f"one outer iteration (CGLS x3 + regulariser) of dose case c, 10 x 256^2, 60 views x 512 "
                      f"bins, from the FBP image; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=50, help="outer iterations per solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 256 MiB device copy (counter scale)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(slices shard across GPUs without communication, see the design notes)"}))
        sys.exit(2)

    import torch
    import synth
    from paper_1009_1351_amd import Recon

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    names = ["C2a", "C2b", "C2c"]
    cases = {n: synth.make_case(n, K=a.iters) for n in names}
    log("inputs generated")
    runs = []
    for n in names:
        c = cases[n]
        rc = Recon.from_geometry(c.geom, patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat, m1=c.m1,
                                 m2=c.m2, max_outer=c.max_outer, tol=0.0)
        y = torch.from_numpy(c.y.astype(np.float32)).to(dev)
        w = torch.from_numpy(c.w.astype(np.float32)).to(dev)
        f = rc.new_image()
        runs.append((n, c, rc, y, w, f))
    torch.cuda.synchronize()

    def step():
        done = 0
        for n, c, rc, y, w, f in runs:
            _, k, _, st = rc.solve(y, w, f)
            done += c.geom.n_phases * c.geom.L ** 2 * k
        return done

    for _ in range(a.warmup):
        step()
    log("warmup done")
    if a.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _, _, rc, _, _, _ in runs:
        rc.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = 0
    for s in range(a.steps):
        units += step()
        log(f"step {s + 1}/{a.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_kind = {}
    algo = {"project": 0.0, "backproject": 0.0, "regularize": 0.0}
    for n, c, rc, _, _, _ in runs:
        t = rc.timing_read()
        rc.timing(False)
        for k, (ms, cnt) in t.items():
            tot = per_kind.setdefault(k, [0.0, 0])
            tot[0] += ms
            tot[1] += cnt
        nz = crossings(c.geom)
        algo["project"] += t["project"][1] * nz * OPS_PER_CROSSING
        algo["backproject"] += t["backproject"][1] * nz * OPS_PER_CROSSING
        algo["regularize"] += t["regularize"][1] * pairs(c) * OPS_PER_PAIR
    dom = max(algo, key=lambda k: per_kind[k][0])
    ms_tot, launches = per_kind[dom]
    achieved = algo[dom] / (ms_tot * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TOPS, 2),
            "unit": "TOP/s", "frac": round(achieved / PEAK_ALU_TOPS, 4),
            "avg_launch_ms": round(ms_tot / max(launches, 1), 4),
            "traffic": traffic_for(dom, launches / a.steps)}
    value = units / dt
    slices = len(runs) * a.steps
    out = {
        "metric": "phase-pixel*iters/s", "value": value, "unit": "phase-pixel*iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "C2: 1 slice x 10 phases, 256x256, 512 bins, doses a (360 views, I0 2e4), "
                               "b (60 views, I0 1e6), c (60 views, I0 2e4); patch 7, window 15, M1 3, M2 1; "
                               f"{a.iters} outer iterations from the FBP of all phases",
                   "slices_per_step": len(runs), "wall_s_per_slice": dt / slices,
                   "parallelism": "single GPU"},
        "kernel_ms": {k: round(v[0] / a.steps, 3) for k, v in per_kind.items()},
        "roofline": roof,
    }
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(lambda n: synth.make_case(n, K=a.iters))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
