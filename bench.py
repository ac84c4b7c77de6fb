#!/usr/bin/env python
"""Benchmark of the TNLM 4DCT reconstruction hot path on one MI355X.

Timed step: the 64-slice mixed batch solved as one batch by the batched
engine -- 64 slices x 10 phases, image sides drawn from {128, 256, 384, 512},
40-360 views per phase, 1.5 L detector bins, I0 log-uniform in [1e4, 1e6];
FBP of all phases' views, then 50 outer iterations of (3 CGLS steps -> patch
weights over a 15x15 window of phases i+-1 with 7x7 patches -> one
Gauss-Jacobi sweep -> positivity), one outer iteration replayed as a captured
HIP graph. Inputs are seeded synthetic phantoms (nested ellipses, moving
tumour, analytic line integrals, Poisson noise) resident in HBM before timing.

Metric: phase-pixel*iterations per second = sum over slices of N*L^2*K / wall
seconds. Per-kernel times and the roofline fractions come from a separate,
untimed pass with per-launch HIP events (which replaces the graph replay by
direct launches). Also reported: the 256^2 paper-size slice in its three dose
cases as one batch; 512^2 slices with the FP32 and the BF16-MFMA regulariser;
and -- when trained warm-start weights are present -- wall seconds per
10-phase slice to a relative update of 1e-4 on the 32-slice 512^2 evaluation
set, learned warm start + batched engine and coarse-to-fine start against the
plain path (cold start, one slice at a time).
Prints one JSON line.
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
WEIGHTS = os.path.join(ROOT, "paper_1009_1351_amd", "weights", "warmstart_c5.npz")
C3_SLICES = 64
C5_EVAL_SLICES = 32
WORKLOAD_KEY = "c3_batch"                  # the workload the stored counter figures were taken on


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def crossings(geom) -> float:
    """Number of nonzeros of P (ray-pixel crossings) over all phases, from the
    chord of each ray through the image square: chord (|ux| + |uy|) / D cells
    per ray in expectation (a chord starts and ends on grid lines)."""
    src, u = geom.rays()
    S = geom.fov_mm
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.stack([(-S / 2 - src[..., 0]) / u[..., 0], (S / 2 - src[..., 0]) / u[..., 0]])
        ty = np.stack([(-S / 2 - src[..., 1]) / u[..., 1], (S / 2 - src[..., 1]) / u[..., 1]])
    chord = np.maximum(np.minimum(tx.max(0), ty.max(0)) - np.maximum(tx.min(0), ty.min(0)), 0.0)
    n = np.where(chord > 0, chord * (np.abs(u[..., 0]) + np.abs(u[..., 1])) / geom.pixel_mm, 0.0)
    return float(n.sum())


def pairs(geom, window) -> float:
    """(pixel, candidate) pairs of one regulariser sweep: both neighbours, window truncated to the image."""
    L, R = geom.L, window // 2
    per_axis = sum(min(x + R, L - 1) - max(x - R, 0) + 1 for x in range(L))
    return 2.0 * geom.n_phases * per_axis * per_axis


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


_COMMON = ["paper_1009_1351_amd/csrc/internal.h", "paper_1009_1351_amd/csrc/devutil.h"]
KERNEL_SOURCES = {
    "backproject": ["paper_1009_1351_amd/csrc/proj.hip"] + _COMMON,
    "project": ["paper_1009_1351_amd/csrc/proj.hip"] + _COMMON,
    "regularize": ["paper_1009_1351_amd/csrc/tnlm_reg.hip"] + _COMMON,
}   # a change to these files invalidates the stored traffic figures


def traffic_for(kernel: str, workload: str = WORKLOAD_KEY):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source and on this workload; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p)).get(kernel)
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    if rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


# ------------------------------------------------------------------- inputs
def _make(spec):
    import synth
    name, s, kw = spec
    c = synth.make_case(name, slice_index=s, **kw)
    c.y = np.asarray(c.y, np.float32)
    c.w = np.asarray(c.w, np.float32)
    return c


def make_cases(specs, workers=None):
    """Seeded cases for [(config, slice, overrides)], generated in worker
    processes (before this process touches the GPU); y and w as float32."""
    n = len(specs)
    workers = workers or min(16, len(os.sched_getaffinity(0)), n)
    if workers <= 1 or n <= 1:
        return [_make(s) for s in specs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_make, specs, chunksize=1)


# ---------------------------------------------------------------- baselines
def cpu_baseline(c3_cases):
    """The FP64 oracle on the host cores: one outer iteration (FBP start) of
    two slices of the mixed batch (the smallest-view 128^2 and 256^2 slices),
    on all the threads this process may use (and on 8 when it may use more),
    and of the 128^2 slice on one thread."""
    import oracle
    oracle.build()
    from oracle import _lib_threads
    picks = [c for c in c3_cases if c.name in ("C3/s6", "C3/s34")]

    def run(cases):
        units, dt = 0, 0.0
        for case in cases:
            G = oracle.Geometry(case.geom)
            y = np.asarray(case.y, np.float64)
            w = np.asarray(case.w, np.float64)
            f0 = oracle.fbp(G, y)
            prm = oracle.case_params(case)
            t0 = time.perf_counter()
            oracle.step(G, prm, y, w, f0)
            dt += time.perf_counter() - t0
            units += case.geom.n_phases * case.geom.L ** 2
        return units, dt

    threads = min(int(os.environ.get("OMP_NUM_THREADS", "0")) or 10**6, len(os.sched_getaffinity(0)))
    with _lib_threads(threads):
        units, dt = run(picks)
    with _lib_threads(1):
        u1, d1 = run(picks[:1])
    out8 = None
    if threads > 8:
        with _lib_threads(8):
            u8, d8 = run(picks)
        out8 = {"value": u8 / d8, "cores": 8, "sample": f"the same 2 slices, {d8:.1f} s"}
    shapes = ", ".join(f"{c.geom.L}^2 x {c.geom.n_views} views x {c.geom.n_bins} bins" for c in picks)
    return {"value": units / dt, "unit": "phase-pixel*iters/s", "cores": threads, "kind": "oracle",
            "sample": f"one outer iteration (CGLS x3 + regulariser, FBP start) of 2 of the 64 slices ({shapes}); "
                      f"{dt:.1f} s on {threads} threads",
            "eight_threads": out8,
            "single_thread": {"value": u1 / d1, "cores": 1,
                              "sample": f"the {picks[0].geom.L}^2 slice alone, {d1:.1f} s"}}


# -------------------------------------------------------------------- legs
def learned_vs_plain(torch, dev, cases, tol=1e-4, restart_after=64):
    """Wall seconds per slice to tol: plain (cold start, one slice at a time)
    against the learned warm start + batched engine, and against the
    coarse-to-fine start, on the 512^2 evaluation slices (all reported)."""
    from paper_1009_1351_amd import Recon
    from paper_1009_1351_amd.warmstart import LearnedSolver, WarmStartNet
    net = WarmStartNet(phases=10, base=32)
    net.load_weights(WEIGHTS)
    n_slices = len(cases)
    c0 = cases[0]
    prm = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat)
    ys = [torch.from_numpy(c.y).to(dev) for c in cases]
    ws = [torch.from_numpy(c.w).to(dev) for c in cases]
    plain = [Recon.from_geometry(c.geom, max_outer=c0.max_outer, tol=tol, device=dev, **prm) for c in cases]
    solver = LearnedSolver([c.geom for c in cases], net, tol=tol, max_outer=c0.max_outer, restart_after=restart_after,
                           device=dev, **prm)
    plain[0].solve(ys[0], ws[0])   # warm-up: library kernels loaded
    net.forward(torch.zeros((1, 10, c0.geom.L, c0.geom.L), device=dev), factor=net.factor_for(c0.geom.L))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [rc.solve(y, w) for rc, y, w in zip(plain, ys, ws)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log("  plain done")
    t0 = time.perf_counter()
    _, it_l, st_l, used, probe = solver.solve(ys, ws, with_probe=True)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    solver.close()
    log("  learned done")
    from paper_1009_1351_amd.multigrid import MultigridSolver
    mg = MultigridSolver([c.geom for c in cases], tol=tol, max_outer=c0.max_outer, restart_after=restart_after,
                         device=dev, **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it_m, it_mc, st_m = mg.solve(ys, ws)
    torch.cuda.synchronize()
    t_mg = time.perf_counter() - t0
    mg.close()
    log("  coarse-to-fine done")
    return {"workload": f"{n_slices} slices x 10 phases, 512^2, 60 views x 720 bins, I0 2e4, h_rel 0.6, "
                        f"to relative update {tol} (cap {c0.max_outer}); slices {cases[0].name}..{cases[-1].name}",
            "plain_wall_s_per_slice": t_plain / n_slices, "plain_iters": [r[1] for r in res],
            "learned_batched_wall_s_per_slice": t_learned / n_slices, "learned_iters": it_l,
            "learned_probe_iters": probe, "warm_start_used": int(sum(used)),
            "plain_reached_tol": int(sum(r[3] == 0 for r in res)),
            "learned_reached_tol": int(sum(s_ == 0 for s_ in st_l)), "speedup": t_plain / t_learned,
            "multigrid_wall_s_per_slice": t_mg / n_slices, "multigrid_iters": it_m, "multigrid_coarse_iters": it_mc,
            "multigrid_reached_tol": int(sum(s_ == 0 for s_ in st_m)), "multigrid_speedup": t_plain / t_mg}


def c2_leg(torch, dev, cases, steps=3):
    """The 256^2 paper-size slice in its three dose cases as one batch, 50
    outer iterations (graph replay)."""
    from paper_1009_1351_amd import Batch
    c0 = cases[0]
    bt = Batch([c.geom for c in cases], patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat,
               max_outer=c0.max_outer, tol=0.0, device=dev)
    ys = [torch.from_numpy(c.y).to(dev) for c in cases]
    ws = [torch.from_numpy(c.w).to(dev) for c in cases]
    fs = bt.new_images()
    bt.solve(ys, ws, fs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = 0
    for _ in range(steps):
        _, iters, _, _, _ = bt.solve(ys, ws, fs)
        units += sum(c.geom.n_phases * c.geom.L ** 2 * k for c, k in zip(cases, iters))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bt.close()
    return {"workload": "3 slices x 10 phases, 256^2, 512 bins, doses a (360 views, I0 2e4), b (60 views, I0 1e6), "
                        "c (60 views, I0 2e4) in one batch; 50 outer iterations",
            "value": units / dt, "ms_per_solve": dt / steps * 1e3}


def precision_leg(torch, dev, cases):
    """512^2 slices (120 views x 720 bins) with the FP32 and the BF16-MFMA
    regulariser, 10 outer iterations each."""
    from paper_1009_1351_amd import Batch
    ys = [torch.from_numpy(c.y).to(dev) for c in cases]
    ws = [torch.from_numpy(c.w).to(dev) for c in cases]
    iters = cases[0].max_outer
    units = sum(c.geom.n_phases * c.geom.L ** 2 * iters for c in cases)
    res = {}
    for mode in ("fp32", "bf16_mfma"):
        bt = Batch([c.geom for c in cases], patch=7, window=15, h=cases[0].h, mu_hat=cases[0].mu_hat,
                   max_outer=iters, tol=0.0, ssd_mode=mode, device=dev)
        bt.solve(ys, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.solve(ys, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bt.timing(True)
        bt.solve(ys, ws)
        t = bt.timing_read()
        bt.close()
        res[mode] = {"value": units / dt,
                     "regularize_ms_per_launch": round(t["regularize"][0] / max(t["regularize"][1], 1), 4)}
    return {"workload": f"{len(cases)} slices x 10 phases, 512^2, 120 views x 720 bins, I0 5e4, {iters} iterations",
            **res, "bf16_over_fp32_regularize": round(res["bf16_mfma"]["regularize_ms_per_launch"] /
                                                      res["fp32"]["regularize_ms_per_launch"], 3)}


def cnn_flops(phases, base, H, W):
    """Multiply-add FLOPs (2 per MAC) of one forward pass of the warm-start
    network on one [phases][H][W] input: (in, out, kernel, grid divisor) of
    each convolution, encoder 4 levels, decoder with skip concatenation, 1x1
    output."""
    b, P = base, phases
    layers = [(P, b, 3, 1), (b, b, 3, 1), (b, 2 * b, 3, 2), (2 * b, 2 * b, 3, 2), (2 * b, 4 * b, 3, 4),
              (4 * b, 4 * b, 3, 4), (4 * b, 8 * b, 3, 8), (8 * b, 8 * b, 3, 8), (12 * b, 4 * b, 3, 4),
              (4 * b, 4 * b, 3, 4), (6 * b, 2 * b, 3, 2), (2 * b, 2 * b, 3, 2), (3 * b, b, 3, 1), (b, b, 3, 1),
              (b, P, 1, 1)]
    return sum(2.0 * ci * co * k * k * (H // d) * (W // d) for ci, co, k, d in layers)


def cnn_leg(torch, dev, n_fwd=8, n_train=8, L=256, reps=5):
    """Throughput of the warm-start network's BF16 MFMA convolutions: forward
    passes of n_fwd inputs at L^2 and Adam training steps (forward, data and
    weight gradients) on n_train pairs, against the dense BF16 MFMA peak."""
    from paper_1009_1351_amd.warmstart import WarmStartNet
    net = WarmStartNet(phases=10, base=32, seed=1, device=dev)
    g = torch.Generator(device="cpu").manual_seed(3)
    x = (0.02 * torch.rand((max(n_fwd, n_train), 10, L, L), generator=g)).to(dev)
    t = (0.02 * torch.rand((n_train, 10, L, L), generator=g)).to(dev)
    xf = x[:n_fwd].contiguous()
    xt = x[:n_train].contiguous()
    out = torch.empty_like(xf)
    net.forward(xf, out)
    net.train_step(xt, t, 1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(xf, out)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(xt, t, 1e-5)
    torch.cuda.synchronize()
    t_tr = (time.perf_counter() - t0) / reps
    net.close()
    ff = cnn_flops(10, 32, L, L)
    peak = 2500.0
    fwd_tf = n_fwd * ff / t_fwd / 1e12
    tr_tf = 3 * n_train * ff / t_tr / 1e12
    return {"workload": f"forward of {n_fwd} x 10 x {L}^2, Adam step on {n_train} pairs at {L}^2 (bf16 MFMA, fp32 "
                        "accumulate); flops = 2 per MAC of the convolutions, training step counted as 3 forwards",
            "forward_ms": round(t_fwd * 1e3, 3), "forward_tflops": round(fwd_tf, 2),
            "train_step_ms": round(t_tr * 1e3, 3), "train_tflops": round(tr_tf, 2),
            "roofline": {"bound": "mfma", "peak": peak, "unit": "TFLOP/s", "forward_frac": round(fwd_tf / peak, 4),
                         "train_frac": round(tr_tf / peak, 4)}}


def omega_star_leg(torch, dev, iters=50):
    """Adaptive weights against fixed weights from the phantom (the method's
    ideal-weight reference) on the three 256^2 dose cases: relative L2 error
    to the phantom after `iters` outer iterations, and that of the FBP start."""
    import synth
    from paper_1009_1351_amd import Recon
    out = {}
    for n in ("C2a", "C2b", "C2c"):
        c = synth.make_case(n, K=iters)
        y = torch.from_numpy(c.y.astype(np.float32)).to(dev)
        w = torch.from_numpy(c.w.astype(np.float32)).to(dev)
        truth = torch.from_numpy(c.truth.astype(np.float32)).to(dev)
        rc = Recon.from_geometry(c.geom, patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat, max_outer=iters)

        def err(f):
            return float(torch.linalg.vector_norm(f - truth) / torch.linalg.vector_norm(truth))
        e_fbp = err(rc.fbp(y))
        fa, _, _, _ = rc.solve(y, w)
        e_a = err(fa)
        rc.set_guide(truth)
        fs, _, _, _ = rc.solve(y, w)
        e_s = err(fs)
        rc.set_guide(None)
        out[n] = {"fbp_all": e_fbp, "adaptive": e_a, "fixed_from_phantom": e_s}
    return {"iters": iters, "rel_l2_error_to_phantom": out}


def quality_leg(torch, dev, iters=50):
    """Image quality of the three 256^2 dose cases in the layout of the
    paper's tables: mean over phases of the CNR of the two regions (Eq. 10)
    and of the SNR (Eq. 11), for FBP of each phase's own views, FBP of all
    phases' views, and TNLM after `iters` outer iterations."""
    import synth
    from synth import quality
    from paper_1009_1351_amd import Recon
    out = {}
    for n in ("C2a", "C2b", "C2c"):
        c = synth.make_case(n, K=iters)
        y = torch.from_numpy(c.y.astype(np.float32)).to(dev)
        w = torch.from_numpy(c.w.astype(np.float32)).to(dev)
        rc = Recon.from_geometry(c.geom, patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat, max_outer=iters)
        host = lambda t: t.cpu().numpy().astype(np.float64)   # noqa: E731
        f_ph = host(rc.fbp(y, all_phases=False))
        f_all = host(rc.fbp(y, all_phases=True))
        f_tnlm = host(rc.solve(y, w)[0])
        out[n] = {"fbp_per_phase": quality.report(f_ph, c), "fbp_all_phases": quality.report(f_all, c),
                  "tnlm": quality.report(f_tnlm, c)}
    return {"iters": iters, "cases": out}


# ------------------------------------------------------- profile summaries
KIND_OF = {"k_project<": "project", "k_backproject(": "backproject", "k_tnlm_reg<": "regularize",
           "k_tnlm_reg_mfma<": "regularize_bf16", "k_tnlm_sym<": "regularize", "k_tnlm_sym_finish": "regularize_finish",
           "k_transpose(": "transpose"}


def kind_of(name):
    for k, v in KIND_OF.items():
        if k in name:
            return v
    return None


def _one(d, pat):
    import glob
    f = glob.glob(os.path.join(d, "**", pat), recursive=True)
    if not f:
        raise SystemExit(f"no {pat} under {d}")
    return f[0]


def summarize_profiles(kt_dir, fetch_dir, write_dir, command, counters_command, bench_json):
    """Write profiles/kernels_c3_batch.md, profiles/traffic_c3_batch.md and
    profiles/traffic.json from rocprofv3 CSV output (kernel stats, and two
    counter runs: FETCH_SIZE, WRITE_SIZE, in KiB per dispatch)."""
    import csv
    from collections import defaultdict

    rows = list(csv.DictReader(open(_one(kt_dir, "*kernel_stats.csv"))))
    bj = json.loads(open(bench_json).read().strip().splitlines()[-1])
    out = ["# Kernel time, 64-slice mixed batch (L 128-512, 40-360 views, B 1.5 L; one batched 50-iteration "
           "solve per step)", "", "Command (repository root):", "", "    " + command, "",
           "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[:16]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    kind_ns = defaultdict(lambda: [0.0, 0])
    for r in rows:
        k = kind_of(r["Name"])
        if k == "regularize_finish":   # the symmetric regulariser's second kernel: one launch with the first
            kind_ns["regularize"][0] += float(r["TotalDurationNs"])
        elif k:
            kind_ns[k][0] += float(r["TotalDurationNs"])
            kind_ns[k][1] += int(r["Calls"])
    out += ["", "Average per launch by kind (all template instances; the symmetric regulariser's two kernels "
                "as one launch), against the HIP-event figures that bench.py measured in the same run:", "",
            "| kind | launches | avg ms (trace) | avg ms (HIP events) |", "|---|---|---|---|"]
    rk = bj.get("roofline_kernels", {})
    for k, (ns, n) in sorted(kind_ns.items()):
        ev = rk.get(k, {}).get("avg_launch_ms")
        out.append(f"| {k} | {n} | {ns / n / 1e6:.4f} | {ev if ev is not None else '-'} |")
    rf = bj.get("roofline", {})
    out += ["", f"bench.py roofline kernel: {rf.get('kernel')}, avg launch {rf.get('avg_launch_ms')} ms "
                f"(HIP events), frac {rf.get('frac')} of {rf.get('peak')} {rf.get('unit')}.", "",
            "The bench line of that run:", "", "    " + json.dumps(bj), ""]
    open(os.path.join(ROOT, "profiles", "kernels_c3_batch.md"), "w").write("\n".join(out))

    def counters(d):
        per = defaultdict(list)
        for r in csv.DictReader(open(_one(d, "*counter_collection.csv"))):
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return per

    fe, wr = counters(fetch_dir), counters(write_dir)
    copy_bytes = 64 * 1024 * 1024 * 4
    cf = copy_bytes / 1024 / max(v for k, vs in fe.items() if "copyBuffer" in k for v in vs)
    cw = copy_bytes / 1024 / max(v for k, vs in wr.items() if "copyBuffer" in k for v in vs)
    out = ["# HBM traffic per dispatch, 64-slice mixed batch", "",
           "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two counter runs:", "",
           "    " + counters_command.replace("COUNTER", "FETCH_SIZE").replace("DIR", "fetch"),
           "    " + counters_command.replace("COUNTER", "WRITE_SIZE").replace("DIR", "write"), "",
           f"Calibration: a 256 MiB device-to-device copy in the same runs reads as "
           f"{copy_bytes / 1024 / cf:.1f} KiB fetched and {copy_bytes / 1024 / cw:.1f} KiB written, "
           f"so fetch counts are scaled by {cf:.4f} and write counts by {cw:.4f}.", "",
           "| kernel | dispatches | fetch KiB (raw) | write KiB (raw) | scaled MB / dispatch |", "|---|---|---|---|---|"]
    by_kind = defaultdict(lambda: [0.0, 0])
    for k in fe:
        if k not in wr or "tnlm::" not in k:
            continue
        f_ = sum(fe[k]) / len(fe[k])
        w_ = sum(wr[k]) / len(wr[k])
        b = (f_ * cf + w_ * cw) * 1024
        out.append(f"| `{k[:80]}` | {len(fe[k])} | {f_:.1f} | {w_:.1f} | {b / 1e6:.2f} |")
        kd = kind_of(k)
        if kd:
            by_kind[kd][0] += b * len(fe[k])
            by_kind[kd][1] += len(fe[k])
    tj = {}
    for kd, (b, n) in by_kind.items():
        if kd in KERNEL_SOURCES:
            tj[kd] = {"source_hash": source_hash(KERNEL_SOURCES[kd]), "workload": WORKLOAD_KEY,
                      "bytes_per_launch": b / n}
    alg = {k: v.get("algorithmic_bytes_per_launch") for k, v in rk.items()}
    out += ["", "Per kind (dispatch-weighted mean, scaled bytes) against the algorithmic bytes per launch "
                "that bench.py counts:", "", "| kind | counted MB / launch | algorithmic MB / launch | ratio |",
            "|---|---|---|---|"]
    for k, v in sorted(tj.items()):
        a_ = alg.get(k)
        out.append(f"| {k} | {v['bytes_per_launch'] / 1e6:.2f} | {a_ / 1e6 if a_ else float('nan'):.2f} | "
                   f"{v['bytes_per_launch'] / a_ if a_ else float('nan'):.2f} |")
    out.append("")
    open(os.path.join(ROOT, "profiles", "traffic_c3_batch.md"), "w").write("\n".join(out))
    json.dump(tj, open(os.path.join(ROOT, "profiles", "traffic.json"), "w"), indent=1)


def summarize_counters(out_md, title, command, dirs):
    """A counter table from one or more rocprofv3 --pmc runs, written to
    profiles/<out_md>: per kernel kind, the mean per dispatch of each counter
    over the dispatches of full size (launches on the whole batch; set-up
    launches of the tile autotuner on one slice are left out), and derived
    figures:
      time       = GRBM_GUI_ACTIVE / 8 XCDs / 2.4 GHz
      VALU issue = SQ_INSTS_VALU / (256 CUs x time cycles): wave-wide VALU
                   instructions per CU per clock; the ceiling depends on the
                   mix (streams of independent FP32 FMAs reach 0.90, compare /
                   select / add 1.33, integer add / shift / xor 1.59)
      lanes      = SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU)
      MFMA busy  = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x time cycles): the
                   counter adds the busy cycles of every SIMD's matrix core (it
                   equals 16 cycles per 16x16x32 BF16 MFMA issued)
      LDS conflict cycles per LDS instruction = SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS"""
    import csv
    from collections import defaultdict
    rows = []
    for d in dirs:
        rows += list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    conv = {"k_conv_fwd": "conv_fwd", "k_conv_wgrad": "conv_wgrad"}

    def kind(name):
        return kind_of(name) or next((v for c, v in conv.items() if c in name), None)
    grid = defaultdict(int)
    for r in rows:
        k = kind(r["Kernel_Name"])
        if k:
            grid[k] = max(grid[k], int(r["Grid_Size"]))
    vals = defaultdict(lambda: defaultdict(list))
    for r in rows:
        k = kind(r["Kernel_Name"])
        if k and (k.startswith("conv") or int(r["Grid_Size"]) * 2 > grid[k]):
            vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for k in vals for c in vals[k]})
    out = [f"# {title}", "", "Commands (repository root):", ""] + ["    " + c for c in command.split(" ;; ")] + [
        "", "Mean per dispatch (full-size dispatches; all dispatches of the network kernels):", "",
        "| kind | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for k in sorted(vals):
        n = max(len(v) for v in vals[k].values())
        cells = [f"{np.mean(vals[k][c]):.4g}" if vals[k].get(c) else "-" for c in names]
        out.append(f"| {k} | {n} | " + " | ".join(cells) + " |")
    out += ["", "Derived (formulas in bench.py summarize_counters):", "",
            "| kind | time ms | VALU issue | lanes active | MFMA busy | LDS conflict cycles / LDS instr |",
            "|---|---|---|---|---|---|"]
    for k in sorted(vals):
        m = {c: float(np.mean(v)) for c, v in vals[k].items()}
        gui = m.get("GRBM_GUI_ACTIVE")
        cyc = gui / 8.0 if gui else None

        def frac(a, den):
            return f"{a / den:.3f}" if a is not None and den else "-"
        out.append(f"| {k} | {cyc / 2.4e6:.3f} | " if cyc else f"| {k} | - | ")
        out[-1] += " | ".join([
            frac(m.get("SQ_INSTS_VALU"), 256 * cyc if cyc else None),
            frac(m.get("SQ_THREAD_CYCLES_VALU"), 64 * m["SQ_ACTIVE_INST_VALU"] if m.get("SQ_ACTIVE_INST_VALU") else None),
            frac(m.get("SQ_VALU_MFMA_BUSY_CYCLES"), 1024 * cyc if cyc else None),
            frac(m.get("SQ_LDS_BANK_CONFLICT"), m.get("SQ_INSTS_LDS"))]) + " |"
    out.append("")
    open(os.path.join(ROOT, "profiles", out_md), "w").write("\n".join(out))


# --------------------------------------------------------------------- main
def roofline_entry(kind, ms_tot, launches, ops_per_launch, bytes_per_launch):
    achieved = ops_per_launch * launches / (ms_tot * 1e-3) / 1e12
    return {"bound": "alu", "kernel": kind, "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TOPS, 2),
            "unit": "TOP/s", "frac": round(achieved / PEAK_ALU_TOPS, 4),
            "avg_launch_ms": round(ms_tot / max(launches, 1), 4), "launches": launches,
            "algorithmic_ops_per_launch": ops_per_launch, "algorithmic_bytes_per_launch": bytes_per_launch,
            "traffic": traffic_for(kind)}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        # bench.py summarize KT_DIR FETCH_DIR WRITE_DIR BENCH_JSON "COMMAND" "COUNTERS_COMMAND"
        # (COUNTERS_COMMAND with COUNTER and DIR standing for the counter and its output folder)
        summarize_profiles(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[6], sys.argv[7], sys.argv[5])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-counters":
        # bench.py summarize-counters OUT_MD "TITLE" "COMMANDS (;; separated)" DIR [DIR ...]
        summarize_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=50, help="outer iterations per solve")
    ap.add_argument("--slices", type=int, default=C3_SLICES, help="slices of the mixed batch (64 = the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the C2, precision and warm-start legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the warm-start leg")
    ap.add_argument("--no-timing-pass", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--learned-slices", type=int, default=C5_EVAL_SLICES)
    ap.add_argument("--ssd-mode", default="fp32_sym", choices=("fp32", "bf16_mfma", "fp32_sym"),
                    help="regulariser of the timed batch: fp32_sym (default) forms each unordered phase pair's "
                         "weights once for both directions, fp32 each phase's two neighbours on its own, bf16_mfma "
                         "the distances on the matrix cores")
    ap.add_argument("--cnn", action="store_true", help="run only the network leg (for profiling)")
    ap.add_argument("--gen-workers", type=int, default=0, help="input generation processes (0: one per core, <= 16)")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 256 MiB device copy (counter scale)")
    ap.add_argument("--omega-star", action="store_true", help="also compare adaptive and phantom-derived weights")
    ap.add_argument("--quality", action="store_true", help="also report CNR and SNR of FBP and TNLM images")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(slices would shard across GPUs without communication)"}))
        sys.exit(2)

    if a.cnn:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        print(json.dumps({"cnn": cnn_leg(torch, dev)}), flush=True)
        return
    # inputs first, in worker processes, before anything touches the GPU
    t_gen = time.perf_counter()
    specs = [("C3", s, dict(K=a.iters)) for s in range(a.slices)]
    extras = not a.no_extras
    learned = extras and not a.no_learned and os.path.exists(WEIGHTS)
    if extras:
        specs += [(n, 0, {}) for n in ("C2a", "C2b", "C2c")] + [("C4", s, dict(K=10)) for s in range(4)]
    if learned:
        specs += [("C5eval", 20_000 + k, {}) for k in range(a.learned_slices)]
    allc = make_cases(specs, a.gen_workers or None)
    cases = allc[:a.slices]
    c2 = allc[a.slices:a.slices + 3] if extras else []
    c4 = allc[a.slices + 3:a.slices + 7] if extras else []
    c5 = allc[a.slices + 7:] if learned else []
    log(f"inputs generated ({len(allc)} slices, {time.perf_counter() - t_gen:.1f} s)")

    import torch
    from paper_1009_1351_amd import Batch

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    c0 = cases[0]
    kw = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat, m1=c0.m1, m2=c0.m2, max_outer=a.iters,
              tol=0.0, ssd_mode=a.ssd_mode, device=dev)
    bt = Batch([c.geom for c in cases], **kw)
    ys = [torch.from_numpy(c.y).to(dev) for c in cases]
    ws = [torch.from_numpy(c.w).to(dev) for c in cases]
    fs = bt.new_images()
    torch.cuda.synchronize()

    def step():
        _, iters, _, st, _ = bt.solve(ys, ws, fs)
        return sum(c.geom.n_phases * c.geom.L ** 2 * k for c, k in zip(cases, iters))

    for s in range(a.warmup):
        step()
        log(f"warmup {s + 1}/{a.warmup}")
    if a.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = 0
    for s in range(a.steps):
        units += step()
        log(f"step {s + 1}/{a.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = units / dt
    slices = len(cases) * a.steps
    out = {
        "metric": "phase-pixel*iters/s", "value": value, "unit": "phase-pixel*iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16" if a.ssd_mode == "bf16_mfma" else "f32",
        "data": "synthetic",
        "config": {"workload": f"mixed batch: {len(cases)} slices x 10 phases, L from {{128,256,384,512}}, 40-360 "
                               "views, 1.5 L bins, I0 1e4-1e6; patch 7, window 15, M1 3, M2 1; "
                               f"{a.iters} outer iterations from the FBP of all phases, one batched solve per step "
                               "(one outer iteration replayed as a HIP graph); regulariser "
                               + {"fp32_sym": "fp32 with the weights of each unordered phase pair formed once for "
                                              "both directions",
                                  "fp32": "fp32, each phase's two neighbours on their own",
                                  "bf16_mfma": "with bf16 MFMA patch distances"}[a.ssd_mode],
                   "slices_per_step": len(cases), "wall_s_per_slice": dt / slices,
                   "phase_pixel_iters_per_step": units // max(a.steps, 1), "parallelism": "single GPU"},
    }
    if not a.no_timing_pass:
        log("per-kernel timing pass ...")
        bt.timing(True)
        step()
        t = bt.timing_read()
        bt.timing(False)
        per_kind = {k: list(v) for k, v in t.items()}
        nz = sum(crossings(c.geom) for c in cases)
        npairs = sum(pairs(c.geom, c.window) for c in cases)
        nimg = sum(c.geom.n_phases * c.geom.L ** 2 for c in cases)
        nsino = sum(c.geom.n_phases * c.geom.n_views * c.geom.n_bins for c in cases)
        # algorithmic bytes per launch (FP32): projector reads the image and its
        # transposed copy and writes q (the residual launch also reads y and
        # sqrt(w) and writes r and sqrt(w) r); back-projector reads q and writes
        # the image; regulariser reads guide/value/g once and writes the output
        algo_bytes = {"project": 4.0 * (2 * nimg + 1.5 * nsino), "backproject": 4.0 * (nimg + nsino),
                      "regularize": 4.0 * 2 * nimg}
        algo_ops = {"project": nz * OPS_PER_CROSSING, "backproject": nz * OPS_PER_CROSSING,
                    "regularize": npairs * OPS_PER_PAIR}
        rk = {k: roofline_entry(k, per_kind[k][0], per_kind[k][1], algo_ops[k], algo_bytes[k])
              for k in algo_ops if per_kind[k][1]}
        dom = max(rk, key=lambda k: per_kind[k][0])
        out["roofline"] = rk[dom]
        out["roofline_kernels"] = rk
        out["kernel_ms_per_step"] = {k: round(v[0], 3) for k, v in per_kind.items()}
        out["kernel_ms_note"] = "one solve with per-launch HIP events (direct launches, no graph replay)"
    if extras:
        log("C2 leg ...")
        out["c2_batch"] = c2_leg(torch, dev, c2)
        log("precision leg ...")
        out["bf16_mfma"] = precision_leg(torch, dev, c4)
        log("network leg ...")
        out["cnn"] = cnn_leg(torch, dev)
        if learned:
            log(f"learned warm start leg ({len(c5)} slices) ...")
            out["learned_vs_plain"] = learned_vs_plain(torch, dev, c5)
        else:
            out["learned_vs_plain"] = None
    if a.quality:
        log("image quality ...")
        out["quality"] = quality_leg(torch, dev)
    if a.omega_star:
        log("fixed-weight reference ...")
        out["omega_star"] = omega_star_leg(torch, dev)
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cases)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
