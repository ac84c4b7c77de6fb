#!/usr/bin/env python
"""Benchmark of the TNLM 4DCT reconstruction hot path on one MI355X.

Timed step: the 256x256 paper-size slice in its three dose cases, solved
together as one batch by the batched engine -- FBP of all phases' views, then
50 outer iterations of (3 CGLS steps -> patch weights over a 15x15 window of
phases i+-1 with 7x7 patches -> one Gauss-Jacobi sweep -> positivity):
    a: 360 views/phase, I0 = 2e4     b: 60 views/phase, I0 = 1e6
    c: 60 views/phase, I0 = 2e4      (10 phases, 512 bins, fan-beam arc)
Inputs are seeded synthetic phantoms (nested ellipses, moving tumour,
analytic line integrals, Poisson noise) resident in HBM before timing.

Metric: phase-pixel*iterations per second = sum over slices of N*L^2*K / wall
seconds. Also reported: the same workload with BF16-MFMA patch distances,
and -- when trained warm-start weights are present -- wall seconds per
10-phase slice to a relative update of 1e-4 for the learned warm start +
batched engine and for the coarse-to-fine start, against the plain path
(cold start, one slice at a time).
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


_COMMON = ["paper_1009_1351_amd/csrc/internal.h", "paper_1009_1351_amd/csrc/devutil.h"]
KERNEL_SOURCES = {
    "backproject": ["paper_1009_1351_amd/csrc/proj.hip"] + _COMMON,
    "project": ["paper_1009_1351_amd/csrc/proj.hip"] + _COMMON,
    "regularize": ["paper_1009_1351_amd/csrc/tnlm_reg.hip"] + _COMMON,
}   # a change to these files invalidates the stored traffic figures


def traffic_for(kernel: str):
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


def learned_vs_plain(torch, dev, n_slices, tol=1e-4, restart_after=64):
    """Wall seconds per slice to tol: plain (cold start, one slice at a time)
    against the learned warm start + batched engine, on 512^2 slices."""
    import synth
    from paper_1009_1351_amd import Recon
    from paper_1009_1351_amd.warmstart import LearnedSolver, WarmStartNet
    net = WarmStartNet(phases=10, base=32)
    net.load_weights(WEIGHTS)
    cases = [synth.make_case("C5eval", slice_index=20_000 + k) for k in range(n_slices)]
    c0 = cases[0]
    prm = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat)
    ys = [torch.from_numpy(np.asarray(c.y, np.float32)).to(dev) for c in cases]
    ws = [torch.from_numpy(np.asarray(c.w, np.float32)).to(dev) for c in cases]
    plain = [Recon.from_geometry(c.geom, max_outer=c0.max_outer, tol=tol, device=dev, **prm) for c in cases]
    solver = LearnedSolver([c.geom for c in cases], net, tol=tol, max_outer=c0.max_outer, restart_after=restart_after,
                           device=dev, **prm)
    plain[0].solve(ys[0], ws[0])   # warm-up of both paths
    solver.solve(ys, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [rc.solve(y, w) for rc, y, w in zip(plain, ys, ws)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it_l, st_l, used = solver.solve(ys, ws)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    solver.close()
    from paper_1009_1351_amd.multigrid import MultigridSolver
    mg = MultigridSolver([c.geom for c in cases], tol=tol, max_outer=c0.max_outer, restart_after=restart_after,
                         device=dev, **prm)
    mg.solve(ys, ws)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it_m, it_mc, st_m = mg.solve(ys, ws)
    torch.cuda.synchronize()
    t_mg = time.perf_counter() - t0
    mg.close()
    return {"workload": f"{n_slices} slices x 10 phases, 512^2, 60 views x 720 bins, I0 2e4, h_rel 0.6, "
                        f"to relative update {tol} (cap {c0.max_outer})",
            "plain_wall_s_per_slice": t_plain / n_slices, "plain_iters": [r[1] for r in res],
            "learned_batched_wall_s_per_slice": t_learned / n_slices, "learned_iters": it_l,
            "warm_start_used": int(sum(used)), "plain_reached_tol": int(sum(r[3] == 0 for r in res)),
            "learned_reached_tol": int(sum(s_ == 0 for s_ in st_l)), "speedup": t_plain / t_learned,
            "multigrid_wall_s_per_slice": t_mg / n_slices, "multigrid_iters": it_m, "multigrid_coarse_iters": it_mc,
            "multigrid_reached_tol": int(sum(s_ == 0 for s_ in st_m)), "multigrid_speedup": t_plain / t_mg}


def batched_legs(torch, dev, n_c3, n_c4, iters=10):
    """Optional legs on the batched and precision workloads: a ragged batch of
    n_c3 slices (L from {128..512}, 40-360 views, B = 1.5 L) solved as one
    batch (graph replay, no per-kernel events) against the same slices solved
    one at a time; and n_c4 slices at 512^2 (720 bins, 120 views) with the
    FP32 and the BF16-MFMA regulariser."""
    import synth
    from paper_1009_1351_amd import Batch, Recon
    out = {}

    def arrays(cases):
        return ([torch.from_numpy(c.y.astype(np.float32)).to(dev) for c in cases],
                [torch.from_numpy(c.w.astype(np.float32)).to(dev) for c in cases])

    def make(name, n):
        cases = []
        for s in range(n):
            cases.append(synth.make_case(name, slice_index=s, K=iters))
            if (s + 1) % 8 == 0 or s + 1 == n:
                log(f"{name}: {s + 1}/{n} slices generated")
        return cases

    if n_c3:
        cases = make("C3", n_c3)
        ys, ws = arrays(cases)
        kw = dict(patch=7, window=15, h=cases[0].h, mu_hat=cases[0].mu_hat, max_outer=iters, tol=0.0, device=dev)
        units = sum(c.geom.n_phases * c.geom.L ** 2 * iters for c in cases)
        bt = Batch([c.geom for c in cases], **kw)
        bt.solve(ys, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.solve(ys, ws)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        bt.close()
        rcs = [Recon.from_geometry(c.geom, **kw) for c in cases]
        rcs[0].solve(ys[0], ws[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for rc, y, w in zip(rcs, ys, ws):
            rc.solve(y, w)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        log(f"C3: batched {tb:.2f} s, one at a time {tp:.2f} s")
        out["batched_c3"] = {"slices": n_c3, "iters": iters, "shapes": [[c.geom.L, c.geom.n_views, c.geom.n_bins]
                                                                        for c in cases],
                             "batched_value": units / tb, "one_at_a_time_value": units / tp, "unit": "phase-pixel*iters/s"}
    if n_c4:
        cases = make("C4", n_c4)
        ys, ws = arrays(cases)
        res = {}
        for mode in ("fp32", "bf16_mfma"):
            bt = Batch([c.geom for c in cases], patch=7, window=15, h=cases[0].h, mu_hat=cases[0].mu_hat,
                       max_outer=iters, tol=0.0, ssd_mode=mode, device=dev)
            bt.solve(ys, ws)
            bt.timing(True)
            t0 = time.perf_counter()
            bt.solve(ys, ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            t = bt.timing_read()
            bt.close()
            units = sum(c.geom.n_phases * c.geom.L ** 2 * iters for c in cases)
            res[mode] = {"value": units / dt, "regularize_ms_per_launch": t["regularize"][0] / max(t["regularize"][1], 1)}
        out["precision_c4"] = {"slices": n_c4, "iters": iters, **res}
    return out


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


KIND_OF = {"k_project<": "project", "k_backproject(": "backproject", "k_tnlm_reg<": "regularize",
           "k_tnlm_reg_mfma<": "regularize_bf16", "k_transpose(": "transpose"}


def kind_of(name):
    for k, v in KIND_OF.items():
        if k in name:
            return v
    return None


def summarize_profiles(kt_dir, fetch_dir, write_dir, command, counters_command, bench_json):
    """Write profiles/kernels_c2_batch.md, profiles/traffic_c2_batch.md and
    profiles/traffic.json from rocprofv3 CSV output (kernel stats, and two
    counter runs: FETCH_SIZE, WRITE_SIZE, in KiB per dispatch)."""
    import csv
    import glob
    from collections import defaultdict

    def one(d, pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        if not f:
            raise SystemExit(f"no {pat} under {d}")
        return f[0]

    rows = list(csv.DictReader(open(one(kt_dir, "*kernel_stats.csv"))))
    bj = json.loads(open(bench_json).read().strip().splitlines()[-1])
    out = ["# Kernel time, C2 batch (3 slices x 10 phases, 256^2, one batched solve per step)", "",
           "Command (repository root):", "", "    " + command, "",
           "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[:16]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    kind_ns = defaultdict(lambda: [0.0, 0])
    for r in rows:
        k = kind_of(r["Name"])
        if k:
            kind_ns[k][0] += float(r["TotalDurationNs"])
            kind_ns[k][1] += int(r["Calls"])
    out += ["", "Average per launch by kind (all template instances), against the HIP-event figure "
                "that bench.py measured in the same run:", "",
            "| kind | launches | avg ms (trace) |", "|---|---|---|"]
    for k, (ns, n) in sorted(kind_ns.items()):
        out.append(f"| {k} | {n} | {ns / n / 1e6:.4f} |")
    rf = bj.get("roofline", {})
    out += ["", f"bench.py roofline kernel: {rf.get('kernel')}, avg launch {rf.get('avg_launch_ms')} ms "
                f"(HIP events), frac {rf.get('frac')} of {rf.get('peak')} {rf.get('unit')}.", "",
            "The bench line of that run:", "", "    " + json.dumps(bj), ""]
    open(os.path.join(ROOT, "profiles", "kernels_c2_batch.md"), "w").write("\n".join(out))

    def counters(d):
        per = defaultdict(list)
        for r in csv.DictReader(open(one(d, "*counter_collection.csv"))):
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return per

    fe, wr = counters(fetch_dir), counters(write_dir)
    copy_bytes = 64 * 1024 * 1024 * 4
    cf = copy_bytes / 1024 / max(v for k, vs in fe.items() if "copyBuffer" in k for v in vs)
    cw = copy_bytes / 1024 / max(v for k, vs in wr.items() if "copyBuffer" in k for v in vs)
    out = ["# HBM traffic per dispatch, C2 batch", "",
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
            tj[kd] = {"source_hash": source_hash(KERNEL_SOURCES[kd]), "bytes_per_launch": b / n}
    out += ["", "Per kind (dispatch-weighted mean, scaled bytes): " +
            ", ".join(f"{k} {v['bytes_per_launch'] / 1e6:.2f} MB" for k, v in sorted(tj.items())), ""]
    open(os.path.join(ROOT, "profiles", "traffic_c2_batch.md"), "w").write("\n".join(out))
    json.dump(tj, open(os.path.join(ROOT, "profiles", "traffic.json"), "w"), indent=1)


def summarize_bf16(kt_dir, command):
    """profiles/regularize_bf16_c2_batch.md: FP32 and BF16-MFMA regulariser
    kernels of one traced run of both bench legs."""
    import csv
    import glob
    f = glob.glob(os.path.join(kt_dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = [r for r in csv.DictReader(open(f)) if kind_of(r["Name"]) in ("regularize", "regularize_bf16")]
    out = ["# Regulariser: FP32 box sums against BF16 MFMA patch distances, C2 batch", "",
           "Command (repository root):", "", "    " + command, "",
           "| kernel | calls | avg us |", "|---|---|---|"]
    for r in rows:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} |")
    avg = {kind_of(r["Name"]): float(r["AverageNs"]) for r in rows}
    if "regularize" in avg and "regularize_bf16" in avg:
        out += ["", f"BF16 MFMA / FP32 time per launch: {avg['regularize_bf16'] / avg['regularize']:.2f}", ""]
    open(os.path.join(ROOT, "profiles", "regularize_bf16_c2_batch.md"), "w").write("\n".join(out))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-bf16":
        summarize_bf16(sys.argv[2], sys.argv[3])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        # bench.py summarize KT_DIR FETCH_DIR WRITE_DIR BENCH_JSON "COMMAND" "COUNTERS_COMMAND"
        # (COUNTERS_COMMAND with COUNTER and DIR standing for the counter and its output folder)
        summarize_profiles(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[6], sys.argv[7], sys.argv[5])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=50, help="outer iterations per solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the BF16 and warm-start legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the warm-start leg")
    ap.add_argument("--learned-slices", type=int, default=4)
    ap.add_argument("--calib-copy", action="store_true", help="also run a 256 MiB device copy (counter scale)")
    ap.add_argument("--c3", type=int, default=0, help="also run a ragged batch of this many slices")
    ap.add_argument("--c4", type=int, default=0, help="also run this many 512^2 slices with both SSD modes")
    ap.add_argument("--omega-star", action="store_true", help="also compare adaptive and phantom-derived weights")
    ap.add_argument("--quality", action="store_true", help="also report CNR and SNR of FBP and TNLM images")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(slices would shard across GPUs without communication)"}))
        sys.exit(2)

    import torch
    import synth
    from paper_1009_1351_amd import Batch

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    names = ["C2a", "C2b", "C2c"]
    cases = [synth.make_case(n, K=a.iters) for n in names]
    log("inputs generated")
    c0 = cases[0]
    kw = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat, m1=c0.m1, m2=c0.m2, max_outer=a.iters,
              tol=0.0, device=dev)
    bt = Batch([c.geom for c in cases], **kw)
    ys = [torch.from_numpy(c.y.astype(np.float32)).to(dev) for c in cases]
    ws = [torch.from_numpy(c.w.astype(np.float32)).to(dev) for c in cases]
    fs = bt.new_images()
    torch.cuda.synchronize()

    def step(b):
        _, iters, _, st, _ = b.solve(ys, ws, fs)
        return sum(c.geom.n_phases * c.geom.L ** 2 * k for c, k in zip(cases, iters))

    for _ in range(a.warmup):
        step(bt)
    log("warmup done")
    if a.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    bt.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = 0
    for s in range(a.steps):
        units += step(bt)
        log(f"step {s + 1}/{a.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t = bt.timing_read()
    bt.timing(False)
    per_kind = {k: list(v) for k, v in t.items()}
    nz = sum(crossings(c.geom) for c in cases)
    npairs = sum(pairs(c) for c in cases)
    algo = {"project": t["project"][1] * nz * OPS_PER_CROSSING,
            "backproject": t["backproject"][1] * nz * OPS_PER_CROSSING,
            "regularize": t["regularize"][1] * npairs * OPS_PER_PAIR}
    dom = max(algo, key=lambda k: per_kind[k][0])
    ms_tot, launches = per_kind[dom]
    achieved = algo[dom] / (ms_tot * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TOPS, 2),
            "unit": "TOP/s", "frac": round(achieved / PEAK_ALU_TOPS, 4),
            "avg_launch_ms": round(ms_tot / max(launches, 1), 4),
            "algorithmic_ops_per_launch": algo[dom] / max(launches, 1),
            "traffic": traffic_for(dom)}
    value = units / dt
    slices = len(cases) * a.steps
    out = {
        "metric": "phase-pixel*iters/s", "value": value, "unit": "phase-pixel*iters/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "C2: 3 slices x 10 phases, 256x256, 512 bins, doses a (360 views, I0 2e4), "
                               "b (60 views, I0 1e6), c (60 views, I0 2e4) in one batch; patch 7, window 15, "
                               f"M1 3, M2 1; {a.iters} outer iterations from the FBP of all phases",
                   "slices_per_step": len(cases), "wall_s_per_slice": dt / slices, "parallelism": "single GPU"},
        "kernel_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in per_kind.items()},
        "roofline": roof,
    }
    if not a.no_extras:
        log("BF16-MFMA leg ...")
        bb = Batch([c.geom for c in cases], ssd_mode="bf16_mfma", **kw)
        step(bb)
        torch.cuda.synchronize()
        bb.timing(True)
        t0 = time.perf_counter()
        u = step(bb)
        torch.cuda.synchronize()
        d2 = time.perf_counter() - t0
        tb = bb.timing_read()
        out["bf16_mfma"] = {"value": u / d2, "regularize_ms_per_step": round(tb["regularize"][0], 3),
                            "fp32_regularize_ms_per_step": round(per_kind["regularize"][0] / a.steps, 3)}
        bb.close()
        if os.path.exists(WEIGHTS) and not a.no_learned:
            log("learned warm start leg ...")
            out["learned_vs_plain"] = learned_vs_plain(torch, dev, a.learned_slices)
        else:
            out["learned_vs_plain"] = None
    if a.quality:
        log("image quality ...")
        out["quality"] = quality_leg(torch, dev)
    if a.omega_star:
        log("fixed-weight reference ...")
        out["omega_star"] = omega_star_leg(torch, dev)
    if a.c3 or a.c4:
        log("batched / precision legs ...")
        out.update(batched_legs(torch, dev, a.c3, a.c4))
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(lambda n: synth.make_case(n, K=a.iters))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
