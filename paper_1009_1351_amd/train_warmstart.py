"""Train and evaluate the learned warm start (command-line tool).

    python -m paper_1009_1351_amd.train_warmstart --pairs 2000 --out net.ckpt
    python -m paper_1009_1351_amd.train_warmstart --eval-only --ckpt net.ckpt

Training pairs are produced by the method: seeded 256^2 slices (60 views,
512 bins, I0 log-uniform in [1e4, 1e5]) solved with the batched engine to a
relative update of 1e-4; input = the per-phase FBP images, target = the
solution. Evaluation: 512^2 slices (60 views, 720 bins, I0 2e4) solved to
relative update 1e-4 from the cold start (FBP of all phases) and from the
warm start (network output, with the data-term fallback), reporting outer
iterations and wall seconds per slice for both, and the distance between
the two final images. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def eval_warm_vs_cold(net, cases, dev, tol=1e-4, max_outer=600, restart_after=64, coarse_max=50):
    """Plain (one slice at a time, cold start) against learned + batched
    (warm starts, one batched solve, cold restart of slices still above the
    tolerance after restart_after iterations) and against the coarse-to-fine
    start (same restart rule), on the same slices."""
    from paper_1009_1351_amd.recon import Batch, Recon
    from paper_1009_1351_amd.warmstart import LearnedSolver
    c0 = cases[0]
    prm = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat)
    ys = [torch.from_numpy(np.asarray(c.y, np.float32)).to(dev) for c in cases]
    ws = [torch.from_numpy(np.asarray(c.w, np.float32)).to(dev) for c in cases]
    geoms = [c.geom for c in cases]
    n = len(cases)
    # warm-up: inference buffers at this size, one plain solve
    net.forward(torch.stack([Recon.from_geometry(geoms[0], device=dev, **prm).fbp(ys[0], all_phases=False)]),
                factor=net.factor_for(c0.geom.L))
    plain = [Recon.from_geometry(g, max_outer=max_outer, tol=tol, device=dev, **prm) for g in geoms]
    plain[0].solve(ys[0], ws[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_p = [rc.solve(y, w) for rc, y, w in zip(plain, ys, ws)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    fp = [r[0] for r in res_p]
    it_p = [r[1] for r in res_p]
    st_p = [r[3] for r in res_p]
    # batched cold (no network), to separate the two effects
    cold_b = Batch(geoms, init="fbp", max_outer=max_outer, tol=tol, device=dev, **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it_c, _, st_c, _ = cold_b.solve(ys, ws)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    cold_b.close()
    # contexts of both arms are built outside the timed regions
    solver = LearnedSolver(geoms, net, tol=tol, max_outer=max_outer, restart_after=restart_after, device=dev, **prm)
    solver.solve(ys, ws)   # warm-up (graph capture, inference buffers), like the plain arm's
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fl, it_l, st_l, used = solver.solve(ys, ws)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    solver.close()
    # coarse-to-fine start (half-resolution solve, upsampled), same restart rule
    from paper_1009_1351_amd.multigrid import MultigridSolver
    mg = MultigridSolver(geoms, tol=tol, max_outer=max_outer, restart_after=restart_after, coarse_max=coarse_max,
                         device=dev, **prm)
    mg.solve(ys, ws)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fm, it_m, it_mc, st_m = mg.solve(ys, ws)
    torch.cuda.synchronize()
    t_mg = time.perf_counter() - t0
    mg.close()
    diff = [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(fl, fp)]
    err_p = [float(np.linalg.norm(f.cpu().numpy() - c.truth) / np.linalg.norm(c.truth)) for f, c in zip(fp, cases)]
    err_l = [float(np.linalg.norm(f.cpu().numpy() - c.truth) / np.linalg.norm(c.truth)) for f, c in zip(fl, cases)]

    def arm(its, sts, t):
        conv = [k for k, s_ in zip(its, sts) if s_ == 0]
        return {"wall_s_per_slice": t / n, "iters_mean": float(np.mean(its)), "iters_median": float(np.median(its)),
                "reached_tol": len(conv), "iters": its}

    both = [j for j in range(n) if st_p[j] == 0 and st_l[j] == 0]
    return {
        "slices": n, "tol": tol, "max_outer": max_outer, "restart_after": restart_after,
        "plain": arm(it_p, st_p, t_plain),
        "batched_cold": arm(it_c, st_c, t_cold),
        "learned_batched": {**arm(it_l, st_l, t_learned), "warm_used": int(sum(used))},
        "speedup_learned_batched_vs_plain": t_plain / t_learned,
        "coarse_to_fine": {**arm(it_m, st_m, t_mg), "coarse_max": coarse_max, "coarse_iters_mean": float(np.mean(it_mc)),
                           "speedup_vs_plain": t_plain / t_mg},
        "on_slices_reaching_tol_in_both": {"count": len(both),
                                           "plain_iters_mean": float(np.mean([it_p[j] for j in both])) if both else None,
                                           "learned_iters_mean": float(np.mean([it_l[j] for j in both])) if both else None},
        "final_rel_diff_learned_vs_plain": {"max": max(diff), "mean": float(np.mean(diff))},
        "rel_err_to_phantom": {"plain_mean": float(np.mean(err_p)), "learned_mean": float(np.mean(err_l))},
    }


def main():
    import synth
    from paper_1009_1351_amd.warmstart import WarmStartNet, make_pairs, train
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--pair-tol", type=float, default=1e-4)
    ap.add_argument("--pair-max-outer", type=int, default=600)
    ap.add_argument("--pair-time", type=float, default=480.0, help="seconds budget for pair generation")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--train-time", type=float, default=420.0)
    ap.add_argument("--eval-slices", type=int, default=32)
    ap.add_argument("--eval-offset", type=int, default=10_000, help="first slice seed of the evaluation set")
    ap.add_argument("--eval-L", type=int, default=512)
    ap.add_argument("--eval-B", type=int, default=720)
    ap.add_argument("--eval-max-outer", type=int, default=600)
    ap.add_argument("--restart-after", type=int, default=64)
    ap.add_argument("--coarse-max", type=int, default=50, help="iteration cap of the coarse level (coarse-to-fine arm)")
    ap.add_argument("--out", default="warmstart.ckpt")
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    net = WarmStartNet(phases=10, base=32, seed=a.seed, train_L=synth.CONFIGS["C5train"]["L"])
    report = {"network": {"levels": 4, "base_channels": 32, "params": net.num_params}}
    if a.ckpt:
        if a.ckpt.endswith(".npz"):
            net.load_weights(a.ckpt)
        else:
            net.load(a.ckpt)
    if not a.eval_only:
        t0 = time.time()
        cases, X, T, its, rels = [], [], [], [], []
        chunk = 32
        s = 0
        while s < a.pairs and time.time() - t0 < a.pair_time:
            cs = [synth.make_case("C5train", slice_index=k) for k in range(s, min(s + chunk, a.pairs))]
            x, t, it, rl = make_pairs(cs, device=dev, chunk=chunk, tol=a.pair_tol, max_outer=a.pair_max_outer)
            X.append(x)
            T.append(t)
            its += it
            rels += rl
            s += len(cs)
            log(f"pairs {s} ({time.time() - t0:.0f} s, iterations {min(it)}..{max(it)})")
        X = torch.cat(X)
        T = torch.cat(T)
        report["pairs"] = {"count": int(X.shape[0]), "tol": a.pair_tol, "max_outer": a.pair_max_outer,
                           "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
                           "reached_tol": int(sum(r < a.pair_tol for r in rels)),
                           "last_rel_update_median": float(np.median(rels)),
                           "last_rel_update_max": float(max(rels)), "gen_s": time.time() - t0}
        t1 = time.time()
        hist = train(net, X, T, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log, time_limit_s=a.train_time)
        report["training"] = {"steps": len(hist), "loss_first": hist[0], "loss_last_mean": float(np.mean(hist[-20:])),
                              "train_s": time.time() - t1, "batch": a.batch}
        net.save(a.out)
        net.save_weights(os.path.splitext(a.out)[0] + "_weights.npz")
        log(f"saved {a.out}")
        del X, T
        torch.cuda.empty_cache()
    if a.eval_slices > 0:
        ev = [synth.make_case("C5eval", slice_index=a.eval_offset + k, L=a.eval_L, B=a.eval_B)
              for k in range(a.eval_slices)]
        log("evaluation ...")
        report["eval"] = eval_warm_vs_cold(net, ev, dev, max_outer=a.eval_max_outer, restart_after=a.restart_after,
                                           coarse_max=a.coarse_max)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
