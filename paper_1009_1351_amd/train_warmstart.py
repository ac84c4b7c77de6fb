"""Train and evaluate the learned warm start (command-line driver).

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


def eval_warm_vs_cold(net, cases, dev, tol=1e-4, max_outer=500):
    from paper_1009_1351_amd.recon import Batch, Recon
    from paper_1009_1351_amd.warmstart import warm_starts
    c0 = cases[0]
    kw = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat, max_outer=max_outer, tol=tol, device=dev)
    ys = [torch.from_numpy(np.asarray(c.y, np.float32)).to(dev) for c in cases]
    ws = [torch.from_numpy(np.asarray(c.w, np.float32)).to(dev) for c in cases]
    geoms = [c.geom for c in cases]
    cold_b = Batch(geoms, init="fbp", **kw)
    warm_b = Batch(geoms, init="user", **kw)
    recons = [Recon.from_geometry(g, patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat, device=dev)
              for g in geoms]
    # warm-up of the inference path (activation buffers at this size); the
    # solves themselves are long enough that graph capture is negligible
    net.forward(torch.stack([recons[0].fbp(ys[0], all_phases=False)]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fc, it_c, rel_c, st_c, _ = cold_b.solve(ys, ws)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    t0 = time.perf_counter()
    f1s, used = warm_starts(recons, ys, ws, net)
    fw, it_w, rel_w, st_w, _ = warm_b.solve(ys, ws, f1s)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    it_w = [k + 1 for k in it_w]   # the first outer iteration ran inside warm_starts
    diff = [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(fw, fc)]
    truth_err_c = [float(np.linalg.norm(f.cpu().numpy() - c.truth) / np.linalg.norm(c.truth)) for f, c in zip(fc, cases)]
    truth_err_w = [float(np.linalg.norm(f.cpu().numpy() - c.truth) / np.linalg.norm(c.truth)) for f, c in zip(fw, cases)]
    n = len(cases)
    return {
        "slices": n, "tol": tol,
        "cold": {"iters_mean": float(np.mean(it_c)), "iters": it_c, "wall_s_per_slice": t_cold / n,
                 "all_reached_tol": bool(all(s == 0 for s in st_c)), "last_rel": rel_c},
        "warm": {"iters_mean": float(np.mean(it_w)), "iters": it_w, "wall_s_per_slice": t_warm / n,
                 "all_reached_tol": bool(all(s == 0 for s in st_w)), "last_rel": rel_w, "warm_used": used},
        "final_rel_diff_warm_vs_cold": {"max": max(diff), "mean": float(np.mean(diff))},
        "rel_err_to_phantom": {"cold_mean": float(np.mean(truth_err_c)), "warm_mean": float(np.mean(truth_err_w))},
        "speedup_wall": (t_cold / n) / (t_warm / n),
    }


def main():
    import synth
    from paper_1009_1351_amd.warmstart import WarmStartNet, make_pairs, train
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--pair-tol", type=float, default=1e-4)
    ap.add_argument("--pair-max-outer", type=int, default=400)
    ap.add_argument("--pair-time", type=float, default=480.0, help="seconds budget for pair generation")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--train-time", type=float, default=420.0)
    ap.add_argument("--eval-slices", type=int, default=32)
    ap.add_argument("--eval-L", type=int, default=512)
    ap.add_argument("--eval-B", type=int, default=720)
    ap.add_argument("--eval-max-outer", type=int, default=500)
    ap.add_argument("--out", default="warmstart.ckpt")
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    net = WarmStartNet(phases=10, base=32, seed=a.seed)
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
    ev = [synth.make_case("C5eval", slice_index=10_000 + k, L=a.eval_L, B=a.eval_B) for k in range(a.eval_slices)]
    log("evaluation ...")
    report["eval"] = eval_warm_vs_cold(net, ev, dev, max_outer=a.eval_max_outer)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
