"""Writes the stored FP64-oracle results that the full-size GPU parity tests
compare against. Calls only the oracle (and the seeded input generators);
nothing here comes from the HIP path.

    python tests/golden/make_golden.py [name ...]      (default: all)

Names and what each file holds (float32 images, float64 histories):
  c2a, c2b, c2c   the 256^2 paper-size slice in its three dose cases, 50 outer
                  iterations from the FBP of all phases (TNLM algorithm box)
  sweep256        one regulariser sweep (Eq. 8 weights over a 15x15 window of
                  phases i+-1 with 7x7 patches, one Gauss-Jacobi sweep of
                  Eq. 7, positivity) of a 10 x 256^2 stack
  c3s6, c3s34,    four slices of the 64-slice mixed batch, one per image side
  c3s4, c3s16     (128^2 with 48 views, 256^2 with 56, 384^2 with 61, 512^2
                  with 48; bins 1.5 L), 50 outer iterations
  c4s0            slice 0 of the 512^2 precision workload (120 views x 720
                  bins), 50 outer iterations
  c1tol           the 64^2 workload solved from the FBP of all phases until
                  the relative update falls below 1e-4 (cap 400 iterations)

Both sides see the same float32-rounded inputs and parameters: y, w and the
regulariser input are rounded to float32 and widened, h and mu_hat likewise.
The arrays are stored byte-plane shuffled (the four bytes of every float32 in
four planes) and deflated, which roughly halves the size of smooth images.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

SWEEP_SEED = 20260301
SWEEP_NOISE = 1e-3

TRAJECTORIES = {
    "c2a": ("C2a", 0),
    "c2b": ("C2b", 0),
    "c2c": ("C2c", 0),
    "c3s6": ("C3", 6),
    "c3s34": ("C3", 34),
    "c3s4": ("C3", 4),
    "c3s16": ("C3", 16),
    "c4s0": ("C4", 0),
    "c1tol": ("C1", 0),
}
TOLERANCES = {"c1tol": (1e-4, 400)}   # (relative-update tolerance, iteration cap) of solves run to a tolerance


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def pack(a: np.ndarray) -> np.ndarray:
    """float32 array -> uint8 byte planes [4][n]."""
    b = np.ascontiguousarray(a, dtype="<f4").view(np.uint8).reshape(-1, 4)
    return np.ascontiguousarray(b.T)


def unpack(planes: np.ndarray, shape) -> np.ndarray:
    return np.ascontiguousarray(planes.T).view("<f4").reshape(shape)


def sweep_input():
    """A 10 x 256^2 stack: the C2 phantom plus seeded Gaussian noise (sigma
    1e-3 / mm), rounded to float32."""
    case = synth.make_case("C2c")
    rng = np.random.Generator(np.random.PCG64(SWEEP_SEED))
    return case, f32(case.truth + SWEEP_NOISE * rng.standard_normal(case.truth.shape))


def path(name):
    return os.path.join(HERE, f"{name}.npz")


def load(name):
    """{'f': float32 images, other keys as stored} of a stored result."""
    z = np.load(path(name), allow_pickle=False)
    out = {k: z[k] for k in z.files if k not in ("f_planes", "shape")}
    out["f"] = unpack(z["f_planes"], tuple(z["shape"]))
    return out


def make_trajectory(name):
    config, s = TRAJECTORIES[name]
    case = synth.make_case(config, slice_index=s)
    y, w = f32(case.y), f32(case.w)
    tol, cap = TOLERANCES.get(name, (case.tol, case.max_outer))
    prm = oracle.case_params(case, h=float(np.float32(case.h)), mu_hat=float(np.float32(case.mu_hat)), tol=tol,
                             max_outer=cap)
    t0 = time.perf_counter()
    f, k, rel, hist = oracle.solve(oracle.Geometry(case.geom), prm, y, w)
    dt = time.perf_counter() - t0
    f = f.astype(np.float32)
    np.savez_compressed(path(name), f_planes=pack(f), shape=np.array(f.shape), hist=hist, iters=np.int32(k),
                        config=np.array(config), slice_index=np.int32(s), oracle_seconds=np.float64(dt))
    print(f"{name}: {config} slice {s}, L {case.geom.L}, {k} iterations, last update {rel:.3e}, {dt:.0f} s",
          flush=True)


def make_sweep():
    case, g = sweep_input()
    h32, mu32 = float(np.float32(case.h)), float(np.float32(case.mu_hat))
    t0 = time.perf_counter()
    out = oracle.regularize(g, g, g, case.patch, case.window, h32, mu32, clamp=True).astype(np.float32)
    dt = time.perf_counter() - t0
    np.savez_compressed(path("sweep256"), f_planes=pack(out), shape=np.array(out.shape),
                        oracle_seconds=np.float64(dt))
    print(f"sweep256: {dt:.0f} s", flush=True)


def main(names):
    oracle.build()
    for n in names:
        if n == "sweep256":
            make_sweep()
        elif n in TRAJECTORIES:
            make_trajectory(n)
        else:
            raise SystemExit(f"unknown golden {n!r}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["sweep256", "c2c", "c2b", "c3s6", "c3s34", "c2a", "c4s0", "c1tol", "c3s4", "c3s16"])
