"""Learned warm start for the TNLM solve (Python face of tnlm_cnn_*).

The network maps the N per-phase FBP images of a slice to an estimate of its
converged TNLM solution; that estimate replaces the FBP of all phases as
f^(0) of the TNLM algorithm box. It is trained on pairs the method itself
produces (per-phase FBP, TNLM solved to a relative-update tolerance). All
computation runs in the library's kernels; this module marshals arguments
and orchestrates.

Resolution: the network runs at the pixel size it was trained at; a slice
whose side is 2, 4 or 8 times the training side is averaged down to it and
the prediction upsampled bilinearly (tnlm_cnn_forward_resampled).

Fallback rule: two outer iterations are run from the network output and two
from the FBP of all phases; the warm branch is used for a slice only if its
iterates are finite and its relative update in the second iteration is not
larger than the cold branch's (a start nearer the fixed point moves less;
the first iteration is not used because it mostly removes the network's
high-frequency error). Otherwise the slice continues from the cold branch.
Either way the solve continues from the kept branch's second iterate.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import _native as nat
from ._native import TnlmError, check, check_cnn
from .recon import _norm_device


# outer iterations that warm_starts runs before handing the slices back
WARM_START_ITERS = 2


class WarmStartNet:
    def __init__(self, phases=10, base=32, seed=0, scale=50.0, train_L=None, device=None):
        self.device = _norm_device(device)
        self.phases, self.base, self.scale = int(phases), int(base), float(scale)
        self.train_L = train_L   # image side of the training pairs (None: run at any size as given)
        self._n = C.c_void_p()
        with torch.cuda.device(self.device):
            check_cnn(nat.lib.tnlm_cnn_create(C.byref(self._n), self.phases, self.base, int(seed), self.scale,
                                              C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))

    def close(self):
        if getattr(self, "_n", None) is not None and self._n.value:
            nat.lib.tnlm_cnn_destroy(self._n)
            self._n = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(nat.lib.tnlm_cnn_num_params(self._n))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, np.float32)
        check_cnn(nat.lib.tnlm_cnn_get_params(self._n, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        check_cnn(nat.lib.tnlm_cnn_set_params(self._n, p.ctypes.data_as(C.POINTER(C.c_float)), p.size))

    def _chk(self, x, name):
        if x.dtype != torch.float32 or x.device != self.device or x.dim() != 4 or not x.is_contiguous() \
                or x.shape[1] != self.phases:
            raise ValueError(f"{name} must be a contiguous float32 [n][{self.phases}][H][W] tensor on {self.device}")
        return C.c_void_p(x.data_ptr())

    def factor_for(self, L):
        """Down-sampling factor that brings side L to the training side (1 if none applies)."""
        if not self.train_L or L % self.train_L:
            return 1
        f = L // self.train_L
        return f if f in (1, 2, 4, 8) else 1

    def forward(self, x, out=None, factor=1):
        out = torch.empty_like(x) if out is None else out
        n, _, H, W = x.shape
        check_cnn(nat.lib.tnlm_cnn_forward_resampled(self._n, self._chk(x, "x"), self._chk(out, "out"), n, H, W,
                                                     int(factor)))
        return out

    def loss_grad(self, x, t, want_grad=True):
        n, _, H, W = x.shape
        loss = C.c_double(0.0)
        g = np.empty(self.num_params, np.float32) if want_grad else None
        check_cnn(nat.lib.tnlm_cnn_loss_grad(self._n, self._chk(x, "x"), self._chk(t, "t"), n, H, W, C.byref(loss),
                                             g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None,
                                             self.num_params if want_grad else 0))
        return loss.value, g

    def train_step(self, x, t, lr):
        n, _, H, W = x.shape
        loss = C.c_double(0.0)
        check_cnn(nat.lib.tnlm_cnn_train_step(self._n, self._chk(x, "x"), self._chk(t, "t"), n, H, W, float(lr),
                                              C.byref(loss)))
        return loss.value

    def save(self, path):
        """Full training checkpoint (parameters, Adam moments, step)."""
        check_cnn(nat.lib.tnlm_cnn_save(self._n, str(path).encode()))

    def save_weights(self, path):
        """Inference weights: convolution weights as BF16 bit patterns (the
        precision the network computes with) and biases as FP32, in an .npz."""
        p = self.get_params()
        nw = self._num_weights()
        bits = p[:nw].view(np.uint32)
        w16 = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)
        np.savez(path, w_bf16=w16, bias=p[nw:], meta=np.array([self.phases, self.base], np.int64),
                 scale=np.array([self.scale], np.float32), train_L=np.array([self.train_L or 0], np.int64))

    def load_weights(self, path):
        z = np.load(path, allow_pickle=False)
        meta = z["meta"]
        if int(meta[0]) != self.phases or int(meta[1]) != self.base or abs(float(z["scale"][0]) - self.scale) > 0:
            raise ValueError("weights are for a different network shape or input scale")
        w = (z["w_bf16"].astype(np.uint32) << 16).view(np.float32)
        self.set_params(np.concatenate([w, z["bias"].astype(np.float32)]))
        if "train_L" in z.files and int(z["train_L"][0]) > 0:
            self.train_L = int(z["train_L"][0])

    def _num_weights(self) -> int:
        b, P = self.base, self.phases
        chans = [(P, b, 3), (b, b, 3), (b, 2 * b, 3), (2 * b, 2 * b, 3), (2 * b, 4 * b, 3), (4 * b, 4 * b, 3),
                 (4 * b, 8 * b, 3), (8 * b, 8 * b, 3), (12 * b, 4 * b, 3), (4 * b, 4 * b, 3), (6 * b, 2 * b, 3),
                 (2 * b, 2 * b, 3), (3 * b, b, 3), (b, b, 3), (b, P, 1)]
        return sum(ci * co * k * k for ci, co, k in chans)

    def load(self, path):
        check_cnn(nat.lib.tnlm_cnn_load(self._n, str(path).encode()))


def data_cost(recon, y, w, f) -> float:
    out = C.c_double(0.0)
    check(nat.lib.tnlm_data_cost(recon._ctx, recon._sino(y, "y"), recon._sino(w, "w"), recon._img(f, "f"),
                                 C.byref(out)))
    return out.value


def rel_change(recon, a, b) -> float:
    """||a - b|| / ||a|| over the slice's image stack (raises TnlmError on non-finite values)."""
    out = C.c_double(0.0)
    check(nat.lib.tnlm_rel_change(recon._ctx, recon._img(a, "a"), recon._img(b, "b"), C.byref(out)))
    return out.value


def _second_move(rc, y, w, f):
    """Two outer iterations in place on f; returns the relative update of the second."""
    rc.step(y, w, f)
    prev = f.clone()
    rc.step(y, w, f)
    return rel_change(rc, f, prev)


def warm_starts(recons, ys, ws, net, batch=4):
    """Start images for each slice (list of Recon contexts of the slices'
    geometries), each WARM_START_ITERS outer iterations in: from the network
    estimate, or from the FBP of all phases when the fallback rule rejects
    it. Returns (images, used_warm flags)."""
    fbps = [rc.fbp(y, all_phases=False) for rc, y in zip(recons, ys)]
    outs = [None] * len(recons)
    # batched inference over slices of equal size
    order = sorted(range(len(recons)), key=lambda k: recons[k].L)
    k = 0
    while k < len(order):
        L = recons[order[k]].L
        grp = [j for j in order[k:k + batch] if recons[j].L == L]
        x = torch.stack([fbps[j] for j in grp])
        o = net.forward(x, factor=net.factor_for(L))
        for t, j in enumerate(grp):
            outs[j] = o[t].contiguous()
        k += len(grp)
    f_out, used = [], []
    for rc, y, w, o in zip(recons, ys, ws, outs):
        cold = rc.fbp(y, all_phases=True)
        m_cold = _second_move(rc, y, w, cold)
        try:
            m_warm = _second_move(rc, y, w, o)
            ok = m_warm <= m_cold
        except TnlmError:   # non-finite iterate
            ok = False
        f_out.append(o if ok else cold)
        used.append(ok)
    return f_out, used


class StartedSolver:
    """Solve of a fixed set of slices to a relative-update tolerance from given
    starting images, batched, with a cold restart (from the FBP of all phases,
    on the slice's own context) of slices that do not converge from them:

    * stall check (stall_window = m, stall_ratio = q): after 2m batched
      iterations, a slice above the tolerance whose relative update did not
      fall below q times its value m iterations earlier restarts at once (the
      outer iteration has settled into its period-2 cycle; converging slices
      contract by about 0.5 per 10 iterations); stall_window=None turns the
      check off;
    * a slice still above the tolerance after restart_after batched
      iterations restarts then.

    A restart gets max_outer - 2m cold iterations (a late restart can so take
    a slice past max_outer; the iterations are reported as taken). Contexts
    are built once, at construction. solve() returns (images, iterations
    counted from the start images, statuses)."""

    def __init__(self, geoms, *, patch, window, h, mu_hat, tol, max_outer, restart_after=None, stall_window=10,
                 stall_ratio=0.6, device=None):
        from .recon import Batch, Recon
        self.n = len(geoms)
        kw = dict(patch=patch, window=window, h=h, mu_hat=mu_hat, device=device)
        self.k1 = max_outer if restart_after is None else min(restart_after, max_outer)
        self.m = stall_window if stall_window and 2 * stall_window <= self.k1 else 0
        self.q = stall_ratio
        self.restart = self.k1 < max_outer or self.m > 0
        self.recons = [Recon.from_geometry(g, max_outer=max(max_outer - 2 * self.m, 1), tol=tol, **kw)
                       for g in geoms]
        self.seg = Batch(geoms, init="user", max_outer=self.m, tol=tol, **kw) if self.m else None
        rest = self.k1 - 2 * self.m
        self.rest = Batch(geoms, init="user", max_outer=rest, tol=tol, **kw) if rest > 0 else None

    def solve(self, ys, ws, fs):
        n = self.n
        iters, done, cont = [0] * n, [False] * n, [True] * n
        if self.seg is not None:
            fs, it1, r1, st1, _ = self.seg.solve(ys, ws, fs)
            act = [s_ != 0 for s_ in st1]
            fs, it2, r2, st2, _ = self.seg.solve(ys, ws, fs, active=act)
            for j in range(n):
                iters[j] = it1[j] + (it2[j] if act[j] else 0)
                done[j] = st1[j] == 0 or (act[j] and st2[j] == 0)
                stalled = act[j] and not done[j] and not (r2[j] < self.q * r1[j])
                cont[j] = not done[j] and not stalled
        if self.rest is not None and any(cont):
            fs, it3, _, st3, _ = self.rest.solve(ys, ws, fs, active=cont)
            for j in range(n):
                if cont[j]:
                    iters[j] += it3[j]
                    done[j] = st3[j] == 0
        st = [0 if d else 1 for d in done]
        if self.restart:
            for j in range(n):
                if not done[j]:
                    fs[j], kj, _, st[j] = self.recons[j].solve(ys[j], ws[j])
                    iters[j] += kj
        return fs, iters, st

    def close(self):
        for b in (self.seg, self.rest):
            if b is not None:
                b.close()
        for rc in self.recons:
            rc.close()


class LearnedSolver:
    """Learned + batched solve of a fixed set of slice geometries to a
    relative-update tolerance (contexts are built once, at construction):
    warm starts (warm_starts) for all slices, then StartedSolver from them
    (batched iterations, stall check, cold restart of the slices that do not
    converge from the warm start: the TNLM outer iteration can settle into a
    period-2 cycle instead of converging). Iterations are counted per slice
    from the first one."""

    def __init__(self, geoms, net, *, patch, window, h, mu_hat, tol, max_outer, restart_after=None, stall_window=10,
                 stall_ratio=0.6, device=None):
        self.net, self.n = net, len(geoms)
        self.inner = StartedSolver(geoms, patch=patch, window=window, h=h, mu_hat=mu_hat, tol=tol,
                                   max_outer=max_outer - WARM_START_ITERS, restart_after=restart_after,
                                   stall_window=stall_window, stall_ratio=stall_ratio, device=device)

    def solve(self, ys, ws, with_probe=False):
        """Returns (images, iterations, statuses, used_warm); iterations count
        the kept start's WARM_START_ITERS and those after it. The fallback
        check also runs WARM_START_ITERS iterations from the start it rejects:
        with_probe=True appends those per slice as a fifth element."""
        fs, used = warm_starts(self.inner.recons, ys, ws, self.net)
        fs, it, st = self.inner.solve(ys, ws, fs)
        out = (fs, [WARM_START_ITERS + k for k in it], st, used)
        return out + ([WARM_START_ITERS] * self.n,) if with_probe else out

    def close(self):
        self.inner.close()


def solve_learned(geoms, ys, ws, net, *, patch, window, h, mu_hat, tol, max_outer, restart_after=None, device=None):
    """One-shot LearnedSolver(...).solve(ys, ws); returns (images, iterations, statuses, used_warm)."""
    sol = LearnedSolver(geoms, net, patch=patch, window=window, h=h, mu_hat=mu_hat, tol=tol, max_outer=max_outer,
                        restart_after=restart_after, device=device)
    out = sol.solve(ys, ws)
    sol.close()
    return out


def make_pairs(cases, *, device, chunk=32, tol=1e-4, max_outer=400, patch=7, window=15, log=None):
    """Training pairs produced by the method: (per-phase FBP, TNLM solved to tol).
    Returns (inputs [n][N][L][L], targets [n][N][L][L]) on the device, the
    iterations taken and the last relative update of each slice."""
    from .recon import Batch, Recon
    xs, ts, its, rels = [], [], [], []
    for s0 in range(0, len(cases), chunk):
        cs = cases[s0:s0 + chunk]
        ys = [torch.from_numpy(np.asarray(c.y, np.float32)).to(device) for c in cs]
        wts = [torch.from_numpy(np.asarray(c.w, np.float32)).to(device) for c in cs]
        bt = Batch([c.geom for c in cs], patch=patch, window=window, h=cs[0].h, mu_hat=cs[0].mu_hat,
                   max_outer=max_outer, tol=tol, device=device)
        fs, iters, rel, sts, st = bt.solve(ys, wts)
        its += iters
        rels += rel
        for c, y, f in zip(cs, ys, fs):
            rc = Recon.from_geometry(c.geom, patch=patch, window=window, h=c.h, mu_hat=c.mu_hat, device=device)
            xs.append(rc.fbp(y, all_phases=False))
            ts.append(f)
        bt.close()
        if log:
            log(f"pairs {min(s0 + chunk, len(cases))}/{len(cases)} (iterations {min(iters)}..{max(iters)})")
    return torch.stack(xs), torch.stack(ts), its, rels


def train(net, X, T, *, epochs=4, batch=8, lr=1e-3, lr_final=1e-4, seed=0, log=None, time_limit_s=None):
    """Adam on the MSE of the network output against the targets; returns the loss history."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * max(1, n // batch)
    hist = []
    t0 = time.time()
    k = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        for b0 in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(perm[b0:b0 + batch], device=X.device)
            frac = k / max(1, steps - 1)
            cur = lr * (lr_final / lr) ** frac
            loss = net.train_step(X.index_select(0, idx).contiguous(), T.index_select(0, idx).contiguous(), cur)
            hist.append(loss)
            k += 1
            if time_limit_s is not None and time.time() - t0 > time_limit_s:
                break
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {np.mean(hist[-max(1, n // batch):]):.4e} ({time.time() - t0:.0f} s)")
        if time_limit_s is not None and time.time() - t0 > time_limit_s:
            break
    return hist


__all__ = ["WarmStartNet", "warm_starts", "StartedSolver", "LearnedSolver", "solve_learned", "make_pairs", "train", "data_cost", "rel_change",
           "WARM_START_ITERS"]
