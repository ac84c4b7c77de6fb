"""Helpers for the GPU parity tests: the same seeded inputs go to the HIP path
(float32 on the device) and to the FP64 oracle (the float32 values widened),
and results are compared per phase."""
import sys

import numpy as np

import synth


def rel_l2_per_phase(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    n = got.shape[0]
    out = []
    for i in range(n):
        den = np.linalg.norm(ref[i])
        out.append(np.linalg.norm(got[i] - ref[i]) / (den if den > 0 else 1.0))
    return np.array(out)


def f32(a):
    """Round to float32 and widen back: the value both sides see."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def recon_for(geom, **kw):
    from paper_1009_1351_amd import Recon
    return Recon.from_geometry(geom, **kw)


def announce(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def case_inputs(case):
    """(y, w) rounded to float32, as float64 arrays."""
    return f32(case.y), f32(case.w)


__all__ = ["rel_l2_per_phase", "f32", "to_dev", "to_host", "recon_for", "announce", "case_inputs", "synth"]
