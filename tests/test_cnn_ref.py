"""Pins of the FP64 reference network (CPU): its gradient equals central finite
differences of its loss, and the initial-identity construction holds."""
import numpy as np

from oracle import cnn_ref


def test_reference_gradient_matches_finite_differences():
    P, b, H, n = 2, 8, 16, 1
    rng = np.random.default_rng(0)
    npar = cnn_ref.num_params(P, b)
    params = np.empty(npar)
    off = 0
    for ci, co, k, _ in cnn_ref.layers(P, b):
        m = co * ci * k * k
        params[off:off + m] = rng.standard_normal(m) * np.sqrt(2.0 / (ci * k * k))
        off += m
    params[off:] = rng.standard_normal(npar - off) * 0.05
    x = rng.uniform(0, 0.03, size=(n, P, H, H))
    t = rng.uniform(0, 0.03, size=(n, P, H, H))
    loss, g = cnn_ref.loss_and_grad(params, x, t, P, b, 50.0)
    idx = rng.choice(npar, size=40, replace=False)
    eps = 1e-6
    for i in idx:
        p1 = params.copy()
        p1[i] += eps
        p2 = params.copy()
        p2[i] -= eps
        fd = (cnn_ref.loss_and_grad(p1, x, t, P, b, 50.0)[0] - cnn_ref.loss_and_grad(p2, x, t, P, b, 50.0)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)) + 1e-7, (i, fd, g[i])


def test_reference_zero_head_is_identity():
    P, b, H = 3, 8, 8
    npar = cnn_ref.num_params(P, b)
    rng = np.random.default_rng(1)
    params = rng.standard_normal(npar) * 0.1
    ws, bs = cnn_ref.unpack(params, P, b)
    ws[-1][:] = 0.0
    bs[-1][:] = 0.0
    x = rng.uniform(0, 0.03, size=(2, P, H, H))
    loss, _ = cnn_ref.loss_and_grad(params, x, x, P, b, 50.0)
    assert loss == 0.0


def test_bf16_rounding_is_round_to_nearest_even():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265])
    r = cnn_ref.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 4 * 2 ** -8 and r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12
