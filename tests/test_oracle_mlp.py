"""Pins of the oracle's surrogate network: finite differences of the loss,
the SiLU derivative, exactness at kappa = 1, and the bfloat16 rounding rule."""
import numpy as np

from oracle import mlp


def test_dsilu_matches_finite_difference():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.dsilu(z))) < 1e-8


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    params = mlp.init_params(5)
    m = 16
    x = rng.uniform(-1, 1, (m, mlp.NFEAT))
    kd = rng.uniform(-0.2, 0.2, m)
    y = rng.normal(0, 0.3, m)
    loss, _, g = mlp.loss_and_grad(params, x, kd, y)
    # a few coordinates in every tensor
    offs, o = {}, 0
    for name, shape in mlp.SIZES:
        offs[name] = (o, int(np.prod(shape)))
        o += int(np.prod(shape))
    picks = []
    for name, (o0, n) in offs.items():
        idx = rng.integers(0, n, 3)
        if name == "W1":
            idx = np.array([r * 64 + c for r, c in zip(rng.integers(0, 256, 3), rng.integers(0, mlp.NFEAT, 3))])
        picks += [o0 + int(i) for i in idx]
    h = 1e-6
    for i in picks:
        pp = params.copy()
        pm = params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, kd, y)[0] - mlp.loss_and_grad(pm, x, kd, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_unused_input_columns_get_zero_gradient():
    rng = np.random.default_rng(4)
    params = mlp.init_params(6)
    x = rng.uniform(-1, 1, (8, mlp.NFEAT))
    _, _, g = mlp.loss_and_grad(params, x, rng.uniform(-.2, .2, 8), rng.normal(size=8))
    W1g = g[:256 * 64].reshape(256, 64)
    assert np.all(W1g[:, mlp.NFEAT:] == 0)


def test_prediction_vanishes_at_kappa_one():
    params = mlp.init_params(7)
    x = np.random.default_rng(5).uniform(-1, 1, (10, mlp.NFEAT))
    yhat, _ = mlp.forward(params, x, np.zeros(10))
    assert np.all(yhat == 0)


def test_bf16_rounding_rule():
    # exactly representable values stay; ties go to even; 1 + 2^-8 is a tie -> 1
    v = np.array([1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0])
    assert np.array_equal(mlp.bf16(v), [1.0, 1.0 + 2 ** -7, 1.0, 1.0 + 4 * 2 ** -8, -2.5, 0.0])
