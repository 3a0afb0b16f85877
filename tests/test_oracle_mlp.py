"""Pins of the oracle MLP: backward against central finite differences of
the loss (h = 1e-6, FP64), SiLU derivative, the zero-weight special case,
and one Adam step against its closed form."""
import numpy as np

from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init(1)
    p = p + rng.normal(size=p.size) * 0.05     # non-zero padding rows too
    x = np.zeros((7, 16))
    x[:, :9] = rng.normal(size=(7, 9))
    t = np.zeros((7, 16))
    t[:, :3] = rng.normal(size=(7, 3))
    y, act = mlp.forward(p, x)
    L, dy = mlp.mse(y, t)
    g = mlp.backward(p, x, act, dy)
    h = 1e-6
    for j in rng.choice(p.size, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (mlp.mse(mlp.forward(pp, x)[0], t)[0] - mlp.mse(mlp.forward(pm, x)[0], t)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, np.abs(g).max()), j


def test_silu_and_zero_network():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.silu_grad(z)).max() < 1e-8
    p = np.zeros(mlp.N_PARAMS)
    w = mlp.unpack(p)
    w["b4"][:] = np.arange(16)
    p = mlp.pack(w)
    y, _ = mlp.forward(p, np.ones((3, 16)))
    assert np.array_equal(y, np.tile(np.arange(16.0), (3, 1)))


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -2.0, 0.5])
    p, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    assert np.allclose(p, -0.1 * np.sign(g))
