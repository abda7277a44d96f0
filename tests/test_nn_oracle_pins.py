"""Pins of the warm-start network oracle (oracle/nn_oracle.py) against
library routines, exact identities and finite differences."""
import numpy as np
import pytest

from oracle import nn_oracle as N


def test_bf16_rounding_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, 3.0e38]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16(x), want)
    assert N.bf16(1 + 2 ** -8) == 1.0                 # halfway, even neighbour below
    assert N.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6     # halfway, even neighbour above


def test_conv3d_matches_scipy_correlate():
    nd = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(6)
    x = rng.standard_normal((6, 5, 7, 3))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    y = N.conv3d(x, w, b)
    for co in range(4):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            ref += nd.correlate(x[..., ci], w[co, :, :, :, ci], mode="constant", cval=0.0)
        assert np.allclose(y[..., co], ref, rtol=1e-13, atol=1e-12)


def test_conv3d_backward_is_the_adjoint():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((5, 6, 4, 3))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    dy = rng.standard_normal((5, 6, 4, 2))
    dx, dw, db = N.conv3d_backward(x, w, dy)
    lin = np.sum((N.conv3d(x, w, b) - b) * dy)
    assert np.isclose(lin, np.sum(x * dx), rtol=1e-12)      # linear in x
    assert np.isclose(lin, np.sum(w * dw), rtol=1e-12)      # linear in w
    assert np.allclose(db, dy.reshape(-1, 2).sum(axis=0), rtol=1e-13)


def test_pool_and_upsample_are_adjoint():
    rng = np.random.default_rng(8)
    a = rng.standard_normal((3, 2, 4, 5))
    c = rng.standard_normal((6, 4, 8, 5))
    assert np.isclose(np.sum(N.up2(a) * c), 8.0 * np.sum(a * N.pool2(c)), rtol=1e-13)
    assert np.allclose(N.pool2(N.up2(a)), a)


def _net(seed, cfg, n):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(N.n_params(cfg)) * 0.3
    x = rng.standard_normal((n, n, n, cfg["cin"]))
    return p, x


@pytest.mark.parametrize("cfg", [{"levels": 2, "ch": [4, 4], "cin": 2}, {"levels": 3, "ch": [3, 4, 5], "cin": 2}])
def test_network_gradient_matches_central_differences(cfg):
    p, x = _net(9, cfg, 8)
    rng = np.random.default_rng(10)
    out, cache = N.forward(p, x, cfg, rounding=False)
    dout = rng.standard_normal(out.shape)
    g = N.backward(p, cache, dout, cfg)
    idx = rng.choice(len(p), 40, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (np.sum(N.forward(pp, x, cfg, rounding=False)[0] * dout) -
              np.sum(N.forward(pm, x, cfg, rounding=False)[0] * dout)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mse_gradient_and_adam_first_step():
    rng = np.random.default_rng(11)
    o, t = rng.standard_normal(50), rng.standard_normal(50)
    loss, d = N.mse(o, t)
    assert np.isclose(loss, np.mean((o - t) ** 2))
    e = np.zeros(50)
    e[3] = 1e-6
    assert np.isclose((N.mse(o + e, t)[0] - N.mse(o - e, t)[0]) / 2e-6, d[3], rtol=1e-7)
    p, g = rng.standard_normal(20), rng.standard_normal(20)
    p1, m, v = N.adam(p, g, np.zeros(20), np.zeros(20), 1, 1e-3)
    # first step: bias-corrected moments are g and g^2
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_ramp_and_scale():
    grid = (8, 4, 4, 0.5, 0.5, 0.5)
    bc = {"kind": [0, 0, 1, 1, 1, 1], "value": [10.0, -30.0, 0, 0, 0, 0]}
    rho = np.ones((4, 4, 8))
    f, V = N.features(rho, grid, bc, 2.0)
    assert V == 30.0
    xc = (np.arange(8) + 0.5) * 0.5
    assert np.allclose(f[0, 0, :, 1], (10.0 - 40.0 * xc / 4.0) / 30.0)
    assert np.allclose(f[..., 0], 1.0 * 16.0 / (2.0 * 30.0))
