"""Pins of the FP64 surrogate oracle: its chain-rule gradient against central
finite differences, Adam's first step in closed form, BF16 rounding on
values with known answers, and the ensemble statistics."""
import numpy as np

from oracle import mlp_oracle as mo


def _rand(H=8, n=13, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.5, mo.n_params(H))
    X = rng.normal(0, 1, (n, 4))
    Y = rng.normal(0, 1, (n, 2))
    return theta, X, Y


def test_param_count():
    assert mo.n_params(128) == 17410


def test_gradient_matches_finite_differences():
    H = 8
    theta, X, Y = _rand(H)
    g = mo.grad(theta, X, Y, H)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (mo.loss(theta + e, X, Y, H) - mo.loss(theta - e, X, Y, H)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.abs(fd).max())


def test_adam_first_step_is_signed_lr():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = mo.adam(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -7), 3.0e-3])
    r = mo.bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2.0 ** -6 and r[3] == -(1 + 2.0 ** -7)
    assert abs(r[4] - 3.0e-3) <= 2.0 ** -8 * 3.0e-3


def test_ensemble_statistics():
    H = 8
    theta, X, _ = _rand(H)
    mu, sd, fb = mo.ensemble([theta, theta, theta], X, H, 0.05)
    assert np.allclose(sd, 0.0) and not fb.any()
    y0 = mo.forward_bf16(theta, X, H)
    assert np.allclose(mu, y0)
    other = theta.copy()
    other[-2:] += 10.0                    # shift the output biases of one member
    mu, sd, fb = mo.ensemble([theta, other], X, H, 0.05)
    assert np.allclose(sd, 5.0) and fb.all()


def test_ensemble_in_caller_units():
    """Outputs mapped to the caller's units before the statistics: the mean
    maps affinely, the spread scales by |scale|, and the fallback test is
    relative to the mapped mean (a network trained on normalised targets has
    means near zero, where a relative test on its raw outputs always fails)."""
    H = 8
    theta, X, _ = _rand(H)
    other = theta.copy()
    other[-2:] += 0.02                    # two members 0.02 apart on both raw outputs
    mu0, sd0, fb0 = mo.ensemble([theta, other], X, H, 0.05)
    scale, shift = np.array([0.5, -2.0]), np.array([3.0, 7.0])
    mu, sd, fb = mo.ensemble([theta, other], X, H, 0.05, out_scale=scale, out_shift=shift)
    assert np.allclose(mu, mu0 * scale + shift) and np.allclose(sd, sd0 * np.abs(scale))
    assert np.allclose(sd0, 0.01)
    # raw: spread 0.01 against means of the size of the raw outputs; mapped:
    # 0.005 and 0.02 against means near 3 and 7, far below 5%
    assert not fb.any()
    small = np.abs(mu0).min(axis=1) < 0.2
    assert small.any() and fb0[small].all()
