"""Pins of the learned-guess reference (oracle/guess.py) against facts that do not depend on
its code: planted solutions of the two target fits, central finite differences of the network
loss, the closed form of Adam's first step, and hand-computed features."""
import numpy as np
import pytest

from oracle import guess


def _sym(rng, P):
    A = rng.standard_normal((P, P))
    return A + A.T


def test_fit_scaling_recovers_a_planted_scaling():
    """T* = diag(1+c) T0 diag(1+c) exactly: Gauss-Newton must return c (the fit is exact)."""
    rng = np.random.default_rng(11)
    for P in (1, 5, 40):
        T0 = _sym(rng, P)
        c = 0.2 * rng.standard_normal(P)
        Ts = (1.0 + c)[:, None] * T0 * (1.0 + c)[None, :]
        assert np.abs(guess.fit_scaling(T0, Ts) - c).max() < 1e-10


def test_fit_scaling_is_the_least_squares_minimum():
    """For a T* that is not an exact scaling, the gradient of ||diag(s) T0 diag(s) - T*||^2 in s
    vanishes at the fit (checked by central differences of the objective)."""
    rng = np.random.default_rng(12)
    P = 9
    T0 = _sym(rng, P)
    Ts = T0 * 1.1 + 0.05 * _sym(rng, P)
    c = guess.fit_scaling(T0, Ts)
    f = lambda cc: np.sum(((1 + cc)[:, None] * T0 * (1 + cc)[None, :] - Ts) ** 2)
    h = 1e-6
    grad = np.array([(f(c + h * np.eye(P)[k]) - f(c - h * np.eye(P)[k])) / (2 * h) for k in range(P)])
    assert np.abs(grad).max() < 1e-6 * max(1.0, f(c))


def test_fit_shift_recovers_a_planted_shift():
    """-sigma0 = (e_P + e_Q + d_P + d_Q) dT exactly: the secant fit must return d."""
    rng = np.random.default_rng(13)
    P = 30
    e = np.sort(rng.uniform(0.5, 6.0, P))
    T0 = _sym(rng, P)
    dT = 0.1 * _sym(rng, P)
    d = 0.2 * rng.standard_normal(P)
    sig0 = -(e[:, None] + e[None, :] + d[:, None] + d[None, :]) * dT
    assert np.abs(guess.fit_shift(e, T0, T0 + dT, sig0) - d).max() < 1e-8


def test_shifted_denominators_clamp():
    e = np.array([1.0, 2.0])
    d = np.array([-10.0, 0.5])
    D = guess.shifted_denominators(e, d)
    assert D[0, 0] == pytest.approx(1.0)          # 2 - 20 clamped to (1 + 1) / 2
    assert D[1, 1] == pytest.approx(5.0)          # 4 + 1
    assert D[0, 1] == pytest.approx(1.5)          # 3 - 9.5 clamped to 3 / 2
    assert np.array_equal(guess.shifted_denominators(e, None), e[:, None] + e[None, :])


def test_network_gradient_matches_central_differences():
    rng = np.random.default_rng(14)
    dims = (guess.N_FEAT, 12, guess.N_OUT)
    p = 0.4 * rng.standard_normal(guess.n_params(*dims))
    X = rng.standard_normal((9, dims[0]))
    T = rng.standard_normal((9, dims[2]))
    norm = (rng.standard_normal(dims[0]), rng.uniform(0.5, 2.0, dims[0]), rng.standard_normal(dims[2]),
            rng.uniform(0.5, 2.0, dims[2]))
    loss, g = guess.loss_and_grad(p, dims, X, T, norm)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd[k] = (guess.loss_and_grad(pp, dims, X, T, norm)[0] - guess.loss_and_grad(pm, dims, X, T, norm)[0]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-7 * np.abs(g).max()
    # the loss itself: mean squared error of standardized outputs, evaluated directly
    y, yn, _ = guess.forward(p, dims, X, norm)
    assert loss == pytest.approx(np.mean((yn - (T - norm[2]) / norm[3]) ** 2), rel=1e-14)
    assert np.allclose(y, yn * norm[3] + norm[2])


def test_silu_and_its_derivative():
    z = np.linspace(-8, 8, 101)
    assert np.allclose(guess.silu(z), z * 0.5 * (1 + np.tanh(z / 2)), rtol=1e-14, atol=1e-15)
    h = 1e-6
    assert np.allclose(guess.silu_prime(z), (guess.silu(z + h) - guess.silu(z - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_closed_form():
    """With zero moments, bias correction makes the first step -lr g / (|g| + eps)."""
    rng = np.random.default_rng(15)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = guess.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(p1 - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_of_a_small_state():
    Th0 = np.array([[2.0, -1.0], [-1.0, 3.0]])
    e = np.array([0.5, 1.5])
    eps = np.array([-1.0, -0.5, 0.2, 0.6, 1.0])  # o = 2
    phi = guess.features(Th0, e, eps, 2)
    want0 = [2.0, 0.5, 1.0, -0.5, 0.2, -0.75, 0.6, 1.0, np.sqrt(15.0 / 2.0), 3.0]
    want1 = [3.0, 1.5, 4.5, -0.5, 0.2, -0.75, 0.6, 1.0, np.sqrt(15.0 / 2.0), 4.0]
    assert np.allclose(phi[0], want0) and np.allclose(phi[1], want1)
