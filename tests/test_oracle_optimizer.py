"""Pins of oracle/optimizer.py: dense BFGS equivalence, secant condition, Armijo by hand, and
convergence on a convex quadratic."""
import numpy as np
import pytest

from oracle import optimizer as O


def _history(n, k, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    A = A @ A.T + n * np.eye(n)
    hist = []
    for _ in range(k):
        s = rng.normal(size=n)
        y = A @ s
        hist.append((s, y, 1.0 / float(s @ y)))
    return hist


def test_two_loop_equals_dense_bfgs():
    n = 12
    hist = _history(n, 5, 0)
    g = np.random.default_rng(1).normal(size=n)
    r = O.two_loop(g, hist)
    H = O.dense_inverse_hessian(hist, n)
    np.testing.assert_allclose(r, H @ g, rtol=1e-10, atol=1e-12)
    # secant condition for the newest pair
    s, y, _ = hist[-1]
    np.testing.assert_allclose(H @ y, s, rtol=1e-10, atol=1e-12)
    # empty history: steepest descent
    np.testing.assert_array_equal(O.two_loop(g, []), g)


def test_armijo_by_hand():
    # f(x) = x^2 at x = 1, g = 2, d = -2: alpha=1 -> x=-1, f=1 (fails 1 <= 1 - 4e-4);
    # alpha=1/2 -> x=0, f=0 (passes)
    cost, gd = 1.0, -4.0
    cand = np.array([1.0, 0.0, 0.5625, 0.5625 ** 1])
    assert O.select(cost, gd, cand) == 1
    # nothing passes Armijo but one candidate lowers the cost -> the lowest one
    assert O.select(1.0, -1e6, np.array([0.99, 0.98, 0.999, 0.995])) == 1
    # nothing lowers the cost -> rejected
    assert O.select(1.0, -1.0, np.array([1.5, 1.2, 1.1, 1.0])) == -1


def test_converges_on_convex_quadratic():
    T, n_ls = 5, 4
    n = T * 7
    rng = np.random.default_rng(2)
    A = rng.normal(size=(n, n))
    A = A @ A.T / n + np.eye(n)
    b = rng.normal(size=n)
    free = np.ones(n, dtype=bool)
    free[:7] = False
    free[-7:] = False
    x0 = O.fp32(rng.normal(size=n))

    def f(x):
        return 0.5 * x @ A @ x - b @ x

    def grad(x):
        return A @ x - b

    st = O.init_state(x0, f(x0), grad(x0), T, max_step=np.inf)
    for _ in range(60):
        cand = O.candidates(st.x, st.d, n_ls)
        costs = np.array([f(c) for c in cand])
        grads = np.array([grad(c) for c in cand])
        O.step(st, costs, grads, T, max_step=np.inf)
    # optimum over the free variables with the pinned rows held at x0
    x_opt = x0.copy()
    Aff = A[np.ix_(free, free)]
    x_opt[free] = np.linalg.solve(Aff, b[free] - A[np.ix_(free, ~free)] @ x0[~free])
    assert f(st.x) - f(x_opt) < 1e-6 * abs(f(x0) - f(x_opt))
    np.testing.assert_array_equal(st.x[~free], x0[~free])


def test_capped_steepest_direction_and_backtracking():
    g = np.array([0.0, 4.0, -1.0, 0.5])
    np.testing.assert_array_equal(O.steepest(g, 0.2), O.fp32([0.0, -0.2, 0.05, -0.025]))
    np.testing.assert_array_equal(O.steepest(g * 0.01, 0.2), O.fp32(-g * 0.01))  # small gradients untouched
    # a rejected line search keeps x and scales the direction by alpha_min / 2 = 1/16
    T = 3
    x = np.zeros(21)
    gg = O.pin_rows(np.arange(21, dtype=float), T)
    st = O.init_state(x, 1.0, gg, T)
    d0 = st.d.copy()
    info = O.step(st, np.array([2.0, 2.0, 2.0, 2.0]), np.zeros((4, 21)), T)
    assert info["accepted"] == -1 and info["reset"]
    np.testing.assert_array_equal(st.x, x)
    np.testing.assert_array_equal(st.d, O.fp32(d0 / 16.0))
    assert np.max(np.abs(d0)) == np.float32(0.2)
