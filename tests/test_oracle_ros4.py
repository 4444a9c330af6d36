"""Pins of the oracle's ROS4 table and integrator on model problems.

The paper names ROS4 with Hairer-Wanner coefficients (Table T:solvers) and
gives the transformed Rosenbrock form (Sec. 2.3) but prints no table.  These
tests pin the oracle's table to what the method must satisfy, independently of
how it was derived: the order conditions of a 4-stage Rosenbrock method
(order 4, embedded order 3), L-stability, and observed convergence order on
problems with closed-form solutions.
"""
import numpy as np
import pytest

import oracle


def untransform(t):
    """Recover (alpha, Gamma, b, bhat) from the transformed coefficients.

    a = alpha Gamma^-1, C = diag(1/gamma) - Gamma^-1, m = b Gamma^-1,
    e = (b - bhat) Gamma^-1 (the reading of the garbled c_ij line in Sec. 2.3).
    """
    g = t["gamma"]
    A = np.zeros((4, 4))
    A[1, 0] = t["a21"]
    A[2, 0], A[2, 1] = t["a31"], t["a32"]
    A[3, 0], A[3, 1] = t["a31"], t["a32"]       # stage 4 reuses stage 3's argument
    Cm = np.zeros((4, 4))
    Cm[1, 0] = t["c21"]
    Cm[2, 0], Cm[2, 1] = t["c31"], t["c32"]
    Cm[3, 0], Cm[3, 1], Cm[3, 2] = t["c41"], t["c42"], t["c43"]
    Ginv = np.diag([1 / g] * 4) - Cm
    G = np.linalg.inv(Ginv)
    alpha = A @ G
    m = np.array([t["m1"], t["m2"], t["m3"], t["m4"]])
    e = np.array([t["e1"], t["e2"], t["e3"], t["e4"]])
    b = m @ G
    bh = b - e @ G
    return g, alpha, G, b, bh


def order_residuals(g, alpha, G, b):
    beta = np.tril(alpha + G, -1)
    bp = beta.sum(1)
    ai = alpha.sum(1)
    return np.array([
        b.sum() - 1,
        b @ bp - (0.5 - g),
        b @ ai ** 2 - 1 / 3,
        b @ (beta @ bp) - (1 / 6 - g + g * g),
        b @ ai ** 3 - 0.25,
        b @ (ai * (alpha @ bp)) - (1 / 8 - g / 3),
        b @ (beta @ ai ** 2) - (1 / 12 - g / 3),
        b @ (beta @ (beta @ bp)) - (1 / 24 - g / 2 + 1.5 * g * g - g ** 3),
    ])


def stability(g, alpha, G, b, z):
    B = alpha + G
    return 1 + z * b @ np.linalg.solve(np.eye(4) - z * B, np.ones(4))


def test_order_conditions():
    g, alpha, G, b, bh = untransform(oracle.ros4_table())
    assert np.all(np.abs(np.diag(G) - g) < 1e-14)
    assert np.abs(order_residuals(g, alpha, G, b)).max() < 1e-13
    # embedded solution: order 3 (first four conditions) but not order 4
    r = order_residuals(g, alpha, G, bh)
    assert np.abs(r[:4]).max() < 1e-13
    assert np.abs(r[4:]).max() > 1e-3
    assert abs(bh[3]) < 1e-13
    # alpha_4j = alpha_3j: the fourth stage needs no new f evaluation
    assert np.allclose(alpha[3], alpha[2], atol=1e-14)


def test_gamma_is_laguerre_root_and_l_stable():
    g, alpha, G, b, bh = untransform(oracle.ros4_table())
    x = 1 / g
    L4 = (x ** 4 - 16 * x ** 3 + 72 * x ** 2 - 96 * x + 24) / 24
    assert abs(L4) < 1e-13
    roots = np.sort(np.roots([1, -16, 72, -96, 24]).real)
    assert abs(x - roots[1]) < 1e-12
    # R(inf) = 0 and |R| <= 1 on the imaginary axis (A-stability)
    assert abs(stability(g, alpha, G, b, -1e12)) < 1e-9
    for y in np.logspace(-3, 6, 60):
        assert abs(stability(g, alpha, G, b, 1j * y)) <= 1 + 1e-12
    # R(z) - e^z = O(z^5)
    for z in (1e-2, -1e-2, 2e-2):
        assert abs(stability(g, alpha, G, b, z) - np.exp(z)) < 5 * abs(z) ** 5


def test_linear_stiff_fixed_step_order():
    rng = np.random.default_rng(7)
    n = 6
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    # two smooth modes and four stiff ones (h * lambda from -30 to -2.5e5); the
    # stiffness is kept where rounding in A y stays below the truncation error
    lam = -np.array([1.0, 0.5, 1e3, 1e4, 1e5, 1e6])
    A = Q @ np.diag(lam) @ Q.T
    y0 = rng.normal(size=n)
    T = 2.0
    exact = Q @ (np.exp(lam * T) * (Q.T @ y0))
    # the stiff modes are damped (R(inf) = 0); the smooth ones converge at order 4
    errs = []
    for steps in (8, 16, 32, 64):
        y, _ = oracle.integrate_linear(A, y0, T, h_fixed=T / steps)
        errs.append(np.abs(y - exact).max())
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4.0) < 0.3), (errs, slopes)


def test_linear_stiff_adaptive_tolerance():
    rng = np.random.default_rng(8)
    n = 5
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = -np.logspace(0, 8, n)
    A = Q @ np.diag(lam) @ Q.T
    y0 = rng.normal(size=n)
    T = 1.0
    exact = Q @ (np.exp(lam * T) * (Q.T @ y0))
    prev = None
    for tol in (1e-4, 1e-6, 1e-8):
        y, nacc = oracle.integrate_linear(A, y0, T, rtol=tol, atol=tol)
        err = np.abs(y - exact).max()
        assert nacc > 0
        assert err < 50 * tol
        if prev is not None:
            assert nacc >= prev
        prev = nacc


def test_riccati_order_four():
    # y' = -y^2, y(t) = y0 / (1 + y0 t)
    y0, T = 2.0, 1.0
    exact = y0 / (1 + y0 * T)
    errs = []
    for steps in (10, 20, 40):
        y, _ = oracle.integrate_riccati(y0, T, h_fixed=T / steps)
        errs.append(abs(y - exact))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4.0) < 0.3), (errs, slopes)


def test_lu_solve_matches_lapack():
    rng = np.random.default_rng(3)
    for n in (1, 2, 11, 54, 112):
        A = rng.normal(size=(n, n))
        if n > 1:
            A[0, 0] = 0.0                          # forces a row interchange
        b = rng.normal(size=n)
        x = oracle.lu_solve(A, b)
        ref = np.linalg.solve(A, b)
        assert np.abs(x - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
        # backward error of partial-pivot LU
        r = np.abs(A @ x - b).max()
        assert r <= 50 * n * np.finfo(float).eps * np.abs(A).max() * np.abs(x).max()
    with pytest.raises(np.linalg.LinAlgError):
        oracle.lu_solve(np.zeros((3, 3)), np.ones(3))
