"""Pins of the oracle's Rosenbrock tables, error estimators and step control.

The paper lists four linearly implicit solvers (Table T:solvers: ROS3 and
RODAS3 of Sandu et al., ROS4 and RODAS4 of Hairer and Wanner) and gives the
transformed Rosenbrock form (Sec. 2.3), but prints no coefficients.  These
tests pin each table the oracle carries to what its method must satisfy,
independently of where the digits came from: the Rosenbrock order conditions
of the method and of its embedded solution, L-stability, stiff accuracy for
the RODAS methods, and observed convergence orders on problems with
closed-form solutions.  They also pin the error estimators through the
stability functions of the two solutions, and the step-size controller
through how work and global error scale with the tolerance.

ROS34PW2 (Rang and Angermann 2005) is the W-method of the paper's future
work (a Rosenbrock method whose order conditions hold for any matrix in the
place of J, so that J can be kept over several steps); its extra pins check
that property: order 3 with a wrong Jacobian and with a Jacobian kept from
earlier steps, where ROS4 loses its order.
"""
import numpy as np
import pytest

import oracle

ORDER = {"ros3": 3, "ros4": 4, "rodas3": 3, "rodas4": 4, "ros34pw2": 3}
METHODS = list(ORDER)


def untransform(t):
    """(gamma, alpha, Gamma, b, bhat) from the transformed coefficients:
    a = alpha Gamma^-1, C = diag(1/gamma) - Gamma^-1, m = b Gamma^-1,
    e = (b - bhat) Gamma^-1 (the reading of the garbled c_ij line of Sec. 2.3)."""
    s, g = t["s"], t["gamma"]
    G = np.linalg.inv(np.diag([1 / g] * s) - t["c"])
    alpha = t["a"] @ G
    b = t["m"] @ G
    bh = b - t["e"] @ G
    return g, alpha, G, b, bh


def order_residuals(g, alpha, G, b):
    """The eight order conditions of a Rosenbrock method up to order 4 (one per
    rooted tree), with beta = alpha + Gamma below the diagonal."""
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


N_COND = {1: 1, 2: 2, 3: 4, 4: 8}     # conditions up to each order


def stability(alpha, G, b, z):
    """R(z) = 1 + z b^T (I - z B)^-1 1 with B = alpha + Gamma."""
    s = b.size
    return 1 + z * b @ np.linalg.solve(np.eye(s) - z * (alpha + G), np.ones(s))


@pytest.mark.parametrize("name", METHODS)
def test_order_conditions(name):
    t = oracle.method_table(name)
    g, alpha, G, b, bh = untransform(t)
    p = ORDER[name]
    assert np.all(np.abs(np.diag(G) - g) < 1e-14)
    r = order_residuals(g, alpha, G, b)
    assert np.abs(r[:N_COND[p]]).max() < 1e-13, r
    if p < 4:
        assert np.abs(r[N_COND[p]:]).max() > 1e-3          # not of a higher order
    rh = order_residuals(g, alpha, G, bh)
    assert np.abs(rh[:N_COND[p - 1]]).max() < 1e-13, rh    # embedded: one order lower
    assert np.abs(rh[N_COND[p - 1]:N_COND[p]]).max() > 1e-3
    assert t["elo"] == p                                    # the estimate is O(h^p)


@pytest.mark.parametrize("name", METHODS)
def test_l_stability_and_accuracy_of_the_stability_function(name):
    g, alpha, G, b, bh = untransform(oracle.method_table(name))
    p = ORDER[name]
    # R(inf) = 0.  ROS4's published gamma, 0.57282, is the L-stable root 1/x2
    # of the Laguerre polynomial L4 rounded to five digits, so its R(inf) is
    # ~1.5e-5 instead of 0.
    Rinf = abs(stability(alpha, G, b, -1e14))
    assert Rinf < (2e-5 if name == "ros4" else 1e-9)
    if name == "ros4":
        x = np.sort(np.roots([1, -16, 72, -96, 24]).real)[1]
        assert abs(g - 1 / x) < 5e-6
    # A-stability on the imaginary axis
    for y in np.logspace(-3, 6, 60):
        assert abs(stability(alpha, G, b, 1j * y)) <= 1 + 1e-12
    # R(z) - e^z = O(z^(p+1))
    for z in (1e-2, -1e-2, 2e-2):
        assert abs(stability(alpha, G, b, z) - np.exp(z)) < 5 * abs(z) ** (p + 1)


@pytest.mark.parametrize("name", ["rodas3", "rodas4", "ros34pw2"])
def test_stiffly_accurate(name):
    """The RODAS solutions (main and embedded) and the ROS34PW2 main solution
    are the last stage arguments: b_i = beta_si, so they damp a stiff mode
    completely."""
    t = oracle.method_table(name)
    g, alpha, G, b, bh = untransform(t)
    B = alpha + G
    assert np.allclose(b, B[-1], atol=1e-13)
    if name != "ros34pw2":
        assert abs(stability(alpha, G, bh, -1e14)) < 1e-9


def test_w_method_order_with_a_wrong_jacobian():
    """y' = A y with every step using A + E in place of the Jacobian: ROS34PW2
    keeps order 3 (its W-order conditions), ROS4 falls to order 2 or below."""
    rng = np.random.default_rng(5)
    lam = -np.array([1.0, 2.0, 0.5, 3.0])
    A, Q, y0 = stiff_linear(4, 9, lam)
    E = 0.5 * rng.normal(size=(4, 4))
    T = 1.0
    exact = Q @ (np.exp(lam * T) * (Q.T @ y0))

    def slopes(name, Aj):
        errs = []
        for steps in (10, 20, 40, 80):
            y = y0.copy()
            for _ in range(steps):
                y = oracle.linear_step(A, y, T / steps, method=name, Ajac=Aj)[0]
            errs.append(np.abs(y - exact).max())
        return np.log2(np.array(errs[:-1]) / np.array(errs[1:]))

    assert np.all(np.abs(slopes("ros34pw2", A + E) - 3) < 0.15)
    assert np.all(np.abs(slopes("ros34pw2", np.zeros((4, 4))) - 3) < 0.15)
    assert np.all(slopes("ros4", A + E) < 2.3)
    assert np.all(np.abs(slopes("ros4", A) - 4) < 0.3)       # the exact Jacobian: order 4


@pytest.mark.parametrize("jac_every", [2, 5])
def test_w_method_keeps_its_order_with_a_kept_jacobian(jac_every):
    """y' = -y^3 with fixed steps and the Jacobian of every jac_every-th
    step's state kept in between: ROS34PW2 converges at order 3, ROS4 does
    not keep its order 4."""
    y0, T = 1.0, 1.0
    exact = y0 / np.sqrt(1 + 2 * y0 ** 2 * T)
    n = np.array([20, 40, 80, 160])

    def slope(name):
        errs = np.array([abs(oracle.integrate_cubic(y0, T, h_fixed=T / k, method=name, jac_every=jac_every)[0]
                             - exact) for k in n])
        return -np.polyfit(np.log(n), np.log(errs), 1)[0]

    assert slope("ros34pw2") == pytest.approx(3.0, abs=0.3)
    assert slope("ros4") < 3.3


def test_jacobian_reuse_under_step_control():
    """Adaptive ROS34PW2 on y' = -y^3 with the Jacobian kept for 1, 3 and 10
    accepted steps: the global error still tracks the tolerance, and keeping
    J changes the result (the kept J is really used)."""
    y0, T = 2.0, 3.0
    exact = y0 / np.sqrt(1 + 2 * y0 ** 2 * T)
    for k in (1, 3, 10):
        tols = 10.0 ** -np.arange(5, 10)
        errs = [abs(oracle.integrate_cubic(y0, T, rtol=t, atol=t, method="ros34pw2", jac_every=k)[0] - exact)
                for t in tols]
        assert np.polyfit(np.log(tols), np.log(errs), 1)[0] == pytest.approx(1.0, abs=0.3), (k, errs)
    y1 = oracle.integrate_cubic(y0, T, rtol=1e-7, atol=1e-7, method="ros34pw2", jac_every=1)[0]
    y3 = oracle.integrate_cubic(y0, T, rtol=1e-7, atol=1e-7, method="ros34pw2", jac_every=3)[0]
    assert y1 != y3


def test_embedded_estimate_of_a_four_stage_method():
    """For any 4-stage method of order 4 with an order-3 embedded solution the
    difference of the two stability functions is E(z) = c z^4 / (1 - gamma z)^4
    (the order conditions of the difference leave only the N^3 term of the
    nilpotent part of B), so its value at infinity, c / gamma^4, is fixed by
    the same constant c that sets the non-stiff estimate: no choice of the free
    parameters damps the stiff response without shrinking the whole estimate.
    For ROS4 the embedded solution keeps 0.55 of a stiff mode."""
    g, alpha, G, b, bh = untransform(oracle.method_table("ros4"))
    zs = np.array([-0.5, -3.0, -40.0, -1e4, 0.7, 1j, -2 + 5j])
    E = np.array([stability(alpha, G, b, z) - stability(alpha, G, bh, z) for z in zs])
    c = E * (1 - g * zs) ** 4 / zs ** 4
    assert np.allclose(c, c[0], rtol=1e-9)
    Rh_inf = stability(alpha, G, bh, -1e14)
    assert Rh_inf == pytest.approx(0.552, abs=2e-3)


@pytest.mark.parametrize("name", METHODS)
@pytest.mark.parametrize("estimator", ["embedded", "filtered"])
def test_step_error_estimate_is_the_stability_difference(name, estimator):
    """One oracle step of y' = lambda y: y_new = R(z) y0 and the estimate is
    (R(z) - Rhat(z)) y0, times (1 - gamma z)^-1 for the filtered estimator,
    which goes to 0 for a strongly damped mode."""
    g, alpha, G, b, bh = untransform(oracle.method_table(name))
    for lam, h in ((-1.0, 0.1), (-50.0, 0.1), (-1e7, 1e-2), (2.0, 0.05)):
        z = lam * h
        y1, e = oracle.linear_step(np.array([[lam]]), np.array([1.0]), h, method=name, estimator=estimator)
        R, Rh = stability(alpha, G, b, z), stability(alpha, G, bh, z)
        # (the stage vectors of a stiff step are ~1/|z| larger than y: rounding)
        assert y1[0] == pytest.approx(R, rel=1e-9, abs=1e-15)
        expect = (R - Rh) / ((1 - g * z) if estimator == "filtered" else 1.0)
        assert e[0] == pytest.approx(expect, rel=1e-9, abs=1e-13)
    if estimator == "filtered":
        _, e = oracle.linear_step(np.array([[-1e9]]), np.array([1.0]), 1.0, method=name, estimator=estimator)
        assert abs(e[0]) < 1e-8


def stiff_linear(n, seed, lam):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return Q @ np.diag(lam) @ Q.T, Q, rng.normal(size=n)


@pytest.mark.parametrize("name", METHODS)
def test_linear_stiff_fixed_step_order(name):
    # two smooth modes and four stiff ones (h * lambda from -30 to -2.5e5): the
    # stiff modes are damped (R(inf) = 0), the smooth ones converge at order p;
    # the stiffness is kept where rounding in A y stays below the truncation error
    lam = -np.array([1.0, 0.5, 1e3, 1e4, 1e5, 1e6])
    A, Q, y0 = stiff_linear(6, 7, lam)
    T = 2.0
    exact = Q @ (np.exp(lam * T) * (Q.T @ y0))
    errs = []
    for steps in (8, 16, 32, 64):
        y, _ = oracle.integrate_linear(A, y0, T, h_fixed=T / steps, method=name)
        errs.append(np.abs(y - exact).max())
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - ORDER[name]) < 0.3), (errs, slopes)


@pytest.mark.parametrize("name", METHODS)
def test_cubic_decay_order(name):
    # y' = -y^3, y(t) = y0 / sqrt(1 + 2 y0^2 t).  (Not y' = -y^2: the first
    # stage of a method with gamma = 1/2 integrates that one exactly.)
    # RODAS4's error constant is small: its observed slope is ~4.4 before the
    # asymptotic regime, still far from the 3 or less of a wrong coefficient.
    y0, T = 1.0, 1.0
    exact = y0 / np.sqrt(1 + 2 * y0 ** 2 * T)
    n = np.array([10, 20, 40, 80, 160])
    errs = np.array([abs(oracle.integrate_cubic(y0, T, h_fixed=T / k, method=name)[0] - exact) for k in n])
    slopes = np.log2(errs[:-1] / errs[1:])
    assert np.all(np.abs(slopes - ORDER[name]) < 0.6), (errs, slopes)
    assert -np.polyfit(np.log(n), np.log(errs), 1)[0] == pytest.approx(ORDER[name], abs=0.5)


@pytest.mark.parametrize("name", METHODS)
def test_controller_scaling_with_tolerance(name):
    """Step control on a smooth problem: the number of accepted steps grows as
    tol^(-1/elo) (each step's estimate, O(h^elo), is held at the tolerance) and
    the global error falls in proportion to tol (the main solution is one order
    more accurate than the estimate).  Fitted over tol = 1e-5 .. 1e-10."""
    y0, T = 2.0, 3.0
    exact = y0 / np.sqrt(1 + 2 * y0 ** 2 * T)
    tols = 10.0 ** -np.arange(5, 11)
    steps, errs = [], []
    for tol in tols:
        y, n = oracle.integrate_cubic(y0, T, rtol=tol, atol=tol, method=name)
        assert n > 0
        steps.append(n)
        errs.append(abs(y - exact))
    s_steps = np.polyfit(np.log(tols), np.log(steps), 1)[0]
    s_err = np.polyfit(np.log(tols), np.log(errs), 1)[0]
    elo = ORDER[name]
    assert s_steps == pytest.approx(-1.0 / elo, abs=0.04), steps
    assert s_err == pytest.approx(1.0, abs=0.25), errs


@pytest.mark.parametrize("estimator", ["embedded", "filtered"])
def test_linear_stiff_adaptive_tolerance(estimator):
    """A stiff linear system under step control: the global error tracks the
    tolerance (fitted slope near 1) and the work grows as it tightens."""
    lam = -np.logspace(0, 8, 5)
    A, Q, y0 = stiff_linear(5, 8, lam)
    T = 1.0
    exact = Q @ (np.exp(lam * T) * (Q.T @ y0))
    tols = 10.0 ** -np.arange(4, 10)
    errs, steps = [], []
    for tol in tols:
        y, nacc = oracle.integrate_linear(A, y0, T, rtol=tol, atol=tol, estimator=estimator)
        assert nacc > 0
        errs.append(np.abs(y - exact).max())
        steps.append(nacc)
    assert np.all(np.diff(steps) >= 0)
    assert np.polyfit(np.log(tols), np.log(errs), 1)[0] == pytest.approx(1.0, abs=0.3), errs
    assert np.all(np.array(errs) < 30 * tols)


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


def _lapack_perm(piv):
    """LAPACK's swap sequence (getrf's ipiv, 0-based) as the row of M taken at each step."""
    p = np.arange(piv.size)
    for k, s in enumerate(piv):
        p[k], p[s] = p[s], p[k]
    return p


def test_lu_factors_match_lapack_getrf():
    """The factors and pivot order of the stage-matrix LU (a6): LAPACK's
    getrf (scipy) makes the same choice - the largest magnitude in the column,
    the first in the current row order on a tie - so on random matrices
    (with and without forced interchanges and exact ties in the first column)
    the permutation agrees exactly and the factors to rounding; P M = L U to
    the backward-error bound, and every multiplier has magnitude <= 1."""
    import scipy.linalg as sl
    rng = np.random.default_rng(21)
    eps = np.finfo(float).eps
    for n in (1, 2, 5, 16, 54, 112, 128):
        for case in range(3):
            M = rng.normal(size=(n, n))
            if case == 1 and n > 1:
                M[0, 0] = 0.0                            # forces an interchange
            if case == 2 and n > 3:
                M[1, 0], M[3, 0] = 7.0, -7.0             # an exact tie in column 0
            F, perm, status, margin = oracle.lu(M)
            assert status == 0
            lu_ref, piv = sl.lu_factor(M)
            assert np.array_equal(perm, _lapack_perm(piv))
            L = np.tril(F, -1) + np.eye(n)
            U = np.triu(F)
            assert np.abs(L).max() <= 1.0
            absLU = np.abs(L) @ np.abs(U)
            assert np.all(np.abs(L @ U - M[perm]) <= 4 * n * eps * absLU + 1e-300)
            assert np.all(np.abs(F - lu_ref) <= 4 * n * eps * (absLU / np.maximum(1.0, np.abs(np.diag(U)))[None, :]
                                                                 + absLU) + 1e-300)
            if case == 2 and n > 3:
                assert perm[0] == 1 and margin == 0.0    # the tie goes to the lower row
            elif n > 1:
                assert margin > 0.0


def test_lu_status_codes():
    """A zero column gives 1, a column with NaN or an infinity gives 2 (the
    first failure in column order); a rank-deficient matrix - two equal rows -
    gives 1 at the step where the repeated row is exhausted."""
    rng = np.random.default_rng(22)
    M = rng.normal(size=(6, 6))
    Z = M.copy(); Z[:, 2] = 0.0
    assert oracle.lu(Z)[2] == 1
    N = M.copy(); N[4, 3] = np.nan
    assert oracle.lu(N)[2] == 2
    I = M.copy(); I[5, 0] = np.inf
    assert oracle.lu(I)[2] == 2
    R = M.copy(); R[3] = R[1]
    assert oracle.lu(R)[2] == 1
