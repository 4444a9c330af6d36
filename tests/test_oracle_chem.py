"""Pins of the oracle's thermochemistry, source terms, Jacobian and integrator.

The paper prints no rate law, thermo fit or worked example (it delegates them
to its code generator, Sec. 2.1), so every pin here is an identity, an
invariant, a limit or a closed-form solution that a mistake in the oracle
would break: cp = dh/dT, element and mass conservation of the production
rates, J against finite differences, conservation of elements, mass and
enthalpy by the integrator, an isothermal A = B reaction with an exponential
solution, relaxation to the Gibbs equilibrium, and tangents against finite
differences along frozen steps.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2205_05681_amd import synth

RU = 8314.462618


def random_phi(o, m, rng, T=None):
    T = rng.uniform(900, 2200) if T is None else T
    if abs(T - 1000.0) < 2.0:
        T += 5.0
    Y = rng.dirichlet(np.ones(o.K))
    P = rng.uniform(1, 5) * 101325.0
    return P, o.to_phi(T, P, Y)


# ------------------------------------------------------------------ thermo
@pytest.mark.parametrize("mech", ["small", "ch4"])
def test_thermo_identities(mech, request):
    path, m, o = request.getfixturevalue(mech)
    for T in (400.0, 850.0, 1500.0, 2600.0):
        d = 1e-3 * T
        cp, h, s = o.thermo(T)
        _, hp, sp = o.thermo(T + d)
        _, hm, sm = o.thermo(T - d)
        # d(h/R)/dT = cp/R with h/R = (h/RT) T ;  d(s/R)/dT = cp/(R T)
        dh = ((hp * (T + d)) - (hm * (T - d))) / (2 * d)
        ds = (sp - sm) / (2 * d)
        assert np.allclose(dh, cp, rtol=1e-6, atol=1e-8)
        assert np.allclose(ds, cp / T, rtol=1e-6, atol=1e-10)
    # continuity at T_mid = 1000 K
    lo = o.thermo(1000.0 - 1e-9)
    hi = o.thermo(1000.0)
    for a, b in zip(lo, hi):
        assert np.allclose(a, b, rtol=1e-8, atol=1e-8)


def test_thermo_matches_the_generating_curve(small):
    """The fits reproduce the smooth cp(T) they were drawn from and h_f(298)."""
    path, m, o = small
    cp, h, s = o.thermo(298.15)
    hf = np.array([sp.hf298 for sp in m.species]) * 1000.0
    assert np.allclose(h * 8.314462618 * 298.15, hf, atol=1.0)     # J/mol
    s298 = np.array([sp.s298 for sp in m.species])
    assert np.allclose(s * 8.314462618, s298, atol=1e-6)


# ------------------------------------------------------------------ kinetics
@pytest.mark.parametrize("mech", ["small", "ch4"])
def test_production_rates_conserve_mass_and_elements(mech, request):
    path, m, o = request.getfixturevalue(mech)
    rng = np.random.default_rng(11)
    for _ in range(5):
        T = rng.uniform(600, 2500)
        Cc = rng.dirichlet(np.ones(o.K)) * 101325.0 / (RU * T)
        q, w, kf, kr = o.kinetics(T, 101325.0, Cc)
        scale = np.abs(q).max() * 4 * max(o.W)
        assert abs(o.W @ w) <= 1e-13 * scale
        for e in range(o.E):
            assert abs(o.comp[:, e] @ w) <= 1e-13 * np.abs(q).max() * 10
        assert w[-1] == 0.0                       # the bath gas is inert


def test_rate_constant_temperature_dependence(ch4):
    """d ln kf / d(1/T) = -(theta + b T) for elementary reactions (Arrhenius),
    and d ln(kf/kr)/dT = (sum nu h)/(R T^2) - (sum nu)/T (van 't Hoff on K_c)."""
    path, m, o = ch4
    Cc = np.full(o.K, 1e-3)
    T = 1400.0
    d = 1e-3
    _, _, kf0, kr0 = o.kinetics(T, 101325.0, Cc)
    _, _, kfp, krp = o.kinetics(T + d, 101325.0, Cc)
    _, _, kfm, krm = o.kinetics(T - d, 101325.0, Cc)
    cp, hRT, sR = o.thermo(T)
    for j, r in enumerate(m.reactions):
        if r.kind == "E":
            slope = (np.log(kfp[j]) - np.log(kfm[j])) / (1 / (T + d) - 1 / (T - d))
            assert slope == pytest.approx(-(r.theta + r.b * T), rel=1e-6, abs=1e-3)
        nu = np.zeros(o.K)
        for i, n in r.reac:
            nu[i] -= n
        for i, n in r.prod:
            nu[i] += n
        dlnK = (np.log(kfp[j] / krp[j]) - np.log(kfm[j] / krm[j])) / (2 * d)
        expect = (nu @ hRT) / T - nu.sum() / T
        assert dlnK == pytest.approx(expect, rel=1e-5, abs=1e-9)


def test_falloff_limits(ch4):
    """Falloff rate constants tend to k0 [M] as Pr -> 0 and to k_inf as Pr -> inf:
    exactly for Lindemann, and up to the Troe broadening factor F in (0, 1]."""
    path, m, o = ch4
    T = 1500.0
    seen = {"low": 0, "high": 0}
    for scale in 10.0 ** np.arange(-24, 25, 4):
        Cc = np.full(o.K, scale)
        _, _, kf, _ = o.kinetics(T, 101325.0, Cc)
        for j, r in enumerate(m.reactions):
            if r.kind not in "LF":
                continue
            alpha = np.ones(o.K)
            for i, a in r.eff:
                alpha[i] = a
            M = alpha @ Cc
            kinf = np.exp(r.lnA + r.b * np.log(T) - r.theta / T)
            k0 = np.exp(r.low[0] + r.low[1] * np.log(T) - r.low[2] / T)
            Pr = k0 * M / kinf
            if Pr < 1e-9:
                seen["low"] += 1
                ratio = kf[j] / (k0 * M)
            elif Pr > 1e9:
                seen["high"] += 1
                ratio = kf[j] / kinf
            else:
                continue
            if r.kind == "L":
                assert ratio == pytest.approx(1.0, rel=1e-6)
            else:
                assert 0.0 < ratio <= 1.0 + 1e-12
    assert seen["low"] > 10 and seen["high"] > 10


def troe_mechanism(path, lnA, lnA0, a, T3, T1, T2):
    """A (+M) = B + C as a Troe falloff reaction with b = theta = 0 for both
    limits (so k_inf = A, k0 = A0) and no listed efficiencies ([M] = sum C)."""
    nasa = "3.5 0 0 0 0 -1000.0 4.0"
    text = ["CHEMMECH 1", "ELEMENTS 2 H O", "SPECIES 4",
            "A 34.0 2 2 1000.0 %s %s" % (nasa, nasa),
            "B 17.0 1 1 1000.0 %s %s" % (nasa, nasa),
            "C 17.0 1 1 1000.0 %s %s" % (nasa, nasa),
            "N2 28.0 0 0 1000.0 %s %s" % (nasa, nasa),
            "REACTIONS 1",
            "F 1 0 1 2 1 1 2 1 %r 0.0 0.0 0 %r 0.0 0.0 %r %r %r %r" % tuple(
                float(v) for v in (lnA, lnA0, a, T3, T1, T2))]
    with open(path, "w") as f:
        f.write("\n".join(text) + "\n")
    return path


def troe_checks(o, T=1200.0, lnA=np.log(1e10), lnA0=np.log(1e12), T1=800.0):
    """The Gilbert-Luther-Troe broadening factor at the points its form fixes.
    With T3 = T1 and no T2 term, F_cent = exp(-T/T1) for any a.  With x =
    log10 Pr + c and y = x / (n - d x), log10 F = log10 F_cent / (1 + y^2):
    F = F_cent where x = 0, F = F_cent^(1/2) where y = +1 or -1, and F ->
    F_cent^(1/(1 + 1/d^2)) as Pr -> 0 or infinity (c = -0.4 - 0.67 log10 F_cent,
    n = 0.75 - 1.27 log10 F_cent, d = 0.14)."""
    Fc = np.exp(-T / T1)
    lFc = np.log10(Fc)
    c = -0.4 - 0.67 * lFc
    n = 0.75 - 1.27 * lFc
    d = 0.14

    def F_at(log10Pr):
        M = 10.0 ** log10Pr * np.exp(lnA) / np.exp(lnA0)
        Cc = np.array([0.25, 0.25, 0.25, 0.25]) * M
        _, _, kf, _ = o.kinetics(T, 101325.0, Cc)
        Pr = np.exp(lnA0) * M / np.exp(lnA)
        return kf[0] / (np.exp(lnA) * Pr / (1.0 + Pr))

    assert F_at(-c) == pytest.approx(Fc, rel=1e-12)
    assert F_at(n / (1 + d) - c) == pytest.approx(np.sqrt(Fc), rel=1e-12)
    assert F_at(-n / (1 - d) - c) == pytest.approx(np.sqrt(Fc), rel=1e-12)
    lim = lFc / (1 + 1 / d ** 2)
    for lp in (250.0, -250.0):
        # x = +-250: y is within n / (d |x|) ~ 3 % of its limit -1/d
        assert np.log10(F_at(lp)) == pytest.approx(lim, rel=0.1)


def test_troe_broadening_special_points(tmp_path):
    for a, T1 in ((0.3, 800.0), (0.8, 3000.0)):
        path = troe_mechanism(str(tmp_path / "troe.txt"), np.log(1e10), np.log(1e12), a, T1, T1, 0.0)
        troe_checks(oracle.Oracle(path), T1=T1)


# ------------------------------------------------------------------ Jacobian
@pytest.mark.parametrize("mech", ["small", "ch4"])
def test_jacobian_vs_central_differences(mech, request):
    path, m, o = request.getfixturevalue(mech)
    rng = np.random.default_rng(5)
    for _ in range(3):
        P, phi = random_phi(o, m, rng)
        J = o.jacobian(P, phi)
        typ = np.r_[phi[0], phi[1], np.full(o.N - 2, 1e-3)]
        for j in range(o.N):
            def central(eps):
                p1, p2 = phi.copy(), phi.copy()
                p1[j] += eps
                p2[j] -= eps
                return (o.rhs(P, p1) - o.rhs(P, p2)) / (2 * eps)
            eps = 3e-3 * max(abs(phi[j]), typ[j])
            fd = (4 * central(eps / 2) - central(eps)) / 3        # Richardson, O(eps^4)
            err = np.abs(fd - J[:, j])
            assert np.all(err <= 1e-6 * (np.abs(J[:, j]).max() + 1e-300) + 1e-7 * np.abs(J[:, j])), j


def test_jacobian_annihilated_by_element_vectors(ch4):
    path, m, o = ch4
    rng = np.random.default_rng(6)
    P, phi = random_phi(o, m, rng)
    J = o.jacobian(P, phi)
    for e in range(o.E):
        w = np.r_[0.0, 0.0, o.comp[:-1, e]]
        assert np.abs(w @ J).max() <= 1e-12 * np.abs(J).max() * np.abs(w).max() * o.N


# ------------------------------------------------------------------ integrator
def element_totals(o, phi):
    return o.comp[:-1].T @ phi[2:]


def enthalpy_and_mass(o, P, phi):
    T, V = phi[0], phi[1]
    n = np.r_[phi[2:], P * V / (RU * T) - phi[2:].sum()]
    cp, hRT, s = o.thermo(T)
    return (n * hRT * RU * T).sum(), n @ o.W


def test_step_conserves_elements_and_energy(small):
    path, m, o = small
    T0, P0, Y0 = synth.states_small(m, n=6, seed=9)
    for c in range(6):
        P = P0[c]
        phi = o.to_phi(T0[c], P, Y0[:, c])
        e0 = element_totals(o, phi)
        H0, m0 = enthalpy_and_mass(o, P, phi)
        hs, Tf, Yf = o.record_steps(T0[c], P, Y0[:, c], 1e-6)
        for h in hs:
            rc, phi, _ = o.step(P, phi, h)
            assert rc == 0
            # element totals are a linear invariant of a Rosenbrock step with the exact J
            assert np.allclose(element_totals(o, phi), e0, rtol=1e-11, atol=0)
        assert phi[0] == pytest.approx(Tf, rel=1e-14)
        # mass (through the bath-gas closure) and enthalpy: conserved by the ODE,
        # kept by the integrator to the order of its tolerance
        H1, m1 = enthalpy_and_mass(o, P, phi)
        assert abs(m1 - m0) <= 10 * 1e-6 * m0
        Habs = np.abs(o.thermo(T0[c])[1] * RU * T0[c] * (Y0[:, c] / o.W)).sum()
        assert abs(H1 - H0) <= 10 * 1e-6 * Habs
        assert abs(Yf.sum() - 1.0) < 1e-14


def test_isothermal_isomerisation_closed_form(tmp_path):
    """A = B with equal enthalpies: T and V stay fixed and C_A relaxes
    exponentially at rate kf + kr towards kr/(kf + kr) C_tot."""
    lo = [4.0, 1e-4, 0.0, 0.0, 0.0, -3000.0, 5.0]
    loB = lo[:6] + [5.6]                      # entropy differs: K = exp(0.6)
    text = ["CHEMMECH 1", "ELEMENTS 2 H O", "SPECIES 3",
            "A 18.0 2 1 1000.0 " + " ".join(map(repr, lo)) + " " + " ".join(map(repr, lo)),
            "B 18.0 2 1 1000.0 " + " ".join(map(repr, loB)) + " " + " ".join(map(repr, loB)),
            "N2 28.0 0 0 1000.0 3.5 0 0 0 0 -1000.0 4.0 3.5 0 0 0 0 -1000.0 4.0",
            "REACTIONS 1",
            "E 1 0 1 1 1 1 %r 0.0 0.0 0" % float(np.log(2e6))]
    p = tmp_path / "iso.txt"
    p.write_text("\n".join(text) + "\n")
    o = oracle.Oracle(str(p))
    kf = 2e6
    kr = kf / np.exp(0.6)
    T, P = 1200.0, 101325.0
    Y = np.array([0.3, 0.1, 0.6])
    dt = 1e-6
    r = o.integrate(np.array([T]), np.array([P]), Y[:, None], dt, rtol=1e-8, atol=1e-14)
    assert r["status"][0] == 0
    assert r["T"][0] == pytest.approx(T, rel=1e-13)
    yA, yB = Y[0], Y[1]
    tot = yA + yB
    exact_A = kr / (kf + kr) * tot + (yA - kr / (kf + kr) * tot) * np.exp(-(kf + kr) * dt)
    assert r["Y"][0, 0] == pytest.approx(exact_A, rel=1e-7)
    assert r["Y"][1, 0] == pytest.approx(tot - exact_A, rel=1e-7)


def test_relaxation_to_gibbs_equilibrium(small):
    path, m, o = small
    T0, P0, Y0 = synth.states_small(m, n=1, seed=21)
    r = o.integrate(T0, P0, Y0, 1e-1, rtol=1e-9, atol=1e-16)
    assert r["status"][0] == 0
    T, Y, P = r["T"][0], r["Y"][:, 0], P0[0]
    phi = o.to_phi(T, P, Y)
    f = o.rhs(P, phi)
    assert abs(f[0]) < 1e-3 * T                    # dT/dt -> 0 (K/s)
    Cc = Y / o.W / phi[1]
    Cc[-1] = P / (RU * T) - Cc[:-1].sum()
    q, w, kf, kr = o.kinetics(T, P, Cc)
    for j, rx in enumerate(m.reactions):
        fwd = kf[j] * np.prod([Cc[i] ** n for i, n in rx.reac])
        rev = kr[j] * np.prod([Cc[i] ** n for i, n in rx.prod])
        if fwd > 1e-20 * max(1.0, np.abs(q).max()) and fwd > 1e-30:
            assert abs(np.log(rev / fwd)) < 1e-4, (j, fwd, rev)
    gibbs_equilibrium_checks(o, m, T, P, Y)


def gibbs_equilibrium_checks(o, m, T, P, Y):
    """At the relaxed state, each reaction's quotient of partial pressures in
    atmospheres equals the thermodynamic K_p = exp(sum_k nu_k (s_k/R - h_k/RT))
    (ideal gas, P_atm standard state).  A wrong standard-state factor in the
    oracle's K_c (for example kmol against mol: 1000^sum nu) moves the
    equilibrium the kinetics relax to, which this sees for reactions whose
    sum nu is not zero."""
    x = (Y / o.W) / (Y / o.W).sum()
    cp, hRT, sR = o.thermo(T)
    g = sR - hRT
    checked = 0
    for rx in m.reactions:
        nu = np.zeros(o.K)
        for i, n in rx.reac:
            nu[i] -= n
        for i, n in rx.prod:
            nu[i] += n
        if nu.sum() == 0 or np.any(x[nu != 0] < 1e-25):
            continue
        lnQ = nu @ np.log(x * P / 101325.0)
        assert lnQ == pytest.approx(nu @ g, abs=1e-4), rx
        checked += 1
    assert checked >= 5


def test_tight_tolerance_self_convergence(ch4):
    """Error of rtol 1e-6 against a rtol 1e-10 oracle run, in the norm of
    eqs. (ivp_norm) and (error_norm): O(1) or below, as tolerances imply."""
    path, m, o = ch4
    T, P, Y = synth.states_mixing(m, 48, 202)
    a = o.integrate(T, P, Y, 1e-6, rtol=1e-6, atol=1e-10)
    b = o.integrate(T, P, Y, 1e-6, rtol=1e-10, atol=1e-16)
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    ya = np.vstack([a["T"], a["Y"]])
    yb = np.vstack([b["T"], b["Y"]])
    E = np.sqrt((((ya - yb) / (1e-10 + 1e-6 * np.abs(yb))) ** 2).sum(0))
    assert np.isfinite(E).all()
    assert E.max() < 10.0


def test_failure_status_codes(small):
    path, m, o = small
    T, P, Y = synth.states_small(m, n=4, seed=3)
    r = o.integrate(T, P, Y, 1e-6, max_steps=1)
    assert np.all(r["status"] == 1)
    T2 = T.copy()
    T2[1] = np.nan
    r = o.integrate(T2, P, Y, 1e-6)
    assert r["status"][1] == 3 and r["status"][0] == 0 and r["status"][2] == 0


# ------------------------------------------------------------------ tangents
def test_tangent_matches_central_differences(ch4):
    path, m, o = ch4
    T, P, Y = synth.states_mixing(m, 64, 205)
    rng = np.random.default_rng(305)
    hot = np.argsort(-T)[:3]
    for c in hot:
        hs, Tf, Yf = o.record_steps(T[c], P[c], Y[:, c], 1e-5)
        v = rng.normal(size=o.Nr)
        dT, dY = o.tangent(T[c], P[c], Y[:, c], hs, v_lnA=v)
        # h = 1e-5: over hundreds of stiff steps the replay's rounding, divided
        # by 2h, is already ~1e-7 of the largest component at h = 1e-6
        h = 1e-5
        Tp, Yp = o.replay(T[c], P[c], Y[:, c], hs, lnA=o.lnA + h * v)
        Tm, Ym = o.replay(T[c], P[c], Y[:, c], hs, lnA=o.lnA - h * v)
        fdT = (Tp - Tm) / (2 * h)
        assert dT == pytest.approx(fdT, rel=1e-5, abs=1e-9 * T[c])
        fdY = (Yp - Ym) / (2 * h)
        # the bath gas closes through P V / (R T): its FD quotient carries ~1e-9 noise
        assert np.allclose(dY, fdY, rtol=1e-5, atol=1e-7 * max(np.abs(fdY).max(), 1e-12))
        # linearity of the tangent in the direction
        dT2, _ = o.tangent(T[c], P[c], Y[:, c], hs, v_lnA=2.5 * v)
        assert dT2 == pytest.approx(2.5 * dT, rel=1e-12, abs=1e-300)
        # the initial-state direction
        dT0, dYT0 = o.tangent(T[c], P[c], Y[:, c], hs, dT0=1.0)
        Tp, _ = o.replay(T[c] + 1e-3, P[c], Y[:, c], hs)
        Tm, _ = o.replay(T[c] - 1e-3, P[c], Y[:, c], hs)
        assert dT0 == pytest.approx((Tp - Tm) / 2e-3, rel=1e-6)


@pytest.mark.parametrize("name,min_steps", [("large", 40), ("n127", 40)])
def test_large_mechanisms_react(mech_dir, name, min_steps):
    """The large synthetic mechanisms (111 and 127 species) are not inert at
    the mixing-layer states the GPU tests and the benchmark use: with dt =
    1e-5 s the hottest cells take many controller steps, so the N = 112 and
    N = 128 paths are compared over long step sequences, not one step."""
    path, m = synth.mechanism_file(name, mech_dir)
    o = oracle.Oracle(path)
    T, P, Y = synth.states_mixing(m, 4096, 210)
    idx = np.argsort(-T)[:8]
    r = o.integrate(T[idx], P[idx], np.ascontiguousarray(Y[:, idx]), 1e-5)
    assert np.all(r["status"] == 0)
    assert r["n_acc"].max() >= min_steps
