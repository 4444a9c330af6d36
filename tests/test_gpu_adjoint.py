"""Discrete adjoint on the GPU against the oracle's exact tangent (replayed
along the GPU's own accepted steps) and extrapolated central differences on
frozen steps.

Workload: the CH4-shaped mechanism, cells drawn like the 16,384-cell
differentiation case (mixing-layer states, seed 205), dt = 1e-5 s; losses
L1 = T_final and L2 = sum_k w_k Y_k,final with w ~ N(0, 1) (seed 305).
"""
import sys

import numpy as np
import pytest

from paper_2205_05681_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05681_amd import chem as C
    C.lib()
    return C


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def case(chem, ch4):
    path, m, o = ch4
    T, P, Y = synth.states_mixing(m, 16384, 205)
    # the 10 hottest cells (many steps) and 6 others
    rng = np.random.default_rng(1)
    idx = np.r_[np.argsort(-T)[:10], rng.choice(16384, 6, replace=False)]
    T, P, Y = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    w = synth.loss_weights(m)
    mech = chem.Mechanism(path)
    say("case: adjoint, ch4 mechanism, 16 cells, dt=1e-5")
    T1, Y1, h1, ns, st, ck = chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-5, checkpoint=True)
    torch.cuda.synchronize()
    off, rec = ck.export()
    n = T.size
    gT = torch.ones(n, dtype=torch.float64, device="cuda")
    gY = torch.zeros((m.n_species, n), dtype=torch.float64, device="cuda")
    g1, gT01, gY01 = chem.adjoint(mech, ck, gT, gY, per_cell=True)
    gT2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    gY2 = dev(np.repeat(w[:, None], n, 1))
    g2, gT02, gY02 = chem.adjoint(mech, ck, gT2, gY2, per_cell=True)
    gsum, _, _ = chem.adjoint(mech, ck, gT2, gY2, per_cell=False)
    torch.cuda.synchronize()
    hs = [rec[off[c]:off[c + 1] - 1, -1].copy() for c in range(n)]
    out = dict(T=T, P=P, Y=Y, w=w, ns=ns.cpu().numpy(), st=st.cpu().numpy(), hs=hs, off=off, rec=rec,
               T1=T1.cpu().numpy(), Y1=Y1.cpu().numpy(),
               g1=g1.cpu().numpy(), g2=g2.cpu().numpy(), gsum=gsum.cpu().numpy(),
               gT01=gT01.cpu().numpy(), gY01=gY01.cpu().numpy(), gT02=gT02.cpu().numpy(),
               gY02=gY02.cpu().numpy())
    ck.close()
    mech.close()
    return out


def test_checkpoint_records_the_forward_steps(case, ch4):
    path, m, o = ch4
    assert np.all(case["st"] == 0)
    for c in range(case["T"].size):
        hs = case["hs"][c]
        assert hs.size == case["ns"][c]
        assert abs(hs.sum() - 1e-5) <= 1e-18
        # replaying the recorded steps on the oracle lands on the GPU result
        To, Yo = o.replay(case["T"][c], case["P"][c], case["Y"][:, c], hs)
        assert To == pytest.approx(case["T1"][c], rel=1e-9)
        assert np.allclose(Yo, case["Y1"][:, c], rtol=1e-7, atol=1e-12)


def test_adjoint_matches_oracle_tangent(case, ch4):
    """<g, v> from the GPU adjoint equals the oracle's forward tangent along v
    (both exact derivatives of the same discrete map)."""
    path, m, o = ch4
    rng = np.random.default_rng(305)
    for c in range(case["T"].size):
        hs = case["hs"][c]
        for _ in range(2):
            v = rng.normal(size=len(m.reactions))
            dT, dY = o.tangent(case["T"][c], case["P"][c], case["Y"][:, c], hs, v_lnA=v)
            a1 = case["g1"][:, c] @ v
            a2 = case["g2"][:, c] @ v
            t2 = case["w"] @ dY
            assert a1 == pytest.approx(dT, rel=1e-6, abs=1e-9 * np.abs(case["g1"][:, c]).sum() + 1e-300)
            assert a2 == pytest.approx(t2, rel=1e-6, abs=1e-9 * np.abs(case["g2"][:, c]).sum() + 1e-300)


def test_initial_state_gradients(case, ch4):
    path, m, o = ch4
    rng = np.random.default_rng(7)
    for c in range(0, case["T"].size, 3):
        hs = case["hs"][c]
        dT, dY = o.tangent(case["T"][c], case["P"][c], case["Y"][:, c], hs, dT0=1.0)
        assert case["gT01"][c] == pytest.approx(dT, rel=1e-6)
        dY0 = rng.normal(size=m.n_species) * 1e-3
        dT, dY = o.tangent(case["T"][c], case["P"][c], case["Y"][:, c], hs, dY0=dY0)
        assert case["gY02"][:, c] @ dY0 == pytest.approx(case["w"] @ dY, rel=1e-6, abs=1e-12)


def test_adjoint_matches_central_differences(case, ch4):
    """d L / d ln A_j against central differences (h = 1e-6) on frozen steps,
    for the four reactions with the largest gradient of each of two cells."""
    path, m, o = ch4
    lnA = o.lnA
    for c in (0, 1):
        hs = case["hs"][c]
        for loss, g in (("T", case["g1"][:, c]), ("wY", case["g2"][:, c])):
            for j in np.argsort(-np.abs(g))[:4]:
                e = np.zeros_like(lnA)
                e[j] = 1e-6
                Tp, Yp = o.replay(case["T"][c], case["P"][c], case["Y"][:, c], hs, lnA=lnA + e)
                Tm, Ym = o.replay(case["T"][c], case["P"][c], case["Y"][:, c], hs, lnA=lnA - e)
                fd = (Tp - Tm) / 2e-6 if loss == "T" else case["w"] @ (Yp - Ym) / 2e-6
                assert g[j] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max()), (c, loss, j)


def test_full_size_adjoint_sampled(chem, ch4):
    """The differentiation case at its full size (16,384 cells, dt = 1e-5 s)
    in the benchmark's launch: per-cell gradients of sum_k w_k Y_k for six
    cells (the three with the most steps, three at random) against the
    oracle's tangent along the GPU's own steps, and the summed gradient
    against the sum of the per-cell ones."""
    path, m, o = ch4
    say("case: adjoint, ch4 mechanism, 16384 cells, dt=1e-5")
    T, P, Y = synth.states_mixing(m, 16384, 205)
    w = synth.loss_weights(m)
    n = T.size
    mech = chem.Mechanism(path)
    T1, Y1, h1, ns, st, ck = chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-5, checkpoint=True)
    gT = torch.zeros(n, dtype=torch.float64, device="cuda")
    gY = dev(np.repeat(w[:, None], n, 1))
    g, _, _ = chem.adjoint(mech, ck, gT, gY, per_cell=True, initial=False)
    gs, _, _ = chem.adjoint(mech, ck, gT, gY, per_cell=False, initial=False)
    torch.cuda.synchronize()
    off, rec = ck.export()
    ck.close()
    mech.close()
    assert np.all(st.cpu().numpy() == 0)
    g = g.cpu().numpy()
    assert np.allclose(gs.cpu().numpy(), g.sum(1), rtol=1e-12, atol=1e-300)
    nsn = ns.cpu().numpy()
    rng = np.random.default_rng(11)
    cells = np.unique(np.r_[np.argsort(-nsn)[:3], rng.choice(n, 3, replace=False)])
    for c in cells:
        hs = rec[off[c]:off[c + 1] - 1, -1].copy()
        v = rng.normal(size=len(m.reactions))
        dT, dY = o.tangent(T[c], P[c], Y[:, c], hs, v_lnA=v)
        assert g[:, c] @ v == pytest.approx(w @ dY, rel=1e-6, abs=1e-9 * np.abs(g[:, c]).sum() + 1e-300), c


@pytest.mark.timeout(600)
def test_differentiation_case_central_differences_64_cells(chem, ch4):
    """The differentiation case's finite-difference check: 64 cells of its
    distribution (the 16 with the most steps and 48 at random), gradients of
    L1 = T_final and L2 = sum_k w_k Y_k,final along a random direction in ln A
    against central differences on the GPU's frozen steps, within 1e-5
    relative.  A plain central difference at h = 1e-6 carries the replays'
    rounding, ~eps |L| / h, which for L2 (|L2| ~ 1, gradients down to 1e-6) is
    already 1e-5 of the gradient; so the differences are Richardson
    extrapolated from h = 2e-3 and 1e-3 (truncation O(h^4)), with a floor of
    100 eps |L| / 1e-3 for the rounding (on 40 cells of this case the oracle's
    own extrapolated differences stay within 3 % of 1e-6 relative plus this
    floor of its exact tangent)."""
    path, m, o = ch4
    say("case: adjoint vs central differences, ch4 mechanism, 64 cells, dt=1e-5")
    T, P, Y = synth.states_mixing(m, 16384, 205)
    w = synth.loss_weights(m)
    mech = chem.Mechanism(path)
    ns = chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-5)[3].cpu().numpy()
    rng = np.random.default_rng(64)
    top = np.argsort(-ns)[:16]
    idx = np.r_[top, rng.choice(np.setdiff1d(np.arange(T.size), top), 48, replace=False)]
    T, P, Y = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    n = idx.size
    T1, Y1, h1, ns, st, ck = chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-5, checkpoint=True)
    gT = torch.ones(n, dtype=torch.float64, device="cuda")
    gY = torch.zeros((m.n_species, n), dtype=torch.float64, device="cuda")
    g1, _, _ = chem.adjoint(mech, ck, gT, gY, per_cell=True, initial=False)
    g2, _, _ = chem.adjoint(mech, ck, torch.zeros_like(gT), dev(np.repeat(w[:, None], n, 1)), per_cell=True,
                            initial=False)
    torch.cuda.synchronize()
    off, rec = ck.export()
    ck.close()
    mech.close()
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    T1, Y1 = T1.cpu().numpy(), Y1.cpu().numpy()
    hstep = 2e-3
    eps = np.finfo(np.float64).eps

    def central(c, hs, v, h):
        Tp, Yp = o.replay(T[c], P[c], Y[:, c], hs, lnA=o.lnA + h * v)
        Tm, Ym = o.replay(T[c], P[c], Y[:, c], hs, lnA=o.lnA - h * v)
        return (Tp - Tm) / (2 * h), w @ (Yp - Ym) / (2 * h)

    for c in range(n):
        hs = rec[off[c]:off[c + 1] - 1, -1].copy()
        v = rng.normal(size=len(m.reactions))
        d_h = central(c, hs, v, hstep)
        d_h2 = central(c, hs, v, hstep / 2)
        fd1, fd2 = ((4 * b - a) / 3 for a, b in zip(d_h, d_h2))
        floor1 = 100 * eps * abs(T1[c]) / (hstep / 2)
        floor2 = 100 * eps * np.abs(w * Y1[:, c]).sum() / (hstep / 2)
        assert g1[:, c] @ v == pytest.approx(fd1, rel=1e-5, abs=floor1), (c, "T")
        assert g2[:, c] @ v == pytest.approx(fd2, rel=1e-5, abs=floor2), (c, "wY")


def test_cell_sum_is_deterministic_reduction(case):
    assert np.allclose(case["gsum"], case["g2"].sum(1), rtol=1e-12, atol=1e-300)


def test_checkpointed_call_matches_plain_call(chem, ch4, case):
    """Recording the steps does not change the integration."""
    path, m, o = ch4
    mech = chem.Mechanism(path)
    T1, Y1, h1, ns, st = chem.integrate(mech, dev(case["T"]), dev(case["P"]), dev(case["Y"]), 1e-5)
    torch.cuda.synchronize()
    assert np.array_equal(T1.cpu().numpy(), case["T1"])
    assert np.array_equal(Y1.cpu().numpy(), case["Y1"])
    mech.close()


def test_checkpoint_arena_refill_and_reuse(chem, small):
    """The record arena is sized from the handle's previous checkpointed call.
    On a fresh handle the small mechanism's cells (hundreds of accepted steps
    each) overflow the first estimate, and the call runs once more with the
    exact size; a second call on the same handle fits in one pass.  Both give
    the plain call's results, one record per accepted step plus the final
    state, and identical records."""
    path, m, o = small
    say("case: checkpoint arena refill, small mechanism, 256 cells, dt=1e-6")
    T, P, Y = synth.states_small(m)
    mech = chem.Mechanism(path)
    T0, Y0, h0, ns0, st0 = chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-6)
    exports = []
    for call in range(2):
        T1, Y1, h1, ns, st, ck = chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-6, checkpoint=True)
        torch.cuda.synchronize()
        assert np.array_equal(T1.cpu().numpy(), T0.cpu().numpy()), call
        assert np.array_equal(Y1.cpu().numpy(), Y0.cpu().numpy()), call
        assert np.array_equal(ns.cpu().numpy(), ns0.cpu().numpy()), call
        off, rec = ck.export()
        nsn = ns.cpu().numpy()
        assert np.array_equal(np.diff(off), nsn + 1), call
        assert nsn.mean() > 100   # well past the first estimate of the arena
        # each record's h is the step taken; the steps of a cell add up to dt
        for c in range(T.size):
            hs = rec[off[c]:off[c + 1] - 1, -1]
            assert hs.sum() == pytest.approx(1e-6, rel=1e-12), (call, c)
            assert rec[off[c + 1] - 1, -1] == 0.0
            assert rec[off[c], 0] == T[c]
        exports.append((off, rec))
        ck.close()
    assert np.array_equal(exports[0][0], exports[1][0])
    assert np.array_equal(exports[0][1], exports[1][1])
    mech.close()


def test_autograd_function(chem, ch4, case):
    path, m, o = ch4
    say("case: autograd IntegrateFn, 16 cells")
    mech = chem.Mechanism(path)
    T = dev(case["T"]).requires_grad_(True)
    Y = dev(case["Y"]).requires_grad_(True)
    lnA = dev(o.lnA).requires_grad_(True)
    T1, Y1 = chem.IntegrateFn.apply(T, dev(case["P"]), Y, lnA, 1e-5, 1e-6, 1e-10, mech)
    loss = (dev(case["w"])[:, None] * Y1).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert np.allclose(lnA.grad.cpu().numpy(), case["gsum"], rtol=1e-10, atol=1e-300)
    assert np.allclose(T.grad.cpu().numpy(), case["gT02"], rtol=1e-10, atol=1e-300)
    assert np.allclose(Y.grad.cpu().numpy(), case["gY02"], rtol=1e-10, atol=1e-300)
    mech.close()
