"""Parity of the HIP integrator with the CPU FP64 oracle (through the C ABI).

Bar, per cell: |T_gpu - T_or| <= 1e-6 T_or and |Y_gpu - Y_or| <= 1e-6 |Y_or|
+ 1e-10 (rtol 1e-6 on T and Y, atol 1e-10).  Both sides run the same
algorithm and controller and differ only in rounding; cells whose result
rounding alone moves past the bar are judged against what rounding does to
the oracle itself (oracle/parity.py: nine rounding-level variants of the
oracle, the same source built with contracted multiply-adds and the input T
moved by one or two ulp).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import parity
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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def assert_h_is_last_proposal(C, mech, o, T, P, Y, dt, mode, hg, rtol=1e-6, atol=1e-10):
    """The returned step is the controller's proposal after the cell's last
    accepted step: h_n clamp(0.9 err^(-1/4), 0.2, 6), capped at 1 when that
    step followed a rejection, with err the RMS error norm of that step.  The
    GPU's own last accepted step (state and h_n, recorded by a checkpointed
    call of the same integration) is replayed in the oracle and the proposal
    recomputed from it.  (Comparing the proposal with the oracle's own run
    instead is ill-posed on cells that run hundreds of steps through a thermal
    runaway: the last step is usually the remainder of dt, which any
    rounding-level change of the step sequence moves.)"""
    T1, Y1, h1, ns, st, ck = C.integrate(mech, dev(T), dev(P), dev(Y), dt,
                                         opts=C.default_opts(mode=mode), checkpoint=True)
    torch.cuda.synchronize()
    off, rec = ck.export()
    ck.close()
    h1 = h1.cpu().numpy()
    assert np.array_equal(h1, hg)            # the checkpointed call takes the same steps
    N = rec.shape[1] - 1
    checked = 0
    for c in range(T.size):
        last = off[c + 1] - 2                # the record before the final state
        if last < off[c]:
            continue
        phi, hn = rec[last, :N], rec[last, N]
        rc, out, err = o.step(P[c], phi, hn)
        assert rc == 0
        sc = atol + rtol * np.maximum(np.abs(phi), np.abs(out))
        e = np.sqrt(np.mean((err / sc) ** 2))
        assert e <= 1.0 + 1e-6, (c, e)
        fac = min(6.0, max(0.2, 0.9 * e ** -0.25)) if e > 0 else 6.0
        cands = np.array([hn * fac, hn * min(fac, 1.0)])
        # err is a cancelled estimate (about rtol of the state's scale, formed
        # from stage vectors that are much larger), so the two sides' values of
        # it agree only to ~1e-5 on stiff cells; h goes as err^(-1/4)
        assert np.min(np.abs(cands - h1[c]) / cands) < 1e-3, (c, h1[c], cands)
        checked += 1
    assert checked > 0


def run_gpu(C, mech, T, P, Y, dt, mode="plain", h=None, **kw):
    opts = C.default_opts(mode=mode, **kw)
    hh = None if h is None else dev(h)
    T1, Y1, h1, ns, st = C.integrate(mech, dev(T), dev(P), dev(Y), dt, h=hh, opts=opts)
    torch.cuda.synchronize()
    return T1.cpu().numpy(), Y1.cpu().numpy(), h1.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("name", ["small", "ch4", "large"])
def test_rhs_and_jacobian_parity(chem, name, request):
    path, m, o = request.getfixturevalue(name)
    say("case: rhs/jacobian parity", name)
    mech = chem.Mechanism(path)
    rng = np.random.default_rng(17)
    n = 70
    phis, Ps = [], []
    for _ in range(n):
        T = rng.uniform(320, 2600)
        if abs(T - 1000) < 1:
            T += 3
        Y = rng.dirichlet(np.ones(o.K))
        P = rng.uniform(1, 5) * 101325.0
        phis.append(o.to_phi(T, P, Y))
        Ps.append(P)
    phi = np.array(phis).T.copy()
    P = np.array(Ps)
    f, J = chem.evaluate(mech, dev(phi), dev(P))
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    J = J.cpu().numpy().reshape(o.N, o.N, n)
    for c in range(n):
        fo = o.rhs(P[c], phi[:, c])
        Jo = o.jacobian(P[c], phi[:, c])
        assert np.allclose(f[:, c], fo, rtol=1e-10, atol=1e-12 * np.abs(fo).max()), c
        # entrywise to 1e-9 of the row scale (J rows mix magnitudes)
        scale = np.abs(Jo).max(1, keepdims=True) + 1e-300
        assert np.abs(J[:, :, c] - Jo).max() <= 1e-9 * scale.max(), c
        assert np.all(np.abs(J[:, :, c] - Jo) <= 1e-9 * scale), c
    mech.close()


@pytest.mark.parametrize("mode", ["plain", "team_persistent"])
def test_small_parity_full_config(chem, small, mode):
    path, m, o = small
    say("case: small mechanism, 256 cells,", mode)
    T, P, Y = synth.states_small(m)
    mech = chem.Mechanism(path)
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode)
    assert np.all(sg == 0)
    r, msg = parity.check_batch(o, T, P, Y, 1e-6, Tg, Yg, ng, "small " + mode)
    say(msg)
    assert np.all(r["status"] == 0)
    assert np.median(np.abs(hg - r["h"]) / r["h"]) < 1e-3
    assert_h_is_last_proposal(chem, mech, o, T, P, Y, 1e-6, mode, hg)
    mech.close()


@pytest.mark.parametrize("mode", ["plain", "persistent", "team", "team_persistent"])
def test_ch4_parity_ragged(chem, ch4, mode):
    """1,000 mixing-layer cells (15 full wavefronts and a ragged tail)."""
    path, m, o = ch4
    say("case: ch4 mechanism, 1000 cells,", mode)
    T, P, Y = synth.states_mixing(m, 1000, 202)
    mech = chem.Mechanism(path)
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode)
    assert np.all(sg == 0)
    r, msg = parity.check_batch(o, T, P, Y, 1e-6, Tg, Yg, ng, "ch4 " + mode)
    say(msg)
    assert np.median(np.abs(hg - r["h"]) / r["h"]) < 1e-6
    assert_h_is_last_proposal(chem, mech, o, T, P, Y, 1e-6, mode, hg)
    mech.close()


@pytest.mark.parametrize("method,estimator", [("ros3", "embedded"), ("rodas3", "embedded"),
                                              ("rodas4", "embedded"), ("ros4", "filtered"),
                                              ("rodas4", "filtered")])
@pytest.mark.parametrize("mode", ["plain", "team_persistent"])
def test_methods_parity(chem, ch4, method, estimator, mode):
    """The other solvers of the paper's solver table, and the filtered error
    estimate, on 1,000 mixing-layer cells in both kinds of launch."""
    path, m, o = ch4
    say("case: ch4 mechanism, 1000 cells,", method, estimator, mode)
    T, P, Y = synth.states_mixing(m, 1000, 202)
    mech = chem.Mechanism(path)
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode, method=method, estimator=estimator)
    assert np.all(sg == 0)
    r, msg = parity.check_batch(o, T, P, Y, 1e-6, Tg, Yg, ng, "ch4 %s %s %s" % (method, estimator, mode),
                                method=method, estimator=estimator)
    say(msg)
    assert np.median(np.abs(hg - r["h"]) / r["h"]) < 1e-6
    mech.close()


@pytest.mark.parametrize("jac_every", [1, 4])
@pytest.mark.parametrize("mode", ["plain", "team_persistent"])
def test_w_method_with_a_kept_jacobian(chem, ch4, jac_every, mode):
    """ROS34PW2, the W-method, with the Jacobian evaluated at every
    jac_every-th accepted state and kept in between: 1,000 mixing-layer cells
    against the oracle running the same policy, and the Jacobian count the
    launch reports (one at every jac_every-th of a cell's accepted states)."""
    path, m, o = ch4
    say("case: ch4 mechanism, 1000 cells, ros34pw2, jac_every", jac_every, mode)
    T, P, Y = synth.states_mixing(m, 1000, 202)
    mech = chem.Mechanism(path)
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode, method="ros34pw2", jac_every=jac_every,
                                 stats=stats)
    assert np.all(sg == 0) and np.all(ng >= 1)
    att, acc, rej, je = (int(x) for x in stats.cpu().numpy())
    assert acc == ng.sum() and att == acc + rej
    assert je == int(np.sum((ng + jac_every - 1) // jac_every))
    r, msg = parity.check_batch(o, T, P, Y, 1e-6, Tg, Yg, ng, "ch4 ros34pw2 jac_every=%d %s" % (jac_every, mode),
                                method="ros34pw2", jac_every=jac_every)
    say(msg)
    mech.close()


def test_kept_jacobian_changes_the_steps_and_needs_a_saved_copy(chem, ch4, large):
    """Keeping J changes the integration (the kept J is used: other results
    than jac_every = 1); with four wavefronts per cell a kept J needs
    the persistent launch's saved copies, and a checkpoint needs a fresh J at
    every step - both refused otherwise."""
    path, m, o = ch4
    T, P, Y = synth.states_mixing(m, 256, 202)
    mech = chem.Mechanism(path)
    a = run_gpu(chem, mech, T, P, Y, 1e-6, mode="team_persistent", method="ros34pw2", jac_every=1)
    b = run_gpu(chem, mech, T, P, Y, 1e-6, mode="team_persistent", method="ros34pw2", jac_every=3)
    assert not np.array_equal(a[0], b[0])
    with pytest.raises(chem.ChemError) as e:
        chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-6, checkpoint=True,
                       opts=chem.default_opts(method="ros34pw2", jac_every=2))
    assert e.value.code == chem.EUNSUPPORTED
    mech.close()
    lpath, lm, lo = large
    T, P, Y = synth.states_mixing(lm, 64, 204)
    mech = chem.Mechanism(lpath)
    with pytest.raises(chem.ChemError) as e:
        run_gpu(chem, mech, T, P, Y, 1e-6, mode="team", method="ros34pw2", jac_every=2)
    assert e.value.code == chem.EUNSUPPORTED
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6, mode="team_persistent", method="ros34pw2",
                                 jac_every=2)
    assert np.all(sg == 0)
    r, msg = parity.check_batch(lo, T, P, Y, 1e-6, Tg, Yg, ng, "large ros34pw2 jac_every=2 team_persistent",
                                method="ros34pw2", jac_every=2)
    say(msg)
    mech.close()


@pytest.mark.timeout(900)
def test_ch4_full_size_all_cells(chem, ch4):
    """65,536 mixing-layer cells in the benchmark's launch (auto), every cell
    against the oracle; the other launch modes are bit-identical to their
    counterparts (plain = persistent, team = team_persistent, a repeated
    launch)."""
    path, m, o = ch4
    say("case: ch4 mechanism, 65536 cells, all launch modes")
    T, P, Y = synth.states_mixing(m, 65536, 202)
    mech = chem.Mechanism(path)
    res = {}
    for key, mode in (("auto", "auto"), ("plain", "plain"), ("persistent", "persistent"), ("team", "team"),
                      ("team_persistent", "team_persistent"), ("team_persistent2", "team_persistent")):
        res[key] = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode)
        say("  ran", key)
    mech.close()
    for a, b in (("plain", "persistent"), ("team", "team_persistent"), ("team_persistent", "team_persistent2"),
                 ("auto", "team_persistent")):
        assert np.array_equal(res[a][0], res[b][0]), (a, b)
        assert np.array_equal(res[a][1], res[b][1]), (a, b)
    for mode in ("auto", "plain"):
        Tg, Yg, hg, ng, sg = res[mode]
        assert np.all(sg == 0)
        r, msg = parity.check_batch(o, T, P, Y, 1e-6, Tg, Yg, ng, "ch4 65536 " + mode)
        say(msg)


@pytest.mark.timeout(900)
def test_batching_full_size_sampled(chem, ch4):
    """The batching mix at its full size, 1,048,576 cells (85 % cold, 10 %
    igniting, 5 % burnt gas; dt = 1e-5 s), in the default launch; 2,048 cells
    re-run on the oracle: the 64 with the most steps, 512 more igniting ones,
    128 burnt-gas ones and 1,344 at random."""
    path, m, o = ch4
    say("case: batching mix, 1048576 cells, auto launch")
    T, P, Y, kind = synth.states_batching(m, 1048576, 203)
    mech = chem.Mechanism(path)
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-5, mode="auto")
    mech.close()
    assert np.all(sg == 0)
    rng = np.random.default_rng(3)
    top = np.argsort(-ng)[:64]
    rest = np.setdiff1d(np.arange(T.size), top)
    ign = rng.choice(np.intersect1d(rest, np.flatnonzero(kind == 1)), 512, replace=False)
    brn = rng.choice(np.intersect1d(rest, np.flatnonzero(kind == 2)), 128, replace=False)
    rnd = rng.choice(np.setdiff1d(rest, np.r_[ign, brn]), 1344, replace=False)
    idx = np.unique(np.r_[top, ign, brn, rnd])
    Ts, Ps, Ys = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    r, msg = parity.check_batch(o, Ts, Ps, Ys, 1e-5, Tg[idx], Yg[:, idx], ng[idx], "batching 2048 of 1048576")
    say(msg)
    assert np.all(r["status"] == 0)
    # the mix spans two orders of magnitude in step count
    assert ng[kind == 0].mean() < 5 and ng[kind == 1].mean() > 50


@pytest.mark.parametrize("name", ["n15", "n30", "n45", "n55", "n62", "n63"])
def test_mechanism_sizes_team_parity(chem, mech_dir, name):
    """Mechanisms of 15, 30, 45, 55, 62 and 63 species (state sizes 16, 31,
    46, 56, 63, 64: the one-wavefront-per-cell kernels compiled for 16, 32,
    48, 56 and 64 rows, with and without identity padding rows, up to one row
    per lane), 300 mixing-layer cells, dt = 1e-6 s, both one-wavefront-per-cell
    launches, and the discrete adjoint of 8 cells against the oracle's
    tangent."""
    import oracle
    path, m = synth.mechanism_file(name, mech_dir)
    o = oracle.Oracle(path)
    say("case: %s mechanism (%d species), 300 cells" % (name, m.n_species))
    T, P, Y = synth.states_mixing(m, 300, 209)
    mech = chem.Mechanism(path)
    r = o.integrate(T, P, Y, 1e-6)
    assert np.all(r["status"] == 0)
    for mode in ("team", "team_persistent"):
        Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode)
        assert np.all(sg == 0)
        say(parity.check_batch(o, T, P, Y, 1e-6, Tg, Yg, ng, name + " " + mode)[1])
    # adjoint: per-cell gradient of T_final along a random ln A direction
    idx = np.r_[np.argsort(-T)[:4], np.arange(4)]
    Ts, Ps, Ys = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    T1, Y1, h1, ns, st, ck = chem.integrate(mech, dev(Ts), dev(Ps), dev(Ys), 1e-6, checkpoint=True)
    gT = torch.ones(idx.size, dtype=torch.float64, device="cuda")
    gY = torch.zeros((m.n_species, idx.size), dtype=torch.float64, device="cuda")
    g, _, _ = chem.adjoint(mech, ck, gT, gY, per_cell=True, initial=False)
    torch.cuda.synchronize()
    off, rec = ck.export()
    ck.close()
    mech.close()
    g = g.cpu().numpy()
    rng = np.random.default_rng(13)
    for c in range(idx.size):
        hs = rec[off[c]:off[c + 1] - 1, -1].copy()
        v = rng.normal(size=len(m.reactions))
        dT, dY = o.tangent(Ts[c], Ps[c], Ys[:, c], hs, v_lnA=v)
        assert g[:, c] @ v == pytest.approx(dT, rel=1e-6, abs=1e-9 * np.abs(g[:, c]).sum() + 1e-300), c


def test_largest_four_wavefront_state(chem, mech_dir):
    """127 species (N = 128, the largest state of the four-wavefront kernels;
    with ROS4's four stages the work-group takes 162,672 of a CU's 163,840
    bytes of LDS): 48 mixing-layer cells (dt = 1e-5 s, up to ~100 steps) in
    both team launches against the oracle.  RODAS4's six stages do not fit, so the team modes run it one cell
    per thread (bit-identical to the plain launch) and the no-allocation entry
    point refuses it."""
    import ctypes as C
    path, m = synth.mechanism_file("n127", mech_dir)
    o = oracle.Oracle(path)
    say("case: n127 mechanism (N = 128), 48 cells")
    T, P, Y = synth.states_mixing(m, 4096, 210)
    idx = np.r_[np.argsort(-T)[:8], np.arange(40)]
    T, P, Y = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    mech = chem.Mechanism(path)
    res = {}
    for mode in ("team", "team_persistent"):
        res[mode] = run_gpu(chem, mech, T, P, Y, 1e-5, mode=mode)
        assert np.all(res[mode][4] == 0)
    for k in range(5):
        assert np.array_equal(res["team"][k], res["team_persistent"][k])
    Tg, Yg, hg, ng, sg = res["team"]
    say(parity.check_batch(o, T, P, Y, 1e-5, Tg, Yg, ng, "n127 team")[1])
    a = run_gpu(chem, mech, T, P, Y, 1e-5, mode="team", method="rodas4")
    b = run_gpu(chem, mech, T, P, Y, 1e-5, mode="plain", method="rodas4")
    for k in range(5):
        assert np.array_equal(a[k], b[k])
    L = chem.lib()
    L.chem_integrate_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(chem.Opts), C.c_void_p]
    Tt, Pt, Yt = dev(T), dev(P), dev(Y)
    T1, Y1 = torch.empty_like(Tt), torch.empty_like(Yt)
    n = T.size
    h1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    ns = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    vp = lambda t: C.c_void_p(t.data_ptr())
    opts = chem.default_opts(mode="team", method="rodas4")
    rc = L.chem_integrate_noalloc(mech.handle, n, vp(Tt), vp(Pt), vp(Yt), n, vp(T1), vp(Y1), 1e-6, 1e-6, 1e-10,
                                  vp(h1), vp(ns), vp(st), None, C.byref(opts),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == chem.EUNSUPPORTED
    torch.cuda.synchronize()
    mech.close()


@pytest.fixture(scope="module")
def large_cells(large):
    """512 of the 111-species mechanism's mixing-layer states (dt = 1e-5 s):
    each takes ~50 accepted steps, so every row of the 112 x 112 LU and many
    controller decisions are compared."""
    path, m, o = large
    T, P, Y = synth.states_mixing(m, 262144, 204)
    rng = np.random.default_rng(5)
    idx = np.unique(np.r_[rng.choice(T.size, 496, replace=False), np.argsort(-T)[:16]])
    return T[idx], P[idx], np.ascontiguousarray(Y[:, idx])


@pytest.mark.timeout(900)
def test_large_parity(chem, large, large_cells):
    """N = 112: every cell against the oracle in the default launch (four
    wavefronts per cell, persistent) and the plain grid of the same kernel,
    which must agree bit for bit; the one-cell-per-thread launch on 64 of the
    cells."""
    path, m, o = large
    T, P, Y = large_cells
    say("case: large mechanism, 512 cells, four-wavefront launches")
    mech = chem.Mechanism(path)
    res = {mode: run_gpu(chem, mech, T, P, Y, 1e-5, mode=mode) for mode in ("auto", "team", "team_persistent")}
    say("case: large mechanism, 64 cells, one cell per thread")
    th = run_gpu(chem, mech, T[:64], P[:64], np.ascontiguousarray(Y[:, :64]), 1e-5, mode="plain")
    mech.close()
    for k in range(5):
        assert np.array_equal(res["team"][k], res["team_persistent"][k])
        assert np.array_equal(res["auto"][k], res["team_persistent"][k])
    Tg, Yg, hg, ng, sg = res["auto"]
    assert np.all(sg == 0)
    r, msg = parity.check_batch(o, T, P, Y, 1e-5, Tg, Yg, ng, "large 512 four-wavefront")
    say(msg)
    assert np.median(r["n_acc"]) > 20
    assert np.median(np.abs(hg - r["h"]) / r["h"]) < 1e-6
    say(parity.check_batch(o, T[:64], P[:64], np.ascontiguousarray(Y[:, :64]), 1e-5, th[0], th[1], th[3],
                           "large 64 one-cell-per-thread")[1])


@pytest.mark.timeout(900)
def test_large_full_size_sampled(chem, large):
    """The 111-species mechanism at its full size, 262,144 mixing-layer cells
    in the default launch; 1,024 cells re-run on the oracle (the 64 with the
    most steps and 960 at random)."""
    path, m, o = large
    say("case: large mechanism, 262144 cells, auto launch")
    T, P, Y = synth.states_mixing(m, 262144, 204)
    mech = chem.Mechanism(path)
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-5, mode="auto")
    mech.close()
    assert np.all(sg == 0)
    rng = np.random.default_rng(6)
    top = np.argsort(-ng)[:64]
    idx = np.unique(np.r_[top, rng.choice(np.setdiff1d(np.arange(T.size), top), 960, replace=False)])
    Ts, Ps, Ys = T[idx], P[idx], np.ascontiguousarray(Y[:, idx])
    say(parity.check_batch(o, Ts, Ps, Ys, 1e-5, Tg[idx], Yg[:, idx], ng[idx], "large 1024 of 262144")[1])


@pytest.mark.parametrize("mode", ["plain", "persistent", "team", "team_persistent"])
def test_dispatch_order_leaves_results_unchanged(chem, small, mode):
    """Hottest-first dispatch only reorders the work: every cell's state, step
    count, status and final h are bit-identical to the index-order run (3,000
    cells over 900-2000 K, a ragged last block of the ordering kernels)."""
    path, m, o = small
    say("case: dispatch order", mode)
    mech = chem.Mechanism(path)
    T, P, Y = synth.states_small(m, n=3000, seed=11)
    a = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode, order=0)
    b = run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode, order=1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    with pytest.raises(chem.ChemError) as ei:
        run_gpu(chem, mech, T, P, Y, 1e-6, mode=mode, order=2)
    assert ei.value.code == chem.EINVAL
    mech.close()


def test_step_carry_over_and_edge_cases(chem, small):
    path, m, o = small
    say("case: edge cases (h carry-over, n=1, max_steps, NaN, T_cut, bad args)")
    mech = chem.Mechanism(path)
    T, P, Y = synth.states_small(m, n=65, seed=7)
    # two consecutive split steps, h carried over like the CFD coupling does
    Tg, Yg, hg, ng, sg = run_gpu(chem, mech, T, P, Y, 1e-6)
    Tg2, Yg2, hg2, ng2, sg2 = run_gpu(chem, mech, Tg, P, Yg, 1e-6, h=hg)
    # the second step starts from slightly different states; compare it from the
    # GPU's own first-step output so that only the second step is tested
    say(parity.check_batch(o, Tg, P, Yg, 1e-6, Tg2, Yg2, ng2, "carry-over", h=hg)[1])
    # a single cell
    Tg1, Yg1, *_ = run_gpu(chem, mech, T[:1], P[:1], Y[:, :1].copy(), 1e-6)
    assert np.array_equal(Tg1, Tg[:1]) and np.array_equal(Yg1, Yg[:, :1])
    # forced failures: max_steps, non-finite state
    *_, st = run_gpu(chem, mech, T, P, Y, 1e-6, max_steps=1)
    assert np.all(st == chem.CELL_MAX_STEPS)
    Tn = T.copy()
    Tn[3] = np.nan
    Tgn, _, _, _, st = run_gpu(chem, mech, Tn, P, Y, 1e-6)
    assert st[3] == chem.CELL_NONFINITE and np.all(np.delete(st, 3) == 0)
    assert np.allclose(np.delete(Tgn, 3), np.delete(Tg, 3), rtol=0, atol=0)
    # cells below T_cut are passed through
    Tc, Yc, _, nc, _ = run_gpu(chem, mech, T, P, Y, 1e-6, T_cut=1500.0)
    cold = T < 1500.0
    assert np.all(nc[cold] == 0) and np.allclose(Tc[cold], T[cold], rtol=1e-15)
    assert np.allclose(Yc[:, cold], Y[:, cold], rtol=1e-12, atol=1e-16)
    assert np.array_equal(Tc[~cold], Tg[~cold]) and np.array_equal(Yc[:, ~cold], Yg[:, ~cold])
    # empty batch and argument errors
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    chem.integrate(mech, e, e, torch.empty((mech.K, 0), dtype=torch.float64, device="cuda"), 1e-6)
    with pytest.raises(chem.ChemError) as ei:
        chem.integrate(mech, dev(T), dev(P), dev(Y), -1.0)
    assert ei.value.code == chem.EINVAL
    with pytest.raises(chem.ChemError):
        chem.integrate(mech, dev(T), dev(P), dev(Y), 1e-6, rtol=0.0)
    mech.close()
