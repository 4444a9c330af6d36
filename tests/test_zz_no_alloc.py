"""chem_integrate_noalloc (the entry point that allocates nothing) against
chem_integrate, through the C ABI: two calls in a row on one mechanism, the
second with a smaller batch, each compared with the allocating entry point on
the same inputs and options (the same kernels run, so the results are equal
bit for bit)."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2205_05681_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def call_noalloc(L, chem, mech, T, P, Y, dt, opts):
    n = T.numel()
    T1, Y1 = torch.empty_like(T), torch.empty_like(Y)
    h = torch.zeros(n, dtype=torch.float64, device="cuda")
    ns = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    rc = L.chem_integrate_noalloc(mech.handle, n, vp(T), vp(P), vp(Y), n, vp(T1), vp(Y1), float(dt), 1e-6, 1e-10,
                                  vp(h), vp(ns), vp(st), None, C.byref(opts),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, T1, Y1, h, ns, st


@pytest.mark.parametrize("mode", ["auto", "team", "team_persistent"])
def test_noalloc_matches_integrate(ch4, mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05681_amd import chem
    L = chem.lib()
    L.chem_integrate_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(chem.Opts), C.c_void_p]
    path, m, o = ch4
    print("case: chem_integrate_noalloc vs chem_integrate, ch4,", mode, flush=True)
    sys.stdout.flush()
    mech = chem.Mechanism(path)
    opts = chem.default_opts(mode=mode)
    for n, seed in ((5000, 202), (1500, 205)):     # the second call is smaller
        T, P, Y = synth.states_mixing(m, n, seed)
        Tt, Pt, Yt = dev(T), dev(P), dev(Y)
        rc, T1, Y1, h1, ns1, st1 = call_noalloc(L, chem, mech, Tt, Pt, Yt, 1e-6, opts)
        assert rc == 0, chem.error_string(rc)
        T2, Y2, h2, ns2, st2 = chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=opts)
        torch.cuda.synchronize()
        for a, b in ((T1, T2), (Y1, Y2), (h1, h2), (ns1, ns2), (st1, st2)):
            assert torch.equal(a, b)
        assert int((st1 != 0).sum()) == 0
    # argument errors: too many cells, a one-cell-per-thread mode
    big = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = L.chem_integrate_noalloc(mech.handle, (1 << 20) + 1, vp(big), vp(big), vp(big), (1 << 20) + 1,
                                  vp(big), vp(big), 1e-6, 1e-6, 1e-10, None, None, None, None,
                                  C.byref(opts), None)
    assert rc == chem.EINVAL
    T, P, Y = synth.states_mixing(m, 64, 3)
    rc, *_ = call_noalloc(L, chem, mech, dev(T), dev(P), dev(Y), 1e-6, chem.default_opts(mode="plain"))
    assert rc == chem.EUNSUPPORTED
    torch.cuda.synchronize()
    mech.close()


@pytest.mark.parametrize("mode", ["team", "team_persistent"])
def test_noalloc_four_wavefronts_matches_integrate(large, mode):
    """The same for the 111-species mechanism (four wavefronts per cell, N =
    112): without a saved J a rejected step evaluates J again at the same
    state, so the results still equal chem_integrate's bit for bit; two calls,
    the second smaller; a kept Jacobian (jac_every > 1) is refused here."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05681_amd import chem
    L = chem.lib()
    L.chem_integrate_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(chem.Opts), C.c_void_p]
    path, m, o = large
    print("case: chem_integrate_noalloc vs chem_integrate, large,", mode, flush=True)
    sys.stdout.flush()
    mech = chem.Mechanism(path)
    opts = chem.default_opts(mode=mode)
    for n, seed in ((512, 204), (96, 205)):
        T, P, Y = synth.states_mixing(m, n, seed)
        Tt, Pt, Yt = dev(T), dev(P), dev(Y)
        rc, T1, Y1, h1, ns1, st1 = call_noalloc(L, chem, mech, Tt, Pt, Yt, 1e-5, opts)
        assert rc == 0, chem.error_string(rc)
        T2, Y2, h2, ns2, st2 = chem.integrate(mech, Tt, Pt, Yt, 1e-5, opts=opts)
        torch.cuda.synchronize()
        for a, b in ((T1, T2), (Y1, Y2), (h1, h2), (ns1, ns2), (st1, st2)):
            assert torch.equal(a, b)
        assert int((st1 != 0).sum()) == 0
    T, P, Y = synth.states_mixing(m, 64, 3)
    rc, *_ = call_noalloc(L, chem, mech, dev(T), dev(P), dev(Y), 1e-6,
                          chem.default_opts(mode=mode, method="ros34pw2", jac_every=2))
    assert rc == chem.EUNSUPPORTED
    torch.cuda.synchronize()
    mech.close()
