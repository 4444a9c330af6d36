"""hipGraph-captured split steps and the autotuner, through the C ABI."""
import os
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


@pytest.mark.parametrize("name,mode,n", [("ch4", "auto", 1000), ("small", "plain", 256),
                                         ("small", "team_persistent", 256)])
def test_graph_replays_equal_direct_launch(chem, name, mode, n, request):
    path, m, o = request.getfixturevalue(name)
    say("case: graph replay", name, mode, n)
    T, P, Y = (synth.states_mixing(m, n, 202) if name == "ch4" else synth.states_small(m, n))
    mech = chem.Mechanism(path)
    Tt, Pt, Yt = dev(T), dev(P), dev(Y)
    opts = chem.default_opts(mode=mode)
    T1, Y1, _, ns, _ = chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=opts)
    torch.cuda.synchronize()
    ref_T, ref_Y, ref_n = T1.cpu().numpy(), Y1.cpu().numpy(), ns.cpu().numpy()
    h = torch.zeros(n, dtype=torch.float64, device="cuda")
    ns_g = torch.empty(n, dtype=torch.int32, device="cuda")
    g = chem.Graph(mech, Tt, Pt, Yt, 1e-6, h=h, n_steps=ns_g, opts=opts)
    for rep in range(3):
        h.zero_()                                   # the step overwrites h
        g.T1.fill_(-1.0)
        g.launch()
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(g.T1.cpu().numpy(), ref_T), rep
        assert np.array_equal(g.Y1.cpu().numpy(), ref_Y), rep
        assert np.array_equal(ns_g.cpu().numpy(), ref_n), rep
    g.close()
    mech.close()


def test_autotuner_choice_is_used_and_cached(chem, ch4, tmp_path):
    path, m, o = ch4
    say("case: autotune ch4 4096 cells")
    cache = tmp_path / "tune.txt"
    os.environ["CHEM_AUTOTUNE_CACHE"] = str(cache)
    try:
        mech = chem.Mechanism(path)
        T, P, Y = synth.states_mixing(m, 4096, 202)
        Tt, Pt, Yt = dev(T), dev(P), dev(Y)
        chosen, ms = chem.autotune(mech, Tt, Pt, Yt, 1e-6)
        assert len(ms) >= 2 and min(ms) > 0
        assert chosen.mode in (1, 2, 3, 4)
        # AUTO now runs the chosen configuration
        a = chem.integrate(mech, Tt, Pt, Yt, 1e-6)
        b = chem.integrate(mech, Tt, Pt, Yt, 1e-6, opts=chosen)
        torch.cuda.synchronize()
        assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
        assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
        mech.close()
        line = cache.read_text().strip().splitlines()[-1]
        assert line.startswith("N54 Nr325 ") and line.endswith(
            "%d %d %d" % (chosen.mode, chosen.wg_size, chosen.waves_per_cu))
        # a new handle of the same shape reads the cache back
        mech2 = chem.Mechanism(path)
        c = chem.integrate(mech2, Tt, Pt, Yt, 1e-6)
        torch.cuda.synchronize()
        assert np.array_equal(c[0].cpu().numpy(), b[0].cpu().numpy())
        mech2.close()
    finally:
        del os.environ["CHEM_AUTOTUNE_CACHE"]
