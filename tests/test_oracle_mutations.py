"""Planted mistakes in the oracle must fail its pins.

Each case copies oracle.cpp, applies one plausible mistake (a swapped
constant, a wrong logarithm base, a wrong standard-state unit, a dropped
term), builds the copy into a scratch library and runs the pins that should
catch it.  Only the scratch copy is changed; the library under test is the
unmodified oracle.
"""
import os

import numpy as np
import pytest

import oracle
from test_oracle_chem import gibbs_equilibrium_checks, troe_checks, troe_mechanism
from paper_2205_05681_amd import synth

SRC = open(oracle.SRC).read()

MUTATIONS = {
    # Troe: the 0.67 and 1.27 of c and n swapped
    "troe_c_n_swapped": [("S c = -0.4 - 0.67 * lFc;", "S c = -0.4 - 1.27 * lFc;"),
                         ("S n = 0.75 - 1.27 * lFc;", "S n = 0.75 - 0.67 * lFc;")],
    # Troe: d = 0.24 instead of 0.14
    "troe_d": [("S y = x / (n - 0.14 * x);", "S y = x / (n - 0.24 * x);")],
    # Troe: natural logarithm of F_cent where log10 is meant
    "troe_ln_fcent": [("S lFc = log_(Fc) / LN10;", "S lFc = log_(Fc);")],
    # Troe: natural logarithm of Pr
    "troe_ln_pr": [("S(log_(Pr) / LN10)", "S(log_(Pr))")],
    # K_c: standard-state concentration in mol instead of kmol per m^3
    "kc_units": [("S lnPref = log_(PATM / (RU * T));", "S lnPref = log_(1000.0 * PATM / (RU * T));")],
    # K_c: the standard-state factor dropped
    "kc_no_pref": [("S lnKc = lnKp + dnu * lnPref;", "S lnKc = lnKp;")],
}


def build_variant(tmp_path, name):
    src = SRC
    for old, new in MUTATIONS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    p = tmp_path / ("oracle_%s.cpp" % name)
    p.write_text(src)
    out = str(tmp_path / ("liboracle_%s.so" % name))
    oracle.build(src=str(p), out=out)
    return oracle.lib(out)


@pytest.mark.parametrize("name", ["troe_c_n_swapped", "troe_d", "troe_ln_fcent", "troe_ln_pr"])
def test_troe_mutation_is_caught(tmp_path, name):
    L = build_variant(tmp_path, name)
    path = troe_mechanism(str(tmp_path / "troe.txt"), np.log(1e10), np.log(1e12), 0.3, 800.0, 800.0, 0.0)
    troe_checks(oracle.Oracle(path, library=oracle.lib()))    # the real oracle passes
    with pytest.raises(AssertionError):
        troe_checks(oracle.Oracle(path, library=L))


@pytest.mark.parametrize("name", ["kc_units", "kc_no_pref"])
def test_kc_mutation_is_caught(tmp_path, name, small):
    path, m, _ = small
    L = build_variant(tmp_path, name)
    o = oracle.Oracle(path, library=L)
    T0, P0, Y0 = synth.states_small(m, n=1, seed=21)
    r = o.integrate(T0, P0, Y0, 1e-1, rtol=1e-9, atol=1e-16)
    with pytest.raises(AssertionError):
        assert r["status"][0] == 0
        gibbs_equilibrium_checks(o, m, r["T"][0], P0[0], r["Y"][:, 0])
