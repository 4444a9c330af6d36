"""The C-ABI library loads and exports every entry point chem.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "chem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chem_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("chem_mech_load", "chem_integrate", "chem_integrate_adjoint", "chem_mech_free",
                 "chem_ckpt_free", "chem_error_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2205_05681_amd import chem
    L = ctypes.CDLL(chem.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(chem.EXPORTS) <= set(declared())


def test_error_strings_and_defaults_without_gpu():
    from paper_2205_05681_amd import chem
    assert chem.error_string(chem.EINVAL) == "invalid argument"
    o = chem.default_opts()
    assert o.rtol == 1e-6 and o.atol == 1e-10 and o.max_steps == 100000
    assert o.safety == 0.9 and o.fac_min == 0.2 and o.fac_max == 6.0


def test_mechanism_parse_errors_without_gpu(tmp_path):
    from paper_2205_05681_amd import chem
    L = chem.lib()
    h = ctypes.c_void_p()
    bad = tmp_path / "bad.txt"
    bad.write_text("CHEMMECH 1\nELEMENTS 1 H\nSPECIES 2\nH 1.0 1 1000\n")
    assert L.chem_mech_load(str(bad).encode(), 0, ctypes.byref(h)) == chem.EPARSE
    assert L.chem_mech_load(str(tmp_path / "missing.txt").encode(), 0, ctypes.byref(h)) == chem.EPARSE
    assert L.chem_mech_load(None, 0, ctypes.byref(h)) == chem.EINVAL


def test_opts_struct_layout_matches_the_header():
    """chem_opts_default writes exactly the Python Opts structure: nothing past
    its end (a sentinel tail survives) and the last field, the stats pointer,
    is set (to null)."""
    from paper_2205_05681_amd import chem
    size = ctypes.sizeof(chem.Opts)
    buf = (ctypes.c_ubyte * (size + 64))(*([0xAB] * (size + 64)))
    chem.lib().chem_opts_default(ctypes.cast(buf, ctypes.POINTER(chem.Opts)))
    assert bytes(buf[size:]) == b"\xab" * 64
    o = chem.Opts.from_buffer(buf)
    assert o.stats is None
    assert o.method == 0 and o.estimator == 0 and o.team_waves == 0 and o.order == 1
    assert o.jac_every == 1
