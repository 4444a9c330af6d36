"""Python binding of libchem.so (the HIP integrator).

Argument marshalling only: torch tensors provide device memory and the
current stream; every step of the integration runs in the library's HIP
kernels.  The binding fails loudly when the library is missing or when a
tensor is not an FP64 device tensor of the expected shape - there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchem.so")

OK, EINVAL, EPARSE, EHIP, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MODE_AUTO, MODE_PLAIN, MODE_PERSISTENT, MODE_TEAM, MODE_TEAM_PERSISTENT = 0, 1, 2, 3, 4
MODES = {"auto": 0, "plain": 1, "persistent": 2, "team": 3, "team_persistent": 4}
CELL_OK, CELL_MAX_STEPS, CELL_H_MIN, CELL_NONFINITE, CELL_SINGULAR = 0, 1, 2, 3, 4


class ChemError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, error_string(code), code))


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h_min", C.c_double),
                ("safety", C.c_double), ("fac_min", C.c_double), ("fac_max", C.c_double),
                ("T_cut", C.c_double), ("max_steps", C.c_int32), ("mode", C.c_int32),
                ("wg_size", C.c_int32), ("waves_per_cu", C.c_int32), ("stats", C.c_void_p)]


_vp = C.c_void_p
_lib = None


def lib():
    """Load libchem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libchem.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.chem_opts_default.argtypes = [C.POINTER(Opts)]
        L.chem_error_string.restype = C.c_char_p
        L.chem_error_string.argtypes = [C.c_int]
        L.chem_mech_load.argtypes = [C.c_char_p, C.c_int, C.POINTER(_vp)]
        L.chem_mech_info.argtypes = [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.chem_mech_free.argtypes = [_vp]
        L.chem_integrate.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.c_int64, _vp, _vp, C.c_double,
                                     C.c_double, C.c_double, _vp, _vp, _vp, _vp, C.POINTER(Opts),
                                     C.POINTER(_vp), _vp]
        L.chem_integrate_adjoint.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, _vp, C.c_int32, _vp, _vp, _vp]
        L.chem_ckpt_free.argtypes = [_vp]
        L.chem_eval.argtypes = [_vp, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp]
        _lib = L
    return _lib


EXPORTS = ("chem_opts_default", "chem_error_string", "chem_mech_load", "chem_mech_info",
           "chem_mech_free", "chem_integrate", "chem_integrate_adjoint", "chem_ckpt_free", "chem_eval")


def error_string(code):
    try:
        return lib().chem_error_string(code).decode()
    except ImportError:
        return "error"


def _check(rc, what):
    if rc != OK:
        raise ChemError(rc, what)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, dtype=torch.float64, shape=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return C.c_void_p(t.data_ptr())


def default_opts(**kw):
    o = Opts()
    lib().chem_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = MODES[v]
        if k == "stats":
            # a (3,) int64 device tensor that the call adds attempts/accepted/rejected to
            v = _ptr(v, "stats", torch.int64, (3,))
        setattr(o, k, v)
    return o


class Mechanism:
    """A mechanism file loaded into device tables (chem_mech_load)."""

    def __init__(self, path, device=None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = C.c_void_p()
        _check(lib().chem_mech_load(str(path).encode(), int(device), C.byref(h)), "chem_mech_load")
        self.handle = h
        K, Nr, E = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().chem_mech_info(h, C.byref(K), C.byref(Nr), C.byref(E)), "chem_mech_info")
        self.K, self.Nr, self.E = K.value, Nr.value, E.value
        self.N = self.K + 1

    def close(self):
        if getattr(self, "handle", None):
            lib().chem_mech_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def integrate(mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, h=None, lnA=None, opts=None,
              out=None, n_steps=None, status=None):
    """Advance every cell over dt.  T, P: (n,); Y: (K, n) SoA.  Returns
    (T1, Y1, h1, n_steps, status); h is updated in place when given."""
    n = T.numel()
    K = mech.K
    dev = T.device
    pT = _ptr(T, "T", shape=(n,))
    pP = _ptr(P, "P", shape=(n,))
    pY = _ptr(Y, "Y", shape=(K, n))
    if out is None:
        T1 = torch.empty_like(T)
        Y1 = torch.empty_like(Y)
    else:
        T1, Y1 = out
    if h is None:
        h = torch.zeros(n, dtype=torch.float64, device=dev)
    if n_steps is None:
        n_steps = torch.empty(n, dtype=torch.int32, device=dev)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=dev)
    o = opts if opts is not None else default_opts()
    rc = lib().chem_integrate(mech.handle, n, pT, pP, pY, n, _ptr(T1, "T_out", shape=(n,)),
                              _ptr(Y1, "Y_out", shape=(K, n)), float(dt), float(rtol), float(atol),
                              _ptr(h, "h", shape=(n,)), _ptr(n_steps, "n_steps", torch.int32, (n,)),
                              _ptr(status, "status", torch.int32, (n,)),
                              _ptr(lnA, "lnA", shape=(mech.Nr,), allow_none=True), C.byref(o), None,
                              _stream())
    _check(rc, "chem_integrate")
    return T1, Y1, h, n_steps, status


def evaluate(mech, phi, P, lnA=None, jacobian=True):
    """f(Phi) (N, n) and, if asked, J (N*N, n) for states phi (N, n)."""
    N, n = phi.shape
    assert N == mech.N
    f = torch.empty_like(phi)
    J = torch.empty((N * N, n), dtype=torch.float64, device=phi.device) if jacobian else None
    rc = lib().chem_eval(mech.handle, n, _ptr(phi, "phi"), n, _ptr(P, "P", shape=(n,)),
                         _ptr(lnA, "lnA", shape=(mech.Nr,), allow_none=True), _ptr(f, "f"),
                         _ptr(J, "J", allow_none=True), _stream())
    _check(rc, "chem_eval")
    return f, J
