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

OK, EINVAL, EPARSE, EHIP, ENOMEM, EUNSUPPORTED, ENONDET = 0, -1, -2, -3, -4, -5, -6
MODE_AUTO, MODE_PLAIN, MODE_PERSISTENT, MODE_TEAM, MODE_TEAM_PERSISTENT = 0, 1, 2, 3, 4
MODES = {"auto": 0, "plain": 1, "persistent": 2, "team": 3, "team_persistent": 4}
METHODS = {"ros4": 0, "ros3": 1, "rodas3": 2, "rodas4": 3, "ros34pw2": 4}
ESTIMATORS = {"embedded": 0, "filtered": 1}
CELL_OK, CELL_MAX_STEPS, CELL_H_MIN, CELL_NONFINITE, CELL_SINGULAR = 0, 1, 2, 3, 4


class ChemError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, error_string(code), code))


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h_min", C.c_double),
                ("safety", C.c_double), ("fac_min", C.c_double), ("fac_max", C.c_double),
                ("T_cut", C.c_double), ("max_steps", C.c_int32), ("mode", C.c_int32),
                ("wg_size", C.c_int32), ("waves_per_cu", C.c_int32), ("order", C.c_int32),
                ("method", C.c_int32), ("estimator", C.c_int32), ("team_waves", C.c_int32),
                ("jac_every", C.c_int32), ("stats", C.c_void_p)]


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
        L.chem_ckpt_records.restype = C.c_int64
        L.chem_ckpt_records.argtypes = [_vp]
        L.chem_ckpt_export.argtypes = [_vp, _vp, _vp]
        L.chem_graph_create.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.c_int64, _vp, _vp, C.c_double,
                                        C.c_double, C.c_double, _vp, _vp, _vp, _vp, C.POINTER(Opts),
                                        C.POINTER(_vp)]
        L.chem_graph_launch.argtypes = [_vp, _vp]
        L.chem_autotune.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.c_int64, C.c_double, C.c_double,
                                    C.c_double, C.POINTER(Opts), _vp, _vp]
        L.chem_graph_free.argtypes = [_vp]
        L.chem_eval.argtypes = [_vp, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp]
        L.chem_lu.argtypes = [C.c_int64, C.c_int32, _vp, C.c_int64, C.c_double, _vp, _vp, _vp, C.c_int32,
                              _vp]
        _lib = L
    return _lib


EXPORTS = ("chem_opts_default", "chem_error_string", "chem_mech_load", "chem_mech_info",
           "chem_mech_free", "chem_integrate", "chem_integrate_adjoint", "chem_ckpt_free", "chem_eval",
           "chem_ckpt_records", "chem_ckpt_export", "chem_graph_create", "chem_graph_launch",
           "chem_graph_free", "chem_autotune", "chem_integrate_noalloc", "chem_lu")


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
        if k == "method" and isinstance(v, str):
            v = METHODS[v]
        if k == "estimator" and isinstance(v, str):
            v = ESTIMATORS[v]
        if k == "stats":
            # a (4,) int64 device tensor that the call adds attempts, accepted,
            # rejected steps and Jacobian evaluations to
            v = _ptr(v, "stats", torch.int64, (4,))
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


class Checkpoint:
    """Accepted steps of a checkpointed integration (chem_ckpt_t)."""

    def __init__(self, mech, handle, n):
        self.mech, self.handle, self.n = mech, handle, n

    def records(self):
        return lib().chem_ckpt_records(self.handle)

    def export(self):
        """(offsets (n+1,), records (R, N+1)) on the host: per cell the accepted
        (Phi_n, h_n), then (Phi_final, 0)."""
        import numpy as np
        off = np.zeros(self.n + 1, np.int64)
        rec = np.zeros((self.records(), self.mech.N + 1))
        _check(lib().chem_ckpt_export(self.handle, off.ctypes.data_as(C.c_void_p),
                                      rec.ctypes.data_as(C.c_void_p)), "chem_ckpt_export")
        return off, rec

    def close(self):
        if getattr(self, "handle", None):
            lib().chem_ckpt_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def integrate(mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, h=None, lnA=None, opts=None,
              out=None, n_steps=None, status=None, checkpoint=False):
    """Advance every cell over dt.  T, P: (n,); Y: (K, n) SoA.  Returns
    (T1, Y1, h1, n_steps, status), plus a Checkpoint when checkpoint=True; h
    is updated in place when given."""
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
    ck = C.c_void_p() if checkpoint else None
    rc = lib().chem_integrate(mech.handle, n, pT, pP, pY, n, _ptr(T1, "T_out", shape=(n,)),
                              _ptr(Y1, "Y_out", shape=(K, n)), float(dt), float(rtol), float(atol),
                              _ptr(h, "h", shape=(n,)), _ptr(n_steps, "n_steps", torch.int32, (n,)),
                              _ptr(status, "status", torch.int32, (n,)),
                              _ptr(lnA, "lnA", shape=(mech.Nr,), allow_none=True), C.byref(o),
                              C.byref(ck) if checkpoint else None, _stream())
    _check(rc, "chem_integrate")
    if checkpoint:
        return T1, Y1, h, n_steps, status, Checkpoint(mech, ck, n)
    return T1, Y1, h, n_steps, status


def adjoint(mech, ckpt, gT, gY, per_cell=False, initial=True):
    """Discrete adjoint of a checkpointed integration.  gT (n,), gY (K, n) are
    dL/dT_final and dL/dY_final.  Returns (g_lnA, gT0, gY0): g_lnA is (Nr,)
    summed over cells, or (Nr, n) per cell; gT0, gY0 are the gradients with
    respect to the initial T and Y (None unless initial)."""
    n = ckpt.n
    dev = gT.device
    g = torch.empty((mech.Nr, n) if per_cell else (mech.Nr,), dtype=torch.float64, device=dev)
    gT0 = torch.empty(n, dtype=torch.float64, device=dev) if initial else None
    gY0 = torch.empty((mech.K, n), dtype=torch.float64, device=dev) if initial else None
    rc = lib().chem_integrate_adjoint(mech.handle, ckpt.handle, _ptr(gT, "gT", shape=(n,)),
                                      _ptr(gY, "gY", shape=(mech.K, n)), n, _ptr(g, "g_lnA"),
                                      1 if per_cell else 0, _ptr(gT0, "gT0", allow_none=True),
                                      _ptr(gY0, "gY0", allow_none=True), _stream())
    _check(rc, "chem_integrate_adjoint")
    return g, gT0, gY0


class IntegrateFn(torch.autograd.Function):
    """(T1, Y1) = IntegrateFn.apply(T, P, Y, lnA, dt, rtol, atol, mech[, opts]):
    the integration as a differentiable function of T, Y and lnA (P, dt and
    the tolerances are constants).  The backward pass is the library's
    discrete adjoint over the checkpointed accepted steps (step sizes
    frozen)."""

    @staticmethod
    def forward(ctx, T, P, Y, lnA, dt, rtol, atol, mech, opts=None):
        T1, Y1, _, _, _, ck = integrate(mech, T.detach().contiguous(), P.detach().contiguous(),
                                        Y.detach().contiguous(), dt, rtol, atol,
                                        lnA=lnA.detach().contiguous(), opts=opts, checkpoint=True)
        ctx.mech, ctx.ck, ctx.device = mech, ck, T.device
        return T1, Y1

    @staticmethod
    def backward(ctx, gT, gY):
        n = ctx.ck.n
        dev = ctx.device
        gT = torch.zeros(n, dtype=torch.float64, device=dev) if gT is None else gT.contiguous()
        gY = torch.zeros((ctx.mech.K, n), dtype=torch.float64, device=dev) if gY is None else gY.contiguous()
        g, gT0, gY0 = adjoint(ctx.mech, ctx.ck, gT, gY, per_cell=False, initial=True)
        ctx.ck.close()
        return gT0, None, gY0, g, None, None, None, None, None


def autotune(mech, T, P, Y, dt, rtol=1e-6, atol=1e-10):
    """Run the library's autotuner on this batch; returns (chosen Opts, list of
    candidate times in ms)."""
    import numpy as np
    n = T.numel()
    o = Opts()
    ms = np.zeros(8)
    rc = lib().chem_autotune(mech.handle, n, _ptr(T, "T", shape=(n,)), _ptr(P, "P", shape=(n,)),
                             _ptr(Y, "Y", shape=(mech.K, n)), n, float(dt), float(rtol), float(atol),
                             C.byref(o), ms.ctypes.data_as(C.c_void_p), _stream())
    _check(rc, "chem_autotune")
    return o, [float(x) for x in ms if x >= 0]


class Graph:
    """One split step captured in a HIP graph (chem_graph_create).  The tensors
    given here are the ones every replay reads and writes."""

    def __init__(self, mech, T, P, Y, dt, rtol=1e-6, atol=1e-10, out=None, h=None, n_steps=None,
                 status=None, lnA=None, opts=None):
        n, K = T.numel(), mech.K
        self.mech = mech
        self.T1, self.Y1 = out if out is not None else (torch.empty_like(T), torch.empty_like(Y))
        self.h, self.n_steps, self.status = h, n_steps, status
        self._keep = (T, P, Y, lnA)
        o = opts if opts is not None else default_opts()
        g = C.c_void_p()
        rc = lib().chem_graph_create(mech.handle, n, _ptr(T, "T", shape=(n,)), _ptr(P, "P", shape=(n,)),
                                     _ptr(Y, "Y", shape=(K, n)), n, _ptr(self.T1, "T_out", shape=(n,)),
                                     _ptr(self.Y1, "Y_out", shape=(K, n)), float(dt), float(rtol),
                                     float(atol), _ptr(h, "h", shape=(n,), allow_none=True),
                                     _ptr(n_steps, "n_steps", torch.int32, (n,), allow_none=True),
                                     _ptr(status, "status", torch.int32, (n,), allow_none=True),
                                     _ptr(lnA, "lnA", shape=(mech.Nr,), allow_none=True), C.byref(o),
                                     C.byref(g))
        _check(rc, "chem_graph_create")
        self.handle = g

    def launch(self):
        _check(lib().chem_graph_launch(self.handle, _stream()), "chem_graph_launch")
        return self.T1, self.Y1

    def close(self):
        if getattr(self, "handle", None):
            lib().chem_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LU_LAUNCHES = {"team": 0, "thread": 1}


def lu(A, d, launch="team"):
    """LU with partial pivoting of M = d I - A for n matrices A (N*N, n) (the
    layout of evaluate's J), by the team launches' routine ("team") or the
    one-cell-per-thread launches' ("thread").  Returns the factors F (N*N, n)
    in pivot order, perm (N, n) int32 (the row of M pivoted at each step) and
    status (n,) int32."""
    NN, n = A.shape
    N = int(round(NN ** 0.5))
    if N * N != NN:
        raise ValueError("A must have N*N rows")
    F = torch.empty_like(A)
    perm = torch.empty((N, n), dtype=torch.int32, device=A.device)
    status = torch.empty((n,), dtype=torch.int32, device=A.device)
    rc = lib().chem_lu(n, N, _ptr(A, "A"), n, float(d), _ptr(F, "F"), _ptr(perm, "perm", dtype=torch.int32),
                       _ptr(status, "status", dtype=torch.int32), LU_LAUNCHES[launch], _stream())
    _check(rc, "chem_lu")
    return F, perm, status


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
