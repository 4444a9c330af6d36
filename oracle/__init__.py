"""ctypes shim for the CPU FP64 oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  It imports nothing
from the library package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.cpp")
# The same source built with fused multiply-adds contracted: a rounding-level
# variant of the oracle (the kind of difference a GPU build has), used by the
# parity tests to measure how far rounding alone moves each cell.
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")
FMA_FLAGS = ("-mfma", "-ffp-contract=fast")

_d = C.POINTER(C.c_double)
_i = C.POINTER(C.c_int32)


FLAGS = ["-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC"]


def build_all(force=True):
    """The oracle and its FMA-contracted variant."""
    build(force)
    build(force, out=LIB_FMA, flags=FMA_FLAGS)


def build(force=True, src=SRC, out=LIB, flags=()):
    """Compile the oracle with g++ (OpenMP over cells).  src/out/flags let a
    test build a variant (other floating-point flags, or a planted mistake)."""
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", *FLAGS, *flags, src, "-o", tmp])
    os.replace(tmp, out)
    return out


_lib = None


def lib(path=None):
    """The oracle library (built on first use), or the one at ``path``."""
    global _lib
    if path is not None or _lib is None:
        if path is None and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = C.CDLL(path or LIB)
        L.or_mech_load.restype = C.c_void_p
        L.or_mech_load.argtypes = [C.c_char_p]
        L.or_mech_free.argtypes = [C.c_void_p]
        L.or_mech_dims.argtypes = [C.c_void_p, _i, _i, _i]
        L.or_mech_arrays.argtypes = [C.c_void_p, _d, _i, _d]
        L.or_thermo.argtypes = [C.c_void_p, C.c_double, _d, _d, _d]
        L.or_kinetics.argtypes = [C.c_void_p, C.c_double, C.c_double, _d, _d, _d, _d, _d, _d]
        L.or_rhs.argtypes = [C.c_void_p, C.c_double, _d, _d, _d]
        L.or_jacobian.argtypes = [C.c_void_p, C.c_double, _d, _d, _d]
        L.or_lu_solve.argtypes = [C.c_int, _d, _d, _d]
        L.or_lu.restype = C.c_int
        L.or_lu.argtypes = [C.c_int, _d, _d, C.POINTER(C.c_int), _d]
        L.or_method_table.argtypes = [C.c_int, _d]
        L.or_step.argtypes = [C.c_void_p, C.c_double, _d, C.c_double, _d, _d, C.c_int, C.c_int]
        L.or_to_phi.argtypes = [C.c_void_p, C.c_double, C.c_double, _d, _d]
        L.or_from_phi.argtypes = [C.c_void_p, C.c_double, _d, _d, _d]
        L.or_integrate.restype = C.c_int
        L.or_integrate.argtypes = [C.c_void_p, C.c_int64, _d, _d, _d, C.c_int64, C.c_double, C.c_double,
                                   C.c_double, _d, _d, _d, _i, _i, _i, _d, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int]
        L.or_record_steps.argtypes = [C.c_void_p, C.c_double, C.c_double, _d, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _d, _d, C.c_int, _d, _d, C.c_int, C.c_int,
                                      C.c_int]
        L.or_replay.argtypes = [C.c_void_p, C.c_double, C.c_double, _d, _d, _d, C.c_int, _d, _d, C.c_int]
        L.or_tangent.argtypes = [C.c_void_p, C.c_double, C.c_double, _d, _d, _d, C.c_int, _d,
                                 C.c_double, _d, _d, _d, C.c_int]
        L.or_integrate_linear.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.c_int]
        L.or_linear_step.argtypes = [C.c_int, _d, _d, C.c_double, _d, _d, C.c_int, C.c_int, _d]
        L.or_integrate_cubic.argtypes = [_d, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                           C.c_int, C.c_int]
        if path is not None:
            return L
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags.c_contiguous
    if a.dtype == np.float64:
        return a.ctypes.data_as(_d)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_i)
    raise TypeError(a.dtype)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


R_U = 8314.462618
P_ATM = 101325.0

# Rosenbrock solvers of the paper's solver table and the error estimators
METHODS = {"ros4": 0, "ros3": 1, "rodas3": 2, "rodas4": 3, "ros34pw2": 4}
ESTIMATORS = {"embedded": 0, "filtered": 1}


def _mid(method):
    return METHODS[method] if isinstance(method, str) else int(method)


def _eid(estimator):
    return ESTIMATORS[estimator] if isinstance(estimator, str) else int(estimator)


class Oracle:
    """One parsed mechanism in the oracle."""

    def __init__(self, path, library=None):
        self.L = library if library is not None else lib()
        self.path = path
        self.h = self.L.or_mech_load(path.encode())
        if not self.h:
            raise ValueError("oracle could not parse %s" % path)
        K, Nr, E = C.c_int32(), C.c_int32(), C.c_int32()
        self.L.or_mech_dims(self.h, C.byref(K), C.byref(Nr), C.byref(E))
        self.K, self.Nr, self.E = K.value, Nr.value, E.value
        self.N = self.K + 1
        self.W = np.zeros(self.K)
        self.comp = np.zeros((self.K, self.E), np.int32)
        self.lnA = np.zeros(self.Nr)
        self.L.or_mech_arrays(self.h, _p(self.W), _p(self.comp), _p(self.lnA))

    def __del__(self):
        try:
            self.L.or_mech_free(self.h)
        except Exception:
            pass

    # -- pieces ---------------------------------------------------------------
    def thermo(self, T):
        cp, h, s = (np.zeros(self.K) for _ in range(3))
        self.L.or_thermo(self.h, float(T), _p(cp), _p(h), _p(s))
        return cp, h, s

    def kinetics(self, T, P, Cc, lnA=None):
        Cc = _f64(Cc)
        q, kf, kr = (np.zeros(self.Nr) for _ in range(3))
        w = np.zeros(self.K)
        self.L.or_kinetics(self.h, float(T), float(P), _p(Cc), _p(_f64(lnA)), _p(q), _p(w), _p(kf), _p(kr))
        return q, w, kf, kr

    def rhs(self, P, phi, lnA=None):
        f = np.zeros(self.N)
        self.L.or_rhs(self.h, float(P), _p(_f64(phi)), _p(_f64(lnA)), _p(f))
        return f

    def jacobian(self, P, phi, lnA=None):
        J = np.zeros((self.N, self.N))
        self.L.or_jacobian(self.h, float(P), _p(_f64(phi)), _p(_f64(lnA)), _p(J))
        return J

    def step(self, P, phi, h, method="ros4", estimator="embedded"):
        out, err = np.zeros(self.N), np.zeros(self.N)
        rc = self.L.or_step(self.h, float(P), _p(_f64(phi)), float(h), _p(out), _p(err), _mid(method),
                            _eid(estimator))
        return rc, out, err

    def to_phi(self, T, P, Y):
        phi = np.zeros(self.N)
        self.L.or_to_phi(self.h, float(T), float(P), _p(_f64(Y)), _p(phi))
        return phi

    def from_phi(self, P, phi):
        T = np.zeros(1)
        Y = np.zeros(self.K)
        self.L.or_from_phi(self.h, float(P), _p(_f64(phi)), _p(T), _p(Y))
        return T[0], Y

    # -- batched integration ---------------------------------------------------
    def integrate(self, T, P, Y, dt, rtol=1e-6, atol=1e-10, h=None, lnA=None, max_steps=0,
                  nthreads=0, method="ros4", estimator="embedded", jac_every=1):
        """Y is (K, n).  Returns dict with T, Y, h, n_acc, n_rej, status, threads.
        jac_every: J evaluated at every jac_every-th accepted state and kept
        in between (a W-method keeps its order with such a J)."""
        T = _f64(T)
        P = _f64(P)
        Y = _f64(Y)
        n = T.size
        assert Y.shape == (self.K, n)
        Tout = np.zeros(n)
        Yout = np.zeros_like(Y)
        hio = np.zeros(n) if h is None else _f64(h).copy()
        na, nr, st = (np.zeros(n, np.int32) for _ in range(3))
        thr = self.L.or_integrate(self.h, n, _p(T), _p(P), _p(Y), n, float(dt), float(rtol), float(atol),
                                  _p(hio), _p(Tout), _p(Yout), _p(na), _p(nr), _p(st), _p(_f64(lnA)),
                                  int(max_steps), int(nthreads), _mid(method), _eid(estimator), int(jac_every))
        if thr < 0:
            raise ValueError("unknown method")
        return dict(T=Tout, Y=Yout, h=hio, n_acc=na, n_rej=nr, status=st, threads=thr)

    def record_steps(self, T, P, Y, dt, rtol=1e-6, atol=1e-10, h0=0.0, lnA=None, cap=1000000,
                     method="ros4", estimator="embedded", jac_every=1):
        hs = np.zeros(cap)
        To = np.zeros(1)
        Yo = np.zeros(self.K)
        n = self.L.or_record_steps(self.h, float(T), float(P), _p(_f64(Y)), float(dt), float(rtol),
                                   float(atol), float(h0), _p(_f64(lnA)), _p(hs), cap, _p(To), _p(Yo),
                                   _mid(method), _eid(estimator), int(jac_every))
        if n < 0:
            raise RuntimeError("oracle integration failed with status %d" % -n)
        return hs[:n].copy(), To[0], Yo

    def replay(self, T, P, Y, hs, lnA=None, method="ros4"):
        To = np.zeros(1)
        Yo = np.zeros(self.K)
        hs = _f64(hs)
        rc = self.L.or_replay(self.h, float(T), float(P), _p(_f64(Y)), _p(_f64(lnA)), _p(hs), hs.size,
                              _p(To), _p(Yo), _mid(method))
        if rc:
            raise RuntimeError("replay failed")
        return To[0], Yo

    def tangent(self, T, P, Y, hs, v_lnA=None, dT0=0.0, dY0=None, lnA=None, method="ros4"):
        dT = np.zeros(1)
        dY = np.zeros(self.K)
        hs = _f64(hs)
        self.L.or_tangent(self.h, float(T), float(P), _p(_f64(Y)), _p(_f64(lnA)), _p(hs), hs.size,
                          _p(_f64(v_lnA)), float(dT0), _p(_f64(dY0)), _p(dT), _p(dY), _mid(method))
        return dT[0], dY


def method_table(method="ros4"):
    """The transformed coefficients of a method: dict with s, gamma, elo and the
    arrays a (s, s), c (s, s), m (s,), e (s,)."""
    t = np.zeros(87)
    if lib().or_method_table(_mid(method), _p(t)):
        raise ValueError(method)
    s = int(t[0])
    return dict(s=s, gamma=t[1], elo=t[2], a=t[3:39].reshape(6, 6)[:s, :s].copy(),
                c=t[39:75].reshape(6, 6)[:s, :s].copy(), m=t[75:75 + s].copy(), e=t[81:81 + s].copy())


def lu_solve(A, b):
    A = _f64(A)
    b = _f64(b)
    x = np.zeros_like(b)
    rc = lib().or_lu_solve(b.size, _p(A), _p(b), _p(x))
    if rc:
        raise np.linalg.LinAlgError("singular")
    return x


def lu(M):
    """LU with partial pivoting of the square matrix M: (F, perm, status,
    margin) - the factors in pivot order (row k: L left of the diagonal, unit
    diagonal implied, U from the diagonal on; row k of L U is row perm[k] of
    M), 0/1/2 as the library's status, and the smallest relative gap between a
    pivot and the runner-up of its column."""
    M = _f64(M)
    n = M.shape[0]
    F = np.zeros_like(M)
    perm = np.zeros(n, dtype=np.intc)
    margin = np.zeros(1)
    rc = lib().or_lu(n, _p(M), _p(F), perm.ctypes.data_as(C.POINTER(C.c_int)), _p(margin))
    return F, perm.astype(np.int64), int(rc), float(margin[0])


def integrate_linear(A, y0, dt, rtol=1e-6, atol=1e-10, h_fixed=0.0, method="ros4", estimator="embedded"):
    A = _f64(A)
    y = _f64(y0).copy()
    n = lib().or_integrate_linear(y.size, _p(A), _p(y), float(dt), float(rtol), float(atol), float(h_fixed),
                                  _mid(method), _eid(estimator))
    return y, n


def linear_step(A, y0, h, method="ros4", estimator="embedded", Ajac=None):
    """One step of y' = A y: (y_new, error estimate).  Ajac (optional) stands
    in for the Jacobian A."""
    A = _f64(A)
    y = _f64(y0)
    out, err = np.zeros_like(y), np.zeros_like(y)
    rc = lib().or_linear_step(y.size, _p(A), _p(y), float(h), _p(out), _p(err), _mid(method), _eid(estimator),
                              _p(_f64(Ajac)))
    if rc:
        raise np.linalg.LinAlgError("step failed")
    return out, err


def integrate_cubic(y0, dt, rtol=1e-6, atol=1e-10, h_fixed=0.0, method="ros4", estimator="embedded",
                    jac_every=1):
    """y' = -y^3 from y0 over [0, dt]; jac_every > 1 keeps the Jacobian of
    every jac_every-th step's state in between."""
    y = np.array([float(y0)])
    n = lib().or_integrate_cubic(_p(y), float(dt), float(rtol), float(atol), float(h_fixed), _mid(method),
                                   _eid(estimator), int(jac_every))
    return y[0], n
