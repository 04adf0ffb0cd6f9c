"""ctypes binding of the plain FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the CPU-baseline leg of the benchmark.  The GPU library never imports,
links or calls it, and it shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "rhs_body.h")]

STATUS = {0: "OK", 1: "MAX_STEPS", 2: "ERR_FAIL", 3: "CONV_FAIL", 4: "NAN"}
COUNTER_NAMES = ("nst", "nfe", "nje", "nni", "netf", "ncfn")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_ip_opt = C.c_void_p

USER_F = C.CFUNCTYPE(None, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-o", LIB_PATH, os.path.join(HERE, "oracle.c"), "-lm"]
        subprocess.check_call(cmd)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.om_load.restype = C.c_void_p
        L.om_load.argtypes = [C.c_char_p]
        L.om_free.argtypes = [C.c_void_p]
        L.om_info.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), _dp]
        L.om_thermo.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp]
        L.om_rates.argtypes = [C.c_void_p, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.om_rhs.argtypes = [C.c_void_p, C.c_double, _dp, _dp]
        L.om_jac.argtypes = [C.c_void_p, C.c_double, _dp, _dp]
        L.om_jac_cs.argtypes = [C.c_void_p, C.c_double, _dp, _dp]
        L.om_enthalpy.restype = C.c_double
        L.om_enthalpy.argtypes = [C.c_void_p, C.c_double, _dp]
        L.om_T_from_h.restype = C.c_double
        L.om_T_from_h.argtypes = [C.c_void_p, C.c_double, _dp, C.c_double, C.POINTER(C.c_int)]
        L.om_lu.argtypes = [C.c_int, _dp, _ip]
        L.om_lu_solve.argtypes = [C.c_int, _dp, _ip, _dp]
        L.om_bdf_coeffs.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp]
        L.om_integrate.restype = C.c_int
        L.om_integrate.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, _dp, C.c_int64, C.c_double,
                                   C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _ip_opt, _ip_opt]
        L.om_bdf_user.argtypes = [C.c_int, USER_F, USER_F, C.c_void_p, _dp, C.c_double, C.c_double,
                                  C.c_double, C.c_int, C.c_int, _ip]
        L.om_bdf_user_trace.argtypes = [C.c_int, USER_F, USER_F, C.c_void_p, _dp, C.c_double, C.c_double,
                                        C.c_double, C.c_int, C.c_int, _ip, _dp, C.c_int, C.POINTER(C.c_int)]
        L.om_order_change.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.om_bdf_prescribed.argtypes = [C.c_int, USER_F, USER_F, C.c_void_p, C.c_int, C.c_double,
                                        _dp, _dp, C.c_int, _dp]
        L.om_rk4.argtypes = [C.c_void_p, C.c_double, _dp, C.c_double, C.c_int64]
        _lib = L
    return _lib


class OracleMech:
    """A mechanism loaded by the oracle's own reader."""

    def __init__(self, path: str):
        self.path = path
        self.h = lib().om_load(path.encode())
        if not self.h:
            raise ValueError(f"oracle could not parse mechanism {path}")
        K, R, E = C.c_int(), C.c_int(), C.c_int()
        W = np.zeros(64)
        lib().om_info(self.h, C.byref(K), C.byref(R), C.byref(E), W)
        self.K, self.R, self.E = K.value, R.value, E.value
        self.N = self.K + 1
        self.W = W[: self.K].copy()

    def __del__(self):
        try:
            if self.h:
                lib().om_free(self.h)
        except Exception:
            pass

    # -- pointwise functions ------------------------------------------------
    def thermo(self, T: float):
        cp, h, s = np.zeros(self.K), np.zeros(self.K), np.zeros(self.K)
        lib().om_thermo(self.h, float(T), cp, h, s)
        return cp, h, s

    def rates(self, T: float, p: float, Y):
        kf, kr, q, wd = np.zeros(max(self.R, 1)), np.zeros(max(self.R, 1)), np.zeros(max(self.R, 1)), np.zeros(self.K)
        lib().om_rates(self.h, float(T), float(p), np.ascontiguousarray(Y, dtype=np.float64), kf, kr, q, wd)
        return kf[: self.R], kr[: self.R], q[: self.R], wd

    def rhs(self, p: float, y):
        f = np.zeros(self.N)
        lib().om_rhs(self.h, float(p), np.ascontiguousarray(y, dtype=np.float64), f)
        return f

    def jac(self, p: float, y):
        J = np.zeros(self.N * self.N)
        lib().om_jac(self.h, float(p), np.ascontiguousarray(y, dtype=np.float64), J)
        return J.reshape(self.N, self.N)

    def jac_cs(self, p: float, y):
        J = np.zeros(self.N * self.N)
        lib().om_jac_cs(self.h, float(p), np.ascontiguousarray(y, dtype=np.float64), J)
        return J.reshape(self.N, self.N)

    def enthalpy(self, T: float, Y) -> float:
        return lib().om_enthalpy(self.h, float(T), np.ascontiguousarray(Y, dtype=np.float64))

    def T_from_h(self, h0: float, Y, T_guess: float):
        it = C.c_int()
        T = lib().om_T_from_h(self.h, float(h0), np.ascontiguousarray(Y, dtype=np.float64),
                              float(T_guess), C.byref(it))
        return T, it.value

    def rk4(self, p: float, y, dt: float, nsteps: int):
        yy = np.array(y, dtype=np.float64)
        bad = lib().om_rk4(self.h, float(p), yy, float(dt), int(nsteps))
        return yy, bad

    # -- batch integration -------------------------------------------------
    def integrate(self, T, p, Y, dt: float, rtol: float = 1e-8, atol: float = 1e-12,
                  max_steps: int = 20000, nthreads: int = 0, qmax: int = 5):
        """Integrate cells over [0, dt] with orders up to qmax.  Returns (T, Y,
        status, counters, threads)."""
        T = np.array(T, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64, order="C")
        n = T.shape[0]
        status = np.zeros(n, dtype=np.int32)
        counters = np.zeros((n, 6), dtype=np.int32)
        used = lib().om_integrate(self.h, n, T, p, Y, Y.shape[1], float(dt), float(rtol), float(atol),
                                  int(max_steps), int(qmax), int(nthreads), status.ctypes.data,
                                  counters.ctypes.data)
        return T, Y, status, counters, used


def lu(M):
    A = np.array(M, dtype=np.float64)
    N = A.shape[0]
    flat = A.reshape(-1).copy()
    piv = np.zeros(N, dtype=np.int32)
    bad = lib().om_lu(N, flat, piv)
    return flat.reshape(N, N), piv, bad


def lu_solve(LU, piv, b):
    x = np.array(b, dtype=np.float64)
    lib().om_lu_solve(LU.shape[0], np.ascontiguousarray(LU).reshape(-1), np.ascontiguousarray(piv, dtype=np.int32), x)
    return x


def bdf_coeffs(q: int, h: float, tau):
    t = np.zeros(8)
    t[: len(tau)] = tau
    xi, l = np.zeros(8), np.zeros(8)
    lib().om_bdf_coeffs(q, float(h), t, xi, l)
    return xi[1: q + 2].copy(), l[: q + 1].copy()


def _wrap_user(N, fn):
    def cb(t, yp, outp, _):
        y = np.ctypeslib.as_array(yp, shape=(N,))
        out = np.ctypeslib.as_array(outp, shape=(fn.__out_size__,))
        out[:] = fn(t, y.copy())
    return USER_F(cb)


def bdf_user(f, jac, y0, t_end: float, rtol=1e-8, atol=1e-12, max_steps=100000, qmax=5):
    """Controlled BDF integration of a user ODE, orders up to qmax (pins of the integrator)."""
    y = np.array(y0, dtype=np.float64)
    N = y.size
    f.__out_size__ = N
    jac.__out_size__ = N * N
    cf, cj = _wrap_user(N, f), _wrap_user(N, lambda t, yy: np.asarray(jac(t, yy)).reshape(-1))
    cj_fn = lambda t, yy: np.asarray(jac(t, yy)).reshape(-1)
    cj_fn.__out_size__ = N * N
    cj = _wrap_user(N, cj_fn)
    counters = np.zeros(6, dtype=np.int32)
    st = lib().om_bdf_user(N, cf, cj, None, y, float(t_end), float(rtol), float(atol), int(max_steps), int(qmax),
                           counters)
    return y, st, counters


def bdf_user_trace(f, jac, y0, t_end: float, rtol=1e-8, atol=1e-12, max_steps=100000, qmax=5, cap=100000):
    """bdf_user, also returning every accepted step as rows (t, h, q, dsm,
    failed attempts before it was accepted)."""
    y = np.array(y0, dtype=np.float64)
    N = y.size
    f.__out_size__ = N
    cj_fn = lambda t, yy: np.asarray(jac(t, yy)).reshape(-1)
    cj_fn.__out_size__ = N * N
    cf, cj = _wrap_user(N, f), _wrap_user(N, cj_fn)
    counters = np.zeros(6, dtype=np.int32)
    trace = np.zeros(5 * cap)
    nrec = C.c_int()
    st = lib().om_bdf_user_trace(N, cf, cj, None, y, float(t_end), float(rtol), float(atol), int(max_steps),
                                 int(qmax), counters, trace, int(cap), C.byref(nrec))
    return y, st, counters, trace[: 5 * nrec.value].reshape(-1, 5).copy()


def order_change(q: int, qnew: int, xi, l, e, z):
    """The integrator's order change of a Nordsieck array z ((max(q,qnew)+1) x N)
    with the step's xi[1..q+1] (xi[0] unused), l[0..q] and correction e."""
    z = np.array(z, dtype=np.float64)
    rows, N = z.shape
    flat = np.ascontiguousarray(z.reshape(-1))
    xi8 = np.zeros(8)
    xi8[: len(xi)] = xi
    l8 = np.zeros(8)
    l8[: len(l)] = l
    lib().om_order_change(N, int(q), int(qnew), xi8, l8, np.ascontiguousarray(e, dtype=np.float64), flat)
    return flat.reshape(rows, N)


def bdf_prescribed(f, jac, q: int, t0: float, z0, tau, hseq):
    """Prescribed-step BDF at fixed order (pins of the coefficients)."""
    z = np.array(z0, dtype=np.float64)
    N = z.shape[1]
    f.__out_size__ = N
    cj_fn = lambda t, yy: np.asarray(jac(t, yy)).reshape(-1)
    cj_fn.__out_size__ = N * N
    cf, cj = _wrap_user(N, f), _wrap_user(N, cj_fn)
    flat = np.zeros((8, N))
    flat[: q + 1] = z[: q + 1]
    flat = flat.reshape(-1).copy()
    t = np.zeros(8)
    t[: len(tau)] = tau
    hs = np.ascontiguousarray(hseq, dtype=np.float64)
    bad = lib().om_bdf_prescribed(N, cf, cj, None, q, float(t0), flat, t, len(hs), hs)
    return flat.reshape(8, N)[: q + 1].copy(), t, bad
