"""Thin ctypes binding of ``libchem.so`` (the C ABI in include/chem.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Tensors must be CUDA (HIP) tensors of the mechanism's
device; the binding passes their data pointers and the current stream.  If the
library has not been built the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchem.so")

CHEM_OK = 0
CELL_STATUS = {0: "OK", 1: "MAX_STEPS", 2: "ERR_FAIL", 3: "CONV_FAIL", 4: "NAN"}
COUNTER_NAMES = ("nst", "nfe", "nje", "nni", "netf", "ncfn")


class ChemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chem error {code}: {msg}")
        self.code = code


class chem_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int32),
                ("precision", C.c_int32), ("schedule", C.c_int32), ("block", C.c_int32),
                ("jac_batch", C.c_int32), ("reserved", C.c_int32 * 7)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(hipcc for gfx950); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32p, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.c_void_p
    L.chem_last_error.restype = C.c_char_p
    L.chem_default_opts.argtypes = [C.POINTER(chem_opts)]
    L.chem_load_mechanism.argtypes = [C.c_char_p, C.c_int, C.POINTER(vp)]
    L.chem_free_mechanism.argtypes = [vp]
    L.chem_free_mechanism.restype = None
    L.chem_mechanism_info.argtypes = [vp, i32p, i32p, i32p, C.POINTER(C.c_double)]
    L.chem_mechanism_variant.restype = C.c_char_p
    L.chem_mechanism_variant.argtypes = [vp]
    L.chem_integrate.argtypes = [vp, dp, dp, dp, i64, i64, C.c_double, C.POINTER(chem_opts), vp, vp, vp]
    L.chem_eval_rhs.argtypes = [vp, dp, dp, dp, i64, i64, dp, i64, vp]
    L.chem_eval_jacobian.argtypes = [vp, dp, dp, dp, i64, i64, dp, i64, vp]
    return L


_lib = _load()

#: Symbols that include/chem.h declares (checked by the ABI test).
EXPORTED = ("chem_default_opts", "chem_load_mechanism", "chem_free_mechanism",
            "chem_mechanism_info", "chem_mechanism_variant", "chem_integrate", "chem_eval_rhs", "chem_eval_jacobian",
            "chem_last_error")


def lib():
    return _lib


def _check(rc: int):
    if rc != CHEM_OK:
        raise ChemError(rc, _lib.chem_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to the chemistry library must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the chemistry library must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def chem_default_opts() -> chem_opts:
    o = chem_opts()
    _check(_lib.chem_default_opts(C.byref(o)))
    return o


def chem_load_mechanism(path: str, device: int = 0) -> int:
    h = C.c_void_p()
    _check(_lib.chem_load_mechanism(path.encode(), int(device), C.byref(h)))
    return h.value


def chem_free_mechanism(handle: int) -> None:
    _lib.chem_free_mechanism(C.c_void_p(handle))


def chem_mechanism_info(handle: int) -> Tuple[int, int, int, list]:
    K, R, E = C.c_int32(), C.c_int32(), C.c_int32()
    W = (C.c_double * 4096)()
    _check(_lib.chem_mechanism_info(C.c_void_p(handle), C.byref(K), C.byref(R), C.byref(E), W))
    return K.value, R.value, E.value, list(W[: K.value])


def chem_mechanism_variant(handle: int) -> str:
    return _lib.chem_mechanism_variant(C.c_void_p(handle)).decode()


def chem_integrate(handle: int, T, p, Y, dt: float, opts: Optional[chem_opts] = None,
                   status=None, counters=None, stream=None, ncells: Optional[int] = None) -> None:
    """Advance the cells in place: T (n,), p (n,), Y (K, ldY) float64 GPU tensors."""
    n = T.shape[0] if ncells is None else int(ncells)
    _check(_lib.chem_integrate(C.c_void_p(handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1], n,
                               float(dt), C.byref(opts) if opts is not None else None,
                               _ptr(status), _ptr(counters), _stream(stream)))


def chem_eval_rhs(handle: int, T, p, Y, F, stream=None) -> None:
    _check(_lib.chem_eval_rhs(C.c_void_p(handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1], T.shape[0],
                              _ptr(F), F.shape[1], _stream(stream)))


def chem_eval_jacobian(handle: int, T, p, Y, J, stream=None) -> None:
    _check(_lib.chem_eval_jacobian(C.c_void_p(handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                   T.shape[0], _ptr(J), J.shape[1], _stream(stream)))


class Mechanism:
    """Owning wrapper of a chem_mech handle."""

    def __init__(self, path: str, device: int = 0):
        self.path = path
        self.device = device
        self.handle = chem_load_mechanism(path, device)
        self.K, self.R, self.E, self.W = chem_mechanism_info(self.handle)
        self.N = self.K + 1
        self.variant = chem_mechanism_variant(self.handle)

    def close(self):
        if self.handle:
            chem_free_mechanism(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, T, p, Y, dt, opts=None, status=None, counters=None, stream=None):
        chem_integrate(self.handle, T, p, Y, dt, opts, status, counters, stream)

    def rhs(self, T, p, Y, F, stream=None):
        chem_eval_rhs(self.handle, T, p, Y, F, stream)

    def jacobian(self, T, p, Y, J, stream=None):
        chem_eval_jacobian(self.handle, T, p, Y, J, stream)
