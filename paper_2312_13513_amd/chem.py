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
                ("jac_batch", C.c_int32), ("qmax", C.c_int32), ("waves_per_simd", C.c_int32),
                ("reserved", C.c_int32 * 5)]


class chem_tune_entry(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("jac_batch", C.c_int32), ("lpt", C.c_int32),
                ("waves_per_simd", C.c_int32), ("ms", C.c_double)]


class chem_stats(C.Structure):
    _fields_ = [("cells", C.c_int64), ("steps_total", C.c_int64), ("rejects", C.c_int64),
                ("newton_iters", C.c_int64), ("jac_evals", C.c_int64), ("rhs_evals", C.c_int64),
                ("fallback_cells", C.c_int64), ("steps_max", C.c_int32), ("reserved", C.c_int32),
                ("status_count", C.c_int64 * 8)]


class chem_surr_checks(C.Structure):
    _fields_ = [("elem_tol", C.c_double), ("sum_tol", C.c_double), ("neg_tol", C.c_double),
                ("T_out_min", C.c_double), ("T_out_max", C.c_double), ("T_in_min", C.c_double),
                ("T_in_max", C.c_double), ("dT_gate", C.c_double), ("reserved", C.c_int32 * 8)]


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
    L.chem_integrate_noalloc.argtypes = [vp, dp, dp, dp, i64, i64, C.c_double, C.POINTER(chem_opts), vp, vp, vp]
    L.chem_eval_rhs.argtypes = [vp, dp, dp, dp, i64, i64, dp, i64, vp]
    L.chem_eval_jacobian.argtypes = [vp, dp, dp, dp, i64, i64, dp, i64, vp]
    L.chem_integrate_indexed.argtypes = [vp, dp, dp, dp, i64, i64, dp, i64, C.c_double, C.POINTER(chem_opts),
                                         vp, vp, vp]
    L.chem_lpt_order.argtypes = [dp, i64, dp, vp]
    L.chem_get_stats.argtypes = [vp, vp, i64, vp, C.POINTER(chem_stats), vp]
    L.chem_autotune.argtypes = [vp, dp, dp, dp, i64, i64, C.c_double, C.POINTER(chem_opts), C.c_int32,
                                C.POINTER(chem_opts), i32p, C.POINTER(C.c_double), vp]
    L.chem_autotune_results.argtypes = [vp, C.POINTER(chem_tune_entry), C.c_int32, i32p]
    L.chem_ldu_create.argtypes = [i64, i64, vp, vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, vp, C.c_int,
                                  C.POINTER(vp)]
    L.chem_free_ldu.argtypes = [vp]
    L.chem_free_ldu.restype = None
    L.chem_ldu_info.argtypes = [vp, C.POINTER(C.c_int64)]
    L.chem_ldu_laplacian.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp, vp]
    L.chem_ldu_to_csr.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, vp]
    L.chem_ldu_csr_pattern.argtypes = [vp, dp, dp, vp]
    L.chem_ldu_laplacian_csr.argtypes = [vp, dp, dp, dp, dp, dp, vp]
    L.chem_mixture_h_cp.argtypes = [vp, dp, dp, i64, i64, dp, dp, vp]
    L.chem_T_from_h.argtypes = [vp, dp, dp, i64, i64, dp, dp, dp, C.c_int32, C.c_double, vp]
    L.chem_set_transport.argtypes = [vp, dp, dp, dp]
    L.chem_transport_field.argtypes = [vp, dp, dp, dp, i64, i64, dp, dp, dp, i64, vp]
    fp, dblp, i64p = C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int64)
    ckp = C.POINTER(chem_surr_checks)
    L.chem_surrogate_default_checks.argtypes = [ckp]
    L.chem_surrogate_create.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vp)]
    L.chem_surrogate_create_species.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vp)]
    L.chem_surrogate_groups.argtypes = [vp, C.POINTER(C.c_int32)]
    L.chem_free_surrogate.argtypes = [vp]
    L.chem_free_surrogate.restype = None
    L.chem_surrogate_info.argtypes = [vp, i64p]
    L.chem_surrogate_set_params.argtypes = [vp, fp, i64]
    L.chem_surrogate_get_params.argtypes = [vp, fp, i64]
    L.chem_surrogate_set_norm.argtypes = [vp, dblp, i64]
    L.chem_surrogate_get_norm.argtypes = [vp, dblp, i64]
    L.chem_surrogate_fit_norm.argtypes = [vp, dp, dp, dp, i64, dp, i64, i64, C.c_double, vp]
    L.chem_surrogate_encode.argtypes = [vp, dp, dp, dp, i64, i64, dp, vp]
    L.chem_surrogate_forward.argtypes = [vp, dp, i64, dp, i64, vp]
    L.chem_surrogate_forward_path.argtypes = [vp, dp, i64, dp, i64, C.c_int32, vp]
    L.chem_surrogate_apply.argtypes = [vp, dp, dp, dp, i64, i64, dp, i64, ckp, dp, vp]
    L.chem_surrogate_infer.argtypes = [vp, dp, dp, dp, i64, i64, C.c_double, C.POINTER(chem_opts), ckp,
                                       dp, dp, dp, vp]
    L.chem_surrogate_grad.argtypes = [vp, dp, dp, i64, i64, dblp, vp]
    L.chem_surrogate_get_grads.argtypes = [vp, fp, i64]
    L.chem_surrogate_set_grads.argtypes = [vp, fp, i64]
    L.chem_surrogate_adam.argtypes = [vp, C.c_double, vp]
    L.chem_surrogate_train.argtypes = [vp, dp, dp, dp, i64, dp, i64, i64, dp, C.c_int32, C.c_int32,
                                       C.c_double, C.c_double, dblp, vp]
    L.chem_surrogate_forward_trace.argtypes = [vp, dp, i64, dp, dp, dp, dp, i64, vp]
    L.chem_surrogate_reserve.argtypes = [vp, i64, vp]
    L.chem_surrogate_set_pass_rows.argtypes = [vp, i64]
    L.chem_surrogate_save.argtypes = [vp, C.c_char_p]
    L.chem_surrogate_load.argtypes = [vp, C.c_char_p, C.POINTER(vp)]
    L.chem_surrogate_train_part.argtypes = [vp, dp, dp, dp, i64, dp, i64, i64, dp, C.c_int32, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_double, C.c_double, dblp, vp]
    L.chem_surrogate_save_checkpoint.argtypes = [vp, C.c_char_p, C.c_char_p, i64]
    L.chem_surrogate_checkpoint_user.argtypes = [C.c_char_p, C.c_char_p, i64, i64p]
    return L


_lib = _load()

#: Symbols that include/chem.h declares (checked by the ABI test).
EXPORTED = ("chem_default_opts", "chem_load_mechanism", "chem_free_mechanism",
            "chem_mechanism_info", "chem_mechanism_variant", "chem_integrate", "chem_eval_rhs", "chem_eval_jacobian",
            "chem_last_error", "chem_integrate_indexed", "chem_lpt_order", "chem_autotune", "chem_get_stats",
            "chem_surrogate_default_checks", "chem_surrogate_create",
            "chem_free_surrogate", "chem_surrogate_info", "chem_surrogate_set_params",
            "chem_surrogate_get_params", "chem_surrogate_set_norm", "chem_surrogate_get_norm",
            "chem_surrogate_fit_norm", "chem_surrogate_encode", "chem_surrogate_forward", "chem_surrogate_forward_path",
            "chem_surrogate_apply", "chem_surrogate_infer", "chem_surrogate_grad",
            "chem_surrogate_get_grads", "chem_surrogate_set_grads", "chem_surrogate_adam",
            "chem_surrogate_train", "chem_surrogate_save", "chem_surrogate_load", "chem_surrogate_reserve",
            "chem_surrogate_set_pass_rows", "chem_surrogate_forward_trace", "chem_integrate_noalloc",
            "chem_surrogate_train_part", "chem_surrogate_save_checkpoint", "chem_surrogate_checkpoint_user",
            "chem_surrogate_create_species", "chem_surrogate_groups",
            "chem_autotune_results", "chem_ldu_create", "chem_free_ldu", "chem_ldu_info", "chem_ldu_laplacian",
            "chem_ldu_to_csr", "chem_ldu_csr_pattern", "chem_ldu_laplacian_csr", "chem_mixture_h_cp",
            "chem_T_from_h", "chem_set_transport", "chem_transport_field")


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


def chem_integrate_noalloc(handle: int, T, p, Y, dt: float, opts: Optional[chem_opts] = None,
                           status=None, counters=None, stream=None, ncells: Optional[int] = None) -> None:
    """chem_integrate with the start-pass workspace in the library's fixed
    per-GPU array (no device allocation; calls overlapping on one GPU race)."""
    n = T.shape[0] if ncells is None else int(ncells)
    _check(_lib.chem_integrate_noalloc(C.c_void_p(handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1], n,
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

    def integrate_noalloc(self, T, p, Y, dt, opts=None, status=None, counters=None, stream=None):
        chem_integrate_noalloc(self.handle, T, p, Y, dt, opts, status, counters, stream)

    def integrate_indexed(self, T, p, Y, idx, dt, opts=None, status=None, counters=None, stream=None):
        """Advance cells idx (int32 GPU tensor) of the arrays, in list order."""
        _check(_lib.chem_integrate_indexed(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                           T.shape[0], _ptr(idx), idx.shape[0], float(dt),
                                           C.byref(opts) if opts is not None else None, _ptr(status),
                                           _ptr(counters), _stream(stream)))

    def autotune(self, T, p, Y, dt, opts=None, max_sample: int = 0, stream=None):
        """Returns (best chem_opts, use_lpt, best_ms) and keeps the choice (schedule -2)."""
        best = chem_opts()
        lpt = C.c_int32()
        ms = C.c_double()
        _check(_lib.chem_autotune(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1], T.shape[0],
                                  float(dt), C.byref(opts) if opts is not None else None, int(max_sample),
                                  C.byref(best), C.byref(lpt), C.byref(ms), _stream(stream)))
        return best, bool(lpt.value), ms.value

    def autotune_results(self) -> list:
        """Measured table of the last autotune: dicts of schedule, jac_batch,
        lpt, waves_per_simd, ms."""
        n = C.c_int32()
        _check(_lib.chem_autotune_results(C.c_void_p(self.handle), None, 0, C.byref(n)))
        buf = (chem_tune_entry * max(1, n.value))()
        _check(_lib.chem_autotune_results(C.c_void_p(self.handle), buf, n.value, C.byref(n)))
        return [{k: getattr(e, k) for k, _ in chem_tune_entry._fields_} for e in buf[:n.value]]

    def rhs(self, T, p, Y, F, stream=None):
        chem_eval_rhs(self.handle, T, p, Y, F, stream)

    def jacobian(self, T, p, Y, J, stream=None):
        chem_eval_jacobian(self.handle, T, p, Y, J, stream)

    # -- field properties (the Thermo class) --------------------------------
    def mixture_h_cp(self, T, Y, h=None, cp=None, stream=None, ncells=None):
        """h, cp (n,) float64 GPU tensors (either may be None) of the mixtures Y at T."""
        n = T.shape[0] if ncells is None else int(ncells)
        _check(_lib.chem_mixture_h_cp(C.c_void_p(self.handle), _ptr(T), _ptr(Y), Y.shape[1], n, _ptr(h),
                                      _ptr(cp), _stream(stream)))

    def T_from_h(self, h, Y, T, cp=None, iters=None, max_iter: int = 20, tol: float = 1e-10, stream=None,
                 ncells=None):
        """T (n,) in: Newton guess, out: temperature with mixture enthalpy h."""
        n = h.shape[0] if ncells is None else int(ncells)
        _check(_lib.chem_T_from_h(C.c_void_p(self.handle), _ptr(h), _ptr(Y), Y.shape[1], n, _ptr(T), _ptr(cp),
                                  _ptr(iters), int(max_iter), float(tol), _stream(stream)))

    def set_transport(self, visc, cond, diff):
        """Species transport fits (numpy, lowest power first): visc (K, 5),
        cond (K, 5), diff (K, K, 5)."""
        import numpy as np
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (visc, cond, diff)]
        if a[0].shape != (self.K, 5) or a[1].shape != (self.K, 5) or a[2].shape != (self.K, self.K, 5):
            raise ValueError("transport fits must be (K, 5), (K, 5) and (K, K, 5)")
        _check(_lib.chem_set_transport(C.c_void_p(self.handle), *(x.ctypes.data for x in a)))

    def transport(self, T, p, Y, mu=None, lam=None, D=None, stream=None, ncells=None):
        """Mixture viscosity, conductivity (n,) and diffusion coefficients D (K, ldD)."""
        n = T.shape[0] if ncells is None else int(ncells)
        _check(_lib.chem_transport_field(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1], n,
                                         _ptr(mu), _ptr(lam), _ptr(D), D.shape[1] if D is not None else 0,
                                         _stream(stream)))


def chem_lpt_order(cost, order, stream=None) -> None:
    """order (int32 GPU tensor) <- indices sorted by descending cost (int32 GPU tensor)."""
    _check(_lib.chem_lpt_order(_ptr(cost), cost.shape[0], _ptr(order), _stream(stream)))


def chem_get_stats(status=None, counters=None, n=None, fallback_count=None, stream=None) -> dict:
    """Totals of one call's per-cell outputs (status: int32 (n,), counters:
    int32 (6*n,) GPU tensors, either may be None; fallback_count: int64 (1,))."""
    if n is None:
        n = status.shape[0] if status is not None else (counters.shape[0] // 6 if counters is not None else 0)
    out = chem_stats()
    _check(_lib.chem_get_stats(_ptr(status), _ptr(counters), int(n), _ptr(fallback_count), C.byref(out),
                               _stream(stream)))
    d = {k: getattr(out, k) for k, _ in chem_stats._fields_ if k not in ("reserved", "status_count")}
    d["status_count"] = list(out.status_count)
    return d


# --------------------------------------------------------------------------- surrogate

def chem_surrogate_default_checks() -> chem_surr_checks:
    c = chem_surr_checks()
    _check(_lib.chem_surrogate_default_checks(C.byref(c)))
    return c


def _host_f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def _host_f64(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


class Surrogate:
    """Owning wrapper of a chem_surr handle (the mechanism must stay open)."""

    def __init__(self, mech: Mechanism, h1: int = 512, h2: int = 256, h3: int = 128, handle: int = 0,
                 per_species: bool = False):
        """per_species: one network nin -> h1 -> h2 -> h3 -> 1 per species (the
        paper's variant) instead of one network with K outputs."""
        self.mech = mech
        if not handle:
            h = C.c_void_p()
            create = _lib.chem_surrogate_create_species if per_species else _lib.chem_surrogate_create
            _check(create(C.c_void_p(mech.handle), int(h1), int(h2), int(h3), C.byref(h)))
            handle = h.value
        self.handle = handle
        dims = (C.c_int64 * 6)()
        _check(_lib.chem_surrogate_info(C.c_void_p(self.handle), dims))
        self.nin, self.h1, self.h2, self.h3, self.K, self.nparams = (int(v) for v in dims)
        g = C.c_int32()
        _check(_lib.chem_surrogate_groups(C.c_void_p(self.handle), C.byref(g)))
        self.groups = g.value
        self.nout_pad = (self.K + 15) // 16 * 16
        self.norm_len = 2 * self.nin + 2 * self.K + 1

    @classmethod
    def load(cls, mech: Mechanism, path: str) -> "Surrogate":
        h = C.c_void_p()
        _check(_lib.chem_surrogate_load(C.c_void_p(mech.handle), path.encode(), C.byref(h)))
        return cls(mech, handle=h.value)

    def close(self):
        if self.handle:
            _lib.chem_free_surrogate(C.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path: str):
        _check(_lib.chem_surrogate_save(C.c_void_p(self.handle), path.encode()))

    def save_checkpoint(self, path: str, user: bytes = b""):
        """Weights, normalisation and optimiser state, plus the caller's bytes."""
        _check(_lib.chem_surrogate_save_checkpoint(C.c_void_p(self.handle), path.encode(), bytes(user), len(user)))

    @staticmethod
    def checkpoint_user(path: str) -> bytes:
        n = C.c_int64(0)
        rc = _lib.chem_surrogate_checkpoint_user(path.encode(), None, 0, C.byref(n))
        if rc != CHEM_OK and n.value == 0:
            _check(rc)
        buf = C.create_string_buffer(max(1, n.value))
        _check(_lib.chem_surrogate_checkpoint_user(path.encode(), buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def set_params(self, params):
        a, p = _host_f32(params)
        _check(_lib.chem_surrogate_set_params(C.c_void_p(self.handle), p, a.size))

    def get_params(self):
        import numpy as np
        a = np.zeros(self.nparams, dtype=np.float32)
        _check(_lib.chem_surrogate_get_params(C.c_void_p(self.handle), a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def set_norm(self, norm):
        a, p = _host_f64(norm)
        _check(_lib.chem_surrogate_set_norm(C.c_void_p(self.handle), p, a.size))

    def get_norm(self):
        import numpy as np
        a = np.zeros(self.norm_len)
        _check(_lib.chem_surrogate_get_norm(C.c_void_p(self.handle), a.ctypes.data_as(C.POINTER(C.c_double)), a.size))
        return a

    def fit_norm(self, T, p, Y, Ynext, dt, stream=None):
        _check(_lib.chem_surrogate_fit_norm(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                            _ptr(Ynext), Ynext.shape[1], T.shape[0], float(dt), _stream(stream)))

    def encode(self, T, p, Y, X, stream=None):
        """X: int16 GPU tensor of shape (n, 64) receiving BF16 bit patterns."""
        _check(_lib.chem_surrogate_encode(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                          T.shape[0], _ptr(X), _stream(stream)))

    def forward(self, X, out, path=0, stream=None):
        """path: 0 library choice, 1 one GEMM per layer, 2 fused kernel."""
        _check(_lib.chem_surrogate_forward_path(C.c_void_p(self.handle), _ptr(X), X.shape[0], _ptr(out),
                                                out.shape[1], int(path), _stream(stream)))

    def forward_trace(self, X, H1, H2, H3, out, stream=None):
        """Per-layer forward keeping the BF16 hidden activations (int16 GPU
        tensors of shape (n, h1), (n, h2), (n, h3))."""
        _check(_lib.chem_surrogate_forward_trace(C.c_void_p(self.handle), _ptr(X), X.shape[0], _ptr(H1), _ptr(H2),
                                                 _ptr(H3), _ptr(out), out.shape[1], _stream(stream)))

    def apply(self, T, p, Y, out, checks=None, mask=None, stream=None):
        _check(_lib.chem_surrogate_apply(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                         T.shape[0], _ptr(out), out.shape[1],
                                         C.byref(checks) if checks is not None else None, _ptr(mask),
                                         _stream(stream)))

    def infer(self, T, p, Y, dt, opts=None, checks=None, mask=None, status=None, fallback_count=None,
              stream=None):
        _check(_lib.chem_surrogate_infer(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                         T.shape[0], float(dt), C.byref(opts) if opts is not None else None,
                                         C.byref(checks) if checks is not None else None, _ptr(mask),
                                         _ptr(status), _ptr(fallback_count), _stream(stream)))

    def reserve(self, ncells: int, stream=None):
        """Size the inference workspace for calls of up to ncells cells."""
        _check(_lib.chem_surrogate_reserve(C.c_void_p(self.handle), int(ncells), _stream(stream)))

    def set_pass_rows(self, rows: int):
        """Rows per inference pass (0 = the library's choice)."""
        _check(_lib.chem_surrogate_set_pass_rows(C.c_void_p(self.handle), int(rows)))

    def grad(self, X, Yt, stream=None) -> float:
        loss = C.c_double()
        _check(_lib.chem_surrogate_grad(C.c_void_p(self.handle), _ptr(X), _ptr(Yt), Yt.shape[1], X.shape[0],
                                        C.byref(loss), _stream(stream)))
        return loss.value

    def get_grads(self):
        import numpy as np
        a = np.zeros(self.nparams, dtype=np.float32)
        _check(_lib.chem_surrogate_get_grads(C.c_void_p(self.handle), a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def set_grads(self, g):
        a, p = _host_f32(g)
        _check(_lib.chem_surrogate_set_grads(C.c_void_p(self.handle), p, a.size))

    def adam(self, lr: float, stream=None):
        _check(_lib.chem_surrogate_adam(C.c_void_p(self.handle), float(lr), _stream(stream)))

    def train(self, T, p, Y, Ynext, epochs: int, batch: int, lr0: float = 1e-3, lr1: float = 1e-5, order=None,
              stream=None):
        import numpy as np
        losses = np.zeros(int(epochs))
        _check(_lib.chem_surrogate_train(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                         _ptr(Ynext), Ynext.shape[1], T.shape[0], _ptr(order), int(epochs), int(batch),
                                         float(lr0), float(lr1), losses.ctypes.data_as(C.POINTER(C.c_double)),
                                         _stream(stream)))
        return losses

    def train_part(self, T, p, Y, Ynext, first_epoch: int, epochs: int, total_epochs: int, batch: int,
                   lr0: float = 1e-3, lr1: float = 1e-5, order=None, stream=None):
        import numpy as np
        losses = np.zeros(int(epochs))
        _check(_lib.chem_surrogate_train_part(C.c_void_p(self.handle), _ptr(T), _ptr(p), _ptr(Y), Y.shape[1],
                                              _ptr(Ynext), Ynext.shape[1], T.shape[0], _ptr(order),
                                              int(first_epoch), int(epochs), int(total_epochs), int(batch),
                                              float(lr0), float(lr1), losses.ctypes.data_as(C.POINTER(C.c_double)),
                                              _stream(stream)))
        return losses


# --------------------------------------------------------------------------- finite-volume Laplacian

class LduMesh:
    """Owning wrapper of a chem_ldu mesh (built from host numpy arrays, e.g.
    chemgen.mesh.BoxMesh)."""

    def __init__(self, mesh, device: int = 0):
        import numpy as np
        a = {k: np.ascontiguousarray(getattr(mesh, k), dtype=t) for k, t in
             (("owner", np.int32), ("neighbour", np.int32), ("weight", np.float64), ("delta", np.float64),
              ("mag_sf", np.float64), ("patch_start", np.int64), ("patch_type", np.int32),
              ("face_cells", np.int32), ("bdelta", np.float64), ("bmag_sf", np.float64))}
        self._keep = a
        h = C.c_void_p()
        _check(_lib.chem_ldu_create(int(mesh.ncells), int(a["owner"].size), *(a[k].ctypes.data for k in
                                    ("owner", "neighbour", "weight", "delta", "mag_sf")),
                                    int(a["patch_type"].size), a["patch_start"].ctypes.data,
                                    a["patch_type"].ctypes.data, a["face_cells"].ctypes.data, a["bdelta"].ctypes.data,
                                    a["bmag_sf"].ctypes.data, int(device), C.byref(h)))
        self.handle = h.value
        dims = (C.c_int64 * 4)()
        _check(_lib.chem_ldu_info(C.c_void_p(self.handle), dims))
        self.ncells, self.nfaces, self.nbfaces, self.nnz = (int(v) for v in dims)

    def close(self):
        if self.handle:
            _lib.chem_free_ldu(C.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def laplacian(self, gamma_c, gamma_b, psi_b, lower, upper, diag, internal, boundary, stream=None):
        _check(_lib.chem_ldu_laplacian(C.c_void_p(self.handle), _ptr(gamma_c), _ptr(gamma_b), _ptr(psi_b),
                                       _ptr(lower), _ptr(upper), _ptr(diag), _ptr(internal), _ptr(boundary),
                                       _stream(stream)))

    def to_csr(self, lower, upper, diag, internal, boundary, csr_val, rhs, stream=None):
        _check(_lib.chem_ldu_to_csr(C.c_void_p(self.handle), _ptr(lower), _ptr(upper), _ptr(diag), _ptr(internal),
                                    _ptr(boundary), _ptr(csr_val), _ptr(rhs), _stream(stream)))

    def laplacian_csr(self, gamma_c, gamma_b, psi_b, csr_val, rhs, stream=None):
        _check(_lib.chem_ldu_laplacian_csr(C.c_void_p(self.handle), _ptr(gamma_c), _ptr(gamma_b), _ptr(psi_b),
                                           _ptr(csr_val), _ptr(rhs), _stream(stream)))

    def csr_pattern(self, row_ptr, col, stream=None):
        _check(_lib.chem_ldu_csr_pattern(C.c_void_p(self.handle), _ptr(row_ptr), _ptr(col), _stream(stream)))
