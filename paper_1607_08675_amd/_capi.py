"""ctypes declarations of the C ABI in ``include/lbmhd.h`` and ``include/lbmhd3.h``
(argument marshalling only).

``torch`` is imported first so that the library resolves its HIP runtime to the
one torch already loaded: device pointers and streams then belong to a single
runtime instance.  Loading fails loudly if ``liblbmhd.so`` has not been built;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading the library, see above)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbmhd.so")

LBMHD_OK = 0
LBMHD_ERR_INVALID_ARG = -1
LBMHD_ERR_NOT_BOUND = -2
LBMHD_ERR_HIP = -3
LBMHD_ERR_NONFINITE = -4
LBMHD_ERR_UNSUPPORTED = -5
LBMHD_FP32 = 0
LBMHD_FP16 = 1

# Every function declared in include/lbmhd.h, in declaration order.
EXPORTS = (
    "lbmhd_strerror", "lbmhd_last_error", "lbmhd_create", "lbmhd_destroy", "lbmhd_sizes",
    "lbmhd_layout", "lbmhd_bind", "lbmhd_init_fields", "lbmhd_step", "lbmhd_steps_per_pass",
    "lbmhd_step_between", "lbmhd_step_store", "lbmhd_step_store_pairs",
    "lbmhd_macro",
    "lbmhd_macro_box", "lbmhd_mismatch", "lbmhd_diag", "lbmhd_run", "lbmhd_get_populations",
    "lbmhd_set_populations", "lbmhd_save_state", "lbmhd_load_state", "lbmhd_get_step",
    "lbmhd_current_state",
    "lbmhd_energy", "lbmhd_adj_seed_energy", "lbmhd_adj_seed_mismatch", "lbmhd_adj_step",
    "lbmhd_adj_sweep", "lbmhd_adj_step2", "lbmhd_adj_sweep_pairs", "lbmhd_adj_acc_total",
    "lbmhd_adj_fields", "lbmhd_diag_noalloc",
)
# Every function declared in include/lbmhd3.h.
EXPORTS3 = (
    "lbmhd3_create", "lbmhd3_destroy", "lbmhd3_sizes", "lbmhd3_bind", "lbmhd3_init_fields",
    "lbmhd3_step", "lbmhd3_macro", "lbmhd3_diag", "lbmhd3_get_populations",
    "lbmhd3_set_populations", "lbmhd3_last_error",
)


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nu", ctypes.c_double), ("eta", ctypes.c_double),
        ("s5", ctypes.c_double), ("s6", ctypes.c_double),
        ("s7", ctypes.c_double), ("s8", ctypes.c_double),
        ("les", ctypes.c_int32),
        ("cs", ctypes.c_double), ("cs_b", ctypes.c_double), ("delta", ctypes.c_double),
        ("storage", ctypes.c_int32), ("inplace", ctypes.c_int32),
        ("steps_per_pass", ctypes.c_int32),
    ]


class Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nu", ctypes.c_double), ("eta", ctypes.c_double), ("les", ctypes.c_int32),
        ("cs", ctypes.c_double), ("cs_b", ctypes.c_double), ("delta", ctypes.c_double),
        ("storage", ctypes.c_int32), ("mrt", ctypes.c_int32),
        ("s5", ctypes.c_double), ("s7", ctypes.c_double), ("s8", ctypes.c_double),
        ("sg", ctypes.c_double), ("szz", ctypes.c_double),
    ]


class Diag3(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "mass", "mom_x", "mom_y", "mom_z", "flux_x", "flux_y", "flux_z", "e_kin", "e_mag",
        "max_abs_divB", "max_u")] + [("nonfinite", ctypes.c_int64), ("step", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "mass", "mom_x", "mom_y", "flux_x", "flux_y", "e_kin", "e_mag", "cross_helicity",
        "max_abs_divB", "enstrophy", "current_sq", "max_u")] + [
        ("nonfinite", ctypes.c_int64), ("step", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class LbmhdError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what} failed: {strerror(code)} ({code})" + (f": {detail}" if detail else ""))


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1607_08675_amd.build` "
                "(there is no non-GPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        P = ctypes.POINTER
        L.lbmhd_strerror.argtypes = [ctypes.c_int]
        L.lbmhd_strerror.restype = ctypes.c_char_p
        L.lbmhd_last_error.argtypes = [vp]
        L.lbmhd_last_error.restype = ctypes.c_char_p
        L.lbmhd3_last_error.argtypes = [vp]
        L.lbmhd3_last_error.restype = ctypes.c_char_p
        sig = {
            "lbmhd_create": [P(Params), P(vp)],
            "lbmhd_destroy": [vp],
            "lbmhd_sizes": [vp, P(sz), P(sz), P(sz), P(sz)],
            "lbmhd_layout": [vp, P(i64), P(i64), P(i64), P(i64)],
            "lbmhd_bind": [vp, vp, sz, vp, sz, vp, sz, vp],
            "lbmhd_init_fields": [vp] * 6,
            "lbmhd_step": [vp, i64],
            "lbmhd_step_between": [vp, vp, vp],
            "lbmhd_step_store": [vp, vp, vp, sz, i64],
            "lbmhd_macro": [vp] * 6,
            "lbmhd_macro_box": [vp, ctypes.c_int32] + [vp] * 5,
            "lbmhd_mismatch": [vp] * 6 + [P(ctypes.c_double)],
            "lbmhd_adj_seed_mismatch": [vp] * 6 + [ctypes.c_double, vp],
            "lbmhd_diag": [vp, P(Diag)],
            "lbmhd_run": [vp, i64, i64, vp, P(Diag), i64],
            "lbmhd_diag_noalloc": [vp, P(Diag)],
            "lbmhd_get_populations": [vp, vp],
            "lbmhd_set_populations": [vp, vp, i64],
            "lbmhd_save_state": [vp, vp],
            "lbmhd_load_state": [vp, vp, i64],
            "lbmhd_get_step": [vp, P(i64)],
            "lbmhd_current_state": [vp, P(vp)],
            "lbmhd_steps_per_pass": [vp, P(ctypes.c_int32)],
            "lbmhd_energy": [vp, vp, P(ctypes.c_double)],
            "lbmhd_adj_seed_energy": [vp, vp, vp],
            "lbmhd_adj_step": [vp, vp, vp, vp, vp],
            "lbmhd_adj_sweep": [vp, vp, vp, sz, i64, vp, vp, vp],
            "lbmhd_step_store_pairs": [vp, vp, vp, sz, i64],
            "lbmhd_adj_step2": [vp, vp, vp, vp, vp],
            "lbmhd_adj_sweep_pairs": [vp, vp, vp, sz, i64, vp, vp, vp],
            "lbmhd_adj_acc_total": [vp, vp, P(ctypes.c_double)],
            "lbmhd_adj_fields": [vp] * 11,
            "lbmhd3_create": [P(Params3), P(vp)],
            "lbmhd3_destroy": [vp],
            "lbmhd3_sizes": [vp, P(sz), P(sz)],
            "lbmhd3_bind": [vp, vp, sz, vp, sz, vp, sz, vp],
            "lbmhd3_init_fields": [vp] * 8,
            "lbmhd3_step": [vp, i64],
            "lbmhd3_macro": [vp] * 4,
            "lbmhd3_diag": [vp, P(Diag3)],
            "lbmhd3_get_populations": [vp, vp],
            "lbmhd3_set_populations": [vp, vp, i64],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().lbmhd_strerror(code).decode()


def check(rc: int, what: str, handle=None, last_error=None):
    if rc != LBMHD_OK:
        fn = last_error or lib().lbmhd_last_error
        detail = fn(handle).decode() if handle else ""
        raise LbmhdError(rc, what, detail)
