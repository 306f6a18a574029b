"""ctypes binding of libwc.so (argument marshalling only; all compute is in the HIP library)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwc.so")

WC_OK = 0
STATUS = {
    0: "WC_OK", -1: "WC_ERR_ARG", -2: "WC_ERR_GEOMETRY", -3: "WC_ERR_HIP", -4: "WC_ERR_OOM",
    -5: "WC_ERR_NOT_CONVERGED", -6: "WC_ERR_BREAKDOWN", -7: "WC_ERR_STATE",
}
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
REGION = {"full": 0, "blocks": 1}


class SolverParams(ctypes.Structure):
    _fields_ = [
        ("nkv", ctypes.c_int), ("ncy", ctypes.c_int), ("nmr", ctypes.c_int), ("sap_prec", ctypes.c_int),
        ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("x0_given", ctypes.c_int),
        ("use_graph", ctypes.c_int), ("nr_dirac", ctypes.c_int), ("nr_sap", ctypes.c_int),
        ("eo", ctypes.c_int), ("dagger", ctypes.c_int), ("stag", ctypes.c_int), ("timing", ctypes.c_int),
        ("basis_prec", ctypes.c_int), ("drop", ctypes.c_double),
    ]


HIST_MAX = 64
OPTIONS = {"sap_cache": 0, "dirac_stage": 1}


class SolverStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("restarts", ctypes.c_int),
        ("breakdown", ctypes.c_int), ("rel_true_res", ctypes.c_double), ("time_ms", ctypes.c_double),
        ("reorth", ctypes.c_int), ("stagnated", ctypes.c_int), ("nhist", ctypes.c_int), ("timed", ctypes.c_int),
        ("t_setup_ms", ctypes.c_double), ("t_cycles_ms", ctypes.c_double), ("t_finish_ms", ctypes.c_double),
        ("t_sap_ms", ctypes.c_double), ("t_dirac_ms", ctypes.c_double), ("t_blas_ms", ctypes.c_double),
        ("res_hist", ctypes.c_double * HIST_MAX),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "res_hist"}
        d["res_hist"] = [self.res_hist[i] for i in range(self.nhist)]
        return d


class WCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "wc_default_params": (None, [ctypes.POINTER(SolverParams)]),
    "wc_create_gauge": (_I, [ctypes.POINTER(_P), ctypes.POINTER(_I), ctypes.POINTER(_I), _P, _I, _P]),
    "wc_create_clover": (_I, [_P, _D, _D, _P]),
    "wc_set_block": (_I, [_P, ctypes.POINTER(_I), _P]),
    "wc_clover_export": (_I, [_P, _P, _P]),
    "wc_apply_D": (_I, [_P, _P, _P, _I, _I, _I, _I, _P]),
    "wc_apply_D_noalloc": (_I, [_P, _P, _P, _I, _I, _I, _I, _P]),
    "wc_harmonic_ritz": (_I, [_I, _P, _P, _P]),
    "wc_fgmres_dr_solve_batch": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                      ctypes.POINTER(_I), ctypes.POINTER(SolverParams), _I, ctypes.POINTER(SolverStats),
                                      _P]),
    "wc_fgmres_dr_solve": (_I, [_P, _P, _P, _I, ctypes.POINTER(SolverParams), _I, ctypes.POINTER(SolverStats), _P]),
    "wc_sap_block_mr": (_I, [_P, _P, _P, _I, _I, _I, _I, _I, _P]),
    "wc_sap": (_I, [_P, _P, _P, _I, _I, _I, _I, _I, _P]),
    "wc_fgcr_solve": (_I, [_P, _P, _P, _I, ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats), _P]),
    "wc_fgcr_solve_batch": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                 ctypes.POINTER(_I), ctypes.POINTER(SolverParams),
                                 ctypes.POINTER(SolverStats), _P]),
    "wc_link_grad": (_I, [_P, _P, _P, _P, _I, _D, _P]),
    "wc_force": (_I, [_P, _P, _P, ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats), _P, _P, _P]),
    "wc_autotune": (_I, [_P, _I, _I, ctypes.POINTER(_I), _P]),
    "wc_set_option": (_I, [_P, _I, _I]),
    "wc_set_tiles": (_I, [_P, _I, _I, _I, _I]),
    "wc_pseudofermion_action": (_I, [_P, _P, ctypes.POINTER(SolverParams), ctypes.POINTER(_D), _P, _P,
                                     ctypes.POINTER(SolverStats), _P]),
    "wc_spinor_scale": (_I, [_P, _P, _P, _I, _D, _P]),
    "wc_autotune_block": (_I, [_P, ctypes.POINTER(SolverParams), ctypes.POINTER(_I), _P]),
    "wc_bench_dirac": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(_D), _P]),
    "wc_bench_sap": (_I, [_P, _I, _I, _I, _I, _I, ctypes.POINTER(_D), _P]),
    "wc_destroy": (None, [_P]),
    "wc_last_error": (ctypes.c_char_p, []),
    "wc_version": (_I, []),
}

_lib = None


def load(path: str | None = None):
    """Load libwc.so (the in-tree build unless `path` is given) and declare every exported
    entry point; raises if it is missing.  torch is imported first so that the library
    binds to the HIP runtime torch already loaded: one runtime per process."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1109_4279_amd.build`")
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> int:
    if code != WC_OK:
        msg = load().wc_last_error().decode(errors="replace")
        raise WCError(code, msg)
    return code


def exported_symbols():
    return list(_SIGS)
