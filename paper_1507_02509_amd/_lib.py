"""ctypes binding of libkbc.so (include/kbc.h).  Argument marshalling only:
every step of the path runs in the library's HIP kernels.

The library must have been built (``python -m paper_1507_02509_amd.build``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkbc.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "kbc.h")

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ENOMEM, LBM_ENONFINITE, LBM_EUNSUPPORTED, LBM_ESYNC = 0, -1, -2, -3, -4, -5, -6
LBM_ENSEMBLE_SPIN_DEFAULT, LBM_ENSEMBLE_SPIN_MAX = 1 << 22, 1 << 26
LBGK, KBC = 0, 1
KBC_A, KBC_B, KBC_C, KBC_D = 0, 1, 2, 3
F16DEV_F32, F32DEV_F32, F64 = 0, 1, 2
GAMMA_ESTIMATE, GAMMA_FIXED, GAMMA_EXACT = 0, 1, 2
INIT_EQ, INIT_GRAD_CD, INIT_GRAD_GIVEN = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("beta", ctypes.c_double),
                ("rho0", ctypes.c_double), ("collision", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("form", ctypes.c_int32), ("gamma_mode", ctypes.c_int32),
                ("gamma_guard", ctypes.c_double), ("gamma_fixed", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


DIAG_FIELDS = ["mass", "jx", "jy", "E", "E_std", "Z", "Z_std", "P", "P_std", "S", "gamma",
               "gamma_std", "n_nonfinite", "n_feq_nonpos", "rho_std", "reserved"]


class Diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in DIAG_FIELDS]


class KbcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libkbc error {code}: {msg}")
        self.code = code


_lib = None

_c = ctypes
_vp, _dp = _c.c_void_p, _c.POINTER(_c.c_double)
_SIGS = {
    "lbm_required_pitch": (_c.c_size_t, [_c.c_int32, _c.c_int32]),
    "lbm_buffer_bytes": (_c.c_size_t, [_c.c_int32, _c.c_int32, _c.c_int32]),
    "lbm_init": (_c.c_int, [_c.POINTER(_vp), _c.POINTER(Params), _vp, _vp, _c.c_size_t, _vp, _vp, _vp,
                            _vp, _c.c_int32]),
    "lbm_step": (_c.c_int, [_vp, _c.c_int32]),
    "lbm_moments": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_get_populations": (_c.c_int, [_vp, _vp]),
    "lbm_set_populations": (_c.c_int, [_vp, _vp]),
    "lbm_diagnostics": (_c.c_int, [_vp, _c.POINTER(Diag)]),
    "lbm_step_count": (_c.c_int64, [_vp]),
    "lbm_set_step": (_c.c_int, [_vp, _c.c_int64]),
    "lbm_state_buffer": (_vp, [_vp]),
    "lbm_work_buffer": (_vp, [_vp]),
    "lbm_set_beta": (_c.c_int, [_vp, _c.c_double]),
    "lbm_set_tile": (_c.c_int, [_vp, _c.c_int32, _c.c_int32, _c.c_int32]),
    "lbm_get_tile": (_c.c_int, [_vp, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "lbm_set_fusion": (_c.c_int, [_vp, _c.c_int32, _c.c_int32]),
    "lbm_spectra": (_c.c_int, [_vp, _c.c_int32, _vp, _vp]),
    "lbm_get_fusion": (_c.c_int, [_vp, _c.POINTER(_c.c_int32)]),
    "lbm_set_graph": (_c.c_int, [_vp, _c.c_int32]),
    "lbm_set_halo": (_c.c_int, [_vp, _vp, _vp]),
    "lbm_get_edge_rows": (_c.c_int, [_vp, _vp, _vp]),
    "lbm_get_graph": (_c.c_int, [_vp]),
    "lbm_free": (_c.c_int, [_vp]),
    "lbm_last_error": (_c.c_char_p, []),
    "lbm_copy_probe": (_c.c_int, [_vp, _vp, _c.c_size_t, _vp]),
    "lbm_ensemble_create": (_c.c_int, [_c.POINTER(_vp), _c.POINTER(_vp), _c.c_int32]),
    "lbm_ensemble_set_tile": (_c.c_int, [_vp, _c.c_int32, _c.c_int32, _c.c_int32]),
    "lbm_ensemble_step": (_c.c_int, [_vp, _c.c_int32, _c.c_int32]),
    "lbm_ensemble_set_fusion": (_c.c_int, [_vp, _c.c_int32, _c.c_int32]),
    "lbm_ensemble_get_fusion": (_c.c_int, [_vp, _c.POINTER(_c.c_int32)]),
    "lbm_ensemble_blocks": (_c.c_int, [_vp]),
    "lbm_ensemble_set_spin_limit": (_c.c_int, [_vp, _c.c_uint32]),
    "lbm_ensemble_check": (_c.c_int, [_vp]),
    "lbm_adjoint_step_noalloc": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_ensemble_free": (_c.c_int, [_vp]),
    "lbm_set_adjoint_gamma": (_c.c_int, [_vp, _c.c_int32]),
    "lbm_adjoint_bytes": (_c.c_size_t, [_c.c_int32, _c.c_int32, _c.c_int32]),
    "lbm_step_buffers": (_c.c_int, [_vp, _vp, _vp]),
    "lbm_adjoint_seed": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_step": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_step_slab": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_segment": (_c.c_int, [_vp, _vp, _c.POINTER(_vp), _c.c_int32, _vp, _vp, _vp,
                                       _c.POINTER(_c.c_int32)]),
    "lbm_adjoint_init": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_int32, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_rollout": (_c.c_int, [_vp, _c.POINTER(_vp), _c.c_int32, _c.c_int32, _c.POINTER(_vp),
                                       _c.POINTER(_vp), _vp, _vp, _vp, _c.POINTER(_c.c_int32)]),
}


def load():
    """Load libkbc.so; raise ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1507_02509_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_functions() -> list[str]:
    """Names of the functions include/kbc.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def check(rc: int, what: str = ""):
    if rc != LBM_OK:
        msg = load().lbm_last_error().decode(errors="replace")
        raise KbcError(rc, f"{what}: {msg}" if what else msg)
    return rc


def ptr(t) -> int | None:
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    return t.data_ptr()
