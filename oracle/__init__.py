"""ctypes wrapper of the FP64 CPU oracle (``libkbc_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the product path never imports it.

Arrays are float64 numpy arrays; a lattice state is ``f[9, ny, nx]`` holding
the pre-collision populations in the velocity order
(0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkbc_oracle.so")

LBGK, KBC = 0, 1
KBC_A, KBC_B, KBC_C, KBC_D = 0, 1, 2, 3
GAMMA_ESTIMATE, GAMMA_FIXED, GAMMA_EXACT = 0, 1, 2
INIT_EQ, INIT_GRAD_CD, INIT_GRAD_GIVEN = 0, 1, 2
VARIANTS = {"A": KBC_A, "B": KBC_B, "C": KBC_C, "D": KBC_D}

DIAG_NAMES = ["mass", "jx", "jy", "E", "E_std", "Z", "Z_std", "P", "P_std", "S",
              "gamma", "gamma_std", "n_nonfinite", "n_feq_nonpos", "rho_std", "unused"]


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("beta", ctypes.c_double),
                ("collision", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("gamma_mode", ctypes.c_int32), ("gamma_guard", ctypes.c_double),
                ("gamma_fixed", ctypes.c_double), ("threads", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b  # noqa: F401  (build script beside the sources)
            _b.build()
        _lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.orc_node_collide.restype = ctypes.c_double
        _lib.orc_node_result1.restype = ctypes.c_double
        _lib.orc_cs2.restype = ctypes.c_double
        _lib.orc_round_f16.restype = ctypes.c_double
        _lib.orc_round_f16.argtypes = [ctypes.c_double]
        del dp
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need C-contiguous float64"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def beta_from_nu(nu: float) -> float:
    """Invert nu = cs2 (1/(2 beta) - 1/2) with cs2 = 1/3, eq. (viscosity)."""
    return 1.0 / (6.0 * nu + 1.0)


@dataclass
class Params:
    nx: int
    ny: int
    beta: float
    collision: int = KBC
    variant: int = KBC_B
    gamma_mode: int = GAMMA_ESTIMATE
    gamma_guard: float = 1e-12
    gamma_fixed: float = 2.0
    threads: int = 0

    def c(self) -> _Params:
        nt = self.threads if self.threads > 0 else min(8, os.cpu_count() or 1)
        return _Params(self.nx, self.ny, self.beta, self.collision, self.variant,
                       self.gamma_mode, self.gamma_guard, self.gamma_fixed, nt)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ------------------------------------------------------------------ constants
def cs2() -> float:
    return lib().orc_cs2()


def velocities():
    cx = (ctypes.c_int32 * 9)()
    cy = (ctypes.c_int32 * 9)()
    lib().orc_velocities(cx, cy)
    return np.array(cx, dtype=np.int64), np.array(cy, dtype=np.int64)


def weights() -> np.ndarray:
    w = np.zeros(9)
    lib().orc_weights(_ptr(w))
    return w


# ------------------------------------------------------------- node functions
def node_equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_node_equilibrium(ctypes.c_double(rho), ctypes.c_double(ux), ctypes.c_double(uy),
                               _ptr(out))
    return out


def node_natural(f) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_node_natural(_ptr(f), _ptr(out))
    return out


def node_central(f) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(6)
    lib().orc_node_central(_ptr(f), _ptr(out))
    return out


def node_central_to_natural(ux, uy, ct, kin=1) -> np.ndarray:
    ct = np.ascontiguousarray(ct, dtype=np.float64)
    out = np.zeros(6)
    lib().orc_node_central_to_natural(ctypes.c_double(ux), ctypes.c_double(uy), _ptr(ct),
                                      ctypes.c_int32(kin), _ptr(out))
    return out


def node_populations(r) -> np.ndarray:
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_node_populations(_ptr(r), _ptr(out))
    return out


def node_split(variant: int, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    k, s, h = np.zeros(9), np.zeros(9), np.zeros(9)
    lib().orc_node_split(ctypes.c_int32(variant), _ptr(f), _ptr(k), _ptr(s), _ptr(h))
    return k, s, h


def node_deviations(variant: int, f):
    """Return (ds, dh, (<ds|dh>, <dh|dh>, <ds|ds>))."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    ds, dh, out = np.zeros(9), np.zeros(9), np.zeros(3)
    lib().orc_node_deviations(ctypes.c_int32(variant), _ptr(f), _ptr(ds), _ptr(dh), _ptr(out))
    return ds, dh, out


def node_collide(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    cp = p.c()
    g = lib().orc_node_collide(ctypes.byref(cp), _ptr(f), _ptr(out))
    return out, g


def node_result1(p: Params, f, gamma: float) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    cp = p.c()
    return lib().orc_node_result1(ctypes.byref(cp), _ptr(f), ctypes.c_double(gamma))


def node_grad(rho, ux, uy, du, beta) -> np.ndarray:
    du = np.ascontiguousarray(du, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_node_grad(ctypes.c_double(rho), ctypes.c_double(ux), ctypes.c_double(uy), _ptr(du),
                        ctypes.c_double(beta), _ptr(out))
    return out


def node_jacobian(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    J, db = np.zeros(81), np.zeros(9)
    cp = p.c()
    lib().orc_node_jacobian(ctypes.byref(cp), _ptr(f), _ptr(J), _ptr(db))
    return J.reshape(9, 9), db


# ----------------------------------------------------------- lattice functions
def init(p: Params, ux, uy, rho=None, rho0: float = 1.0, mode: int = INIT_GRAD_CD, grad=None):
    ux = np.ascontiguousarray(ux, dtype=np.float64)
    uy = np.ascontiguousarray(uy, dtype=np.float64)
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    grad = None if grad is None else np.ascontiguousarray(grad, dtype=np.float64)
    f = np.zeros((9, p.ny, p.nx))
    cp = p.c()
    _check(lib().orc_init(ctypes.byref(cp), _ptr(rho), ctypes.c_double(rho0), _ptr(ux), _ptr(uy),
                          _ptr(grad), ctypes.c_int32(mode), _ptr(f)), "init")
    return f


def step(p: Params, f, want_gamma: bool = False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    gam = np.zeros((p.ny, p.nx)) if want_gamma else None
    cp = p.c()
    _check(lib().orc_step(ctypes.byref(cp), _ptr(f), _ptr(out), _ptr(gam)), "step")
    return (out, gam) if want_gamma else out


STORE_F64, STORE_F32, STORE_F16 = 0, 1, 2
STORAGE = {"f64": STORE_F64, "f32": STORE_F32, "f16": STORE_F16}


def run(p: Params, f, nsteps: int, storage: str | None = None, rho0: float = 1.0):
    """nsteps steps from f; with storage "f32" or "f16" the state is rounded
    to that deviation storage after every step (the caller rounds the initial
    state with round_storage)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    work = np.zeros_like(f)
    cp = p.c()
    if storage is None:
        _check(lib().orc_run(ctypes.byref(cp), _ptr(f), _ptr(work), ctypes.c_int32(nsteps)), "run")
    else:
        _check(lib().orc_run_stored(ctypes.byref(cp), ctypes.c_double(rho0), ctypes.c_int32(STORAGE[storage]),
                                    _ptr(f), _ptr(work), ctypes.c_int32(nsteps)), "run_stored")
    return f


def round_storage(p: Params, f, storage: str, rho0: float = 1.0):
    """A copy of state f with every deviation rounded to the given storage."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    cp = p.c()
    _check(lib().orc_round_storage(ctypes.byref(cp), ctypes.c_double(rho0), ctypes.c_int32(STORAGE[storage]),
                                   _ptr(f)), "round_storage")
    return f


def round_f16(x: float) -> float:
    return lib().orc_round_f16(float(x))


def moments(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho, ux, uy = (np.zeros((p.ny, p.nx)) for _ in range(3))
    cp = p.c()
    _check(lib().orc_moments(ctypes.byref(cp), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy)), "moments")
    return rho, ux, uy


def gamma_field(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.zeros((p.ny, p.nx))
    cp = p.c()
    _check(lib().orc_gamma_field(ctypes.byref(cp), _ptr(f), _ptr(g)), "gamma_field")
    return g


def diagnostics(p: Params, f) -> dict:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(16)
    cp = p.c()
    _check(lib().orc_diagnostics(ctypes.byref(cp), _ptr(f), _ptr(out)), "diagnostics")
    return {k: float(v) for k, v in zip(DIAG_NAMES, out)}


def adjoint_step(p: Params, f, lam_next):
    f = np.ascontiguousarray(f, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    lam = np.zeros_like(lam_next)
    db = np.zeros((p.ny, p.nx))
    cp = p.c()
    _check(lib().orc_adjoint_step(ctypes.byref(cp), _ptr(f), _ptr(lam_next), _ptr(lam), _ptr(db)),
           "adjoint_step")
    return lam, db


def init_adjoint(p: Params, ux, uy, lam0, rho0: float = 1.0, mode: int = INIT_GRAD_CD):
    ux = np.ascontiguousarray(ux, dtype=np.float64)
    uy = np.ascontiguousarray(uy, dtype=np.float64)
    lam0 = np.ascontiguousarray(lam0, dtype=np.float64)
    gux, guy, db = (np.zeros((p.ny, p.nx)) for _ in range(3))
    cp = p.c()
    _check(lib().orc_init_adjoint(ctypes.byref(cp), ctypes.c_double(rho0), _ptr(ux), _ptr(uy),
                                  ctypes.c_int32(mode), _ptr(lam0), _ptr(gux), _ptr(guy), _ptr(db)),
           "init_adjoint")
    return gux, guy, db


# ------------------------------------------------------------ statistics
def spectra(ux, uy, kmax: int):
    """Shell-summed kinetic-energy and enstrophy spectra of a velocity field on
    an N x N periodic lattice (turbulence statistics of section "Decaying
    Two-Dimensional Turbulence"), written out from the definition over the
    full plane of integer wavevectors k (|k_a| <= N/2):
      e(k) = (|ux_hat(k)|^2 + |uy_hat(k)|^2) / (2 N^4),
      E[s] = sum of e(k) over round(|k|) = s,
      Z[s] = sum of e(k) (2 pi |k| / N)^2 over the same shell,
    with u_hat the unnormalised discrete Fourier transform (numpy's fft2), so
    that sum_s E[s] = <|u|^2> / 2 (Parseval) and sum_s Z[s] is the enstrophy
    with the exact derivative.  Shells above kmax are dropped."""
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    n = ux.shape[0]
    assert ux.shape == (n, n) and uy.shape == (n, n)
    e = (np.abs(np.fft.fft2(ux)) ** 2 + np.abs(np.fft.fft2(uy)) ** 2) / (2.0 * float(n) ** 4)
    k = np.fft.fftfreq(n, d=1.0 / n)                 # integer wavenumbers 0..n/2-1, -n/2..-1
    k2 = k[None, :] ** 2 + k[:, None] ** 2
    shell = np.floor(np.sqrt(k2) + 0.5).astype(np.int64)
    keep = shell <= kmax
    E = np.bincount(shell[keep], weights=e[keep], minlength=kmax + 1)[: kmax + 1]
    Z = np.bincount(shell[keep], weights=(e * k2 * (2.0 * np.pi / n) ** 2)[keep], minlength=kmax + 1)[: kmax + 1]
    return E, Z
