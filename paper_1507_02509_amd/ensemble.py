"""Ensembles of independent lattices of different sizes advanced by one kernel
(include/kbc.h, "ensemble").  Members are ordinary Sim objects; the ensemble
only steps them."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from . import inputs
from .sim import Sim, beta_from_nu


class Ensemble:
    def __init__(self, members: list[Sim]):
        if not members:
            raise ValueError("empty ensemble")
        self.lib = L.load()
        self.members = list(members)
        arr = (ctypes.c_void_p * len(members))(*[m.ctx.value for m in members])
        self.h = ctypes.c_void_p()
        L.check(self.lib.lbm_ensemble_create(ctypes.byref(self.h), arr, len(members)), "lbm_ensemble_create")

    @property
    def nodes(self) -> int:
        return sum(m.nx * m.ny for m in self.members)

    @property
    def blocks(self) -> int:
        """Grid size of the persistent launch for the current fusion and tiles."""
        b = int(self.lib.lbm_ensemble_blocks(self.h))
        if b < 0:
            L.check(b, "lbm_ensemble_blocks")
        return b

    def set_spin_limit(self, polls: int):
        """Barrier polls after which a persistent launch gives up (see check())."""
        L.check(self.lib.lbm_ensemble_set_spin_limit(self.h, int(polls)), "lbm_ensemble_set_spin_limit")

    def check(self) -> "Ensemble":
        """Synchronise and raise KbcError (LBM_ESYNC) if a persistent launch
        since the last check gave up at a grid barrier."""
        L.check(self.lib.lbm_ensemble_check(self.h), "lbm_ensemble_check")
        return self

    def set_tile(self, width: int, rows_per_thread: int, nontemporal: bool = False):
        L.check(self.lib.lbm_ensemble_set_tile(self.h, int(width), int(rows_per_thread), 1 if nontemporal else 0),
                "lbm_ensemble_set_tile")

    def set_fusion(self, steps_per_launch: int, rows: int = 0):
        """Steps per launch (1, or 2 = two fused steps) and the fused tile
        height (8 or 16 rows; 0 keeps the current one)."""
        L.check(self.lib.lbm_ensemble_set_fusion(self.h, int(steps_per_launch), int(rows)), "lbm_ensemble_set_fusion")

    @property
    def fusion(self) -> int:
        return int(self.lib.lbm_ensemble_get_fusion(self.h, None))

    def step(self, n: int = 1, persistent: bool = False) -> "Ensemble":
        """n steps of every member: one launch per step (or pair of fused
        steps), or with persistent=True one launch for all of them."""
        L.check(self.lib.lbm_ensemble_step(self.h, int(n), 1 if persistent else 0), "lbm_ensemble_step")
        return self

    def free(self):
        if self.h:
            L.check(self.lib.lbm_ensemble_free(self.h), "lbm_ensemble_free")
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.h and L._lib is not None:
                L._lib.lbm_ensemble_free(self.h)
        except Exception:
            pass


def make_members(specs, form: str = "f32", collision: str = "kbc", variant: str = "B", k0: float = 8,
                 u_rms: float = 0.05, device="cuda:0") -> list[Sim]:
    """Sims for (n, nu, seed) specs (see inputs.ensemble_members), each
    initialised with Grad's approximation of its seeded spectral field."""
    out = []
    for n, nu, seed in specs:
        ux, uy = inputs.spectral(n, k0, u_rms, seed=seed, device=device)
        s = Sim(n, n, beta_from_nu(nu), collision=collision, variant=variant, form=form, device=device)
        s.init(ux, uy)
        out.append(s)
    torch.cuda.synchronize(device)
    return out
