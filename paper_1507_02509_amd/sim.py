"""A lattice on one GPU behind the C ABI: torch allocates the population
buffers and the macroscopic fields and provides the stream; libkbc does all
of the work."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

_FORMS = {"f16": L.F16DEV_F32, "f32": L.F32DEV_F32, "f64": L.F64}
_TORCH_STORE = {L.F16DEV_F32: torch.float16, L.F32DEV_F32: torch.float32, L.F64: torch.float64}
_VARIANTS = {"A": L.KBC_A, "B": L.KBC_B, "C": L.KBC_C, "D": L.KBC_D}
_GMODES = {"estimate": L.GAMMA_ESTIMATE, "fixed": L.GAMMA_FIXED, "exact": L.GAMMA_EXACT}
_INIT = {"eq": L.INIT_EQ, "grad_cd": L.INIT_GRAD_CD, "grad_given": L.INIT_GRAD_GIVEN}


def beta_from_nu(nu: float) -> float:
    """beta from the kinematic viscosity, eq. (viscosity) with cs2 = 1/3."""
    return 1.0 / (6.0 * nu + 1.0)


def _dev64(a, device) -> torch.Tensor | None:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    return a.to(device=device, dtype=torch.float64).contiguous()


class Sim:
    """One periodic nx x ny lattice.

    collision: "kbc" or "lbgk"; variant: "A".."D" (Table kbc_moment_grouping);
    form: "f16" | "f32" | "f64" (storage form, see include/kbc.h).
    """

    def __init__(self, nx: int, ny: int, beta: float, collision: str = "kbc", variant: str = "B",
                 form: str = "f32", gamma_mode: str = "estimate", gamma_guard: float = 1e-12,
                 gamma_fixed: float = 2.0, rho0: float = 1.0, device="cuda:0", tile: tuple | None = None,
                 pitch_pad: int = 0, fusion: int | None = None, graph: int = 0):
        self.lib = L.load()
        self.device = torch.device(device)
        self.nx, self.ny = int(nx), int(ny)
        self.form = _FORMS[form]
        self.pitch = int(self.lib.lbm_required_pitch(self.nx, self.form))
        if self.pitch == 0:
            raise ValueError("invalid lattice size or form")
        if pitch_pad % 64:
            raise ValueError("pitch_pad must be a multiple of 64 elements")
        self.pitch += int(pitch_pad)
        dt = _TORCH_STORE[self.form]
        # population buffers are [ny][9][pitch]: the nine population rows of
        # each lattice row one after another
        self.buf_a = torch.empty((self.ny, 9, self.pitch), dtype=dt, device=self.device)
        self.buf_b = torch.empty((self.ny, 9, self.pitch), dtype=dt, device=self.device)
        self.params = L.Params()
        self.params.nx, self.params.ny = self.nx, self.ny
        self.params.beta = float(beta)
        self.params.rho0 = float(rho0)
        self.params.collision = L.LBGK if collision.lower() == "lbgk" else L.KBC
        self.params.variant = _VARIANTS[variant.upper()]
        self.params.form = self.form
        self.params.gamma_mode = _GMODES[gamma_mode]
        self.params.gamma_guard = float(gamma_guard)
        self.params.gamma_fixed = float(gamma_fixed)
        self.params.stream = torch.cuda.current_stream(self.device).cuda_stream
        self.ctx = ctypes.c_void_p()
        self._tile = tile
        self._fusion = fusion
        self._graph = int(graph)
        self._inputs = None

    # ------------------------------------------------------------------ setup
    def init(self, ux, uy, rho=None, mode: str = "grad_cd", grad=None) -> "Sim":
        ux, uy = _dev64(ux, self.device), _dev64(uy, self.device)
        rho, grad = _dev64(rho, self.device), _dev64(grad, self.device)
        for a in (ux, uy):
            assert a.shape == (self.ny, self.nx), "velocity fields must be [ny, nx]"
        if self.ctx:
            self.free()
        L.check(self.lib.lbm_init(ctypes.byref(self.ctx), ctypes.byref(self.params), L.ptr(self.buf_a),
                                  L.ptr(self.buf_b), self.pitch, L.ptr(rho), L.ptr(ux), L.ptr(uy),
                                  L.ptr(grad), _INIT[mode]), "lbm_init")
        self._inputs = (ux, uy, rho, grad)   # alive until the init kernel has run
        if self._tile is not None:
            self.set_tile(*self._tile)
        if self._fusion is not None:
            self.set_fusion(*(self._fusion if isinstance(self._fusion, tuple) else (self._fusion,)))
        if self._graph:
            self.set_graph(self._graph)
        return self

    def set_graph(self, chunk: int):
        """Replay every whole `chunk` steps of step() as one HIP graph launch
        (captured once per start buffer from the same kernel launches; bitwise
        identical to launching them one by one); 0 launches every kernel
        directly.  Pays off on small, launch-bound lattices."""
        self._graph = int(chunk)
        if self.ctx:
            L.check(self.lib.lbm_set_graph(self.ctx, self._graph), "lbm_set_graph")

    @property
    def graph(self) -> int:
        """Steps per graph replay (0: none)."""
        return int(self.lib.lbm_get_graph(self.ctx))

    def set_fusion(self, steps_per_launch: int, rows: int = 0):
        """Time steps per kernel launch (1, or 2 = two fused steps) and the
        fused tile height (8, 16, 24 or 32 rows; 0 keeps the current one)."""
        self._fusion = (int(steps_per_launch), int(rows))
        if self.ctx:
            L.check(self.lib.lbm_set_fusion(self.ctx, *self._fusion), "lbm_set_fusion")

    @property
    def fusion(self) -> int:
        """Time steps per kernel launch."""
        return int(self.lib.lbm_get_fusion(self.ctx, None))

    @property
    def fusion_rows(self) -> int:
        """Output tile height of the fused launch."""
        r = ctypes.c_int32(0)
        self.lib.lbm_get_fusion(self.ctx, ctypes.byref(r))
        return int(r.value)

    # ------------------------------------------------------- slab of a domain
    def halo_buffers(self) -> tuple[torch.Tensor, torch.Tensor]:
        """Two zeroed [2, 9, pitch] buffers of the storage dtype: the shape of
        a slab's halo (lbm_set_halo) and of its edge rows (lbm_get_edge_rows)."""
        dt = _TORCH_STORE[self.form]
        return (torch.zeros((2, 9, self.pitch), dtype=dt, device=self.device),
                torch.zeros((2, 9, self.pitch), dtype=dt, device=self.device))

    def set_halo(self, lo: torch.Tensor | None, hi: torch.Tensor | None):
        """Make this lattice one slab of a domain split in y: rows -2, -1
        come from `lo` and rows ny, ny + 1 from `hi` ([2, 9, pitch] each, kept
        alive by the caller and refreshed between steps); None, None returns
        to periodic rows (include/kbc.h, lbm_set_halo)."""
        for t in (lo, hi):
            if t is not None:
                assert t.shape == (2, 9, self.pitch) and t.dtype == _TORCH_STORE[self.form] and t.is_contiguous()
        self._halo = (lo, hi)
        L.check(self.lib.lbm_set_halo(self.ctx, L.ptr(lo), L.ptr(hi)), "lbm_set_halo")

    def edge_rows(self, lo_rows: torch.Tensor, hi_rows: torch.Tensor):
        """Rows 0, 1 into lo_rows and rows ny - 2, ny - 1 into hi_rows (the
        neighbours' halos), enqueued on the library's stream."""
        for t in (lo_rows, hi_rows):
            assert t.shape == (2, 9, self.pitch) and t.dtype == _TORCH_STORE[self.form] and t.is_contiguous()
        L.check(self.lib.lbm_get_edge_rows(self.ctx, L.ptr(lo_rows), L.ptr(hi_rows)), "lbm_get_edge_rows")

    def set_tile(self, width: int, rows_per_thread: int = 1, nontemporal: bool = False):
        L.check(self.lib.lbm_set_tile(self.ctx, int(width), int(rows_per_thread), 1 if nontemporal else 0),
                "lbm_set_tile")

    @property
    def tile(self) -> tuple[int, int, bool]:
        """(width, rows_per_thread, nontemporal) of the step kernel's tile,
        the flag also being the store kind of the fused launch."""
        w, r, f = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        L.check(self.lib.lbm_get_tile(self.ctx, ctypes.byref(w), ctypes.byref(r), ctypes.byref(f)), "lbm_get_tile")
        return int(w.value), int(r.value), bool(f.value & 1)

    def set_beta(self, beta: float):
        self.params.beta = float(beta)
        if self.ctx:
            L.check(self.lib.lbm_set_beta(self.ctx, float(beta)), "lbm_set_beta")

    # ------------------------------------------------------------------- run
    def step(self, n: int = 1) -> "Sim":
        L.check(self.lib.lbm_step(self.ctx, int(n)), "lbm_step")
        return self

    def step_checked(self, n: int, every: int = 100) -> "Sim":
        """n steps, reading the diagnostics every `every` steps and at the end;
        raises NonFiniteState (code LBM_ENONFINITE) at the first check that
        finds a non-finite density or velocity.  The step kernels themselves
        never check values."""
        done = 0
        while done < n:
            k = min(every, n - done)
            self.step(k)
            done += k
            d = self.diagnostics()
            if d["n_nonfinite"]:
                raise NonFiniteState(self.steps, int(d["n_nonfinite"]))
        return self

    @property
    def steps(self) -> int:
        return int(self.lib.lbm_step_count(self.ctx))

    def moments(self, gamma: bool = False):
        shape = (self.ny, self.nx)
        rho, ux, uy = (torch.empty(shape, dtype=torch.float64, device=self.device) for _ in range(3))
        g = torch.empty(shape, dtype=torch.float64, device=self.device) if gamma else None
        L.check(self.lib.lbm_moments(self.ctx, L.ptr(rho), L.ptr(ux), L.ptr(uy), L.ptr(g)), "lbm_moments")
        return (rho, ux, uy, g) if gamma else (rho, ux, uy)

    def get_populations(self) -> torch.Tensor:
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_get_populations(self.ctx, L.ptr(f)), "lbm_get_populations")
        return f

    def set_populations(self, f):
        f = _dev64(f, self.device)
        assert f.shape == (9, self.ny, self.nx)
        L.check(self.lib.lbm_set_populations(self.ctx, L.ptr(f)), "lbm_set_populations")
        self._inputs = (f,)

    def spectra(self, kmax: int | None = None):
        """Shell-summed kinetic-energy and enstrophy spectra (E_k, Z_k), FP64
        tensors of kmax + 1 shells (default: every shell, ceil(N/sqrt 2))."""
        if kmax is None:
            kmax = int(np.ceil(self.nx / np.sqrt(2.0)))
        ek = torch.empty(kmax + 1, dtype=torch.float64, device=self.device)
        zk = torch.empty(kmax + 1, dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_spectra(self.ctx, int(kmax), L.ptr(ek), L.ptr(zk)), "lbm_spectra")
        return ek, zk

    def diagnostics(self) -> dict:
        d = L.Diag()
        L.check(self.lib.lbm_diagnostics(self.ctx, ctypes.byref(d)), "lbm_diagnostics")
        return {k: getattr(d, k) for k in L.DIAG_FIELDS if k != "reserved"}

    # ------------------------------------------------------------- adjoint
    @property
    def adjoint_dtype(self):
        return torch.float64 if self.form == L.F64 else torch.float32

    def set_adjoint_gamma(self, frozen: bool):
        L.check(self.lib.lbm_set_adjoint_gamma(self.ctx, 1 if frozen else 0), "lbm_set_adjoint_gamma")

    def new_adjoint(self) -> torch.Tensor:
        return torch.empty((self.ny, 9, self.pitch), dtype=self.adjoint_dtype, device=self.device)

    def planes(self, buf: torch.Tensor) -> torch.Tensor:
        """View of a [ny][9][pitch] state or adjoint buffer as [9][ny][nx]
        (no copy; writes through the view change the buffer)."""
        return buf.permute(1, 0, 2)[:, :, :self.nx]

    def new_state(self) -> torch.Tensor:
        return torch.empty_like(self.buf_a)

    def step_buffers(self, src: torch.Tensor, dst: torch.Tensor):
        L.check(self.lib.lbm_step_buffers(self.ctx, L.ptr(src), L.ptr(dst)), "lbm_step_buffers")

    def adjoint_seed(self, state, lam, drho=None, dux=None, duy=None):
        drho, dux, duy = (None if a is None else _dev64(a, self.device) for a in (drho, dux, duy))
        L.check(self.lib.lbm_adjoint_seed(self.ctx, L.ptr(state), L.ptr(drho), L.ptr(dux), L.ptr(duy),
                                          L.ptr(lam)), "lbm_adjoint_seed")
        self._inputs = (drho, dux, duy)

    def adjoint_step(self, state, lam_in, lam_out, dbeta=None):
        L.check(self.lib.lbm_adjoint_step(self.ctx, L.ptr(state), L.ptr(lam_in), L.ptr(lam_out), L.ptr(dbeta)),
                "lbm_adjoint_step")

    def adjoint_step_slab(self, state, state_lo, state_hi, lam_in, lam_lo, lam_hi, lam_out, dbeta=None):
        """The adjoint step of a slab (lbm_adjoint_step_slab): rows -2, -1 and
        ny, ny + 1 of the state and of lam_in from the given [2, 9, pitch]
        halo tensors."""
        L.check(self.lib.lbm_adjoint_step_slab(self.ctx, L.ptr(state), L.ptr(state_lo), L.ptr(state_hi),
                                               L.ptr(lam_in), L.ptr(lam_lo), L.ptr(lam_hi), L.ptr(lam_out),
                                               L.ptr(dbeta)), "lbm_adjoint_step_slab")

    def adjoint_step_noalloc(self, state, lam_in, lam_out, dbeta=None):
        """lbm_adjoint_step_noalloc: the same step with the library's fixed
        per-GPU scratch array (allocates nothing; overlapping calls on one
        GPU race)."""
        L.check(self.lib.lbm_adjoint_step_noalloc(self.ctx, L.ptr(state), L.ptr(lam_in), L.ptr(lam_out),
                                                  L.ptr(dbeta)), "lbm_adjoint_step_noalloc")

    def adjoint_segment(self, state0, slots, k: int, lam_in, lam_out, dbeta=None) -> int:
        """Recompute and back-propagate one checkpoint segment (see
        lbm_adjoint_segment); returns 0 if the result is in lam_in, 1 if in lam_out."""
        arr = (ctypes.c_void_p * max(1, k - 1))(*[L.ptr(t) for t in slots[:k - 1]]) if k > 1 else None
        which = ctypes.c_int32(-1)
        L.check(self.lib.lbm_adjoint_segment(self.ctx, L.ptr(state0), arr, int(k), L.ptr(lam_in), L.ptr(lam_out),
                                             L.ptr(dbeta), ctypes.byref(which)), "lbm_adjoint_segment")
        return int(which.value)

    def adjoint_rollout(self, ckpts, nsteps: int, seglen: int, slots_a, slots_b, lam_in, lam_out,
                        dbeta=None) -> int:
        """The whole backward pass over checkpoints ckpts (f^0, f^seglen, ...),
        each launch running one adjoint step and one recomputation step of the
        next segment (see lbm_adjoint_rollout); returns 0 if dL/df^0 is in
        lam_in, 1 if in lam_out."""
        def arr(ts):
            return (ctypes.c_void_p * max(1, len(ts)))(*[L.ptr(t) for t in ts]) if ts else None
        which = ctypes.c_int32(-1)
        L.check(self.lib.lbm_adjoint_rollout(self.ctx, arr(ckpts), int(nsteps), int(seglen), arr(slots_a),
                                             arr(slots_b), L.ptr(lam_in), L.ptr(lam_out), L.ptr(dbeta),
                                             ctypes.byref(which)), "lbm_adjoint_rollout")
        return int(which.value)

    def adjoint_init(self, ux0, uy0, lam0, grad_ux, grad_uy, dbeta=None, rho=None, mode: str = "grad_cd"):
        L.check(self.lib.lbm_adjoint_init(self.ctx, L.ptr(rho), L.ptr(ux0), L.ptr(uy0), _INIT[mode], L.ptr(lam0),
                                          L.ptr(grad_ux), L.ptr(grad_uy), L.ptr(dbeta)), "lbm_adjoint_init")

    def state_buffer(self) -> torch.Tensor:
        p = self.lib.lbm_state_buffer(self.ctx)
        return self.buf_a if p == self.buf_a.data_ptr() else self.buf_b

    def free(self):
        if self.ctx:
            L.check(self.lib.lbm_free(self.ctx), "lbm_free")
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.ctx and L._lib is not None:
                L._lib.lbm_free(self.ctx)
        except Exception:
            pass


class NonFiniteState(RuntimeError):
    """A checked run found non-finite values (LBM_ENONFINITE)."""
    code = L.LBM_ENONFINITE

    def __init__(self, step: int, count: int):
        super().__init__(f"non-finite state at step {step}: {count} nodes")
        self.step, self.count = step, count


def copy_probe(dst: torch.Tensor, src: torch.Tensor):
    """dst <- src through the library's streaming copy kernel (4-byte words)."""
    lib = L.load()
    n = src.numel() * src.element_size() // 4
    L.check(lib.lbm_copy_probe(L.ptr(dst), L.ptr(src), n, torch.cuda.current_stream(dst.device).cuda_stream),
            "lbm_copy_probe")
