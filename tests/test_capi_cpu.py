"""CPU tests of the C ABI: the library loads, exports every function
include/kbc.h declares, and rejects invalid arguments before any HIP call
(no GPU is needed for that)."""
import ctypes

import pytest

from paper_1507_02509_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_exports_every_declared_function(lib):
    names = L.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_sizes():
    assert ctypes.sizeof(L.Params) == 64
    assert ctypes.sizeof(L.Diag) == 16 * 8


def test_pitch_and_bytes(lib):
    assert lib.lbm_required_pitch(1, L.F32DEV_F32) == 64
    assert lib.lbm_required_pitch(64, L.F32DEV_F32) == 64
    assert lib.lbm_required_pitch(65, L.F16DEV_F32) == 128
    assert lib.lbm_required_pitch(16384, L.F64) == 16384
    assert lib.lbm_required_pitch(0, L.F64) == 0
    assert lib.lbm_required_pitch(10, 7) == 0
    assert lib.lbm_buffer_bytes(100, 10, L.F32DEV_F32) == 9 * 10 * 128 * 4
    assert lib.lbm_buffer_bytes(100, 10, L.F16DEV_F32) == 9 * 10 * 128 * 2
    assert lib.lbm_buffer_bytes(100, 10, L.F64) == 9 * 10 * 128 * 8
    # sides are at most 2^28 nodes (32-bit byte offsets within a row)
    assert lib.lbm_required_pitch(1 << 28, L.F64) == 1 << 28
    assert lib.lbm_required_pitch((1 << 28) + 1, L.F16DEV_F32) == 0
    assert lib.lbm_buffer_bytes((1 << 28) + 1, 3, L.F32DEV_F32) == 0
    assert lib.lbm_buffer_bytes(65536, 65536, L.F16DEV_F32) == 9 * 65536 * 65536 * 2


def _params(**kw):
    p = L.Params()
    p.nx, p.ny, p.beta, p.rho0 = 16, 16, 0.9, 1.0
    p.collision, p.variant, p.form, p.gamma_mode = L.KBC, L.KBC_B, L.F32DEV_F32, L.GAMMA_ESTIMATE
    p.gamma_guard, p.gamma_fixed, p.stream = 1e-12, 2.0, None
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# fake, never dereferenced device addresses: every case fails validation first
A, B, U, V, G = 0x100000, 0x200000, 0x300000, 0x400000, 0x500000


@pytest.mark.parametrize("kw,args,code", [
    (dict(nx=2), {}, L.LBM_EINVAL),
    (dict(ny=1), {}, L.LBM_EINVAL),
    (dict(nx=(1 << 28) + 1), {}, L.LBM_EINVAL),
    (dict(ny=(1 << 28) + 1), {}, L.LBM_EINVAL),
    (dict(beta=0.0), {}, L.LBM_EINVAL),
    (dict(beta=1.5), {}, L.LBM_EINVAL),
    (dict(beta=float("nan")), {}, L.LBM_EINVAL),
    (dict(rho0=0.0), {}, L.LBM_EINVAL),
    (dict(collision=3), {}, L.LBM_EINVAL),
    (dict(variant=4), {}, L.LBM_EINVAL),
    (dict(form=5), {}, L.LBM_EINVAL),
    (dict(gamma_mode=9), {}, L.LBM_EINVAL),
    (dict(gamma_guard=-1.0), {}, L.LBM_EINVAL),
    (dict(gamma_mode=L.GAMMA_FIXED, gamma_fixed=float("inf")), {}, L.LBM_EINVAL),
    ({}, dict(buf_a=None), L.LBM_EINVAL),
    ({}, dict(pitch=32), L.LBM_EINVAL),
    ({}, dict(pitch=96), L.LBM_EINVAL),
    ({}, dict(buf_b=A + 64), L.LBM_EINVAL),          # overlapping buffers
    ({}, dict(ux=None), L.LBM_EINVAL),
    ({}, dict(mode=L.INIT_GRAD_GIVEN, grad=None), L.LBM_EINVAL),
    ({}, dict(mode=7), L.LBM_EINVAL),
])
def test_init_rejects_invalid_arguments(lib, kw, args, code):
    p = _params(**kw)
    a = dict(buf_a=A, buf_b=B, pitch=64, rho=None, ux=U, uy=V, grad=None, mode=L.INIT_GRAD_CD)
    a.update(args)
    ctx = ctypes.c_void_p()
    rc = lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), a["buf_a"], a["buf_b"], a["pitch"], a["rho"],
                      a["ux"], a["uy"], a["grad"], a["mode"])
    assert rc == code
    assert not ctx
    assert lib.lbm_last_error()


def test_null_context_calls_fail_cleanly(lib):
    assert lib.lbm_step(None, 1) == L.LBM_EINVAL
    assert lib.lbm_moments(None, None, None, None, None) == L.LBM_EINVAL
    assert lib.lbm_get_populations(None, None) == L.LBM_EINVAL
    assert lib.lbm_set_populations(None, None) == L.LBM_EINVAL
    assert lib.lbm_diagnostics(None, None) == L.LBM_EINVAL
    assert lib.lbm_set_tile(None, 256, 1, 0) == L.LBM_EINVAL
    assert lib.lbm_get_tile(None, None, None, None) == L.LBM_EINVAL
    assert lib.lbm_set_graph(None, 8) == L.LBM_EINVAL
    assert lib.lbm_set_halo(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_get_edge_rows(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_adjoint_step_slab(None, None, None, None, None, None, None, None, None) == L.LBM_EINVAL
    assert lib.lbm_get_graph(None) == -1
    assert lib.lbm_step_count(None) == -1
    assert lib.lbm_free(None) == L.LBM_OK
    assert lib.lbm_copy_probe(None, None, 4, None) == L.LBM_EINVAL
    which = ctypes.c_int32(-1)
    assert lib.lbm_adjoint_rollout(None, None, 10, 3, None, None, None, None, None,
                                   ctypes.byref(which)) == L.LBM_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        L.load()


def test_ensemble_entry_points_reject_null(lib):
    """The ensemble calls validate their handle before any HIP call."""
    assert lib.lbm_ensemble_step(None, 2, 1) == L.LBM_EINVAL
    assert lib.lbm_ensemble_set_spin_limit(None, 5) == L.LBM_EINVAL
    assert lib.lbm_ensemble_check(None) == L.LBM_EINVAL
    assert lib.lbm_ensemble_blocks(None) < 0
    assert lib.lbm_ensemble_free(None) == L.LBM_OK
    assert L.LBM_ESYNC == -6 and L.LBM_ENSEMBLE_SPIN_MAX == 1 << 26
