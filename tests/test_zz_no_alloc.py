"""lbm_adjoint_step_noalloc, the adjoint step for callers that cannot
allocate: through the C ABI, bitwise equal to lbm_adjoint_step on two calls in
a row (the second on a smaller lattice), no device memory allocated by the
call (free device memory unchanged on a context whose own scratch was never
allocated), the full-size FP32 lattice accepted and the full-size FP64
lattice refused before any launch (above the fixed scratch)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import _lib as L
from paper_1507_02509_amd import inputs
from paper_1507_02509_amd.sim import Sim, beta_from_nu

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def lattice(nx, ny, form, seed, k0=3):
    ux, uy = inputs.spectral(nx, k0, 0.05, seed=seed, ny=ny)
    return Sim(nx, ny, beta_from_nu(1e-4), variant="B", form=form).init(ux, uy)


def both(s, seed):
    """lambda_out and dL/dbeta from the allocating step and from the
    no-alloc step, from the same seeded lambda_in."""
    lam = s.new_adjoint()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    lam.normal_(generator=gen)
    out_a, out_b = s.new_adjoint(), s.new_adjoint()
    acc_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    acc_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    L.check(s.lib.lbm_adjoint_step_noalloc(s.ctx, L.ptr(s.state_buffer()), L.ptr(lam), L.ptr(out_b),
                                           L.ptr(acc_b)), "lbm_adjoint_step_noalloc")
    s.adjoint_step(s.state_buffer(), lam, out_a, acc_a)
    torch.cuda.synchronize()
    return s.planes(out_a), s.planes(out_b), acc_a.item(), acc_b.item()


def test_noalloc_equals_adjoint_step_two_calls():
    for (nx, ny, form), seed in (((300, 170, "f32"), 1), ((67, 45, "f64"), 2)):   # the second smaller
        say("noalloc vs adjoint step", nx, ny, form)
        s = lattice(nx, ny, form, seed)
        a, b, da, db = both(s, seed)
        assert torch.equal(a, b), (nx, ny, form)
        assert da == db and np.isfinite(da)
        s.free()


def test_noalloc_full_size_limits():
    n = 16384
    say("noalloc full-size FP32: accepted, no allocation, equal")
    s = lattice(n, n, "f32", 3, k0=32)
    lam = s.new_adjoint()
    lam.normal_()
    out_a, out_b = s.new_adjoint(), s.new_adjoint()
    acc_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    acc_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    # a first call looks the array's address up (which may load the code
    # object holding it); the calls measured below follow it
    warm = torch.zeros(1, dtype=torch.float64, device="cuda")
    L.check(s.lib.lbm_adjoint_step_noalloc(s.ctx, L.ptr(s.state_buffer()), L.ptr(lam), L.ptr(out_b),
                                           L.ptr(warm)), "lbm_adjoint_step_noalloc")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(2):
        L.check(s.lib.lbm_adjoint_step_noalloc(s.ctx, L.ptr(s.state_buffer()), L.ptr(lam), L.ptr(out_b),
                                               L.ptr(acc_b)), "lbm_adjoint_step_noalloc")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    s.adjoint_step(s.state_buffer(), lam, out_a, acc_a)   # allocates the context's scratch (4 MB here)
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    say(f"  free device memory: {free0} -> {free1} (no-alloc) -> {free2} (allocating step)")
    assert free1 == free0
    assert torch.equal(s.planes(out_a), s.planes(out_b))
    assert acc_b.item() == 2 * acc_a.item()
    del lam, out_a, out_b
    s.free()
    del s
    torch.cuda.empty_cache()
    say("noalloc full-size FP64: refused")
    s = lattice(n, n, "f64", 3, k0=32)
    la, lb = s.new_adjoint(), s.new_adjoint()
    rc = s.lib.lbm_adjoint_step_noalloc(s.ctx, L.ptr(s.state_buffer()), L.ptr(la), L.ptr(lb), None)
    assert rc == L.LBM_EINVAL
    assert b"fixed" in s.lib.lbm_last_error()
    s.free()
