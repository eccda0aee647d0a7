"""One GPU's share of a domain split in y: slabs stepped with halo rows from
their neighbours (lbm_set_halo / lbm_get_edge_rows) equal, bit for bit, the
whole domain stepped as one periodic lattice.  The exchange between slabs is
done here with device copies on the library's stream, in the pattern a
multi-GPU run would do with point-to-point sends: before every launch, each
slab's two top and two bottom rows go to its neighbours' halos."""
import numpy as np
import pytest
import torch

from paper_1507_02509_amd import inputs
from paper_1507_02509_amd._lib import KbcError
from paper_1507_02509_amd.sim import Sim, beta_from_nu

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make_slabs(nx, heights, form, coll, var, fusion, gamma_mode="estimate"):
    ny = sum(heights)
    beta = beta_from_nu(1e-4)
    ux, uy = inputs.spectral(nx, 4, 0.05, seed=31, ny=ny)
    full = Sim(nx, ny, beta, collision=coll, variant=var, form=form, fusion=fusion,
               gamma_mode=gamma_mode).init(ux, uy)
    f0 = full.state_buffer()   # [ny][9][pitch] in the storage form: copied bit for bit
    slabs = []
    y = 0
    for h in heights:
        s = Sim(nx, h, beta, collision=coll, variant=var, form=form, fusion=fusion, gamma_mode=gamma_mode)
        s.init(np.zeros((h, nx)), np.zeros((h, nx)), mode="eq")
        assert s.pitch == full.pitch
        s.state_buffer().copy_(f0[y:y + h])
        lo, hi = s.halo_buffers()
        s.set_halo(lo, hi)
        send_lo, send_hi = s.halo_buffers()
        slabs.append({"sim": s, "lo": lo, "hi": hi, "send_lo": send_lo, "send_hi": send_hi})
        y += h
    return full, slabs


def exchange(slabs):
    """Rows -2, -1 of slab k are rows ny - 2, ny - 1 of slab k - 1; rows ny,
    ny + 1 are rows 0, 1 of slab k + 1 (the domain is periodic in y)."""
    k = len(slabs)
    for d in slabs:
        d["sim"].edge_rows(d["send_lo"], d["send_hi"])
    for i, d in enumerate(slabs):
        d["lo"].copy_(slabs[(i - 1) % k]["send_hi"])
        d["hi"].copy_(slabs[(i + 1) % k]["send_lo"])


def assert_slabs_equal_full(full, slabs):
    nx = full.nx
    got = torch.cat([d["sim"].state_buffer()[:, :, :nx] for d in slabs], dim=0)
    want = full.state_buffer()[:, :, :nx]
    assert got.shape == want.shape
    assert torch.equal(got, want), float((got.double() - want.double()).abs().max())


SCHEDULE = (2, 2, 1, 2, 1, 1, 2)


@pytest.mark.parametrize("form", ["f32", "f16", "f64"])
@pytest.mark.parametrize("coll,var", [("kbc", "B"), ("lbgk", "A"), ("kbc", "C")])
@pytest.mark.parametrize("fusion", [(2, 16), (2, 8), (1, 0)])
def test_slabs_equal_periodic_domain(form, coll, var, fusion):
    """Four ragged slabs (16, 20, 9 and 19 rows, 150 columns: tiles ragged
    in x, slabs shorter than a fused tile) over seven launches of one or two
    steps."""
    say("slabs", form, coll, var, fusion)
    full, slabs = make_slabs(150, (16, 20, 9, 19), form, coll, var, fusion)
    for n in SCHEDULE:
        if n > fusion[0]:
            n = fusion[0]
        exchange(slabs)
        for d in slabs:
            d["sim"].step(n)
        full.step(n)
    assert_slabs_equal_full(full, slabs)


@pytest.mark.parametrize("heights", [(3, 3, 5), (37,), (2 * 16 + 3, 16)])
def test_slab_edge_cases(heights):
    """Three-row slabs (the fused tile's ring rows both come from halos), one
    slab that is its own neighbour, and slabs taller than one fused tile."""
    say("slab edges", heights)
    full, slabs = make_slabs(70, heights, "f32", "kbc", "B", (2, 16))
    for n in (2, 1, 2, 2):
        exchange(slabs)
        for d in slabs:
            d["sim"].step(n)
        full.step(n)
    assert_slabs_equal_full(full, slabs)


def test_slab_exact_stabilizer():
    full, slabs = make_slabs(96, (12, 20), "f64", "kbc", "B", (2, 16), gamma_mode="exact")
    for n in (2, 2, 1):
        exchange(slabs)
        for d in slabs:
            d["sim"].step(n)
        full.step(n)
    assert_slabs_equal_full(full, slabs)


def test_slab_rules():
    """A slab steps at most one launch per call, takes both halo buffers or
    neither, and returns to periodic rows when both are cleared."""
    full, slabs = make_slabs(64, (16, 16), "f32", "kbc", "B", (2, 16))
    s = slabs[0]["sim"]
    with pytest.raises(KbcError):
        s.step(3)
    with pytest.raises(KbcError):
        s.set_halo(slabs[0]["lo"], None)
    with pytest.raises(KbcError):
        s.set_graph(4)
    with pytest.raises(KbcError):
        s.set_fusion(2, 24)
    s.set_halo(None, None)
    s.step(3)
    periodic = Sim(64, 16, beta_from_nu(1e-4), collision="kbc", variant="B", form="f32", fusion=(2, 16))
    periodic.init(np.zeros((16, 64)), np.zeros((16, 64)), mode="eq")
    periodic.state_buffer().copy_(full.state_buffer()[:16])
    periodic.step(3)
    assert torch.equal(s.state_buffer()[:, :, :64], periodic.state_buffer()[:, :, :64])


def two_rows(t, r0, ny):
    """Rows r0 and r0 + 1 (periodic in the domain) of a [ny, 9, pitch] field."""
    return torch.stack([t[r0 % ny], t[(r0 + 1) % ny]]).contiguous()


@pytest.mark.parametrize("form", ["f32", "f64", "f16"])
@pytest.mark.parametrize("coll,var", [("kbc", "B"), ("lbgk", "A"), ("kbc", "D")])
def test_slab_adjoint_step_equals_domain(form, coll, var):
    """The adjoint step of each slab (lbm_adjoint_step_slab), with the state's
    and the incoming adjoint's rows beyond the slab taken from the
    neighbouring slabs, equals the whole domain's adjoint step on those rows
    bit for bit; the slabs' dL/dbeta shares add up to the domain's."""
    nx, heights = 100, (13, 20, 7)
    ny = sum(heights)
    say("slab adjoint", form, coll, var)
    beta = beta_from_nu(1e-3)
    ux, uy = inputs.spectral(nx, 3, 0.05, seed=33, ny=ny)
    full = Sim(nx, ny, beta, collision=coll, variant=var, form=form).init(ux, uy)
    full.step(3)
    state = full.state_buffer()
    lin = full.new_adjoint()
    g = torch.Generator(device="cuda").manual_seed(34)
    lin.copy_(torch.randn(lin.shape, generator=g, device="cuda", dtype=torch.float64).to(lin.dtype))
    lout = full.new_adjoint().zero_()
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    full.adjoint_step(state, lin, lout, acc)
    y, total = 0, 0.0
    for h in heights:
        s = Sim(nx, h, beta, collision=coll, variant=var, form=form)
        s.init(np.zeros((h, nx)), np.zeros((h, nx)), mode="eq")
        st = state[y:y + h].contiguous()
        li = lin[y:y + h].contiguous()
        out = s.new_adjoint().zero_()
        a = torch.zeros(1, dtype=torch.float64, device="cuda")
        s.adjoint_step_slab(st, two_rows(state, y - 2, ny), two_rows(state, y + h, ny), li,
                            two_rows(lin, y - 2, ny), two_rows(lin, y + h, ny), out, a)
        assert torch.equal(out[:, :, :nx], lout[y:y + h, :, :nx])
        total += a.item()
        y += h
    assert total == pytest.approx(acc.item(), rel=1e-9, abs=1e-12)
