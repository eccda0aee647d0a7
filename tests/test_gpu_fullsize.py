"""Parity at the full roofline size: the 16384^2 decaying-turbulence lattice
(k0 = 32, u_rms = 0.05, nu = 1e-4, seed 3, Grad initialisation with central
differences, KBC-B), stepped on the GPU in the launch configuration the
benchmark times (the default tile of each storage form), checked against the
oracle on sampled nodes.

The oracle cannot hold this lattice, but one step at a node depends only on a
5 x 5 patch of the initial velocity: f^1_i(x) is component i of the collision
at the source node x - v_i, whose Grad populations need u there and at its
four neighbours (central differences).  So for every sampled node the oracle
builds the nine source nodes' populations (node_grad) and collides them
(node_collide), and the GPU's f^1 at that node must match.  Samples include
the four corners and the edges, where the periodic wrap is taken, and nodes on
tile edges.

Tolerances (max |gpu - oracle| / max |oracle - W| over the samples): FP64
1e-12, FP32 2e-5, FP16 5e-3, as for one step on the small lattices.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import inputs
from paper_1507_02509_amd.sim import Sim, beta_from_nu
from oracle_sensitivity import K_SENS, SEEDS, perturbed

pytestmark = pytest.mark.gpu

N, K0, URMS, NU, SEED = 16384, 32, 0.05, 1e-4, 3
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
TOL = {"f64": 1e-12, "f32": 2e-5, "f16": 5e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def field():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("full-size field", N, "k0", K0, "seed", SEED)
    ux, uy = inputs.spectral(N, K0, URMS, seed=SEED, device="cuda")
    return ux, uy


def sample_nodes():
    rng = np.random.default_rng(11)
    pts = [(0, 0), (N - 1, 0), (0, N - 1), (N - 1, N - 1), (0, N // 2), (N // 2, 0), (N - 1, N // 3),
           (N // 3, N - 1), (255, 77), (256, 77), (127, 4095), (128, 4096)]
    pts += [tuple(int(v) for v in rng.integers(0, N, 2)) for _ in range(40)]
    return pts


def oracle_f1(orc, ux, uy, beta, x, y):
    """f^1 at (x, y) from the oracle's node functions."""
    dx = np.arange(-2, 3)
    ys = (y + dx) % N
    xs = (x + dx) % N
    # 5 x 5 velocity patch around (x, y), patch[j, i] = u(x + i - 2, y + j - 2)
    iy = torch.as_tensor(ys, device=ux.device)[:, None]
    ix = torch.as_tensor(xs, device=ux.device)[None, :]
    pu = ux[iy, ix].cpu().numpy()
    pv = uy[iy, ix].cpu().numpy()
    p = orc.Params(N, N, beta, collision=orc.KBC, variant=orc.VARIANTS["B"])
    out = np.zeros(9)
    for i in range(9):
        # source node x - v_i, at patch index (2 - c_y, 2 - c_x)
        j, k = 2 - CY[i], 2 - CX[i]
        du = [0.5 * (pu[j, k + 1] - pu[j, k - 1]), 0.5 * (pu[j + 1, k] - pu[j - 1, k]),
              0.5 * (pv[j, k + 1] - pv[j, k - 1]), 0.5 * (pv[j + 1, k] - pv[j - 1, k])]
        f0 = orc.node_grad(1.0, pu[j, k], pv[j, k], du, beta)
        post, _ = orc.node_collide(p, f0)
        out[i] = post[i]
    return out


@pytest.mark.parametrize("form", ["f32", "f64", "f16"])
def test_fullsize_one_step_sampled(orc, field, form):
    ux, uy = field
    beta = beta_from_nu(NU)
    say("full-size one step", form)
    s = Sim(N, N, beta, collision="kbc", variant="B", form=form).init(ux, uy)
    s.step(1)
    torch.cuda.synchronize()
    pts = sample_nodes()
    xs = torch.as_tensor([p[0] for p in pts], device="cuda")
    ys = torch.as_tensor([p[1] for p in pts], device="cuda")
    f = s.get_populations()
    fg = f[:, ys, xs].cpu().numpy().T          # [samples, 9]
    del f, s
    torch.cuda.empty_cache()
    fo = np.array([oracle_f1(orc, ux, uy, beta, x, y) for x, y in pts])
    err = np.abs(fg - fo).max() / np.abs(fo - W).max()
    say("  samples", len(pts), "err", err)
    assert np.isfinite(fg).all()
    assert err < TOL[form]


def oracle_window(orc, ux, uy, beta, x, y, nsteps, collision="kbc", variant="B", storage=None, perturb_seed=None):
    """f^nsteps at (x, y) from the oracle run on a periodic window of half-width
    nsteps + 2 cut from the full field around (x, y).  After n steps a node
    depends on the initial velocity within distance n + 1 (n streaming steps
    and the central-difference gradient of Grad's state); the window's own
    wrap-around spreads inward one node per step from its edge, so its centre
    is exact."""
    h = nsteps + 2
    d = np.arange(-h, h + 1)
    iy = torch.as_tensor((y + d) % N, device=ux.device)[:, None]
    ix = torch.as_tensor((x + d) % N, device=ux.device)[None, :]
    pu = np.ascontiguousarray(ux[iy, ix].cpu().numpy())
    pv = np.ascontiguousarray(uy[iy, ix].cpu().numpy())
    p = orc.Params(2 * h + 1, 2 * h + 1, beta, collision=orc.LBGK if collision == "lbgk" else orc.KBC,
                   variant=orc.VARIANTS[variant], threads=4)
    f0 = orc.init(p, pu, pv)
    if perturb_seed is not None:
        f0 = perturbed(f0, perturb_seed)
    if storage is not None:
        f0 = orc.round_storage(p, f0, storage)
    f = orc.run(p, f0, nsteps, storage=storage)
    return f[:, h, h]


MULTI_TOL = {"f64": 1e-12, "f32": 1e-4, "f16": 1e-2}


@pytest.mark.parametrize("form", ["f32", "f64", "f16"])
def test_fullsize_steps_10_and_50_sampled(orc, field, form):
    """As the one-step test, after 10 and 50 steps of the full lattice in the
    default launch configuration (two fused steps per launch), against the
    oracle on windows around 12 sampled nodes (corners, edges, random).
    Bars (max |gpu - oracle| / max |oracle - W| over the samples): FP64 1e-12,
    FP32 1e-4, FP16 1e-2 (binary16 rounding of every stored deviation, about
    5e-4 of its size, over up to 50 steps)."""
    ux, uy = field
    beta = beta_from_nu(NU)
    say("full-size steps 10 and 50", form)
    pts = sample_nodes()[:8] + sample_nodes()[-4:]
    xs = torch.as_tensor([q[0] for q in pts], device="cuda")
    ys = torch.as_tensor([q[1] for q in pts], device="cuda")
    s = Sim(N, N, beta, collision="kbc", variant="B", form=form).init(ux, uy)
    done = 0
    for nsteps in (10, 50):
        s.step(nsteps - done)
        done = nsteps
        torch.cuda.synchronize()
        f = s.get_populations()
        fg = f[:, ys, xs].cpu().numpy().T
        del f
        torch.cuda.empty_cache()
        fo = np.array([oracle_window(orc, ux, uy, beta, x, y, nsteps) for x, y in pts])
        err = np.abs(fg - fo).max() / np.abs(fo - W).max()
        say(f"  {form} after {nsteps} steps: samples {len(pts)}, err {err:.3e} (bar {MULTI_TOL[form]:.0e})")
        assert np.isfinite(fg).all()
        assert err < MULTI_TOL[form]


@pytest.mark.parametrize("form", ["f32", "f64", "f16"])
@pytest.mark.parametrize("coll,var", [("lbgk", "B"), ("kbc", "A"), ("kbc", "C"), ("kbc", "D")])
def test_fullsize_other_collisions_10_steps_sampled(orc, field, coll, var, form):
    """The other collisions at the full size, in every storage form, in the
    default launch configuration (two fused steps per launch): after 10
    steps, against the oracle on windows around 12 sampled nodes.

    Bar: max(MULTI_TOL, 5 s), s = how far the form's own rounding alone moves
    the oracle (FP32 / FP16: the oracle re-run with every stored state rounded
    to the form; FP64: 1e-15 relative perturbations of the start, the largest
    of three seeds), measured from the oracle alone, no GPU value.  Variants C and D
    leave only third- and fourth-order moments in dh, so <dh|dh> is tiny and
    gamma's ratio amplifies rounding: in FP32, s is about 6e-5 for them on
    this field against 5e-8 for B and LBGK and 4e-6 for A, and the GPU, which
    also computes in FP32, lands at about 2 s.  This is the self-sensitivity
    rule the ill-conditioned small-lattice cases use."""
    ux, uy = field
    beta = beta_from_nu(NU)
    say("full-size 10 steps", coll, var, form)
    pts = sample_nodes()[:8] + sample_nodes()[-4:]
    xs = torch.as_tensor([q[0] for q in pts], device="cuda")
    ys = torch.as_tensor([q[1] for q in pts], device="cuda")
    s = Sim(N, N, beta, collision=coll, variant=var, form=form).init(ux, uy)
    assert s.fusion == 2
    s.step(10)
    torch.cuda.synchronize()
    f = s.get_populations()
    fg = f[:, ys, xs].cpu().numpy().T
    del f, s
    torch.cuda.empty_cache()
    fo = np.array([oracle_window(orc, ux, uy, beta, x, y, 10, coll, var) for x, y in pts])
    scale = np.abs(fo - W).max()
    if form == "f64":
        sens = max(np.abs(np.array([oracle_window(orc, ux, uy, beta, x, y, 10, coll, var, perturb_seed=sd)
                                    for x, y in pts]) - fo).max() for sd in SEEDS) / scale
    else:
        fs = np.array([oracle_window(orc, ux, uy, beta, x, y, 10, coll, var, storage=form) for x, y in pts])
        sens = np.abs(fs - fo).max() / scale
    bar = max(MULTI_TOL[form], K_SENS * sens)
    err = np.abs(fg - fo).max() / scale
    say(f"  {coll} {var} {form} after 10 steps: samples {len(pts)}, err {err:.3e}, sensitivity {sens:.3e}, "
        f"bar {bar:.3e}, err/bar {err / bar:.3f}")
    assert np.isfinite(fg).all()
    assert err < bar


def test_fullsize_adjoint_step_sampled(orc, field):
    """The adjoint step at the full size in the configuration the benchmark
    times (FP32 KBC-B, gamma differentiated, state f^0 of the turbulence
    field, a seeded normal adjoint field lambda^(n+1)): lambda^n at 52 sampled
    nodes against the oracle's adjoint step on a 5 x 5 periodic window around
    each.  lambda^n(x) needs only f^n(x) and lambda^(n+1) at x + v_i, so the
    window's centre is exact; the oracle builds f^0 there itself from the
    velocity patch (central differences) and rounds it to binary32 as stored.
    Bar 1e-4 relative, as for the FP32 adjoint on small lattices (the
    derivative of gamma carries 1 / <dh|dh>)."""
    ux, uy = field
    beta = beta_from_nu(NU)
    say("full-size adjoint step")
    s = Sim(N, N, beta, collision="kbc", variant="B", form="f32").init(ux, uy)
    la, lb = s.new_adjoint(), s.new_adjoint()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    la.normal_(generator=gen)
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(s.state_buffer(), la, lb, acc)
    torch.cuda.synchronize()
    pin, pout = s.planes(la), s.planes(lb)
    p5 = orc.Params(5, 5, beta, collision=orc.KBC, variant=orc.VARIANTS["B"])
    d = np.arange(-2, 3)
    lg, lo = [], []
    for x, y in sample_nodes():
        iy = torch.as_tensor((y + d) % N, device="cuda")[:, None]
        ix = torch.as_tensor((x + d) % N, device="cuda")[None, :]
        lam_w = np.ascontiguousarray(pin[:, iy, ix].double().cpu().numpy())
        pu = np.ascontiguousarray(ux[iy, ix].cpu().numpy())
        pv = np.ascontiguousarray(uy[iy, ix].cpu().numpy())
        f_w = orc.round_storage(p5, orc.init(p5, pu, pv), "f32")
        lam_o, _ = orc.adjoint_step(p5, f_w, lam_w)
        lo.append(lam_o[:, 2, 2])
        lg.append(pout[:, y, x].double().cpu().numpy())
    lg, lo = np.array(lg), np.array(lo)
    err = np.abs(lg - lo).max() / np.abs(lo).max()
    say(f"  adjoint samples {len(lo)}, err {err:.3e}, dL/dbeta partial sum {acc.item():.6e}")
    del s, la, lb
    torch.cuda.empty_cache()
    assert np.isfinite(lg).all() and np.isfinite(acc.item())
    assert err < 1e-4
