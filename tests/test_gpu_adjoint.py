"""GPU parity of the discrete adjoint (hand-written reverse mode of the
collision, gamma(f) differentiated) against the FP64 oracle's adjoint, whose
per-node Jacobians come from complex-step differentiation of the oracle's own
collision; plus finite differences of the GPU forward and checkpoint
invariance of the autograd rollout."""
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import inputs
from paper_1507_02509_amd.autograd import rollout
from paper_1507_02509_amd.sim import Sim, beta_from_nu
from oracle_sensitivity import K_SENS, SEEDS, perturbed

pytestmark = pytest.mark.gpu

VEL = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], float)
CASES = [("lbgk", "A"), ("kbc", "A"), ("kbc", "B"), ("kbc", "C"), ("kbc", "D")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oparams(orc, nx, ny, beta, coll, var):
    return orc.Params(nx, ny, beta, collision=orc.LBGK if coll == "lbgk" else orc.KBC,
                      variant=orc.VARIANTS[var])


def random_state(orc, nx, ny, beta, seed, eps=2e-3):
    ux, uy = inputs.spectral(nx, 3, 0.05, seed=seed, ny=ny)
    f = orc.init(oparams(orc, nx, ny, beta, "kbc", "B"), ux, uy)
    rng = np.random.default_rng(seed)
    return f * (1 + eps * rng.standard_normal(f.shape))


def field_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


EPS32 = 2.0 ** -24


def f32_adjoint_bars(orc, p, f, lam_next):
    """Bars of an FP32 adjoint step against the FP64 oracle's at the stored
    state f (max |diff| / max |oracle| for lambda, relative for the summed
    dL/dbeta), from the oracle alone: the kernel computes in binary32, so
    its lambda moves at least as much as the oracle's does when the stored
    deviations g = f - W are perturbed by one binary32 rounding,
    g (1 + 2^-24 xi) (largest of three seeds, s_lam and s_beta); the bar is
    K_SENS times that, but not below 16 binary32 units for lambda (the
    arithmetic of an O(1) adjoint field) and 4 kappa binary32 units for
    dL/dbeta, kappa = sum |dbeta_x| / |sum dbeta_x| being the condition number
    of the sum of per-node terms each formed in binary32.  Model C's
    <dh|dh> holds only third- and fourth-order moments, so the 1/<dh|dh> in
    the derivative of gamma* makes its s_lam about 20 times B's."""
    lo, db = orc.adjoint_step(p, f, lam_next)
    W = orc.weights()[:, None, None]
    s_lam = s_beta = 0.0
    for seed in SEEDS:
        xi = np.random.default_rng(seed).standard_normal(f.shape)
        lp, dbp = orc.adjoint_step(p, W + (f - W) * (1.0 + EPS32 * xi), lam_next)
        s_lam = max(s_lam, field_err(lp, lo))
        s_beta = max(s_beta, abs(dbp.sum() - db.sum()) / abs(db.sum()))
    kappa = np.abs(db).sum() / abs(db.sum())
    return lo, db, max(16 * EPS32, K_SENS * s_lam), max(4 * kappa * EPS32, K_SENS * s_beta)


def to_lam(sim, lam_np):
    lam = sim.new_adjoint().zero_()
    sim.planes(lam)[...] = torch.from_numpy(lam_np).to(device="cuda", dtype=sim.adjoint_dtype)
    return lam


@pytest.mark.parametrize("coll,var", CASES)
def test_adjoint_step_parity_f64(orc, coll, var):
    nx, ny = 67, 45
    say("adjoint step f64", coll, var)
    beta = beta_from_nu(1e-3)
    f0 = random_state(orc, nx, ny, beta, seed=40)
    lam_next = np.random.default_rng(41).standard_normal((9, ny, nx))
    s = Sim(nx, ny, beta, collision=coll, variant=var, form="f64")
    s.init(np.zeros((ny, nx)), np.zeros((ny, nx)), mode="eq")
    s.set_populations(f0)
    lin = to_lam(s, lam_next)
    lout = s.new_adjoint()
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(s.state_buffer(), lin, lout, acc)
    lg = s.planes(lout).cpu().numpy()
    lo, dbo = orc.adjoint_step(oparams(orc, nx, ny, beta, coll, var), f0, lam_next)
    err = field_err(lg, lo)
    say("  lam err", err, "dbeta", acc.item(), dbo.sum())
    assert err < 1e-11
    assert acc.item() == pytest.approx(dbo.sum(), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("coll,var", [("lbgk", "A"), ("kbc", "B"), ("kbc", "C")])
def test_adjoint_step_parity_f32(orc, coll, var):
    nx, ny = 67, 45
    say("adjoint step f32", coll, var)
    beta = beta_from_nu(1e-3)
    f0 = random_state(orc, nx, ny, beta, seed=42, eps=1e-3)
    lam_next = np.random.default_rng(43).standard_normal((9, ny, nx))
    s = Sim(nx, ny, beta, collision=coll, variant=var, form="f32")
    s.init(np.zeros((ny, nx)), np.zeros((ny, nx)), mode="eq")
    f0r = orc.round_storage(orc.Params(nx, ny, beta), f0, "f32")
    s.set_populations(f0)
    assert np.abs(s.get_populations().cpu().numpy() - f0r).max() < 1e-15
    lam_next = lam_next.astype(np.float32).astype(np.float64)
    lout = s.new_adjoint()
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(s.state_buffer(), to_lam(s, lam_next), lout, acc)
    lo, dbo, bar, bar_b = f32_adjoint_bars(orc, oparams(orc, nx, ny, beta, coll, var), f0r, lam_next)
    err = field_err(s.planes(lout).cpu().numpy(), lo)
    eb = abs(acc.item() - dbo.sum()) / abs(dbo.sum())
    say(f"  f32 lam err {err:.3e} (bar {bar:.3e}), dbeta err {eb:.3e} (bar {bar_b:.3e})")
    assert err < bar and bar <= 2e-3
    assert eb < bar_b


@pytest.mark.parametrize("coll,var", [("lbgk", "A"), ("kbc", "B")])
def test_adjoint_step_parity_f16(orc, coll, var):
    """The adjoint step of the FP16 storage form (FP32 arithmetic) from the
    oracle's binary16 rounding of the state, which the form decodes exactly:
    what separates it from the FP64 oracle adjoint at that state is FP32
    arithmetic alone, so the FP32 bars (f32_adjoint_bars) apply."""
    nx, ny = 67, 45
    say("adjoint step f16", coll, var)
    beta = beta_from_nu(1e-3)
    f0 = random_state(orc, nx, ny, beta, seed=46, eps=1e-3)
    lam_next = np.random.default_rng(47).standard_normal((9, ny, nx)).astype(np.float32).astype(np.float64)
    s = Sim(nx, ny, beta, collision=coll, variant=var, form="f16")
    s.init(np.zeros((ny, nx)), np.zeros((ny, nx)), mode="eq")
    f0r = orc.round_storage(orc.Params(nx, ny, beta), f0, "f16")
    s.set_populations(f0)
    assert np.abs(s.get_populations().cpu().numpy() - f0r).max() < 1e-15
    lout = s.new_adjoint()
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(s.state_buffer(), to_lam(s, lam_next), lout, acc)
    lo, dbo, bar, bar_b = f32_adjoint_bars(orc, oparams(orc, nx, ny, beta, coll, var), f0r, lam_next)
    err = field_err(s.planes(lout).cpu().numpy(), lo)
    eb = abs(acc.item() - dbo.sum()) / abs(dbo.sum())
    say(f"  f16 lam err {err:.3e} (bar {bar:.3e}), dbeta err {eb:.3e} (bar {bar_b:.3e})")
    assert err < bar and bar <= 2e-3
    assert eb < bar_b


@pytest.mark.parametrize("mode", ["eq", "grad_cd"])
def test_adjoint_init_parity(orc, mode):
    nx, ny = 67, 45
    say("adjoint init", mode)
    beta = beta_from_nu(1e-3)
    ux, uy = inputs.spectral(nx, 3, 0.05, seed=44, ny=ny)
    lam0 = np.random.default_rng(45).standard_normal((9, ny, nx))
    s = Sim(nx, ny, beta, form="f64").init(ux, uy, mode=mode)
    gx = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
    gy = torch.empty_like(gx)
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    ux_t = torch.from_numpy(ux).cuda()
    uy_t = torch.from_numpy(uy).cuda()
    s.adjoint_init(ux_t, uy_t, to_lam(s, lam0), gx, gy, acc, mode=mode)
    omode = orc.INIT_EQ if mode == "eq" else orc.INIT_GRAD_CD
    ogx, ogy, odb = orc.init_adjoint(oparams(orc, nx, ny, beta, "kbc", "B"), ux, uy, lam0, mode=omode)
    assert field_err(gx.cpu().numpy(), ogx) < 1e-12
    assert field_err(gy.cpu().numpy(), ogy) < 1e-12
    assert acc.item() == pytest.approx(odb.sum(), rel=1e-10, abs=1e-14)


def velocity_loss(ux, uy, tx, ty):
    return 0.5 * (((ux - tx) ** 2).sum() + ((uy - ty) ** 2).sum())


def oracle_gradient(orc, p, ux0, uy0, tx, ty, nsteps):
    states = [orc.init(p, ux0, uy0)]
    for _ in range(nsteps):
        states.append(orc.step(p, states[-1]))
    rho, ux, uy = orc.moments(p, states[-1])
    dx, dy = ux - tx, uy - ty
    lam = (dx[None] * (VEL[:, 0, None, None] - ux[None]) + dy[None] * (VEL[:, 1, None, None] - uy[None])) / rho[None]
    db = 0.0
    for k in range(nsteps - 1, -1, -1):
        lam, d = orc.adjoint_step(p, states[k], lam)
        db += d.sum()
    gx, gy, d0 = orc.init_adjoint(p, ux0, uy0, lam)
    return gx, gy, db + d0.sum()


@pytest.mark.parametrize("coll,var", [("kbc", "B"), ("kbc", "A"), ("kbc", "D"), ("lbgk", "A")])
def test_rollout_gradient_matches_oracle_f64(orc, coll, var):
    nx, ny, nsteps = 21, 18, 12
    say("rollout grad vs oracle", coll, var)
    beta = beta_from_nu(1e-3)
    ux0, uy0 = inputs.spectral(nx, 2, 0.05, seed=46, ny=ny)
    tx, ty = inputs.spectral(nx, 2, 0.03, seed=47, ny=ny)
    u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
    u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    rho, ux, uy = rollout(u0x, u0y, b, nsteps, collision=coll, variant=var, form="f64", checkpoint_every=5)
    loss = velocity_loss(ux, uy, torch.from_numpy(tx).cuda(), torch.from_numpy(ty).cuda())
    loss.backward()
    ogx, ogy, odb = oracle_gradient(orc, oparams(orc, nx, ny, beta, coll, var), ux0, uy0, tx, ty, nsteps)
    errs = (field_err(u0x.grad.cpu().numpy(), ogx), field_err(u0y.grad.cpu().numpy(), ogy),
            abs(b.grad.item() - odb) / abs(odb))
    say("  grad errors", errs)
    assert max(errs) < 1e-9


def test_rollout_gradient_matches_finite_differences_f64():
    nx, ny, nsteps = 24, 20, 40
    say("rollout grad vs FD")
    beta = beta_from_nu(1e-3)
    ux0, uy0 = inputs.spectral(nx, 2, 0.05, seed=48, ny=ny)
    tx, ty = (torch.from_numpy(a).cuda() for a in inputs.spectral(nx, 2, 0.03, seed=49, ny=ny))
    u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
    u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    _, ux, uy = rollout(u0x, u0y, b, nsteps, form="f64")
    velocity_loss(ux, uy, tx, ty).backward()
    rng = np.random.default_rng(50)
    vx = torch.from_numpy(rng.standard_normal((ny, nx))).cuda()
    vy = torch.from_numpy(rng.standard_normal((ny, nx))).cuda()

    def L(ex, ey, bb):
        with torch.no_grad():
            _, a, c = rollout(u0x.detach() + ex, u0y.detach() + ey, bb, nsteps, form="f64")
            return velocity_loss(a, c, tx, ty).item()
    h = 1e-6
    fd = (L(h * vx, h * vy, beta) - L(-h * vx, -h * vy, beta)) / (2 * h)
    ad = float((u0x.grad * vx).sum() + (u0y.grad * vy).sum())
    assert ad == pytest.approx(fd, rel=1e-6)
    hb = 1e-7
    fdb = (L(0, 0, beta + hb) - L(0, 0, beta - hb)) / (2 * hb)
    assert b.grad.item() == pytest.approx(fdb, rel=1e-5)


# FP32 bars: the measured FP32 vs FP64 gradient differences are 7.0e-7 (B,
# 300 steps) and 1.75e-3 (D, 2000 steps)
@pytest.mark.parametrize("variant,guard,nsteps,f32_tol", [("B", 1e-12, 300, 5e-6), ("D", 1e-4, 2000, 1e-2)])
def test_rollout_gradient_16x16_finite_differences(variant, guard, nsteps, f32_tol):
    """The adjoint workload's loss and gradient on a 16 x 16 lattice (KBC,
    seeded turbulence-like start, nu = 1e-3, loss 1/2 |u(T) - u_t|^2): the
    FP64 rollout gradient against central finite differences of the FP64
    forward along a seeded direction (and in beta), and the FP32 rollout
    gradient against the FP64 one.  Variant D with guard 1e-4 is the KBC
    configuration the 2000-step benchmark rollout uses; model B with the
    default guard is checked over 300 steps, where its gradient still means
    something."""
    n = 16
    say("16x16 rollout grad vs FD", variant, guard, nsteps)
    beta = beta_from_nu(1e-3)
    ux0, uy0 = inputs.spectral(n, 2, 0.05, seed=61)
    tx, ty = (torch.from_numpy(a).cuda() for a in inputs.spectral(n, 2, 0.03, seed=62))
    kw = dict(variant=variant, gamma_guard=guard)
    grads = {}
    for form in ("f64", "f32"):
        u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
        u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
        b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
        _, ux, uy = rollout(u0x, u0y, b, nsteps, form=form, **kw)
        velocity_loss(ux, uy, tx, ty).backward()
        grads[form] = (torch.cat([u0x.grad.flatten(), u0y.grad.flatten()]), b.grad.item())
    rng = np.random.default_rng(63)
    vx = torch.from_numpy(rng.standard_normal((n, n))).cuda()
    vy = torch.from_numpy(rng.standard_normal((n, n))).cuda()

    def L(ex, ey, bb):
        with torch.no_grad():
            _, a, c = rollout(torch.from_numpy(ux0).cuda() + ex, torch.from_numpy(uy0).cuda() + ey, bb, nsteps,
                              form="f64", **kw)
            return velocity_loss(a, c, tx, ty).item()
    # steps small enough that no node's guard decision changes between the
    # two evaluations (as in the 512^2 test)
    h = 1e-9
    fd = (L(h * vx, h * vy, beta) - L(-h * vx, -h * vy, beta)) / (2 * h)
    g64, b64 = grads["f64"]
    ad = float((g64 * torch.cat([vx.flatten(), vy.flatten()])).sum())
    hb = 1e-9
    fdb = (L(0, 0, beta + hb) - L(0, 0, beta - hb)) / (2 * hb)
    g32, b32 = grads["f32"]
    rel32 = float(torch.linalg.norm(g32 - g64) / torch.linalg.norm(g64))
    say(f"  directional {ad:.6e} FD {fd:.6e}; dL/dbeta {b64:.6e} FD {fdb:.6e}; FP32 vs FP64 {rel32:.2e}")
    assert ad == pytest.approx(fd, rel=1e-5)
    assert b64 == pytest.approx(fdb, rel=1e-4)
    assert rel32 < f32_tol
    assert b32 == pytest.approx(b64, rel=f32_tol)


def test_checkpoint_interval_does_not_change_the_gradient():
    nx, ny, nsteps = 70, 33, 23
    say("checkpoint invariance")
    ux0, uy0 = inputs.spectral(nx, 3, 0.05, seed=51, ny=ny)
    grads = []
    for K in (1, 4, 23, None):
        u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
        u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
        b = torch.tensor(beta_from_nu(1e-4), dtype=torch.float64, device="cuda", requires_grad=True)
        _, ux, uy = rollout(u0x, u0y, b, nsteps, form="f32", checkpoint_every=K)
        (0.5 * (ux ** 2 + uy ** 2).sum()).backward()
        grads.append((u0x.grad.clone(), u0y.grad.clone(), b.grad.clone()))
    for g in grads[1:]:
        for a, c in zip(g, grads[0]):
            assert torch.equal(a, c)


@pytest.mark.parametrize("form,nsteps,K,kw", [("f32", 23, 4, {}), ("f32", 40, 5, {}), ("f64", 17, 3, {}),
                                             ("f32", 9, 2, {}), ("f32", 21, 5, {}),
                                             ("f32", 23, 4, {"gamma_grad": "frozen"}),
                                             ("f64", 19, 4, {"collision": "lbgk"}),
                                             ("f32", 19, 4, {"variant": "D", "gamma_guard": 1e-4}),
                                             ("f32", 19, 4, {"gamma_mode": "exact"}),
                                             ("f64", 17, 3, {"gamma_mode": "exact", "variant": "A"})])
def test_overlapped_backward_is_bitwise_identical(form, nsteps, K, kw):
    """The backward pass whose launches each run one adjoint step and one
    recomputation step of the next segment (two slot sets) returns the
    gradients of the one that recomputes and runs back each segment in turn,
    bit for bit (ragged last segments included, shorter and longer than the
    recomputation they share launches with)."""
    nx, ny = 70, 33
    say("overlapped backward", form, nsteps, K, kw)
    ux0, uy0 = inputs.spectral(nx, 3, 0.05, seed=52, ny=ny)
    grads = []
    for overlap in (False, True):
        u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
        u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
        b = torch.tensor(beta_from_nu(1e-4), dtype=torch.float64, device="cuda", requires_grad=True)
        _, ux, uy = rollout(u0x, u0y, b, nsteps, form=form, checkpoint_every=K, overlap=overlap, **kw)
        (0.5 * (ux ** 2 + uy ** 2).sum()).backward()
        torch.cuda.synchronize()
        grads.append((u0x.grad.clone(), u0y.grad.clone(), b.grad.clone()))
    for a, c in zip(grads[1], grads[0]):
        assert torch.equal(a, c)


def c5_setup():
    n = 512
    ux0, uy0 = inputs.spectral(n, 8, 0.05, seed=5)
    tx, ty = (torch.from_numpy(a).cuda() for a in inputs.spectral(n, 8, 0.03, seed=55))
    rng = np.random.default_rng(56)
    vx = torch.from_numpy(rng.standard_normal((n, n))).cuda()
    vy = torch.from_numpy(rng.standard_normal((n, n))).cuda()
    return n, ux0, uy0, tx, ty, vx, vy


def c5_grad(form, nsteps, ux0, uy0, tx, ty, **kw):
    u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
    u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
    b = torch.tensor(beta_from_nu(1e-3), dtype=torch.float64, device="cuda", requires_grad=True)
    _, ux, uy = rollout(u0x, u0y, b, nsteps, form=form, **kw)
    velocity_loss(ux, uy, tx, ty).backward()
    return torch.cat([u0x.grad.flatten(), u0y.grad.flatten()]), b.grad.item()


def c5_fd(h, nsteps, ux0, uy0, tx, ty, vx, vy, **kw):
    def L(e):
        with torch.no_grad():
            _, a, c = rollout(torch.from_numpy(ux0).cuda() + e * vx, torch.from_numpy(uy0).cuda() + e * vy,
                              beta_from_nu(1e-3), nsteps, form="f64", **kw)
            return velocity_loss(a, c, tx, ty).item()
    return (L(h) - L(-h)) / (2 * h)


@pytest.mark.parametrize("coll,var,nsteps,guard,h,fd_tol,f32_tol", [
    ("lbgk", "A", 2000, 1e-12, 1e-6, 1e-6, 2e-3),
    ("kbc", "B", 300, 1e-12, 1e-9, 1e-5, 2e-2),
    ("kbc", "D", 2000, 1e-4, 1e-9, 1e-5, 5e-2),
])
def test_turbulence_512_gradient(coll, var, nsteps, guard, h, fd_tol, f32_tol):
    """The adjoint workload: 512^2 decaying turbulence (k0 = 8, u_rms = 0.05,
    nu = 1e-3), loss 1/2 |u(T) - u_t|^2 with a seeded target (u_rms = 0.03),
    sqrt(N) checkpoints.  The FP64 gradient along a random direction agrees
    with central finite differences of the FP64 forward, and the FP32
    gradient with the FP64 one.  Horizons and guards are those where the loss
    is differentiable at the finite-difference scale: the exact derivative of
    gamma* grows without bound over long KBC-A/B rollouts (|grad| ~ 1e30 after
    2000 steps with the default guard) and a large guard makes the loss jump
    where nodes switch branch."""
    n, ux0, uy0, tx, ty, vx, vy = c5_setup()
    say("512 gradient", coll, var, nsteps, guard)
    kw = dict(collision=coll, variant=var, gamma_guard=guard)
    g64, b64 = c5_grad("f64", nsteps, ux0, uy0, tx, ty, **kw)
    g32, b32 = c5_grad("f32", nsteps, ux0, uy0, tx, ty, **kw)
    rel = float(torch.linalg.norm(g32 - g64) / torch.linalg.norm(g64))
    ad = float((g64[:n * n].reshape(n, n) * vx).sum() + (g64[n * n:].reshape(n, n) * vy).sum())
    fd = c5_fd(h, nsteps, ux0, uy0, tx, ty, vx, vy, **kw)
    say("  |g64|", float(torch.linalg.norm(g64)), "fp32 vs fp64", rel, "beta", b32, b64, "FD", fd, "adj", ad)
    assert ad == pytest.approx(fd, rel=fd_tol)
    assert rel < f32_tol
    assert b32 == pytest.approx(b64, rel=f32_tol)


@pytest.mark.parametrize("var,guard", [("B", 1e-12), ("D", 1e-4)])
def test_turbulence_512_adjoint_matches_oracle(orc, var, guard):
    """Full 512^2 lattice against the FP64 CPU discrete adjoint (complex-step
    Jacobians of the oracle's collision) over 50 steps in FP64: KBC-B with the
    default guard, and KBC-D with guard 1e-4, the configuration whose
    2000-step gradient the benchmark times.  dL/dbeta to 1e-10 relative; the
    gradient w.r.t. the initial velocity (max |diff| / max |oracle|) to
    max(1e-10, 5 s), s being how far the oracle's own gradient moves when
    its initial velocity is perturbed by 1e-15 relative (one seed: each
    oracle gradient takes tens of seconds): over 50 steps the derivative of
    gamma* carries rounding differences of the trajectory to about 1e-9."""
    n, ux0, uy0, tx, ty, _, _ = c5_setup()
    say("512 adjoint vs oracle", var, guard)
    beta, nsteps = beta_from_nu(1e-3), 50
    g64, b64 = c5_grad("f64", nsteps, ux0, uy0, tx, ty, variant=var, gamma_guard=guard)
    p = oparams(orc, n, n, beta, "kbc", var)
    p.gamma_guard = guard
    p.threads = 16
    txn, tyn = tx.cpu().numpy(), ty.cpu().numpy()
    ogx, ogy, odb = oracle_gradient(orc, p, ux0, uy0, txn, tyn, nsteps)
    og = np.concatenate([ogx.ravel(), ogy.ravel()])
    err = float(np.abs(g64.cpu().numpy() - og).max() / np.abs(og).max())
    px, py, _ = oracle_gradient(orc, p, perturbed(ux0, 0), perturbed(uy0, 0), txn, tyn, nsteps)
    sens = float(np.abs(np.concatenate([px.ravel(), py.ravel()]) - og).max() / np.abs(og).max())
    bar = max(1e-10, K_SENS * sens)
    say(f"  grad err {err:.3e}, oracle self-sensitivity {sens:.3e}, bar {bar:.3e}; dL/dbeta {b64!r} vs {odb!r}")
    assert err < bar
    assert b64 == pytest.approx(odb, rel=1e-10)


def test_seed_matches_loss_derivative(orc):
    nx, ny = 33, 20
    say("seed")
    beta = beta_from_nu(1e-3)
    f0 = random_state(orc, nx, ny, beta, seed=52)
    s = Sim(nx, ny, beta, form="f64")
    s.init(np.zeros((ny, nx)), np.zeros((ny, nx)), mode="eq")
    s.set_populations(f0)
    rng = np.random.default_rng(53)
    a, bx, by = (rng.standard_normal((ny, nx)) for _ in range(3))
    lam = s.new_adjoint()
    s.adjoint_seed(s.state_buffer(), lam, a, bx, by)
    rho, ux, uy = orc.moments(oparams(orc, nx, ny, beta, "kbc", "B"), f0)
    want = a[None] + (bx[None] * (VEL[:, 0, None, None] - ux[None]) + by[None] * (VEL[:, 1, None, None] - uy[None])) / rho[None]
    assert field_err(s.planes(lam).cpu().numpy(), want) < 1e-13


def oparams_exact(orc, nx, ny, beta, var):
    return orc.Params(nx, ny, beta, collision=orc.KBC, variant=orc.VARIANTS[var], gamma_mode=orc.GAMMA_EXACT)


@pytest.mark.parametrize("form,var", [("f64", "A"), ("f64", "B"), ("f64", "C"), ("f64", "D"), ("f32", "B")])
def test_adjoint_step_parity_exact_stabilizer(orc, form, var):
    """The adjoint of a step with the exact stabiliser (the root of eq.
    (result1), differentiated by the implicit function theorem on the GPU)
    against the oracle's complex-step adjoint through its own Newton
    iteration.  FP64 bar 1e-10 (both roots are solved to 1e-15 relative; the
    derivative carries 1 / F'(gamma)); FP32 bars as for the estimate
    (f32_adjoint_bars)."""
    nx, ny = 67, 45
    say("adjoint step exact", form, var)
    beta = beta_from_nu(1e-3)
    f0 = random_state(orc, nx, ny, beta, seed=60, eps=2e-3)
    lam_next = np.random.default_rng(61).standard_normal((9, ny, nx))
    s = Sim(nx, ny, beta, variant=var, form=form, gamma_mode="exact")
    s.init(np.zeros((ny, nx)), np.zeros((ny, nx)), mode="eq")
    s.set_populations(f0)
    if form == "f32":
        f0 = orc.round_storage(orc.Params(nx, ny, beta), f0, "f32")
        lam_next = lam_next.astype(np.float32).astype(np.float64)
    lout = s.new_adjoint()
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(s.state_buffer(), to_lam(s, lam_next), lout, acc)
    lo, dbo = orc.adjoint_step(oparams_exact(orc, nx, ny, beta, var), f0, lam_next)
    lg = s.planes(lout).cpu().numpy()
    err = field_err(lg, lo)
    # the exact root's adjoint differs from the estimate's: the test can tell them apart
    le, _ = orc.adjoint_step(oparams(orc, nx, ny, beta, "kbc", var), f0, lam_next)
    gap = field_err(le, lo)
    say(f"  lam err {err:.3e} (estimate's adjoint is {gap:.3e} away), dbeta {acc.item():.9e} {dbo.sum():.9e}")
    assert gap > 1e-6
    if form == "f64":
        assert err < 1e-10
        assert acc.item() == pytest.approx(dbo.sum(), rel=1e-8, abs=1e-12)
    else:
        _, _, bar, bar_b = f32_adjoint_bars(orc, oparams_exact(orc, nx, ny, beta, var), f0, lam_next)
        eb = abs(acc.item() - dbo.sum()) / abs(dbo.sum())
        say(f"  bars: lam {bar:.3e}, dbeta {bar_b:.3e} (dbeta err {eb:.3e})")
        assert err < bar and bar <= 2e-3
        assert eb < bar_b


def test_rollout_gradient_exact_stabilizer_matches_oracle_f64(orc):
    """Gradient of a final-time velocity loss through 12 steps with the exact
    stabiliser (checkpointed rollout, initial state included) against the
    oracle's discrete adjoint with its complex-step Jacobians."""
    nx, ny, nsteps = 21, 18, 12
    say("rollout grad exact vs oracle")
    beta = beta_from_nu(1e-3)
    ux0, uy0 = inputs.spectral(nx, 2, 0.05, seed=62, ny=ny)
    tx, ty = inputs.spectral(nx, 2, 0.03, seed=63, ny=ny)
    u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
    u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    rho, ux, uy = rollout(u0x, u0y, b, nsteps, variant="B", form="f64", gamma_mode="exact", checkpoint_every=5)
    loss = velocity_loss(ux, uy, torch.from_numpy(tx).cuda(), torch.from_numpy(ty).cuda())
    loss.backward()
    ogx, ogy, odb = oracle_gradient(orc, oparams_exact(orc, nx, ny, beta, "B"), ux0, uy0, tx, ty, nsteps)
    errs = (field_err(u0x.grad.cpu().numpy(), ogx), field_err(u0y.grad.cpu().numpy(), ogy),
            abs(b.grad.item() - odb) / abs(odb))
    say("  grad errors", errs)
    assert max(errs) < 1e-9


def test_adjoint_two_rows_per_thread_f32(orc):
    """FP32 lattices with at least 8192 tiles of 128 x 4 run the adjoint with
    two nodes per thread (rows r and r + 2).  On a ragged 1030 x 3650 lattice
    (the last tile column 6 nodes wide, the last tile row 2 rows high) the
    adjoint step matches the oracle's to the FP32 bar of the small lattices,
    and the overlapped backward pass equals the plain one bit for bit."""
    nx, ny = 1030, 3650
    say("adjoint two rows per thread", nx, ny)
    beta = beta_from_nu(1e-3)
    f0 = random_state(orc, nx, ny, beta, seed=64, eps=1e-3)
    lam_next = np.random.default_rng(65).standard_normal((9, ny, nx)).astype(np.float32).astype(np.float64)
    s = Sim(nx, ny, beta, variant="B", form="f32")
    s.init(np.zeros((ny, nx)), np.zeros((ny, nx)), mode="eq")
    s.set_populations(f0)
    f0r = orc.round_storage(orc.Params(nx, ny, beta), f0, "f32")
    lout = s.new_adjoint()
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(s.state_buffer(), to_lam(s, lam_next), lout, acc)
    lg = s.planes(lout).cpu().numpy()
    del s, lout
    torch.cuda.empty_cache()
    p = oparams(orc, nx, ny, beta, "kbc", "B")
    p.threads = 16
    lo, dbo = orc.adjoint_step(p, f0r, lam_next)
    err = field_err(lg, lo)
    say(f"  lam err {err:.3e}, dbeta {acc.item():.9e} {dbo.sum():.9e}")
    assert err < 1e-4
    assert acc.item() == pytest.approx(dbo.sum(), rel=1e-4)
    ux0, uy0 = inputs.spectral(nx, 3, 0.05, seed=66, ny=ny)
    grads = []
    for overlap in (False, True):
        u0x = torch.from_numpy(ux0).cuda().requires_grad_(True)
        u0y = torch.from_numpy(uy0).cuda().requires_grad_(True)
        b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
        _, ux, uy = rollout(u0x, u0y, b, 9, form="f32", checkpoint_every=3, overlap=overlap)
        (0.5 * (ux ** 2 + uy ** 2).sum()).backward()
        torch.cuda.synchronize()
        grads.append((u0x.grad.clone(), u0y.grad.clone(), b.grad.clone()))
    for a, c in zip(grads[1], grads[0]):
        assert torch.equal(a, c)
