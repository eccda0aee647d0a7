"""Parity on the paper-shaped turbulence workloads beyond the small lattices.

* The 1024^2 decaying-turbulence run (spectrum k^4 exp(-2 (k/8)^2), seed 2,
  u_rms = 0.05, nu = 1e-5, Grad initialisation; under-resolved for LBGK in
  the turbulence section): KBC-B in FP64 and FP32 for 200 steps against the
  FP64 oracle -- the velocity field pointwise after 200 steps and the energy
  and enstrophy every 50 steps.  Bars (max |diff| / max |field|): FP64
  1e-10 for the traces and, pointwise, 1e-10 or 5 times the oracle's own
  sensitivity (its run repeated from the initial state perturbed by 1e-15
  relative, largest of three seeds), whichever is larger: at this Reynolds number rounding-order
  differences grow to about 1e-7 in 200 steps on their own (measured 9.9e-8;
  the GPU's difference from the oracle, 2.7e-8, is below it).  FP32: 1e-4
  pointwise, |dE| / E(0) <= 1e-3 and |dZ| / Z(0) <= 1e-2 (the proposed trace
  bounds; measured values are printed).
* The 256-lattice uneven ensemble (master seed 4, N drawn from
  {128, 256, 512, 1024}, nu log-uniform in [1e-5, 1e-3]), all members stepped
  together for 50 steps in FP32: 16 members, four of each lattice size drawn
  with a fixed seed, against the oracle run of each member alone (FP32 bar
  1e-4 on the velocity field).  The members' initial fields come from the
  input module's torch transform on the GPU, the oracle's from its numpy
  transform of the same coefficients: they differ at rounding level only.

Both sides start from the same seeded velocity arrays (numpy transforms).
"""
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import inputs
from paper_1507_02509_amd.ensemble import Ensemble
from paper_1507_02509_amd.sim import Sim, beta_from_nu
from oracle_sensitivity import K_SENS, self_sensitivity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


N2, NU2, SEED2, STEPS2 = 1024, 1e-5, 2, 200


@pytest.fixture(scope="module")
def c2_oracle(orc):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ux, uy = inputs.spectral(N2, 8, 0.05, seed=SEED2)
    p = orc.Params(N2, N2, beta_from_nu(NU2), collision=orc.KBC, variant=orc.KBC_B, threads=16)
    f = orc.init(p, ux, uy)
    trace = [orc.diagnostics(p, f)]
    for _ in range(STEPS2 // 50):
        f = orc.run(p, f, 50)
        trace.append(orc.diagnostics(p, f))
    _, ox, oy = orc.moments(p, f)
    f0 = orc.init(p, ux, uy)
    sens = self_sensitivity(lambda f: orc.moments(p, orc.run(p, f, STEPS2))[1:], f0, (ox, oy),
                            lambda a, b: max(field_err(a[0], b[0]), field_err(a[1], b[1])))
    say("c2 oracle done: E", [round(d["E"], 9) for d in trace], "self-sensitivity", sens)
    return ux, uy, ox, oy, trace, sens


@pytest.mark.parametrize("form,bar_u,bar_e,bar_z", [("f64", 1e-10, 1e-10, 1e-10), ("f32", 1e-4, 1e-3, 1e-2)])
def test_c2_turbulence_1024(c2_oracle, form, bar_u, bar_e, bar_z):
    ux, uy, ox, oy, trace, sens = c2_oracle
    if form == "f64":
        bar_u = max(bar_u, K_SENS * sens)
    s = Sim(N2, N2, beta_from_nu(NU2), collision="kbc", variant="B", form=form).init(ux, uy)
    d0 = s.diagnostics()
    e_errs, z_errs = [], []
    for k in range(STEPS2 // 50 + 1):
        if k:
            s.step(50)
        d = s.diagnostics()
        e_errs.append(abs(d["E"] - trace[k]["E"]) / trace[0]["E"])
        z_errs.append(abs(d["Z"] - trace[k]["Z"]) / trace[0]["Z"])
        assert d["n_nonfinite"] == 0
    _, gx, gy = (t.cpu().numpy() for t in s.moments())
    eu = max(field_err(gx, ox), field_err(gy, oy))
    say(f"  c2 {form}: u err {eu:.3e} (bar {bar_u:.1e}), E errs {max(e_errs):.3e}, Z errs {max(z_errs):.3e}, "
        f"mass drift {(d['mass'] - d0['mass']) / d0['mass']:.2e}")
    assert eu < bar_u
    assert max(e_errs) < bar_e and max(z_errs) < bar_z


def test_c4_members_vs_oracle(orc):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1507_02509_amd.ensemble import make_members
    specs = inputs.ensemble_members(256, master_seed=4)
    rng = np.random.default_rng(44)
    pick = []
    for n in (128, 256, 512, 1024):
        idx = [i for i, m in enumerate(specs) if m[0] == n]
        pick += sorted(rng.choice(idx, size=min(4, len(idx)), replace=False).tolist())
    sims = make_members(specs, form="f32")
    Ensemble(sims).step(50)
    torch.cuda.synchronize()
    for i in pick:
        n, nu, seed = specs[i]
        ux, uy = inputs.spectral(n, 8, 0.05, seed=seed)
        p = orc.Params(n, n, beta_from_nu(nu), collision=orc.KBC, variant=orc.KBC_B, threads=16)
        _, ox, oy = orc.moments(p, orc.run(p, orc.init(p, ux, uy), 50))
        _, gx, gy = (t.cpu().numpy() for t in sims[i].moments())
        err = max(field_err(gx, ox), field_err(gy, oy))
        say(f"  c4 member {i}: n={n} nu={nu:.2e} seed={seed}: u err {err:.3e}")
        assert err < 1e-4


def test_c2_long_run_all_models():
    """The c2 workload over 10^4 steps (1024^2, nu = 1e-5, seed 2): every KBC
    model and LBGK in FP32 and KBC-B in FP64, with E and Z every 50 steps.
    Pointwise parity with the oracle is the 200-step test above; over 10^4
    steps the flow decorrelates, so the FP32 KBC-B traces are held to the
    proposed statistical bounds against the FP64 run: |dE| / E(0) <= 1e-3 and
    |dZ| / Z(0) <= 1e-2 at every sample.  Every KBC model stays finite (the
    paper reports no instability in any KBC run); the spatial mean of gamma of
    KBC-B stays within 10 % of 1 (its stabiliser sits near the regularised
    value, section on the entropic stabiliser); LBGK's first non-finite step,
    if any, is printed, not asserted."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    steps, every = 10000, 50
    ux, uy = inputs.spectral(N2, 8, 0.05, seed=SEED2)
    beta = beta_from_nu(NU2)

    def trace(coll, var, form):
        s = Sim(N2, N2, beta, collision=coll, variant=var, form=form).init(ux, uy)
        out, blown = [s.diagnostics()], None
        for k in range(steps // every):
            s.step(every)
            d = s.diagnostics()
            out.append(d)
            if d["n_nonfinite"] and blown is None:
                blown = (k + 1) * every
                break
        return out, blown

    ref, blown = trace("kbc", "B", "f64")
    assert blown is None
    e0, z0 = ref[0]["E"], ref[0]["Z"]
    for coll, var in [("kbc", "A"), ("kbc", "B"), ("kbc", "C"), ("kbc", "D"), ("lbgk", "A")]:
        tr, blown = trace(coll, var, "f32")
        if coll == "lbgk":
            say(f"  c2 long run LBGK f32: first non-finite sample at step {blown}" if blown
                else f"  c2 long run LBGK f32: finite to step {steps}, E {tr[-1]['E']:.5e}")
            continue
        assert blown is None, (var, blown)
        g = np.mean([d["gamma"] for d in tr[1:]])
        msg = f"  c2 long run KBC-{var} f32: E {tr[-1]['E']:.5e} Z {tr[-1]['Z']:.5e} mean gamma {g:.4f}"
        if var == "B":
            de = max(abs(a["E"] - b["E"]) for a, b in zip(tr, ref)) / e0
            dz = max(abs(a["Z"] - b["Z"]) for a, b in zip(tr, ref)) / z0
            msg += f"; vs FP64 max |dE|/E0 {de:.2e} |dZ|/Z0 {dz:.2e}"
            assert de <= 1e-3 and dz <= 1e-2
            assert abs(g - 1.0) < 0.1
        say(msg)


def test_c4_2000_steps_one_persistent_launch(orc):
    """The ensemble workload as stated: 256 members (N in {128, 256, 512,
    1024}, nu log-uniform in [1e-5, 1e-3], per-member seeds), KBC-B FP32,
    2000 steps in ONE persistent launch (pairs of fused steps, grid barrier
    between pairs).  (a) No barrier gave up, and four members, one of each
    size, equal the same members stepped alone, bit for bit.  (b) The most
    viscous 128^2 member (nu = 9.7e-4) against the oracle run with the same
    binary32 storage rounding after every step: velocity field within
    max(1e-4, 5 s), s being how far that rounding alone moves the FP64
    oracle after 2000 steps (measured from the oracle)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1507_02509_amd.ensemble import make_members
    specs = inputs.ensemble_members(256, master_seed=4)
    pick = [next(i for i, m in enumerate(specs) if m[0] == n) for n in (128, 256, 512, 1024)]
    visc = max((m[1], i) for i, m in enumerate(specs) if m[0] == 128)[1]
    sims = make_members(specs, form="f32")
    snaps = {i: sims[i].state_buffer().clone() for i in pick + [visc]}
    ens = Ensemble(sims)
    ens.step(2000, persistent=True)
    ens.check()
    for i in pick:
        s = sims[i]
        ref = Sim(s.nx, s.ny, s.params.beta, variant="B", form="f32")
        ref.init(np.zeros((s.ny, s.nx)), np.zeros((s.ny, s.nx)), mode="eq")
        ref.state_buffer().copy_(snaps[i])
        ref.step(2000)
        assert torch.equal(ref.planes(ref.state_buffer()), s.planes(s.state_buffer())), i
    n, nu, seed = specs[visc]
    ux, uy = inputs.spectral(n, 8, 0.05, seed=seed)
    p = orc.Params(n, n, beta_from_nu(nu), collision=orc.KBC, variant=orc.KBC_B, threads=16)
    f0 = orc.init(p, ux, uy)
    _, ox, oy = orc.moments(p, orc.run(p, f0, 2000))
    _, sx, sy = orc.moments(p, orc.run(p, orc.round_storage(p, f0, "f32"), 2000, storage="f32"))
    _, gx, gy = (t.cpu().numpy() for t in sims[visc].moments())
    sens = max(field_err(sx, ox), field_err(sy, oy))
    err = max(field_err(gx, sx), field_err(gy, sy))
    bar = max(1e-4, K_SENS * sens)
    say(f"  c4 2000 steps, member {visc} (n={n}, nu={nu:.2e}): u err vs storage-rounded oracle {err:.3e}, "
        f"storage sensitivity {sens:.3e}, bar {bar:.3e}")
    assert err < bar
    ens.free()
