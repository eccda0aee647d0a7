"""GPU tests of the ensemble kernels (uneven lattices in one launch, single
or two fused steps per launch, or one persistent launch for many steps with a
bounded grid barrier) and of the tile autotuner.
The per-node code is shared with the single-lattice step, so an ensemble step
must equal stepping every member alone, bit for bit."""
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import autotune, inputs
from paper_1507_02509_amd.ensemble import Ensemble, make_members
from paper_1507_02509_amd.sim import Sim, beta_from_nu

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_specs():
    # ragged sizes: tails in x and y for every tile shape
    return [(67, 45, 1e-3, 1), (128, 128, 1e-4, 2), (131, 37, 3e-5, 3), (64, 200, 1e-3, 4), (3, 3, 1e-3, 5)]


def build(specs, form, coll="kbc", var="B"):
    sims = []
    for nx, ny, nu, seed in specs:
        if nx >= 8 and ny >= 8:
            ux, uy = inputs.spectral(nx, 3, 0.05, seed=seed, ny=ny)
        else:
            ux, uy = np.full((ny, nx), 0.01), np.full((ny, nx), -0.02)
        s = Sim(nx, ny, beta_from_nu(nu), collision=coll, variant=var, form=form)
        sims.append(s.init(ux, uy))
    return sims


def states(sims):
    return [s.planes(s.state_buffer()).clone() for s in sims]


@pytest.mark.parametrize("form", ["f32", "f64", "f16"])
@pytest.mark.parametrize("coll,var", [("kbc", "B"), ("lbgk", "A"), ("kbc", "A")])
def test_ensemble_equals_individual_steps(form, coll, var):
    say("ensemble vs individual", form, coll, var)
    ref = build(small_specs(), form, coll, var)
    for s in ref:
        s.step(9)
    want = states(ref)
    persistent = False
    configs = [(tile, (1, 0)) for tile in ((128, 2, False), (256, 1, True), (256, 2, False))]
    configs += [((256, 1, nt), fusion) for nt in (False, True) for fusion in ((2, 8), (2, 16))]
    for tile, fusion in configs:
        sims = build(small_specs(), form, coll, var)
        ens = Ensemble(sims)
        ens.set_tile(*tile)
        ens.set_fusion(*fusion)
        assert ens.fusion == fusion[0]
        ens.step(4, persistent).step(5, persistent)   # pairs, then pairs and one single step
        got = states(sims)
        for a, b in zip(got, want):
            assert torch.equal(a, b), (tile, fusion)
        assert all(s.steps == 9 for s in sims)
        ens.free()


def test_ensemble_members_match_oracle(orc):
    say("ensemble vs oracle")
    sims = build(small_specs(), "f64")
    Ensemble(sims).step(12, False)
    for (nx, ny, nu, seed), s in zip(small_specs(), sims):
        if nx < 8:
            continue
        ux, uy = inputs.spectral(nx, 3, 0.05, seed=seed, ny=ny)
        p = orc.Params(nx, ny, beta_from_nu(nu), collision=orc.KBC, variant=orc.KBC_B)
        fo = orc.run(p, orc.init(p, ux, uy), 12)
        fg = s.get_populations().cpu().numpy()
        err = np.abs(fg - fo).max() / np.abs(fo).max()
        assert err < 1e-12, (nx, ny, err)


def test_member_beta_change_and_member_lifetime():
    """A member's new beta (lbm_set_beta) is taken up at the ensemble's next
    step, which stays bitwise equal to stepping every member alone; a member
    cannot be freed or re-initialised while the ensemble lives (its context
    would be left dangling), and can be once the ensemble is freed."""
    from paper_1507_02509_amd._lib import KbcError
    say("ensemble member beta and lifetime")
    specs = small_specs()[:3]
    sims, ref = build(specs, "f32"), build(specs, "f32")
    ens = Ensemble(sims)
    ens.step(3)
    for s in ref:
        s.step(3)
    for s in (sims[1], ref[1]):
        s.set_beta(0.9)
    ens.step(5)
    for s in ref:
        s.step(5)
    for a, b in zip(states(sims), states(ref)):
        assert torch.equal(a, b)
    with pytest.raises(KbcError, match="live ensemble"):
        sims[0].free()
    ux, uy = inputs.spectral(specs[0][0], 3, 0.05, seed=1, ny=specs[0][1])
    with pytest.raises(KbcError, match="live ensemble"):
        sims[0].init(ux, uy)
    ens.step(2)                       # the member context is intact
    for s in ref:
        s.step(2)
    for a, b in zip(states(sims), states(ref)):
        assert torch.equal(a, b)
    ens.free()
    sims[0].init(ux, uy)              # allowed again
    sims[0].free()


@pytest.mark.parametrize("form", ["f32", "f64", "f16"])
def test_persistent_ensemble_equals_individual_steps(form):
    """One persistent launch for all the steps (grid barrier between steps),
    with single steps and with two fused steps per barrier, for several
    tiles: bitwise equal to stepping every member alone; the launch reports
    no barrier give-up."""
    say("persistent ensemble vs individual", form)
    ref = build(small_specs(), form)
    for s in ref:
        s.step(9)
    want = states(ref)
    configs = [((128, 2, False), (1, 0)), ((256, 1, True), (1, 0)), ((256, 1, True), (2, 8)),
               ((256, 1, False), (2, 16))]
    for tile, fusion in configs:
        sims = build(small_specs(), form)
        ens = Ensemble(sims)
        ens.set_tile(*tile)
        ens.set_fusion(*fusion)
        blocks = ens.blocks
        say("  tile", tile, "fusion", fusion, "grid", blocks)
        assert blocks >= 8 and blocks % 8 == 0
        ens.step(4, persistent=True).step(5, persistent=True)   # pairs; pairs and one single step
        ens.check()
        for a, b in zip(states(sims), want):
            assert torch.equal(a, b), (tile, fusion)
        assert all(s.steps == 9 for s in sims)
        ens.free()


def test_persistent_barrier_gives_up_and_reports():
    """The grid barrier's wait is bounded: with a spin limit of 0 a workgroup
    that finds the barrier still closed at its first poll gives up, every
    wait of the launch ends at once, and lbm_ensemble_check reports
    LBM_ESYNC (the states are invalid).  The ensemble then recovers: states
    restored, default limit, the persistent launch equals stepping alone."""
    from paper_1507_02509_amd._lib import KbcError
    say("persistent barrier give-up")
    specs = [(512, 512, 1e-4, 7)] + small_specs()[:2]
    sims, ref = build(specs, "f32"), build(specs, "f32")
    snaps = [s.state_buffer().clone() for s in sims]
    ens = Ensemble(sims)
    ens.set_spin_limit(0)
    ens.step(12, persistent=True)
    with pytest.raises(KbcError, match="grid barrier"):
        ens.check()
    ens.check()                      # the flag was cleared by the report
    for s, snap in zip(sims, snaps):      # 12 steps: the state is back in the same buffer
        s.state_buffer().copy_(snap)
        s.lib.lbm_set_step(s.ctx, 0)
    ens.set_spin_limit(1 << 22)
    ens.step(12, persistent=True).check()
    for s in ref:
        s.step(12)
    for a, b in zip(states(sims), states(ref)):
        assert torch.equal(a, b)
    ens.free()


@pytest.mark.parametrize("persistent", [False, True])
def test_uneven_ensemble_256_members(persistent):
    """The ensemble workload: 256 members, N uniform over {128, 256, 512, 1024},
    nu log-uniform over [1e-5, 1e-3], per-member seeds; KBC-B, FP32.  50
    steps (per-step launches, or one persistent launch) equal per-member
    stepping bit for bit (checked on 8 members drawn across the sizes)."""
    specs = inputs.ensemble_members(256, master_seed=4)
    say("256-member ensemble; nodes", sum(n * n for n, _, _ in specs), "persistent", persistent)
    sims = make_members(specs, form="f32")
    pick = [0, 1, 2, 3, 64, 127, 200, 255]
    snaps = [sims[i].state_buffer().clone() for i in pick]
    ens = Ensemble(sims)
    ens.step(50, persistent=persistent)
    ens.check()
    for i, snap in zip(pick, snaps):
        s = sims[i]
        ref = Sim(s.nx, s.ny, s.params.beta, variant="B", form="f32")
        ref.init(np.zeros((s.ny, s.nx)), np.zeros((s.ny, s.nx)), mode="eq")
        ref.state_buffer().copy_(snap)
        ref.step(50)
        assert torch.equal(ref.planes(ref.state_buffer()), s.planes(s.state_buffer())), i
    d = sims[255].diagnostics()
    assert d["n_nonfinite"] == 0


def test_autotuner_restores_state_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("KBC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    say("autotune")
    s = build([(300, 170, 1e-4, 9)], "f32")[0]
    s.step(3)
    before = s.planes(s.state_buffer()).clone()
    n0 = s.steps
    best, timings = autotune.tune_sim(s, steps=4, reps=1)
    assert best in autotune.STEP_CANDIDATES and len(timings) == len(autotune.STEP_CANDIDATES)
    assert torch.equal(s.planes(s.state_buffer()), before) and s.steps == n0
    again, _ = autotune.tune_sim(s)
    assert again == best
    sims = build(small_specs(), "f32")
    ens = Ensemble(sims)
    b2, t2 = autotune.tune_ensemble(ens, steps=2, reps=1)
    assert b2 in autotune.ENSEMBLE_CANDIDATES
    b3, t3 = autotune.tune_ensemble(ens, steps=2, reps=1, persistent=True)
    assert b3 in autotune.ENSEMBLE_CANDIDATES and len(t3) == len(autotune.ENSEMBLE_CANDIDATES)
    ens.check()
    ref = build(small_specs(), "f32")
    for a, b in zip(states(sims), states(ref)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("form", ["f32", "f64"])
def test_ensemble_exact_stabilizer_equals_individual_steps(form):
    """The exact stabiliser (Newton on eq. (result1)) inside the ensemble
    kernels: single and fused launches equal stepping every member alone with
    the same stabiliser, bit for bit (the same per-node code)."""
    say("ensemble exact gamma", form)

    def build_exact():
        sims = []
        for nx, ny, nu, seed in small_specs():
            if nx >= 8 and ny >= 8:
                ux, uy = inputs.spectral(nx, 3, 0.05, seed=seed, ny=ny)
            else:
                ux, uy = np.full((ny, nx), 0.01), np.full((ny, nx), -0.02)
            s = Sim(nx, ny, beta_from_nu(nu), variant="B", form=form, gamma_mode="exact")
            sims.append(s.init(ux, uy))
        return sims

    ref = build_exact()
    for s in ref:
        s.step(9)
    want = states(ref)
    for fusion in ((1, 0), (2, 8), (2, 16)):
        sims = build_exact()
        ens = Ensemble(sims)
        ens.set_fusion(*fusion)
        ens.step(4).step(5)
        for a, b in zip(states(sims), want):
            assert torch.equal(a, b), fusion
        ens.free()
