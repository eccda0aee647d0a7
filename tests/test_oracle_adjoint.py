"""CPU pins of the adjoint oracle: its complex-step Jacobian against central
finite differences of the real collision, and the gradient of a final-time
velocity loss through a full rollout (initial state included) against central
finite differences of the forward oracle."""
import numpy as np
import pytest

from paper_1507_02509_amd import inputs

VEL = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], float)


def random_state(rng, eps=0.05):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    u = rng.uniform(-0.08, 0.08, 2)
    return w * (1 + 3 * (VEL @ u)) * (1 + eps * rng.standard_normal(9))


@pytest.mark.parametrize("coll,variant", [(0, 0), (1, 0), (1, 1), (1, 2), (1, 3)])
def test_node_jacobian_matches_finite_differences(orc, coll, variant):
    rng = np.random.default_rng(100 + variant)
    p = orc.Params(1, 1, 0.93, collision=coll, variant=variant)
    for _ in range(5):
        f = random_state(rng)
        J, db = orc.node_jacobian(p, f)
        h = 1e-7
        Jfd = np.zeros((9, 9))
        for j in range(9):
            e = np.zeros(9)
            e[j] = h
            Jfd[:, j] = (orc.node_collide(p, f + e)[0] - orc.node_collide(p, f - e)[0]) / (2 * h)
        np.testing.assert_allclose(J, Jfd, atol=2e-7 * np.abs(J).max())
        pb, pm = (orc.Params(1, 1, 0.93 + s * h, collision=coll, variant=variant) for s in (1, -1))
        dbfd = (orc.node_collide(pb, f)[0] - orc.node_collide(pm, f)[0]) / (2 * h)
        np.testing.assert_allclose(db, dbfd, atol=1e-6 * max(np.abs(db).max(), 1e-12))


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_node_jacobian_exact_stabilizer_matches_finite_differences(orc, variant):
    """With the exact stabiliser the oracle's Newton iteration runs in complex
    arithmetic too; once F(gamma) is at rounding level its imaginary part is
    the implicit derivative -F_theta / F_gamma of the root.  Pinned against
    central differences of the real collision, whose Newton iteration is
    solved to 1e-15 relative at every perturbed state."""
    rng = np.random.default_rng(300 + variant)
    p = orc.Params(1, 1, 0.93, collision=orc.KBC, variant=variant, gamma_mode=orc.GAMMA_EXACT)
    pe = orc.Params(1, 1, 0.93, collision=orc.KBC, variant=variant)
    for _ in range(5):
        f = random_state(rng)
        J, db = orc.node_jacobian(p, f)
        Je, _ = orc.node_jacobian(pe, f)
        h = 1e-6
        Jfd = np.zeros((9, 9))
        for j in range(9):
            e = np.zeros(9)
            e[j] = h
            Jfd[:, j] = (orc.node_collide(p, f + e)[0] - orc.node_collide(p, f - e)[0]) / (2 * h)
        np.testing.assert_allclose(J, Jfd, atol=1e-6 * np.abs(J).max())
        # the exact root's derivative is not the estimate's
        assert np.abs(J - Je).max() > 1e-4 * np.abs(J).max()
        pb, pm = (orc.Params(1, 1, 0.93 + s * h, collision=orc.KBC, variant=variant, gamma_mode=orc.GAMMA_EXACT)
                  for s in (1, -1))
        dbfd = (orc.node_collide(pb, f)[0] - orc.node_collide(pm, f)[0]) / (2 * h)
        np.testing.assert_allclose(db, dbfd, atol=1e-6 * max(np.abs(db).max(), 1e-12))


def velocity_loss_and_seed(orc, p, f, utx, uty):
    """L = 1/2 sum |u - u_t|^2 over nodes and dL/df_i = (u - u_t) . (v_i - u) / rho."""
    rho, ux, uy = orc.moments(p, f)
    dx, dy = ux - utx, uy - uty
    L = 0.5 * float((dx * dx + dy * dy).sum())
    lam = (dx[None] * (VEL[:, 0, None, None] - ux[None]) + dy[None] * (VEL[:, 1, None, None] - uy[None])) / rho[None]
    return L, lam


def rollout_loss(orc, p, ux0, uy0, utx, uty, nsteps):
    f = orc.run(p, orc.init(p, ux0, uy0), nsteps)
    return velocity_loss_and_seed(orc, p, f, utx, uty)[0]


@pytest.mark.parametrize("coll,variant", [(1, 1), (1, 0), (0, 0)])
def test_rollout_gradient_matches_finite_differences(orc, coll, variant):
    n, nsteps = 12, 15
    nu = 1e-3
    ux0, uy0 = inputs.spectral(n, 2, 0.05, seed=5)
    utx, uty = inputs.spectral(n, 2, 0.03, seed=55)
    p = orc.Params(n, n, orc.beta_from_nu(nu), collision=coll, variant=variant)
    states = [orc.init(p, ux0, uy0)]
    for _ in range(nsteps):
        states.append(orc.step(p, states[-1]))
    L, lam = velocity_loss_and_seed(orc, p, states[-1], utx, uty)
    dbeta = 0.0
    for k in range(nsteps - 1, -1, -1):
        lam, db = orc.adjoint_step(p, states[k], lam)
        dbeta += db.sum()
    gux, guy, db0 = orc.init_adjoint(p, ux0, uy0, lam)
    dbeta += db0.sum()

    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(4):
        y, x = rng.integers(0, n, 2)
        for comp, g in ((0, gux), (1, guy)):
            up = [ux0.copy(), uy0.copy()]
            um = [ux0.copy(), uy0.copy()]
            up[comp][y, x] += h
            um[comp][y, x] -= h
            fd = (rollout_loss(orc, p, *up, utx, uty, nsteps) - rollout_loss(orc, p, *um, utx, uty, nsteps)) / (2 * h)
            assert g[y, x] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max())
    hb = 1e-7
    pp = orc.Params(n, n, p.beta + hb, collision=coll, variant=variant)
    pm = orc.Params(n, n, p.beta - hb, collision=coll, variant=variant)
    fd = (rollout_loss(orc, pp, ux0, uy0, utx, uty, nsteps) - rollout_loss(orc, pm, ux0, uy0, utx, uty, nsteps)) / (2 * hb)
    assert dbeta == pytest.approx(fd, rel=1e-5)
