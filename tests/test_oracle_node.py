"""CPU pins of the oracle's single-node arithmetic against what the paper and
the mathematics fix.  Each test names the passage it checks.  The tests build
their inputs with plain numpy sums over the nine velocities and never reuse
the oracle's formula for the quantity under test."""
import numpy as np
import pytest

VEL = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
CX, CY = VEL[:, 0].astype(float), VEL[:, 1].astype(float)


def moment(f, p, q):
    return float(np.sum(f * CX ** p * CY ** q))


def random_state(rng, rho=1.0, u=(0.03, -0.02), eps=0.05):
    """A positive population vector near rest with a random non-equilibrium part."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    base = rho * w * (1 + 3 * (CX * u[0] + CY * u[1]))
    return base * (1 + eps * rng.standard_normal(9))


def state_with_central_moments(rho, ux, uy, ct):
    """Populations with the given density, velocity and central moments
    (T~, N~, Pi~, Q~xyy, Q~yxx, A~): solve the 9x9 moment system directly,
    <f (v_x-u_x)^p (v_y-u_y)^q> = rho M~_pq."""
    T, N, P, Qx, Qy, A = ct
    target = {(0, 0): 1.0, (1, 0): 0.0, (0, 1): 0.0, (2, 0): 0.5 * (T + N), (0, 2): 0.5 * (T - N),
              (1, 1): P, (1, 2): Qx, (2, 1): Qy, (2, 2): A}
    rows, rhs = [], []
    for (p, q), v in target.items():
        rows.append((CX - ux) ** p * (CY - uy) ** q)
        rhs.append(rho * v)
    return np.linalg.solve(np.array(rows), np.array(rhs))


# ----------------------------------------------------------------- lattice
def test_velocity_order(orc):
    cx, cy = orc.velocities()
    assert np.array_equal(cx, CX.astype(int)) and np.array_equal(cy, CY.astype(int))


def test_weights_isotropy(orc):
    """The weights reproduce the lattice moments that make eq. (Eq) give
    Pi^eq and Q^eq of eqs. (Peq), (Qeq): sum W = 1, sum W v_a v_b = cs2 d_ab,
    sum W v_x^4 = 3 cs2^2, sum W v_x^2 v_y^2 = cs2^2, odd moments zero."""
    W = orc.weights()
    cs2 = orc.cs2()
    assert cs2 == pytest.approx(1.0 / 3.0, abs=1e-16)
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    assert moment(W, 2, 0) == pytest.approx(cs2, abs=1e-15)
    assert moment(W, 0, 2) == pytest.approx(cs2, abs=1e-15)
    assert moment(W, 1, 1) == pytest.approx(0.0, abs=1e-16)
    assert moment(W, 4, 0) == pytest.approx(3 * cs2 ** 2, abs=1e-15)
    assert moment(W, 2, 2) == pytest.approx(cs2 ** 2, abs=1e-15)
    for p, q in [(1, 0), (0, 1), (3, 0), (2, 1), (1, 2)]:
        assert moment(W, p, q) == pytest.approx(0.0, abs=1e-16)


def test_weights_from_moment_representation(orc):
    """At rest with the equilibrium moments T = 2 cs2, A = cs2^2 (the rest of
    the set zero), eq. (momentsD2Q9) must give f = W rho: 4/9, 1/9, 1/36."""
    rho = 1.3
    cs2 = 1.0 / 3.0
    r = rho * np.array([1, 0, 0, 2 * cs2, 0, 0, 0, 0, cs2 ** 2])
    f = orc.node_populations(r)
    np.testing.assert_allclose(f, rho * np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4), atol=1e-15)
    np.testing.assert_allclose(orc.weights(), f / rho, atol=1e-15)


# -------------------------------------------------------------- equilibrium
@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.02, 0.05, -0.03), (0.97, -0.1, 0.08)])
def test_equilibrium_moments(orc, rho, ux, uy):
    """eq. (Eq): conserves rho and rho u; its second and third moments are
    eqs. (Peq), (Qeq) exactly on D2Q9 (u is carried to second order)."""
    feq = orc.node_equilibrium(rho, ux, uy)
    cs2 = 1.0 / 3.0
    u = (ux, uy)
    assert moment(feq, 0, 0) == pytest.approx(rho, abs=1e-15)
    assert moment(feq, 1, 0) == pytest.approx(rho * ux, abs=1e-15)
    assert moment(feq, 0, 1) == pytest.approx(rho * uy, abs=1e-15)
    for (p, q), (a, b) in {(2, 0): (0, 0), (0, 2): (1, 1), (1, 1): (0, 1)}.items():
        want = rho * cs2 * (a == b) + rho * u[a] * u[b]
        assert moment(feq, p, q) == pytest.approx(want, abs=1e-15)
    # Q_abm = rho cs2 (u_a d_bm + u_b d_am + u_m d_ab); on D2Q9 v^3 = v
    assert moment(feq, 1, 2) == pytest.approx(rho * cs2 * ux, abs=1e-15)   # Q_xyy
    assert moment(feq, 2, 1) == pytest.approx(rho * cs2 * uy, abs=1e-15)   # Q_yxx
    assert moment(feq, 3, 0) == pytest.approx(3 * rho * cs2 * ux, abs=1e-15)
    if ux == 0 and uy == 0:
        np.testing.assert_allclose(feq, rho * orc.weights(), atol=1e-16)


# ------------------------------------------------------------ moment algebra
def test_natural_moments_of_unit_populations(orc):
    """eq. (natmoments1) on a single unit population f = e_i gives the monomials
    of v_i: (1, v_x, v_y, v_x^2+v_y^2, v_x^2-v_y^2, v_x v_y, v_x v_y^2, v_x^2 v_y, v_x^2 v_y^2)."""
    for i in range(9):
        e = np.zeros(9)
        e[i] = 1.0
        vx, vy = CX[i], CY[i]
        want = [1, vx, vy, vx * vx + vy * vy, vx * vx - vy * vy, vx * vy, vx * vy * vy,
                vx * vx * vy, vx * vx * vy * vy]
        np.testing.assert_array_equal(orc.node_natural(e), want)


def test_populations_invert_moments(orc):
    """eq. (momentsD2Q9) is the inverse of the moment map: f -> r -> f."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        f = random_state(rng, rho=rng.uniform(0.8, 1.2), u=rng.uniform(-0.1, 0.1, 2), eps=0.3)
        np.testing.assert_allclose(orc.node_populations(orc.node_natural(f)), f, atol=2e-16)


def test_central_to_natural_relation(orc):
    """eq. (cm): natural moments from the central ones agree with the natural
    moments summed directly (both moment sets computed by explicit sums)."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        f = random_state(rng, rho=rng.uniform(0.8, 1.2), u=rng.uniform(-0.15, 0.15, 2), eps=0.3)
        rho = moment(f, 0, 0)
        ux, uy = moment(f, 1, 0) / rho, moment(f, 0, 1) / rho
        ct = np.array([moment_c(f, ux, uy, 2, 0) + moment_c(f, ux, uy, 0, 2),
                       moment_c(f, ux, uy, 2, 0) - moment_c(f, ux, uy, 0, 2),
                       moment_c(f, ux, uy, 1, 1), moment_c(f, ux, uy, 1, 2),
                       moment_c(f, ux, uy, 2, 1), moment_c(f, ux, uy, 2, 2)]) / rho
        np.testing.assert_allclose(orc.node_central(f), ct, atol=1e-15)
        nat = np.array([moment(f, 2, 0) + moment(f, 0, 2), moment(f, 2, 0) - moment(f, 0, 2),
                        moment(f, 1, 1), moment(f, 1, 2), moment(f, 2, 1), moment(f, 2, 2)]) / rho
        np.testing.assert_allclose(orc.node_central_to_natural(ux, uy, ct, 1), nat, atol=1e-15)


def moment_c(f, ux, uy, p, q):
    return float(np.sum(f * (CX - ux) ** p * (CY - uy) ** q))


# --------------------------------------------------------------- k / s / h
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_split_sums_to_f_and_conserves(orc, variant):
    """eq. (ksh-representation) f = k + s + h; eqs. (k_conservation),
    (sh_conservation): <k {1, v}> = {rho, rho u}, <s {1, v}> = <h {1, v}> = 0;
    the higher moments of k vanish in its own basis."""
    rng = np.random.default_rng(3 + variant)
    for _ in range(10):
        f = random_state(rng, rho=rng.uniform(0.9, 1.1), u=rng.uniform(-0.1, 0.1, 2), eps=0.2)
        k, s, h = orc.node_split(variant, f)
        np.testing.assert_allclose(k + s + h, f, atol=3e-16)
        rho = moment(f, 0, 0)
        ux, uy = moment(f, 1, 0) / rho, moment(f, 0, 1) / rho
        assert moment(k, 0, 0) == pytest.approx(rho, abs=1e-15)
        assert moment(k, 1, 0) == pytest.approx(rho * ux, abs=1e-15)
        assert moment(k, 0, 1) == pytest.approx(rho * uy, abs=1e-15)
        for part in (s, h):
            for p, q in [(0, 0), (1, 0), (0, 1)]:
                assert moment(part, p, q) == pytest.approx(0.0, abs=1e-15)
        for p, q in [(2, 0), (0, 2), (1, 1), (1, 2), (2, 1), (2, 2)]:
            if variant >= 2:
                assert moment(k, p, q) == pytest.approx(0.0, abs=1e-15)
            else:
                assert moment_c(k, ux, uy, p, q) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_table_sh_moments2(orc, variant):
    """Table sh_moments2: second moments of s and h for models A-D."""
    rng = np.random.default_rng(10 + variant)
    for _ in range(10):
        f = random_state(rng, rho=rng.uniform(0.9, 1.1), u=rng.uniform(-0.1, 0.1, 2), eps=0.2)
        k, s, h = orc.node_split(variant, f)
        rho = moment(f, 0, 0)
        ux, uy = moment(f, 1, 0) / rho, moment(f, 0, 1) / rho
        if variant < 2:   # central moments
            cxx, cyy, cxy = (moment_c(f, ux, uy, 2, 0), moment_c(f, ux, uy, 0, 2),
                             moment_c(f, ux, uy, 1, 1))
        else:
            cxx, cyy, cxy = moment(f, 2, 0), moment(f, 0, 2), moment(f, 1, 1)
        T, N, P = (cxx + cyy) / rho, (cxx - cyy) / rho, cxy / rho
        if variant in (0, 2):   # A, C
            want_s = (0.5 * rho * (T + N), 0.5 * rho * (T - N), rho * P)
            want_h = (0.0, 0.0, 0.0)
        else:                   # B, D
            want_s = (0.5 * rho * N, -0.5 * rho * N, rho * P)
            want_h = (0.5 * rho * T, 0.5 * rho * T, 0.0)
        got_s = (moment(s, 2, 0), moment(s, 0, 2), moment(s, 1, 1))
        got_h = (moment(h, 2, 0), moment(h, 0, 2), moment(h, 1, 1))
        np.testing.assert_allclose(got_s, want_s, atol=2e-15)
        np.testing.assert_allclose(got_h, want_h, atol=2e-15)


# ------------------------------------------------- entropic scalar products
def test_zeroth_order_products(orc):
    """Section 'Entropic Stabilizer', zeroth order in u: at u = 0,
    <ds|dh> = -rho (9 A~ - 1)(3 T~ - 2) / 4 for models A and C, and 0 for B and D."""
    rng = np.random.default_rng(20)
    for _ in range(10):
        rho = rng.uniform(0.9, 1.1)
        ct = np.array([2 / 3, 0, 0, 0, 0, 1 / 9]) + 0.02 * rng.standard_normal(6)
        f = state_with_central_moments(rho, 0.0, 0.0, ct)
        want = -0.25 * rho * (9 * ct[5] - 1) * (3 * ct[0] - 2)
        for variant, w in [(0, want), (1, 0.0), (2, want), (3, 0.0)]:
            a = orc.node_deviations(variant, f)[2][0]
            assert a == pytest.approx(w, abs=1e-17 + 1e-12 * abs(want))


def test_first_order_products(orc):
    """First order in u with the central moments held fixed: zero for A and B,
    the printed expressions for C and D (P~_xy read as Pi~_xy)."""
    rng = np.random.default_rng(21)
    for _ in range(5):
        rho = rng.uniform(0.9, 1.1)
        ct = np.array([2 / 3, 0, 0, 0, 0, 1 / 9]) + 0.02 * rng.standard_normal(6)
        T, N, P, Qx, Qy, A = ct
        d = rng.standard_normal(2)
        d /= np.linalg.norm(d)
        eps = 1e-4
        ux, uy = eps * d

        def a_at(sign, variant):
            f = state_with_central_moments(rho, sign * ux, sign * uy, ct)
            return orc.node_deviations(variant, f)[2][0]

        c1 = 9 / 4 * rho * (Qx * ((2 + 3 * N - 3 * T) * ux - 12 * P * uy)
                            - Qy * (12 * P * ux + (-2 + 3 * N + 3 * T) * uy))
        d1 = -27 / 4 * rho * (-N * Qx * ux + 4 * P * Qy * ux + 4 * P * Qx * uy + N * Qy * uy)
        for variant, want in [(0, 0.0), (1, 0.0), (2, c1), (3, d1)]:
            odd = 0.5 * (a_at(1, variant) - a_at(-1, variant))
            scale = abs(c1) + abs(d1)
            assert abs(odd - want) <= 1e-6 * scale, (variant, odd, want)


# ---------------------------------------------------------------- collision
def params(orc, **kw):
    base = dict(nx=1, ny=1, beta=0.9, collision=orc.KBC, variant=orc.KBC_B)
    base.update(kw)
    return orc.Params(**base)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_gamma_two_is_lbgk(orc, variant):
    """eq. (ksh-mirror) with gamma = 2 coincides with LBGK, eq. (LBGKmirr)."""
    rng = np.random.default_rng(30 + variant)
    for _ in range(10):
        f = random_state(rng, u=rng.uniform(-0.1, 0.1, 2), eps=0.1)
        beta = rng.uniform(0.5, 1.0)
        out_k, g = orc.node_collide(params(orc, beta=beta, variant=variant,
                                           gamma_mode=orc.GAMMA_FIXED, gamma_fixed=2.0), f)
        out_l, gl = orc.node_collide(params(orc, beta=beta, collision=orc.LBGK), f)
        assert g == 2.0 and gl == 2.0
        np.testing.assert_allclose(out_k, out_l, atol=5e-16)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_gamma_inverse_beta_is_regularized(orc, variant):
    """gamma = 1/beta brings the higher-order part to its equilibrium value
    (regularized LB): h(f') = h(feq); the shear deviation flips as
    ds' = (1 - 2 beta) ds."""
    rng = np.random.default_rng(40 + variant)
    for _ in range(10):
        f = random_state(rng, u=rng.uniform(-0.1, 0.1, 2), eps=0.1)
        beta = rng.uniform(0.5, 1.0)
        out, g = orc.node_collide(params(orc, beta=beta, variant=variant,
                                         gamma_mode=orc.GAMMA_FIXED, gamma_fixed=1.0 / beta), f)
        ds0, dh0, _ = orc.node_deviations(variant, f)
        ds1, dh1, _ = orc.node_deviations(variant, out)
        np.testing.assert_allclose(dh1, 0.0, atol=1e-15)
        np.testing.assert_allclose(ds1, (1 - 2 * beta) * ds0, atol=1e-15)


@pytest.mark.parametrize("coll,variant", [(0, 0), (1, 0), (1, 1), (1, 2), (1, 3)])
def test_collision_conserves_and_keeps_equilibrium(orc, coll, variant):
    """The collision conserves rho and rho u; f = feq is a fixed point (to
    rounding: at f = feq the deviations are rounding noise, and gamma * dh is
    bounded by |ds| through the Cauchy-Schwarz inequality)."""
    rng = np.random.default_rng(50 + variant)
    p = params(orc, collision=coll, variant=variant, beta=0.97)
    for _ in range(10):
        f = random_state(rng, u=rng.uniform(-0.1, 0.1, 2), eps=0.1)
        out, _ = orc.node_collide(p, f)
        for pq in [(0, 0), (1, 0), (0, 1)]:
            assert moment(out, *pq) == pytest.approx(moment(f, *pq), abs=1e-15)
        feq = orc.node_equilibrium(1.01, 0.04, -0.07)
        out, g = orc.node_collide(p, feq)
        np.testing.assert_allclose(out, feq, atol=1e-15)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_gamma_star_solves_linearised_condition(orc, variant):
    """gamma* of eq. (result21) satisfies the linearisation of eq. (result1):
    (1 - beta gamma) <dh|dh> = (2 beta - 1) <ds|dh>."""
    rng = np.random.default_rng(60 + variant)
    beta = 0.95
    for _ in range(10):
        f = random_state(rng, u=rng.uniform(-0.1, 0.1, 2), eps=0.05)
        _, g = orc.node_collide(params(orc, beta=beta, variant=variant), f)
        a, b, c = orc.node_deviations(variant, f)[2]
        assert b > 1e-12 * c
        assert (1 - beta * g) * b == pytest.approx((2 * beta - 1) * a, abs=1e-14 * b)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_exact_gamma_root_and_limit(orc, variant):
    """The exact stabiliser is the root of eq. (result1), and gamma* is its
    first-order estimate: |gamma_exact - gamma*| shrinks linearly with the
    size of the non-equilibrium part."""
    rng = np.random.default_rng(70 + variant)
    beta = 0.95
    f0 = random_state(rng, u=(0.04, -0.03), eps=0.0)
    rho = moment(f0, 0, 0)
    feq = orc.node_equilibrium(rho, moment(f0, 1, 0) / rho, moment(f0, 0, 1) / rho)
    direction = rng.standard_normal(9) * feq
    # keep rho and rho u: remove the projection on 1, v_x, v_y
    basis = np.vstack([np.ones(9), CX, CY])
    direction -= basis.T @ np.linalg.lstsq(basis.T, direction, rcond=None)[0]
    gaps = []
    for scale in [1e-2, 1e-3]:
        f = feq + scale * direction / np.abs(direction / feq).max()
        _, g_est = orc.node_collide(params(orc, beta=beta, variant=variant), f)
        pe = params(orc, beta=beta, variant=variant, gamma_mode=orc.GAMMA_EXACT)
        _, g_ex = orc.node_collide(pe, f)
        dh = orc.node_deviations(variant, f)[1]
        assert abs(orc.node_result1(pe, f, g_ex)) <= 1e-14 * np.abs(dh).sum() + 1e-22
        gaps.append(abs(g_ex - g_est))
    assert gaps[1] < 0.2 * gaps[0]


def test_guard_gives_gamma_two(orc):
    """Reading of the denominator guard: with dh = 0 (models C/D on a state whose
    only deviation is in Pi and N) gamma is 2."""
    rho, ux, uy = 1.0, 0.02, -0.01
    feq = orc.node_equilibrium(rho, ux, uy)
    d = np.zeros(9)
    # a pure Pi_xy deviation built from the diagonal populations: (+,-,+,-)/4
    d[5], d[6], d[7], d[8] = 1e-4, -1e-4, 1e-4, -1e-4
    for variant in (2, 3):
        _, g = orc.node_collide(params(orc, variant=variant), feq + d)
        assert g == 2.0
