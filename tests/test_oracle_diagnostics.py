"""CPU pins of the oracle's diagnostics (orc_diagnostics) against closed forms.

The paper reports the kinetic energy and enstrophy and their mean and RMS
fluctuations (section *Doubly Periodic Shear Layer*) and the palinstrophy
(section *Decaying Two-Dimensional Turbulence*).  The oracle reads them as
E = <|u|^2 / 2>, Z = <omega^2 / 2>, P = <|grad omega|^2 / 2> with omega and its
gradient from second-order central differences, each with its spatial
standard deviation, plus the density fluctuation and the mean and standard
deviation of the stabiliser gamma.

Every state here is an equilibrium f = feq(rho, u) of a single lattice Fourier
mode, so the moments are (rho, u) exactly and every statistic has a closed
form: a central difference of sin(k.x) is sin(k_a) cos(k.x), and over a whole
period the lattice means of cos and of cos(2 .) vanish while the mean of cos^2
is 1/2.  A dropped factor 1/2, a one-sided difference, a swapped derivative
component or a divisor other than the node count changes at least one of the
values below.
"""
import numpy as np
import pytest

N = 32
SQ2 = np.sqrt(2.0)


def eq_state(orc, p, ux, uy, rho=None):
    return orc.init(p, ux, uy, rho=rho, mode=orc.INIT_EQ)


def mode(m, n, phase=0.3):
    """phi = 2 pi (m x + n y) / N + phase on the N x N lattice, and k = (k_x, k_y)."""
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    kx, ky = 2.0 * np.pi * m / N, 2.0 * np.pi * n / N
    return kx * x + ky * y + phase, kx, ky


@pytest.mark.parametrize("coll", [0, 1])
def test_axis_shear_mode(orc, coll):
    """u_x = a sin(k y), u_y = 0: omega = -a sin(k) cos(k y) and
    d_y omega = a sin(k)^2 sin(k y) with central differences, so
    E = a^2/4, Z = a^2 sin(k)^2 / 4, P = a^2 sin(k)^4 / 4, each standard
    deviation being its mean over sqrt(2)."""
    a = 0.03
    phi, _, k = mode(0, 3)
    ux, uy = a * np.sin(phi), np.zeros((N, N))
    p = orc.Params(N, N, 0.99, collision=coll, variant=orc.KBC_B)
    d = orc.diagnostics(p, eq_state(orc, p, ux, uy))
    E = a * a / 4.0
    Z = a * a * np.sin(k) ** 2 / 4.0
    P = a * a * np.sin(k) ** 4 / 4.0
    for key, want in (("E", E), ("Z", Z), ("P", P)):
        assert d[key] == pytest.approx(want, rel=1e-12), key
        assert d[key + "_std"] == pytest.approx(want / SQ2, rel=1e-12), key + "_std"
    assert abs(d["mass"] - N * N) < 1e-12 * N * N
    assert abs(d["rho_std"]) < 1e-15
    if coll == 0:
        # LBGK: gamma = 2 by definition (at an equilibrium state KBC's gamma is
        # a ratio of rounding-level scalar products and carries no meaning)
        assert d["gamma"] == 2.0 and d["gamma_std"] == 0.0
    assert d["n_nonfinite"] == 0 and d["n_feq_nonpos"] == 0


def test_oblique_mode_cross_terms(orc):
    """u = (A, B) sin(k.x) with k = 2 pi (m, n) / N, m != n: omega =
    C cos(k.x), C = B sin(k_x) - A sin(k_y); grad omega =
    -C (sin k_x, sin k_y) sin(k.x); hence E = (A^2 + B^2)/4, Z = C^2/4,
    P = C^2 (sin^2 k_x + sin^2 k_y) / 4, standard deviations mean / sqrt(2)."""
    A, B = 0.02, -0.035
    phi, kx, ky = mode(2, 5)
    ux, uy = A * np.sin(phi), B * np.sin(phi)
    p = orc.Params(N, N, 0.95, collision=orc.KBC, variant=orc.KBC_A)
    d = orc.diagnostics(p, eq_state(orc, p, ux, uy))
    C = B * np.sin(kx) - A * np.sin(ky)
    E = (A * A + B * B) / 4.0
    Z = C * C / 4.0
    P = C * C * (np.sin(kx) ** 2 + np.sin(ky) ** 2) / 4.0
    for key, want in (("E", E), ("Z", Z), ("P", P)):
        assert d[key] == pytest.approx(want, rel=1e-12), key
        assert d[key + "_std"] == pytest.approx(want / SQ2, rel=1e-12), key + "_std"
    assert abs(d["jx"]) < 1e-13 and abs(d["jy"]) < 1e-13


def test_two_modes_palinstrophy_weights_each_component(orc):
    """u_x = a sin(k1 y), u_y = b sin(k2 x) (k1 != k2): omega =
    b sin(k2) cos(k2 x) - a sin(k1) cos(k1 y), and the two gradient components
    come from different modes: P = (b^2 sin(k2)^4 + a^2 sin(k1)^4) / 4, which a
    stencil applied to the wrong direction would not give."""
    a, b = 0.025, 0.04
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    k1, k2 = 2.0 * np.pi * 2 / N, 2.0 * np.pi * 5 / N
    ux, uy = a * np.sin(k1 * y + 0.1), b * np.sin(k2 * x + 0.7)
    p = orc.Params(N, N, 0.97, collision=orc.LBGK)
    d = orc.diagnostics(p, eq_state(orc, p, ux, uy))
    assert d["E"] == pytest.approx((a * a + b * b) / 4.0, rel=1e-12)
    assert d["Z"] == pytest.approx((a * a * np.sin(k1) ** 2 + b * b * np.sin(k2) ** 2) / 4.0, rel=1e-12)
    assert d["P"] == pytest.approx((a * a * np.sin(k1) ** 4 + b * b * np.sin(k2) ** 4) / 4.0, rel=1e-12)


def test_density_fluctuation_and_entropy_at_rest(orc):
    """rho = 1 + eps cos(k.x), u = 0: the density's spatial standard deviation
    is eps / sqrt(2) and its mean 1; at rest f = W rho, so the entropy of
    eq. (S) per node is -rho ln rho; E = Z = P = 0."""
    eps = 0.01
    phi, _, _ = mode(3, 1)
    rho = 1.0 + eps * np.cos(phi)
    z = np.zeros((N, N))
    p = orc.Params(N, N, 0.9, collision=orc.KBC, variant=orc.KBC_D)
    f = eq_state(orc, p, z, z, rho=rho)
    d = orc.diagnostics(p, f)
    assert d["rho_std"] == pytest.approx(eps / SQ2, rel=1e-12)
    assert d["mass"] == pytest.approx(N * N, rel=1e-14)
    assert d["S"] == pytest.approx(float(np.mean(-rho * np.log(rho))), rel=1e-10)
    for key in ("E", "Z", "P", "E_std", "Z_std", "P_std"):
        assert abs(d[key]) < 1e-30, key


def test_gamma_mean_and_std_of_a_two_valued_field(orc):
    """gamma is gamma_1 at n_1 copies of one non-equilibrium node and gamma_2 at
    the n_2 copies of another, so its mean is (n_1 gamma_1 + n_2 gamma_2) / N
    and its standard deviation |gamma_1 - gamma_2| sqrt(n_1 n_2) / N
    (population form)."""
    n = 8
    p = orc.Params(n, n, 0.98, collision=orc.KBC, variant=orc.KBC_A)
    pert = np.array([1, -1, 2, 0, -2, 1, 3, -1, 0], dtype=np.float64)
    node1 = orc.node_equilibrium(1.0, 0.02, -0.01) * (1.0 + 2e-2 * pert)
    node2 = orc.node_equilibrium(1.01, -0.03, 0.015) * (1.0 + 1e-2 * pert[::-1])
    _, g1 = orc.node_collide(p, node1)
    _, g2 = orc.node_collide(p, node2)
    assert abs(g1 - g2) > 1e-3
    f = np.empty((9, n, n))
    f[:] = node2[:, None, None]
    rows = [1, 4, 6]            # n_1 = 24 nodes
    for r in rows:
        f[:, r, :] = node1[:, None]
    n1 = len(rows) * n
    n2 = n * n - n1
    gam = orc.gamma_field(p, f)
    assert np.all(gam[rows, :] == g1) and np.all(np.delete(gam, rows, axis=0) == g2)
    d = orc.diagnostics(p, f)
    assert d["gamma"] == pytest.approx((n1 * g1 + n2 * g2) / (n * n), rel=1e-13)
    assert d["gamma_std"] == pytest.approx(abs(g1 - g2) * np.sqrt(n1 * n2) / (n * n), rel=1e-11)
