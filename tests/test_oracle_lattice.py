"""Pins of the oracle's single-cell arithmetic (Section 3.1) against properties
the mathematics fixes: D3Q19 isotropy, equilibrium moments, exact force
injection of the collision, which rate relaxes which moment, and the BGK
special case written out from the textbook Guo scheme."""
import itertools

import numpy as np
import pytest


@pytest.fixture(scope="module")
def vel(orc):
    return orc.velocities()


def test_velocity_set_is_d3q19(vel):
    c, w = vel
    assert c.shape == (19, 3)
    assert len({tuple(v) for v in c}) == 19
    norms = (c * c).sum(1)
    assert sorted(norms.tolist()) == [0] + [1] * 6 + [2] * 12
    # textbook isotropy of the D3Q19 weights
    assert abs(w.sum() - 1.0) < 1e-15
    d = np.eye(3)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(m4, iso, atol=1e-16)


def test_equilibrium_moments(orc, vel):
    c, w = vel
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        feq = orc.equilibrium(rho, u)
        assert abs(feq.sum() - rho) < 1e-15
        np.testing.assert_allclose(feq @ c, rho * u, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", feq, c, c),
                                   rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_collision_injects_exactly_the_force(orc, vel):
    c, w = vel
    rng = np.random.default_rng(12)
    for _ in range(20):
        f = orc.equilibrium(1.0, 0.01 * rng.standard_normal(3)) + 1e-3 * w * rng.standard_normal(19)
        F = 1e-4 * rng.standard_normal(3)
        wp, wm = rng.uniform(0.3, 1.9, 2)
        fout, rho, u = orc.collide_cell(f, F, wp, wm)
        assert abs(fout.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(fout @ c - f @ c, F, atol=1e-16)
        # reported velocity is the half-force velocity
        np.testing.assert_allclose(u, (f @ c + F / 2) / f.sum(), atol=1e-17)


def test_rates_act_on_even_and_odd_moments(orc, vel):
    """omega+ relaxes the (even) second moment, omega- the (odd) third moment."""
    c, w = vel
    rng = np.random.default_rng(13)
    f = orc.equilibrium(1.02, [0.01, -0.02, 0.005]) + 1e-3 * w * rng.standard_normal(19)
    wp, wm = 0.7, 1.3
    fout, rho, u = orc.collide_cell(f, [0, 0, 0], wp, wm)
    feq = orc.equilibrium(rho, u)
    for a, b in itertools.product(range(3), range(3)):
        m_in = np.sum(c[:, a] * c[:, b] * (f - feq))
        m_out = np.sum(c[:, a] * c[:, b] * (fout - feq))
        assert abs(m_out - (1 - wp) * m_in) < 1e-16
    for a, b in itertools.permutations(range(3), 2):
        m_in = np.sum(c[:, a] * c[:, b] ** 2 * (f - feq))
        m_out = np.sum(c[:, a] * c[:, b] ** 2 * (fout - feq))
        assert abs(m_out - (1 - wm) * m_in) < 1e-16


def test_bgk_case_is_textbook_guo(orc, vel):
    """With omega- = omega+ the collision is BGK with Guo's forcing term
    (1 - w/2) w_i [3 (c - u).F + 9 (c.u)(c.F)], written out here directly."""
    c, w = vel
    rng = np.random.default_rng(14)
    for _ in range(10):
        f = orc.equilibrium(1.0, 0.02 * rng.standard_normal(3)) + 1e-3 * w * rng.standard_normal(19)
        F = 1e-4 * rng.standard_normal(3)
        om = rng.uniform(0.5, 1.8)
        fout, rho, u = orc.collide_cell(f, F, om, om)
        cu = c @ u
        uu = u @ u
        feq = w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu)
        guo = (1 - om / 2) * w * (3 * ((c - u) @ F) + 9 * cu * (c @ F))
        np.testing.assert_allclose(fout, f - om * (f - feq) + guo, atol=2e-17)


def test_relaxation_rates_from_viscosity(orc):
    # TRT: (1/w+ - 1/2)(1/w- - 1/2) equals the magic parameter; BGK: equal rates
    for eta, beta in [(1 / 3, 0.5), (1.0, 0.2), (1 / 6, 0.0)]:
        wp, wm = orc.rates(eta, beta, 3 / 16)
        assert abs((1 / wp - 0.5) / 3 - (1 - beta) * eta) < 1e-15
        assert abs((1 / wp - 0.5) * (1 / wm - 0.5) - 3 / 16) < 1e-15
        wp2, wm2 = orc.rates(eta, beta, -1.0)
        assert wp2 == wm2 == wp
