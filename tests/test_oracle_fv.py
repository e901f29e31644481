"""Pins of the oracle's finite-volume stress update and polymer force
(Section 3.3) against closed forms: pure relaxation, donor-cell advection
(a binomial law), the corner-transport-upwind face overlap computed
geometrically, the Oldroyd-B shear recurrences, zero flux through solid
faces, exact divergence of linear stress fields and the telescoping of the
polymer force to boundary faces."""
import itertools
import math

import numpy as np
import pytest

TAU_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def full(tau6):
    """[6,...] components -> [3,3,...] symmetric tensor"""
    t = np.zeros((3, 3) + tau6.shape[1:])
    for k, (i, j) in enumerate(TAU_PAIRS):
        t[i, j] = tau6[k]
        t[j, i] = tau6[k]
    return t


def test_pure_relaxation_with_zero_velocity(orc):
    rng = np.random.default_rng(1)
    shape = (5, 4, 3)  # nz, ny, nx
    mask = np.zeros(shape, np.uint8)
    tau0 = rng.standard_normal((6,) + shape)
    u = np.zeros((3,) + shape)
    lam = 7.0
    t = tau0
    for _ in range(25):
        t = orc.fv_apply(mask, t, u, 0.3, lam)
    np.testing.assert_allclose(t, (1 - 1 / lam) ** 25 * tau0, rtol=1e-13)


def test_uniform_advection_is_binomial(orc):
    """u = (a,0,0) on a periodic ring: tau' (x) = (1-a-1/lam) tau(x) + a tau(x-1),
    so after n steps tau = sum_k C(n,k) a^k (1-a-1/lam)^(n-k) tau0(x-k)."""
    rng = np.random.default_rng(2)
    nx = 16
    shape = (1, 1, nx)
    mask = np.zeros(shape, np.uint8)
    tau0 = rng.standard_normal((6,) + shape)
    a, lam, n = 0.03, 50.0, 12
    u = np.zeros((3,) + shape)
    u[0] = a
    t = tau0
    for _ in range(n):
        t = orc.fv_apply(mask, t, u, 0.1, lam)
    expect = np.zeros_like(tau0)
    for k in range(n + 1):
        expect += math.comb(n, k) * a ** k * (1 - a - 1 / lam) ** (n - k) * np.roll(tau0, k, axis=3)
    np.testing.assert_allclose(t, expect, rtol=1e-12, atol=1e-15)


def _overlap_1d(d, s):
    """length of [d, d+1] intersected with [s, s+1]"""
    return max(0.0, min(d + 1, s + 1) - max(d, s))


@pytest.mark.parametrize("u", [(0.02, 0.01, -0.03), (-0.04, 0.0, 0.02), (0.01, -0.05, -0.01)])
def test_face_fluxes_are_displaced_cell_overlaps(orc, u):
    """Uniform u: each face neighbour receives the exact overlap volume of the
    displaced unit cell with it (computed here from intervals); overlaps with
    edge/corner neighbours stay in the cell."""
    rng = np.random.default_rng(3)
    shape = (4, 5, 6)
    mask = np.zeros(shape, np.uint8)
    tau0 = rng.standard_normal((6,) + shape)
    uu = np.zeros((3,) + shape)
    for a in range(3):
        uu[a] = u[a]
    lam = 9.0
    out = orc.fv_apply(mask, tau0, uu, 0.2, lam)
    expect = tau0 * (1 - 1 / lam)
    for e in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        ov = np.prod([_overlap_1d(u[a], e[a]) for a in range(3)])
        # (x,y,z) loses ov*tau(x) to x+e and gains ov*tau(x-e) from x-e
        shifted = np.roll(tau0, shift=(e[2], e[1], e[0]), axis=(1, 2, 3))
        expect += ov * (shifted - tau0)
    np.testing.assert_allclose(out, expect, rtol=1e-13, atol=1e-15)


def test_no_flux_through_solid_faces(orc):
    """Uniform u (also prescribed on solid nodes, so the gradient vanishes):
    stress piles up against walls but the fluid total only relaxes."""
    rng = np.random.default_rng(4)
    nx, ny, nz = 6, 7, 5
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    mask[0, :, :] = 1
    mask[-1, :, :] = 1
    tau = rng.standard_normal((6, nz, ny, nx))
    tau[:, mask != 0] = 0
    u = np.zeros((3, nz, ny, nx))
    u[0], u[1], u[2] = 0.02, 0.04, -0.03
    lam = 20.0
    fl = mask == 0
    total0 = tau[:, fl].sum(1)
    for n in range(1, 6):
        tau = orc.fv_apply(mask, tau, u, 0.2, lam)
        np.testing.assert_allclose(tau[:, fl].sum(1), (1 - 1 / lam) ** n * total0, rtol=1e-13,
                                   atol=1e-13)


def test_steady_shear_source_recurrences(orc):
    """u_x = g*y with y walls far away, everything uniform in x: interior cells
    follow the explicit-Euler Oldroyd-B recurrences
        tau_yy' = q tau_yy,  tau_xy' = q tau_xy + g tau_yy + eta_p g / lam,
        tau_xx' = q tau_xx + 2 g tau_xy,  q = 1 - 1/lam,
    whose closed forms from rest are tau_xy = eta_p g (1 - q^n) and
    tau_xx = 2 eta_p g^2 (lam (1 - q^n) - n q^(n-1))."""
    nx, ny, nz = 3, 12, 3
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    gam, eta_p, lam = 2e-3, 0.25, 40.0
    u = np.zeros((3, nz, ny, nx))
    y = np.arange(ny, dtype=float)
    u[0] = (gam * y)[None, :, None]
    tau = np.zeros((6, nz, ny, nx))
    q = 1 - 1 / lam
    for n in range(1, 31):
        tau = orc.fv_apply(mask, tau, u, eta_p, lam)
        inner = tau[:, :, 2:-2, :]
        txy = eta_p * gam * (1 - q ** n)
        txx = 2 * eta_p * gam ** 2 * (lam * (1 - q ** n) - n * q ** (n - 1))
        np.testing.assert_allclose(inner[3], txy, rtol=1e-12)
        np.testing.assert_allclose(inner[0], txx, rtol=1e-11,
                                   atol=1e-12 * 2 * lam * eta_p * gam ** 2)
        np.testing.assert_allclose(inner[1], 0.0, atol=1e-30)
        np.testing.assert_allclose(inner[[2, 4, 5]], 0.0, atol=1e-30)
    # the steady values eta_p g and 2 lam eta_p g^2 are approached
    for _ in range(3000):
        tau = orc.fv_apply(mask, tau, u, eta_p, lam)
    inner = tau[:, :, 2:-2, :]
    np.testing.assert_allclose(inner[3], eta_p * gam, rtol=1e-12)
    np.testing.assert_allclose(inner[0], 2 * lam * eta_p * gam ** 2, rtol=1e-10)


def test_polymer_force_of_linear_stress_is_its_divergence(orc):
    rng = np.random.default_rng(5)
    nx, ny, nz = 7, 8, 9
    mask = np.zeros((nz, ny, nx), np.uint8)
    A = rng.standard_normal(6)
    B = rng.standard_normal((6, 3))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tau = np.stack([A[k] + B[k, 0] * x + B[k, 1] * y + B[k, 2] * z for k in range(6)])
    fp = orc.polymer_force(mask, tau)
    t3 = np.zeros((3, 3, 3))  # d tau_ij / d r_k
    for k, (i, j) in enumerate(TAU_PAIRS):
        t3[i, j] = t3[j, i] = B[k]
    div = np.array([sum(t3[k, j, k] for k in range(3)) for j in range(3)])
    inner = fp[:, 1:-1, 1:-1, 1:-1]
    for j in range(3):
        np.testing.assert_allclose(inner[j], div[j], rtol=1e-12, atol=1e-12)


def test_polymer_force_telescopes_to_boundary_faces(orc):
    """Summed over fluid cells the discrete force is the sum over fluid->solid
    faces of n.tau(fluid cell): interior face contributions cancel."""
    rng = np.random.default_rng(6)
    nx, ny, nz = 8, 7, 6
    mask = (rng.uniform(size=(nz, ny, nx)) < 0.25).astype(np.uint8)
    tau = rng.standard_normal((6, nz, ny, nx))
    tau[:, mask != 0] = 0
    fp = orc.polymer_force(mask, tau)
    total = fp[:, mask == 0].sum(1)
    t = full(tau)
    expect = np.zeros(3)
    for zz, yy, xx in itertools.product(range(nz), range(ny), range(nx)):
        if mask[zz, yy, xx]:
            continue
        for a, s in itertools.product(range(3), (1, -1)):
            p = [xx, yy, zz]
            p[a] = (p[a] + s) % (nx, ny, nz)[a]
            if mask[p[2], p[1], p[0]]:
                expect += s * t[a, :, zz, yy, xx]
    np.testing.assert_allclose(total, expect, rtol=1e-12, atol=1e-12)


def test_giesekus_steady_shear_matches_the_constitutive_equations(orc):
    """Giesekus (Section 2.2 names it among the models the scheme extends
    to): in steady simple shear u_x = g y the stress solves the algebraic
    equations that tau + lam tau^del + (alpha lam / eta_p) tau.tau =
    eta_p (grad u + grad u^T) reduces to, written out by component:
        xx: t_xx - 2 W t_xy + a (t_xx^2 + t_xy^2) = 0
        yy: t_yy + a (t_xy^2 + t_yy^2) = 0
        xy: t_xy - W t_yy + a t_xy (t_xx + t_yy) = W,   t_zz = 0,
    with tau = (eta_p / lam) t and W = lam g.  The explicit FV update with a
    prescribed shear relaxes to that solution; alpha = 0 stays Oldroyd-B
    and alpha > 0 thins the shear stress and turns tau_yy negative."""
    from scipy.optimize import fsolve

    nx, ny, nz = 3, 12, 3
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    gam, eta_p, lam = 2e-3, 0.25, 400.0
    W = lam * gam
    u = np.zeros((3, nz, ny, nx))
    u[0] = (gam * np.arange(ny, dtype=float))[None, :, None]
    for a in (0.0, 0.1, 0.3, 0.5):
        def eqs(v):
            txx, tyy, txy = v
            return [txx - 2 * W * txy + a * (txx ** 2 + txy ** 2),
                    tyy + a * (txy ** 2 + tyy ** 2),
                    txy - W * tyy + a * txy * (txx + tyy) - W]
        sol = fsolve(eqs, [2 * W * W, 0.0, W], xtol=1e-12)
        assert np.max(np.abs(eqs(sol))) < 1e-12
        expect = eta_p / lam * sol
        tau = np.zeros((6, nz, ny, nx))
        for _ in range(12000):
            tau = orc.fv_apply(mask, tau, u, eta_p, lam, alpha=a)
        inner = tau[:, :, 2:-2, :]
        np.testing.assert_allclose(inner[0], expect[0], rtol=1e-9)
        np.testing.assert_allclose(inner[1], expect[1], rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(inner[3], expect[2], rtol=1e-9)
        np.testing.assert_allclose(inner[[2, 4, 5]], 0.0, atol=1e-30)
        if a == 0.0:
            np.testing.assert_allclose(expect, [2 * lam * eta_p * gam ** 2, 0.0, eta_p * gam],
                                       rtol=1e-12, atol=1e-20)
        else:
            assert expect[2] < eta_p * gam and expect[1] < 0


def test_fene_p_steady_shear_matches_the_conformation_solution(orc):
    """FENE-P (Section 2.2 names it as the model the scheme extends to), in
    the stored variable T = (eta_p/lam)(A - I).  In steady simple shear the
    conformation equation A^del = -(f A - I)/lam with f = (L^2-3)/(L^2-tr A)
    gives, by component, A_yy = A_zz = 1/f, A_xy = W/f^2 and
    A_xx = 1/f + 2 W^2/f^3 (W = lam g), with f the root of
    f (L^2 - 3/f - 2 W^2/f^3) = L^2 - 3.  The explicit FV update with a
    prescribed shear relaxes to exactly that; huge L^2 is Oldroyd-B."""
    from scipy.optimize import brentq

    nx, ny, nz = 3, 12, 3
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    gam, eta_p, lam = 2e-3, 0.25, 400.0
    W = lam * gam
    u = np.zeros((3, nz, ny, nx))
    u[0] = (gam * np.arange(ny, dtype=float))[None, :, None]
    for L2 in (10.0, 50.0):
        f = brentq(lambda f: f * (L2 - 3 / f - 2 * W ** 2 / f ** 3) - (L2 - 3), 1.0, 50.0,
                   xtol=1e-15)
        T = np.zeros((6, nz, ny, nx))
        for _ in range(20000):
            T = orc.fv_apply(mask, T, u, eta_p, lam, L2=L2)
        A = T[:, :, 2:-2, :] * (lam / eta_p)  # A - I
        np.testing.assert_allclose(A[1] + 1, 1 / f, rtol=1e-9)
        np.testing.assert_allclose(A[2] + 1, 1 / f, rtol=1e-9)
        np.testing.assert_allclose(A[3], W / f ** 2, rtol=1e-9)
        np.testing.assert_allclose(A[0] + 1, 1 / f + 2 * W ** 2 / f ** 3, rtol=1e-9)
        np.testing.assert_allclose(A[[4, 5]], 0.0, atol=1e-30)
        assert f > 1.01  # the finite extensibility matters at this W
    T_ob = np.zeros((6, nz, ny, nx))
    T_fe = np.zeros((6, nz, ny, nx))
    for _ in range(300):
        T_ob = orc.fv_apply(mask, T_ob, u, eta_p, lam)
        T_fe = orc.fv_apply(mask, T_fe, u, eta_p, lam, L2=1e12)
    np.testing.assert_allclose(T_fe, T_ob, rtol=1e-8, atol=1e-9 * np.abs(T_ob).max())


def test_quadratic_extrapolation_reproduces_the_divergence_next_to_walls(orc):
    """With quadratic extrapolation the discrete force of a stress field
    quadratic in the wall-normal coordinate is its divergence in every fluid
    cell with two fluid layers behind it (central differences are exact for
    quadratics); linear extrapolation misses the curvature in the cells next
    to the walls, and with a single fluid layer behind a wall the quadratic
    order falls back to the linear one."""
    rng = np.random.default_rng(16)
    nx, ny, nz = 6, 12, 5
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    A, B, Cq = rng.standard_normal(6), rng.standard_normal(6), rng.standard_normal(6)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    yy = y.astype(float)
    tau = np.stack([A[k] + B[k] * yy + Cq[k] * yy ** 2 for k in range(6)])
    # divergence: F_j = d tau_yj / dy at cell centres
    dtau = np.stack([B[k] + 2 * Cq[k] * yy for k in range(6)])
    div = np.stack([dtau[3], dtau[1], dtau[5]])   # (tau_xy, tau_yy, tau_yz) along y
    quad = orc.polymer_force(mask, tau, order=2)
    lin = orc.polymer_force(mask, tau, order=1)
    fluid = mask == 0
    np.testing.assert_allclose(quad[:, fluid], div[:, fluid], rtol=0, atol=1e-11)
    wall_rows = (slice(None), slice(None), [1, -2], slice(None))
    assert np.max(np.abs(lin[wall_rows] - div[wall_rows])) > 0.1 * np.abs(Cq[[3, 1, 5]]).min()
    # one fluid layer behind the wall: quadratic = linear there
    mask2 = mask.copy()
    mask2[:, 3, :] = 1            # fluid rows 1, 2 between two walls
    q2 = orc.polymer_force(mask2, tau, order=2)
    l2 = orc.polymer_force(mask2, tau, order=1)
    np.testing.assert_array_equal(q2[:, :, 1:3, :], l2[:, :, 1:3, :])


def test_linear_extrapolation_reproduces_the_divergence_next_to_walls(orc):
    """With linear extrapolation into solid neighbours (Section 3.3 offers it
    beside the constant one) the discrete force of a linear stress field is
    its divergence also in cells next to a wall (two fluid layers behind
    them), where constant extrapolation is off by half a gradient."""
    rng = np.random.default_rng(15)
    nx, ny, nz = 7, 10, 9
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    A = rng.standard_normal(6)
    B = rng.standard_normal((6, 3))
    B[:, 0] = 0.0  # x periodic: no x gradient
    B[:, 2] = 0.0  # z periodic: no z gradient
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tau = np.stack([A[k] + B[k, 1] * y for k in range(6)])
    t3 = np.zeros((3, 3, 3))
    for k, (i, j) in enumerate(TAU_PAIRS):
        t3[i, j] = t3[j, i] = B[k]
    div = np.array([sum(t3[k, j, k] for k in range(3)) for j in range(3)])
    lin = orc.polymer_force(mask, tau, order=1)
    const = orc.polymer_force(mask, tau, order=0)
    fluid = mask == 0
    for j in range(3):
        np.testing.assert_allclose(lin[j][fluid], div[j], rtol=1e-12, atol=1e-12)
    # constant extrapolation: the wall rows see half the normal gradient
    wall_rows = const[:, :, [1, -2], :]
    assert np.max(np.abs(wall_rows[1] - div[1])) > 0.1 * np.abs(div[1])
