"""Force densities that vary from cell to cell (Section 3.1 Guo forcing), as
the four-roll mill of Section 4.4 is driven.  Its force, with the sign of the
y-component taken so that the field is not a pure gradient (the printed
form, with equal signs, is the gradient of cos(kx) cos(ky) and would drive
no flow), is 2 k^2 eta_n u0 (sin kx cos ky, -cos kx sin ky), k = 2 pi / L.
The velocity u0 (sin kx cos ky, -cos kx sin ky) then solves the Stokes and
the Navier-Stokes equations exactly (its inertia is a gradient), which pins
the oracle on plain and on 45-degree rotated lattices."""
import numpy as np

SQ2 = np.sqrt(2.0)


def four_roll_mill(M, rotated, eta_n, u0):
    """Force density and exact Newtonian velocity on an M x M x 1 lattice,
    shapes (3, 1, M, M).  Rotated: the lattice axes run along the diagonals
    of the system, cell (i, j) sits at X = (i - j)/sqrt2 + L/2,
    Y = (i + j)/sqrt2 with L = M sqrt2, so that the lattice's periodicity M
    is the flow's half-period shift (L/2, L/2), a symmetry of the field, and
    cell (M/2, M/2) is the system's centre (L/2, L/2).  Vector components
    are returned in the lattice frame."""
    i = np.arange(M)[None, :].astype(float)
    j = np.arange(M)[:, None].astype(float)
    if rotated:
        L = M * SQ2
        X, Y = (i - j) / SQ2 + L / 2, (i + j) / SQ2
    else:
        L = float(M)
        X, Y = i + 0 * j, j + 0 * i
    k = 2 * np.pi / L
    A = 2 * k * k * eta_n * u0
    sx, cx, sy, cy = np.sin(k * X), np.cos(k * X), np.sin(k * Y), np.cos(k * Y)
    fx, fy = A * sx * cy, -A * cx * sy
    vx, vy = u0 * sx * cy, -u0 * cx * sy
    if rotated:  # system components -> lattice components
        fx, fy = (fx + fy) / SQ2, (fy - fx) / SQ2
        vx, vy = (vx + vy) / SQ2, (vy - vx) / SQ2
    F = np.zeros((3, 1, M, M))
    U = np.zeros((3, 1, M, M))
    F[0, 0], F[1, 0] = fx, fy
    U[0, 0], U[1, 0] = vx, vy
    return F, U, L


def test_uniform_force_field_equals_body_force(orc):
    shape = (10, 9, 8)
    mask = np.zeros(shape[::-1], np.uint8)
    g = (2e-5, -1e-5, 3e-6)
    a = orc.Lattice(shape, mask, (1, 1, 1))
    b = orc.Lattice(shape, mask, (1, 1, 1))
    a.set_params(eta=1 / 3, beta=0.5, lambda_p=20.0, magic=3 / 16, body_force=g)
    b.set_params(eta=1 / 3, beta=0.5, lambda_p=20.0, magic=3 / 16)
    F = np.zeros((3,) + shape[::-1])
    for c in range(3):
        F[c] = g[c]
    b.set_force_field(F)
    a.step(30)
    b.step(30)
    np.testing.assert_array_equal(a.populations(), b.populations())
    np.testing.assert_array_equal(a.stress(), b.stress())
    np.testing.assert_array_equal(a.velocity(), b.velocity())


def test_four_roll_mill_newtonian_exact_solution(orc):
    """eta_n = 1.5 (the paper's), u0 = 1e-3, 400 steps (the slowest mode decays
    as exp(-2 k^2 nu t)).  Second-order convergence to the exact field on the
    plain lattice (M = 16, 32) and on the rotated one (M = 16, 32)."""
    eta_n, u0 = 1.5, 1e-3
    for rotated, bound in ((False, 0.005), (True, 0.0015)):
        err = []
        for M in (16, 32):
            F, U, _ = four_roll_mill(M, rotated, eta_n, u0)
            o = orc.Lattice((M, M, 1), np.zeros((1, M, M), np.uint8), (1, 1, 1))
            o.set_params(eta=eta_n, beta=0.0, lambda_p=1.0, magic=3 / 16)
            o.set_force_field(F)
            o.step(400)
            err.append(np.abs(o.velocity() - U).max() / u0)
            o.close()
        assert err[1] < bound, (rotated, err)
        assert 3.5 < err[0] / err[1] < 4.5, (rotated, err)
