"""Walls whose velocity varies from cell to cell (Section 3.1 velocity
boundary condition), as the lid-driven cavity of Section 4.3 needs with its
regularized lid velocity 16 u0 (x/L)^2 (1 - x/L)^2.  The oracle is pinned
against an independent finite-difference solution of the Stokes problem
(the cavity runs at Re = 0.02, where inertia is negligible) and against the
per-id wall table it generalises."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from paper_2009_12279_amd import inputs


def stokes_cavity(n):
    """Stream function of Stokes flow in the unit square, no slip on three
    sides and the regularized lid velocity along y = 1: the biharmonic
    equation for psi (u = dpsi/dy, v = -dpsi/dx) with the 13-point stencil on
    (n+1)^2 nodes, psi = 0 on the boundary and the normal derivative imposed
    through mirrored ghost nodes.  Returns the node coordinates and psi[j, i]
    (y index first)."""
    h = 1.0 / n
    xs = np.linspace(0.0, 1.0, n + 1)
    lid = 16 * xs ** 2 * (1 - xs) ** 2
    m = n - 1

    def idx(i, j):
        return (j - 1) * m + (i - 1)

    stencil = {(0, 0): 20.0, (1, 0): -8.0, (-1, 0): -8.0, (0, 1): -8.0, (0, -1): -8.0,
               (1, 1): 2.0, (1, -1): 2.0, (-1, 1): 2.0, (-1, -1): 2.0,
               (2, 0): 1.0, (-2, 0): 1.0, (0, 2): 1.0, (0, -2): 1.0}
    rows, cols, vals = [], [], []
    rhs = np.zeros(m * m)
    for j in range(1, n):
        for i in range(1, n):
            r = idx(i, j)
            for (di, dj), c in stencil.items():
                ii, jj = i + di, j + dj
                if 1 <= ii <= m and 1 <= jj <= m:
                    rows.append(r), cols.append(idx(ii, jj)), vals.append(c)
                elif ii in (0, n) or jj in (0, n):
                    continue                                   # psi = 0 on the wall
                elif ii == -1 or ii == n + 1:                  # side walls: v = 0
                    rows.append(r), cols.append(idx(1 if ii == -1 else n - 1, jj)), vals.append(c)
                elif jj == -1:                                 # bottom: u = 0
                    rows.append(r), cols.append(idx(ii, 1)), vals.append(c)
                else:                                          # lid: dpsi/dy = u_lid
                    rows.append(r), cols.append(idx(ii, n - 1)), vals.append(c)
                    rhs[r] -= c * 2 * h * lid[ii]
    A = sp.csc_matrix((vals, (rows, cols)), shape=(m * m, m * m))
    psi = np.zeros((n + 1, n + 1))
    psi[1:n, 1:n] = spl.spsolve(A, rhs).reshape(m, m)
    return xs, psi


def stokes_centrelines(n):
    """u_x / u0 along x = 1/2 and u_y / u0 along y = 1/2 of the Stokes
    solution, on the nodes: central differences of psi inside, the boundary
    values themselves (lid velocity, no slip) on the walls."""
    xs, psi = stokes_cavity(n)
    h = 1.0 / n
    us = np.zeros(n + 1)
    vs = np.zeros(n + 1)
    us[1:n] = (psi[2:, n // 2] - psi[:-2, n // 2]) / (2 * h)
    vs[1:n] = -(psi[n // 2, 2:] - psi[n // 2, :-2]) / (2 * h)
    us[n] = 16 * 0.5 ** 2 * 0.5 ** 2
    return xs, us, vs


def cavity_lattice(orc, L, u0, table_lid=False):
    """(L+2)^2 x 1 cavity, lid along y = L+1.  With table_lid the lid is wall
    id 2 moving at the constant u0 from the per-id table instead."""
    shape = (L + 2, L + 2, 1)
    mask = inputs.channel_mask(shape, wall_axes=(0, 1))
    if table_lid:
        mask[0, L + 1, 1:L + 1] = 2
        o = orc.Lattice(shape, mask, (0, 0, 1), [[0, 0, 0], [u0, 0, 0]])
    else:
        o = orc.Lattice(shape, mask, (0, 0, 1))
    o.set_params(eta=1.0, beta=0.0, lambda_p=1.0, magic=3 / 16)
    return o


def regularized_lid(L, u0):
    fld = np.zeros((3, 1, L + 2, L + 2))
    X = np.clip((np.arange(L + 2) - 0.5) / L, 0.0, 1.0)   # wall halfway between cells
    fld[0, 0, L + 1, :] = 16 * u0 * X ** 2 * (1 - X) ** 2
    return fld


def centrelines(u, L, u0):
    """u_x along x = L/2 and u_y along y = L/2 at the cell centres, / u0."""
    ux = 0.5 * (u[0, 0, 1:L + 1, L // 2] + u[0, 0, 1:L + 1, L // 2 + 1]) / u0
    uy = 0.5 * (u[1, 0, L // 2, 1:L + 1] + u[1, 0, L // 2 + 1, 1:L + 1]) / u0
    return ux, uy


def test_stokes_reference_converges():
    """The finite-difference reference itself: second-order convergence of the
    centreline minimum, and the symmetry u_y(x) = -u_y(1 - x) of the
    symmetric lid."""
    mins = []
    for n in (32, 64, 128):
        xs, psi = stokes_cavity(n)
        mins.append(np.gradient(psi[:, n // 2], 1.0 / n).min())
    r = (mins[0] - mins[1]) / (mins[1] - mins[2])
    assert 3.0 < r < 5.0, mins
    v = -np.gradient(psi[64, :], 1.0 / 128)
    np.testing.assert_allclose(v, -v[::-1], atol=1e-12)


def test_wall_field_equal_to_table_gives_same_bits(orc):
    L, u0 = 12, 1e-3
    a = cavity_lattice(orc, L, u0, table_lid=True)
    b = cavity_lattice(orc, L, u0)
    fld = np.zeros((3, 1, L + 2, L + 2))
    fld[0, 0, L + 1, 1:L + 1] = u0
    b.set_wall_velocity_field(fld)
    a.step(50)
    b.step(50)
    np.testing.assert_array_equal(a.populations(), b.populations())
    # and clearing the field returns to the table (all walls at rest here)
    b.set_wall_velocity_field(None)
    c = cavity_lattice(orc, L, u0)
    b.set_populations(c.populations())
    b.step(5)
    c.step(5)
    np.testing.assert_array_equal(b.populations(), c.populations())


def test_regularized_lid_cavity_matches_stokes(orc):
    """Newtonian cavity at L = 32 and 64 (Re = u0 L / nu <= 0.0064) against the
    Stokes solution on a 256^2 grid.  The wall velocity of a diagonal link is
    taken at the solid node, not at the crossing point, so the error falls
    at first order: it must halve from L = 32 to L = 64 and be below
    0.006 u0 at L = 64."""
    u0 = 1e-4
    xs, us, vs = stokes_centrelines(256)
    orc.set_threads(4)
    dev = []
    for L in (32, 64):
        o = cavity_lattice(orc, L, u0)
        o.set_wall_velocity_field(regularized_lid(L, u0))
        o.step(25 * L)                      # slowest Stokes mode decays in ~L^2/52 steps
        ux, uy = centrelines(o.velocity(), L, u0)
        Y = (np.arange(1, L + 1) - 0.5) / L
        dev.append(max(np.abs(ux - np.interp(Y, xs, us)).max(),
                       np.abs(uy - np.interp(Y, xs, vs)).max()))
        # extrema where the Stokes flow has them, to within a cell
        assert abs(Y[ux.argmin()] - xs[us.argmin()]) <= 1.0 / L
        assert abs(Y[uy.argmax()] - xs[vs.argmax()]) <= 1.0 / L
        assert abs(Y[uy.argmin()] - xs[vs.argmin()]) <= 1.0 / L
        o.close()
    assert dev[1] < 0.006, dev
    assert 1.6 < dev[0] / dev[1] < 2.4, dev
