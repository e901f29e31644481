"""Two-dimensional flows.  A lattice one cell thick in z (periodic) with
z-symmetric populations is the D2Q9 / D2Q5 method the paper uses for its
two-dimensional benchmarks (Section 4): the D3Q19 populations that share an
in-plane velocity sum to a D2Q9 population (weights 1/3 + 2/18 = 4/9,
1/18 + 2/36 = 1/9 and 1/36), the TRT collision and the Guo source are linear
in the populations and depend only on in-plane moments, and the z faces of
the finite-volume stencil carry nothing.  The pin runs an independent D2Q9
TRT-Guo program written out here and compares it with the oracle's sums."""
import numpy as np

from paper_2009_12279_amd import inputs

C2 = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)])
W2 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP2 = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7])


def d2q9_step(f, mask, F, wp, wm):
    """One D2Q9 TRT step with Guo forcing (symmetric source part scaled by
    1 - w+/2, antisymmetric by 1 - w-/2, u = (sum f c + F/2)/rho) and push
    streaming with halfway bounce-back at solid cells.  f: [9, ny, nx]."""
    fl = mask == 0
    rho = f.sum(0)
    j = np.einsum("iyx,ia->ayx", f, C2.astype(float))
    u = (j + 0.5 * F[:, None, None]) / np.where(fl, rho, 1.0)
    cu = np.einsum("ia,ayx->iyx", C2.astype(float), u)
    uu = (u * u).sum(0)
    feq = W2[:, None, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu)
    cF = (C2 * F).sum(1)[:, None, None]
    uF = (u * F[:, None, None]).sum(0)
    S = W2[:, None, None] * (3 * cF + 9 * cu * cF - 3 * uF)
    sym = lambda a: 0.5 * (a + a[OPP2])
    asym = lambda a: 0.5 * (a - a[OPP2])
    fs = (f - wp * (sym(f) - sym(feq)) - wm * (asym(f) - asym(feq))
          + (1 - wp / 2) * sym(S) + (1 - wm / 2) * asym(S))
    ny, nx = mask.shape
    out = np.zeros_like(f)
    for i, (cx, cy) in enumerate(C2):
        for y in range(ny):
            for x in range(nx):
                if not fl[y, x]:
                    continue
                xd, yd = (x + cx) % nx, (y + cy) % ny
                if fl[yd, xd]:
                    out[i, yd, xd] = fs[i, y, x]
                else:
                    out[OPP2[i], y, x] = fs[i, y, x]
    return out


def test_one_cell_thick_lattice_is_d2q9(orc):
    rng = np.random.default_rng(31)
    nx, ny = 9, 11
    shape = (nx, ny, 1)
    mask = inputs.channel_mask(shape, wall_axes=(1,))
    eta, magic = 0.2, 3 / 16
    wp, wm = orc.rates(eta, 0.0, magic)
    F = np.array([1e-5, -3e-6])
    c3, w3 = orc.velocities()
    # random near-equilibrium D2Q9 state on fluid cells, split z-symmetrically
    # over the D3Q19 populations of each in-plane velocity in weight ratio
    u = 2e-3 * rng.standard_normal((2, ny, nx))
    f2 = np.zeros((9, ny, nx))
    for i, c in enumerate(C2):
        cu = c[0] * u[0] + c[1] * u[1]
        f2[i] = W2[i] * (1 + 3 * cu + 4.5 * cu ** 2) + 1e-4 * W2[i] * rng.standard_normal((ny, nx))
    m2 = mask[0] != 0
    f2[:, m2] = 0.0
    group = [int(np.where((C2 == c[:2]).all(1))[0][0]) for c in c3]
    gw = np.array([w3[[k for k in range(19) if group[k] == g]].sum() for g in range(9)])
    np.testing.assert_allclose(gw, W2, rtol=1e-15)
    f3 = np.zeros((19, 1, ny, nx))
    for k in range(19):
        f3[k, 0] = f2[group[k]] * w3[k] / W2[group[k]]
    L = orc.Lattice(shape, mask, periodic=(1, 0, 1))
    L.set_params(eta=eta, beta=0.0, lambda_p=1.0, magic=magic, body_force=(F[0], F[1], 0.0))
    L.set_populations(f3)
    for _ in range(40):
        L.step(1)
        f2 = d2q9_step(f2, mask[0], F, wp, wm)
    f3 = L.populations()[:, 0]
    lumped = np.zeros((9, ny, nx))
    for k in range(19):
        lumped[group[k]] += f3[k]
    fl = mask[0] == 0
    dev = lambda a: a[:, fl] - W2[:, None]
    np.testing.assert_allclose(dev(lumped), dev(f2), rtol=0, atol=1e-15)
    # and the z-symmetry that the reduction needs is kept (to rounding)
    assert np.max(np.abs(L.velocity()[2])) < 1e-15


def test_one_cell_thick_stress_update_is_d2q5(orc):
    """The stress update on one z-layer equals that on four identical layers
    (the z faces contribute nothing) and leaves tau_xz, tau_yz, tau_zz at zero
    for in-plane flow."""
    rng = np.random.default_rng(32)
    nx, ny = 8, 10
    mask1 = inputs.channel_mask((nx, ny, 1), wall_axes=(1,))
    mask4 = np.repeat(mask1, 4, axis=0)
    u1 = np.zeros((3, 1, ny, nx))
    u1[:2] = 3e-3 * rng.standard_normal((2, 1, ny, nx))
    u1[:, mask1 != 0] = 0
    t1 = np.zeros((6, 1, ny, nx))
    t1[[0, 1, 3]] = 1e-3 * rng.standard_normal((3, 1, ny, nx))
    u4, t4 = np.repeat(u1, 4, axis=1), np.repeat(t1, 4, axis=1)
    for _ in range(5):
        t1 = orc.fv_apply(mask1, t1, u1, 0.1, 30.0)
        t4 = orc.fv_apply(mask4, t4, u4, 0.1, 30.0)
    for zz in range(4):
        np.testing.assert_array_equal(t4[:, zz], t1[:, 0])
    assert np.all(t1[[2, 4, 5]] == 0.0)
