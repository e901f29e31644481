"""Pins of the oracle's overlap-fraction smoothing of conversions
(Section 3.4 names the overlapped fraction of a cell as a way to smooth the
conversion of cells between fluid and solid; the reading is in the oracle).

* The sub-sampled overlap fraction is the midpoint rule for the volume of
  the sphere inside the cell: 1 well inside, 0 well outside, the coverage
  test itself with one sample, and summed over the lattice it converges to
  the sphere's volume.
* With one sample per cell the overlap is 0 or 1, nothing is handed over
  before a cover, and the run is bit for bit the binary conversion.
* With smoothing the conversions still conserve the fluid's total stress
  and the momentum of fluid + particle + pending conversion momentum.
* Smoothing acts where it should and nowhere else: one smoothed step
  changes the stress only next to the moving surface, moves it out of the
  cells the sphere advances into, and creates none."""
import numpy as np
import pytest


def _box(orc, samples, shape=(16, 16, 16)):
    L = orc.Lattice(shape)
    L.set_params(eta=1 / 6, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(0, 0, 0))
    pid = L.add_sphere([7.5, 7.3, 7.6], 3.1, density_ratio=5.0, movable=True,
                       f_ext=[8e-3, -4e-3, 1.2e-2], t_ext=[0.0, 0.0, 4e-2])
    L.set_counter_force(True)
    if samples is not None:
        L.set_conversion_smoothing(samples)
    L.init_equilibrium()
    return L, pid


def test_overlap_fraction_is_the_sphere_volume_per_cell(orc):
    shape = (20, 20, 20)
    L = orc.Lattice(shape)
    r = 4.3
    c = np.array([9.7, 10.2, 9.9])
    pid = L.add_sphere(c, r)
    total = 0.0
    for z in range(3, 17):
        for y in range(3, 17):
            for x in range(3, 17):
                d = np.linalg.norm(np.array([x, y, z]) - c)
                phi = L.overlap_fraction(pid, x, y, z, 8)
                total += phi
                if d + np.sqrt(3) / 2 < r:
                    assert phi == 1.0
                if d - np.sqrt(3) / 2 > r:
                    assert phi == 0.0
                # one sample: the coverage test at the cell centre
                assert L.overlap_fraction(pid, x, y, z, 1) == (1.0 if d * d < r * r else 0.0)
    assert total == pytest.approx(4 / 3 * np.pi * r ** 3, rel=2e-3)


def test_one_sample_per_cell_is_the_binary_conversion(orc):
    """Overlap fractions of 0 and 1 only: the smoothing path gives the bits
    of the binary conversion (populations, stress, mask, trajectory)."""
    runs = []
    for samples in (None, 1):
        L, pid = _box(orc, samples)
        L.step(120)
        p = L.particle(pid)
        runs.append((L.populations(), L.stress(), L.mask(), p["pos"], p["vel"], p["omega"]))
        L.close()
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


def test_smoothed_conversion_conserves_stress_and_momentum(orc):
    """Sub-sampled overlaps (4^3 per cell): the fluid's total stress is the
    same before and after every conversion, and fluid + particle momentum +
    momentum owed by the last conversion stays constant under the
    counter-force, while the sphere moves across cells."""
    L, pid = _box(orc, 4)
    M = 5.0 * 4 / 3 * np.pi * 3.1 ** 3

    def ledger():
        _, pf = L.sums()
        return pf + M * L.particle(pid)["vel"] + L.pending_conversion()

    led0 = ledger()
    n_conv = 0
    for _ in range(200):
        L.step(1)
        np.testing.assert_allclose(ledger() - led0, 0.0, rtol=0, atol=1e-12)
        (c, u), before, after = L.conversion_stats()
        n_conv += c + u
        np.testing.assert_allclose(after + L.dropped_stress() * 0, before, rtol=0,
                                   atol=1e-15 + 1e-12 * np.abs(before).max())
    assert n_conv > 0


def test_smoothing_moves_stress_out_of_cells_the_sphere_advances_into(orc):
    """Two identical runs of a moving sphere, the second with 4^3 samples
    per cell for one step: the stress fields then differ only within two
    cells of the sphere's surface, the differences sum to zero (stress is
    moved, not made), and the cells whose overlap grew in that step (the
    senders) hold less stress in the smoothed run, since part of theirs went
    to neighbours behind them."""
    runs = []
    for samples in (None, 4):
        L, pid = _box(orc, None)
        tau0 = np.zeros((6,) + L.mask().shape)
        tau0[0:3] = 1e-4
        tau0[:, L.mask() != 0] = 0
        L.set_stress(tau0)
        L.step(20)
        if samples:
            L.set_conversion_smoothing(samples)
        runs.append(L)
    Lb, Ls = runs
    nz, ny, nx = Lb.mask().shape
    phi0 = np.array([[[Lb.overlap_fraction(pid, x, y, z, 4) for x in range(nx)]
                      for y in range(ny)] for z in range(nz)])
    for L in runs:
        L.step(1)
    phi1 = np.array([[[Lb.overlap_fraction(pid, x, y, z, 4) for x in range(nx)]
                      for y in range(ny)] for z in range(nz)])
    mask = Lb.mask()
    assert np.array_equal(mask, Ls.mask())
    d = Ls.stress() - Lb.stress()
    fl = mask == 0
    scale = np.abs(Lb.stress()[:, fl]).sum(axis=1)
    assert np.all(np.abs(d[:, fl].sum(axis=1)) <= 1e-13 * scale)
    R = Lb.particle(pid)["pos"]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dist = np.sqrt((x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2)
    assert np.all(d[:, dist > 3.1 + 2.5] == 0)
    senders = fl & (phi1 > phi0)
    assert senders.sum() > 0
    assert d[0][senders].sum() < 0 and d[1][senders].sum() < 0 and d[2][senders].sum() < 0
    for L in runs:
        L.close()
