"""Overlap-fraction smoothing of conversions on the GPU against the FP64
oracle, and its binary limit: with one sample per cell the smoothing path
gives the bits of the binary conversion."""
import numpy as np
import pytest

import oracle
from paper_2009_12279_amd import vlb
from parity import log

pytestmark = pytest.mark.gpu


def _box(mk, samples):
    shape = (16, 16, 16)
    L = mk(shape, np.zeros(shape[::-1], np.uint8), (1, 1, 1))
    L.set_params(eta=1 / 6, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(0, 0, 0))
    L.add_sphere([7.5, 7.3, 7.6], 3.1, density_ratio=5.0, movable=True,
                 f_ext=[8e-3, -4e-3, 1.2e-2], t_ext=[0.0, 0.0, 4e-2])
    L.set_counter_force(True)
    if samples is not None:
        L.set_conversion_smoothing(samples)
    L.init_equilibrium()
    return L


def test_one_sample_gives_the_binary_bits():
    runs = []
    for samples in (None, 1):
        log(f"[smoothing] binary limit samples={samples}")
        L = _box(vlb.Lattice, samples)
        L.step(150)
        p = L.particle(0)
        runs.append((L.populations(), L.stress(), L.mask(), p["pos"], p["vel"], p["omega"]))
        L.close()
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("samples", [2, 4])
def test_smoothed_conversion_matches_the_oracle(samples):
    """A free sphere driven through a periodic box with the counter-force,
    smoothed conversions with samples^3 points per cell: masks equal, fields
    within 1e-5, trajectory agreeing, after 150 steps with conversions."""
    log(f"[smoothing] oracle parity samples={samples}")
    g, o = _box(vlb.Lattice, samples), _box(oracle.Lattice, samples)
    for _ in range(3):
        g.step(50)
        o.step(50)
        assert np.array_equal(g.mask(), o.mask())
        pg, po = g.particle(0), o.particle(0)
        np.testing.assert_allclose(pg["pos"], po["pos"], rtol=0, atol=1e-8)
        for k in ("vel", "omega"):
            np.testing.assert_allclose(pg[k], po[k], rtol=0, atol=1e-6 * np.abs(po[k]).max())
    fl = o.mask() == 0
    for name, a, b in (("u", g.velocity(), o.velocity()), ("tau", g.stress(), o.stress())):
        err = np.linalg.norm(a[:, fl] - b[:, fl]) / np.linalg.norm(b[:, fl])
        mx = np.abs(a[:, fl] - b[:, fl]).max() / np.abs(b[:, fl]).max()
        log(f"[smoothing]   {name} L2 {err:.3e} max {mx:.3e}")
        assert err < 1e-5 and mx < 1e-5
    g.close()
    o.close()
