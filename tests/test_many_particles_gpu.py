"""Several movable spheres at once (Section 3.4 coupling and conversion for
each particle).

The conversion runs one block per particle when no particle's cells come
near another's, and one block for all of them otherwise.  The per-particle
blocks must give the bits of the one-block order (VLB_CONV_SERIAL=1 forces
it), both must match the FP64 oracle, and spheres close enough to share cells
take the one-block path by themselves."""
import numpy as np
import pytest

from paper_2009_12279_amd import vlb
from parity import Case, build, compare, log

pytestmark = pytest.mark.gpu

ETA = 1.0 / 6.0


def _case(name, shape, spheres):
    return Case(name, shape, np.zeros(shape[::-1], np.uint8), (1, 1, 1), None,
                dict(eta=ETA, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(0, 0, 0)),
                spheres=[dict(center=c, radius=r, density_ratio=2.0, movable=True, f_ext=f,
                              t_ext=t) for c, r, f, t in spheres])


# six spheres whose boxes stay far apart, pushed in different directions
APART = [((8.3, 8.6, 8.2), 3.1, (4e-2, 0, 0), (0, 0, 1e-2)),
         ((30.4, 8.1, 8.7), 2.7, (0, 3e-2, 0), (0, 0, 0)),
         ((52.6, 9.2, 8.4), 3.3, (0, 0, -4e-2), (1e-2, 0, 0)),
         ((8.8, 30.3, 30.1), 2.9, (-3e-2, 2e-2, 0), (0, 0, 0)),
         ((30.2, 31.4, 29.6), 3.0, (0, -4e-2, 1e-2), (0, 1e-2, 0)),
         ((52.1, 29.7, 30.9), 3.2, (2e-2, 0, 3e-2), (0, 0, -1e-2))]

# two spheres three cells apart (their cells meet) plus one far away
CLOSE = [((20.3, 16.2, 15.8), 3.0, (3e-2, 0, 0), (0, 0, 0)),
         ((29.6, 16.4, 16.1), 3.0, (-3e-2, 0, 0), (0, 0, 1e-2)),
         ((52.0, 30.0, 30.0), 3.0, (0, 3e-2, 0), (0, 0, 0))]


def _run(monkeypatch, spheres, serial, steps=(60, 60, 60)):
    if serial:
        monkeypatch.setenv("VLB_CONV_SERIAL", "1")
    else:
        monkeypatch.delenv("VLB_CONV_SERIAL", raising=False)
    shape = (64, 40, 40)
    L = vlb.Lattice(shape, np.zeros(shape[::-1], np.uint8), (1, 1, 1))
    L.set_params(eta=ETA, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(0, 0, 0))
    for c, r, f, t in spheres:
        L.add_sphere(center=c, radius=r, density_ratio=2.0, movable=True, f_ext=f, t_ext=t)
    L.set_counter_force(True)
    L.set_check_interval(0)
    L.init_equilibrium()
    out = []
    for n in steps:
        L.step(n)
        out += [L.populations(), L.stress(), L.mask()]
        for k in range(len(spheres)):
            p = L.particle(k)
            out += [p["pos"], p["vel"], p["omega"]]
    L.close()
    return out


@pytest.mark.parametrize("which", ["apart", "close"])
def test_per_particle_conversion_gives_the_one_block_bits(monkeypatch, which):
    spheres = APART if which == "apart" else CLOSE
    runs = []
    for serial in (True, False):
        log(f"[particles] {which}: {len(spheres)} movable spheres, serial={serial}")
        runs.append(_run(monkeypatch, spheres, serial))
    masks = runs[0][2::3 + 3 * len(spheres)]
    # the spheres really moved across cells
    assert not np.array_equal(masks[0], masks[-1])
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("which", ["apart", "close"])
def test_many_movable_spheres_match_the_oracle(which):
    spheres = APART if which == "apart" else CLOSE
    case = _case(which, (64, 40, 40), spheres)
    log(f"[particles] {which} against the oracle, 150 steps")
    g, o = build(case, threads=16)
    g.set_counter_force(True)
    o.set_counter_force(True)
    g.step(150)
    o.step(150)
    e = compare(g, o, case)
    log(f"[particles]   errors {e}")
    assert e["mask_equal"]
    for k in ("f", "u", "tau"):
        assert e[k][0] < 1e-5, (k, e[k])
    for k in range(len(spheres)):
        pg, po = g.particle(k), o.particle(k)
        np.testing.assert_allclose(pg["pos"], po["pos"], rtol=0, atol=1e-8)
        # within 1e-5 of each vector's largest component (the cross components
        # the neighbours induce are 1e-4 of it)
        for q in ("vel", "omega"):
            np.testing.assert_allclose(pg[q], po[q], rtol=0, atol=1e-5 * np.abs(po[q]).max())
    g.close()
    o.close()
