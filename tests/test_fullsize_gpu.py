"""GPU against the FP64 oracle at the full sizes of the workloads, in the
launch configuration the benchmark times (same grid, block order and
rounding): the 256^3 box with 64 fixed spheres, the 128x64x64 duct with a
fixed sphere, and the 64x64x256 closed box with a settling sphere.  Every
case prints its name and size before touching the GPU."""
import os

import numpy as np
import pytest

import oracle
from paper_2009_12279_amd import inputs
from parity import Case, build, compare, log

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def test_box_256_cubed_benchmark_workload():
    """The benchmark workload itself, 10 steps from rest (whole fields)."""
    import bench

    shape, spheres, params = bench.build_workload("f32")
    mask = np.zeros(shape[::-1], np.uint8)
    case = Case("box256", shape, mask, (1, 1, 1), None, params,
                spheres=[dict(center=c, radius=r) for c, r in spheres])
    log(f"[fullsize] 256^3 box, {len(spheres)} spheres, 10 steps, oracle threads {THREADS}")
    g, o = build(case, threads=THREADS)
    g.step(10)
    o.step(10)
    e = compare(g, o, case, what=("u", "tau", "rho"))
    log(f"[fullsize]   errors {e}")
    assert e["mask_equal"]
    for k in ("u", "tau", "rho"):
        assert e[k][0] < 1e-5 and e[k][1] < 1e-5, (k, e[k])
    for p in range(0, len(spheres), 9):
        fg, fo = g.particle(p)["force"], o.particle(p)["force"]
        np.testing.assert_allclose(fg, fo, rtol=0, atol=1e-5 * np.abs(fo).max())
    m_g, p_g = g.sums()
    m_o, p_o = o.sums()
    assert abs(m_g - m_o) < 1e-6 * m_o
    g.close()
    o.close()


@pytest.mark.parametrize("lam", [1000.0])
def test_duct_128x64x64_fixed_sphere(lam):
    shape = (128, 64, 64)
    mask = inputs.channel_mask(shape, wall_axes=(1, 2))
    case = Case("duct128", shape, mask, (1, 0, 0), None,
                dict(eta=1 / 3, beta=0.5, lambda_p=lam, magic=3 / 16, body_force=(1e-6, 0, 0)),
                spheres=[dict(center=(63.5, 31.5, 31.5), radius=8.0)])
    log(f"[fullsize] duct 128x64x64, sphere r=8, lambda={lam}, 200 steps")
    g, o = build(case, threads=THREADS)
    g.step(200)
    o.step(200)
    e = compare(g, o, case, what=("u", "tau", "rho"))
    log(f"[fullsize]   errors {e}")
    for k in ("u", "tau"):
        assert e[k][0] < 1e-5 and e[k][1] < 1e-5, (k, e[k])
    pg, po = g.particle(0), o.particle(0)
    np.testing.assert_allclose(pg["force"], po["force"], rtol=0,
                               atol=1e-5 * np.abs(po["force"]).max())
    g.close()
    o.close()


def test_closed_box_64x64x256_settling_sphere():
    """Density ratio 1.5, external force -0.004 along z, Wi = 1 (lambda from
    the Stokes settling speed), 300 steps."""
    shape = (64, 64, 256)
    mask = inputs.channel_mask(shape, wall_axes=(0, 1, 2))
    eta, r, F = 1 / 3, 6.0, 0.004
    v_s = F / (6 * np.pi * eta * r)
    lam = 1.0 * r / v_s
    case = Case("settle", shape, mask, (0, 0, 0), None,
                dict(eta=eta, beta=0.5, lambda_p=lam, magic=3 / 16),
                spheres=[dict(center=(31.5, 31.5, 191.5), radius=r, density_ratio=1.5,
                              movable=True, f_ext=(0.0, 0.0, -F))])
    log(f"[fullsize] closed box 64x64x256, settling sphere, lambda={lam:.0f}, 300 steps")
    g, o = build(case, threads=THREADS)
    vg, vo = [], []
    for _ in range(3):
        g.step(100)
        o.step(100)
        vg.append(g.particle(0)["vel"][2])
        vo.append(o.particle(0)["vel"][2])
    e = compare(g, o, case, what=("u", "tau"))
    log(f"[fullsize]   errors {e}; v_z gpu {vg} oracle {vo}")
    assert e["mask_equal"]
    np.testing.assert_allclose(vg, vo, rtol=1e-5)
    np.testing.assert_allclose(g.particle(0)["pos"], o.particle(0)["pos"], rtol=0, atol=1e-8)
    for k in ("u", "tau"):
        assert e[k][0] < 1e-5, (k, e[k])
    g.close()
    o.close()
