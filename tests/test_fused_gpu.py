"""The fused step kernel (stream-collide and stress update in one pass, the
ring of neighbour velocities recomputed in the block) against the two-kernel
step (velocity through HBM) and against the FP64 oracle.

The two paths run the same arithmetic on the same inputs, so they must agree
bit for bit after any number of steps: on ragged tiles (rows and planes that
do not fill a tile), one-cell-thick lattices, moving walls, fixed and moving
spheres, every constitutive law, linear and quadratic extrapolation, both
rounding modes and all three storage formats.  The fused kernel is measured
slower than the two kernels on MI355X and runs only when asked: VLB_FUSED=1
for lattices that fill the chip with its tiles, -1 for any polymer lattice."""
import numpy as np
import pytest

from paper_2009_12279_amd import inputs, vlb
from parity import build, compare, log
from test_parity_gpu import random_case

pytestmark = pytest.mark.gpu


def _channel(name, shape=(70, 22, 13)):
    storage = {"f16": "f16", "bf16": "bf16"}.get(name, "f32")
    mask = inputs.channel_mask(shape, wall_axes=(1,), top_id=2)
    L = vlb.Lattice(shape, mask, (1, 0, 1), [[0, 0, 0], [2e-3, 0, 1e-3]], storage=storage)
    L.set_params(eta=1 / 4, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(2e-5, 0, 0))
    if shape[2] > 1:
        L.add_sphere(center=(30.5, 10.5, 6.5), radius=3.3)
    if name == "fene":
        L.set_fene_p(50.0)
    elif name == "giesekus":
        L.set_giesekus(0.2)
    elif name == "extrap2":
        L.set_extrapolation(2)
    elif name == "nearest":
        L.set_rounding("nearest")
    u0 = inputs.noise_field(3, 0, shape, 2e-3)
    u0[:, L.mask() != 0] = 0
    L.init_equilibrium(u0)
    return L


def _moving():
    shape = (64, 20, 18)
    L = vlb.Lattice(shape, np.zeros(shape[::-1], np.uint8), (1, 1, 1))
    L.set_params(eta=1 / 6, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(0, 0, 0))
    L.add_sphere(center=(31.5, 9.3, 8.6), radius=3.1, density_ratio=5.0, movable=True,
                 f_ext=(8e-3, -4e-3, 1.2e-2), t_ext=(0, 0, 4e-2))
    L.set_counter_force(True)
    L.init_equilibrium()
    return L


CASES = ["plain", "fene", "giesekus", "extrap2", "nearest", "f16", "bf16", "thin", "moving"]


@pytest.mark.parametrize("name", CASES)
def test_fused_step_gives_the_two_kernel_bits(monkeypatch, name):
    runs = []
    for mode in ("0", "-1"):
        monkeypatch.setenv("VLB_FUSED", mode)
        log(f"[fused] {name} VLB_FUSED={mode}")
        if name == "moving":
            L = _moving()
        elif name == "thin":
            L = _channel("plain", (70, 22, 1))
        else:
            L = _channel(name)
        out = []
        for n in (1, 16, 23):
            L.step(n)
            out += [L.populations(), L.stress(), L.velocity(), L.mask()]
            if name == "moving":
                out += [L.particle(0)["pos"], L.particle(0)["omega"]]
        runs.append(out)
        L.close()
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("seed,shape,periodic,moving,sphere", [
    (3, (9, 9, 9), (0, 0, 0), True, ((4.3, 4.6, 4.4), 1.8)),
    (5, (12, 10, 11), (1, 0, 0), True, ((6.2, 4.9, 5.1), 2.5)),
    (6, (67, 9, 10), (1, 0, 1), True, ((30.2, 4.4, 4.9), 2.6)),
])
def test_fused_step_matches_the_oracle(monkeypatch, seed, shape, periodic, moving, sphere):
    """Random masks (12 % solid), moving walls, a fixed sphere, random
    populations and stress: the fused step against the FP64 oracle after 30
    steps, as the brute-force parity of the two-kernel step."""
    monkeypatch.setenv("VLB_FUSED", "-1")
    case = random_case(seed, shape, periodic, moving, sphere)
    log(f"[fused] oracle parity seed={seed} shape={shape}")
    g, o = build(case)
    g.step(30)
    o.step(30)
    e = compare(g, o, case)
    log(f"[fused]   errors {e}")
    assert e["mask_equal"]
    for k in ("f", "u", "tau", "rho"):
        assert e[k][0] < 1e-5, (k, e[k])
    g.close()


def test_large_box_fused_step_on_request(monkeypatch):
    """The 256^3 box with 64 fixed spheres runs the fused kernel when
    VLB_FUSED=1 (no separate stress-update launch), the two kernels by
    default, and both give the same bits."""
    shape = (256, 256, 256)
    spheres = inputs.place_spheres(4, 0, shape, 64, 6.0, 6.0, min_gap=2.0, periodic=(1, 1, 1))
    out = []
    for mode in ("1", None):
        if mode is None:
            monkeypatch.delenv("VLB_FUSED", raising=False)
        else:
            monkeypatch.setenv("VLB_FUSED", mode)
        log(f"[fused] 256^3 VLB_FUSED={mode}")
        L = vlb.Lattice(shape, np.zeros(shape[::-1], np.uint8), (1, 1, 1))
        L.set_params(eta=1 / 3, beta=0.5, lambda_p=1000.0, magic=3 / 16,
                     body_force=(1e-6, 0, 0))
        for c, r in spheres:
            L.add_sphere(center=c, radius=r)
        L.set_check_interval(0)
        L.init_equilibrium()
        L.set_timing(True)
        L.step(3)
        fused = L.kernel_time_ms(1) < 0
        assert fused == (mode == "1")
        L.set_timing(False)
        L.step(4)
        out.append((L.stress(), L.velocity()))
        L.close()
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
