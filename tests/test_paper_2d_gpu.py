"""The paper's two-dimensional benchmarks (Sections 4.1 and 4.2) on the GPU,
on lattices one cell thick (the D2Q9 / D2Q5 reduction the oracle tests pin):
the Reynolds number of start-up Poiseuille flow and the first normal stress
difference of steady shear flow, against the values the paper states and
against the oracle."""
import json
import os

import numpy as np
import pytest

from paper_2009_12279_amd import inputs
from parity import Case, build, compare, log

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_startup_poiseuille_reynolds_number():
    gold = json.load(open(os.path.join(GOLDEN, "poiseuille_startup.json")))
    Lw, F, eta = gold["L"], gold["F"], gold["eta"]
    shape = (1, Lw + 2, 1)
    mask = inputs.channel_mask(shape, wall_axes=(1,))
    case = Case("poiseuille-2d", shape, mask, (1, 0, 1), None,
                dict(eta=eta, beta=0.0, lambda_p=1.0, magic=3 / 16, body_force=(F, 0, 0)))
    log("[paper-2d] start-up Poiseuille, L = 28, 6000 steps")
    g, o = build(case)
    g.step(6000)
    o.step(6000)
    ux = g.velocity()[0, 0, :, 0]
    centre = 0.5 * (ux[Lw // 2] + ux[Lw // 2 + 1])
    Re = centre * Lw / eta
    log(f"[paper-2d]   Re = {Re:.5f} (paper: {gold['Re_quoted']})")
    assert abs(Re - gold["Re_quoted"]) < gold["Re_rounding"]
    e = compare(g, o, case, what=("u",))
    assert e["u"][0] < 1e-5, e


@pytest.mark.parametrize("case_i", [0, 1])
def test_steady_shear_first_normal_stress_difference(case_i):
    gold = json.load(open(os.path.join(GOLDEN, "couette_steady_shear.json")))
    c = gold["cases"][case_i]
    Lw, u0, eta = gold["L"], gold["u0"], gold["eta"]
    beta, lam = c["beta"], float(c["lambda_p"])
    shape = (1, Lw + 2, 1)
    mask = inputs.channel_mask(shape, wall_axes=(1,), top_id=2)
    case = Case("couette-2d", shape, mask, (1, 0, 1), [[0, 0, 0], [u0, 0, 0]],
                dict(eta=eta, beta=beta, lambda_p=lam, magic=3 / 16))
    steps = int(gold["run_lambdas"] * lam)
    log(f"[paper-2d] steady shear beta={beta} lambda={lam}, {steps} steps")
    g, o = build(case)
    g.step(steps)
    o.step(steps)
    u, tau = g.velocity(), g.stress()
    ux = u[0, 0, 1:-1, 0]
    txx, tyy, txy = (tau[k, 0, 1:-1, 0] for k in (0, 1, 3))
    eta_p = beta * eta
    bulk = slice(6, -6)
    slope = np.polyfit(np.arange(Lw)[bulk], ux[bulk], 1)[0]
    L_eff = u0 / slope
    N1 = (txx - tyy)[bulk]
    rel = np.max(np.abs(N1 / (2 * eta_p * lam * (u0 / L_eff) ** 2) - 1))
    log(f"[paper-2d]   L_eff = {L_eff:.3f}, bulk N1 deviation {rel:.2e} "
        f"(paper: {gold['N1_rel_tol_bulk']})")
    assert abs(L_eff - Lw) < 0.6
    assert rel < gold["N1_rel_tol_bulk"]
    e = compare(g, o, case, what=("u", "tau"))
    log(f"[paper-2d]   vs oracle {e}")
    assert e["u"][0] < 1e-5 and e["tau"][0] < 1e-5
