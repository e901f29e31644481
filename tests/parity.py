"""Helpers for GPU-vs-oracle parity: build the same seeded case on both sides,
step both, and compare fields over fluid cells."""
from __future__ import annotations

import sys
from dataclasses import dataclass, field

import numpy as np

import oracle
from paper_2009_12279_amd import vlb


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def public_from_oracle_perm():
    """perm[i] = oracle index of public direction i (matched by velocity)."""
    c_or, _ = oracle.velocities()
    perm = []
    for i in range(19):
        c, _ = vlb.vlb_velocity(i)
        perm.append(int(np.where((c_or == np.array(c)).all(1))[0][0]))
    return np.array(perm)


@dataclass
class Case:
    name: str
    shape: tuple
    mask: np.ndarray
    periodic: tuple = (1, 1, 1)
    wall_velocity: object = None
    params: dict = field(default_factory=dict)
    spheres: list = field(default_factory=list)   # dicts for add_sphere
    u0: object = None                             # [3,nz,ny,nx] or None
    f0: object = None                             # raw populations, public order
    tau0: object = None


def build(case: Case, storage="f32", threads=None):
    """(gpu Lattice, oracle Lattice) set up identically."""
    if threads:
        oracle.set_threads(threads)
    g = vlb.Lattice(case.shape, case.mask, case.periodic, case.wall_velocity, storage=storage)
    o = oracle.Lattice(case.shape, case.mask, case.periodic, case.wall_velocity)
    g.set_params(**case.params)
    o.set_params(**case.params)
    g.set_check_interval(0)
    for s in case.spheres:
        pg = g.add_sphere(**s)
        po = o.add_sphere(**s)
        assert pg == po
    if case.f0 is not None:
        perm = public_from_oracle_perm()
        f_or = np.empty_like(case.f0)
        f_or[perm] = case.f0
        g.set_populations(case.f0)
        o.set_populations(f_or)
    else:
        g.init_equilibrium(case.u0)
        o.init_equilibrium(case.u0)
    if case.tau0 is not None:
        g.set_stress(case.tau0)
        o.set_stress(case.tau0)
    return g, o


def rel_err(a, b, fluid):
    """(max|a-b| / max|b|, ||a-b||_2 / ||b||_2) over fluid cells, all components."""
    da = a[..., fluid] if a.ndim == 4 else a[fluid]
    db = b[..., fluid] if b.ndim == 4 else b[fluid]
    scale_max = np.max(np.abs(db))
    scale_l2 = np.sqrt(np.sum(db ** 2))
    if scale_max == 0:
        return float(np.max(np.abs(da))), float(np.sqrt(np.sum(da ** 2)))
    return float(np.max(np.abs(da - db)) / scale_max), float(np.sqrt(np.sum((da - db) ** 2)) / scale_l2)


def compare(g, o, case: Case, what=("u", "tau", "rho", "f")):
    """Per-field errors of the GPU state against the oracle state."""
    mask_g = g.mask()
    mask_o = o.mask()
    out = {"mask_equal": bool(np.array_equal(mask_g, mask_o))}
    fluid = mask_o == 0
    if "u" in what:
        out["u"] = rel_err(g.velocity(), o.velocity(), fluid)
    if "tau" in what:
        out["tau"] = rel_err(g.stress(), o.stress(), fluid)
    if "rho" in what:
        # compare density deviations from 1
        out["rho"] = rel_err(g.density() - 1.0, o.density() - 1.0, fluid)
    if "f" in what:
        perm = public_from_oracle_perm()
        c, w = zip(*[vlb.vlb_velocity(i) for i in range(19)])
        w = np.array(w)[:, None, None, None]
        fo = o.populations()[perm]
        out["f"] = rel_err(g.populations() - w, fo - w, fluid)
    return out
