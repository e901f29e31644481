"""Plain FP64 CPU oracle (test infrastructure only).

The slow, obviously correct reference implementation of the lattice
Boltzmann + Oldroyd-B method of arXiv 2009.12279 (Sections 3.1, 3.3, 3.4).
Only the tests, the smoke check and the CPU-baseline leg of the benchmark
load it; the GPU library never does.  ``build()`` compiles ``oracle.c`` into
``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

Q = 19


def build() -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O3", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", tmp, src, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.c_int
        L.or_create.restype = P
        L.or_create.argtypes = [I, I, I, ctypes.POINTER(I), ctypes.c_char_p, D, I]
        L.or_destroy.argtypes = [P]
        L.or_set_params.restype = I
        L.or_set_params.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, D]
        L.or_set_counter_force.argtypes = [P, I]
        L.or_set_giesekus.restype = I
        L.or_set_giesekus.argtypes = [P, ctypes.c_double]
        L.or_set_fene_p.restype = I
        L.or_set_fene_p.argtypes = [P, ctypes.c_double]
        L.or_init_equilibrium.argtypes = [P, D]
        L.or_set_populations.argtypes = [P, D]
        L.or_set_stress.argtypes = [P, D]
        L.or_add_sphere.restype = I
        L.or_add_sphere.argtypes = [P, D, ctypes.c_double, ctypes.c_double, I, D, D]
        L.or_step.argtypes = [P, ctypes.c_long]
        for name in ("or_read_populations", "or_read_stress", "or_read_density",
                     "or_read_velocity"):
            getattr(L, name).argtypes = [P, D]
        L.or_read_mask.argtypes = [P, ctypes.c_char_p]
        L.or_read_particle.argtypes = [P, I, D, D, D, D, D]
        L.or_read_particle_parts.argtypes = [P, I, D, D, D]
        L.or_read_sums.argtypes = [P, D, D]
        L.or_read_wall_force.argtypes = [P, D]
        L.or_read_pending_conversion.argtypes = [P, D]
        L.or_read_dropped_stress.argtypes = [P, D]
        L.or_read_conversion_stats.argtypes = [P, ctypes.POINTER(I), D, D]
        L.or_step_count.restype = ctypes.c_long
        L.or_step_count.argtypes = [P]
        L.or_velocity.restype = I
        L.or_velocity.argtypes = [I, ctypes.POINTER(I), D]
        L.or_equilibrium.argtypes = [ctypes.c_double, D, D]
        L.or_collide_cell.argtypes = [D, D, ctypes.c_double, ctypes.c_double, D, D, D]
        L.or_rates.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, D, D]
        L.or_fv_apply.argtypes = [I, I, I, ctypes.c_char_p, D, D, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, D]
        L.or_polymer_force.argtypes = [I, I, I, ctypes.c_char_p, D, D]
        L.or_polymer_force_ext.argtypes = [I, I, I, ctypes.c_char_p, D, I, D]
        L.or_set_extrapolation.restype = I
        L.or_set_wall_velocity_field.argtypes = [P, D]
        L.or_set_force_field.argtypes = [P, D]
        L.or_set_extrapolation.argtypes = [P, I]
        L.or_set_conversion_smoothing.restype = I
        L.or_set_conversion_smoothing.argtypes = [P, I]
        L.or_overlap_fraction.restype = ctypes.c_double
        L.or_overlap_fraction.argtypes = [P, I, I, I, I, I]
        L.or_set_threads.argtypes = [I]
        L.or_get_threads.restype = I
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(v, n=3):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))


def velocities():
    """(c[19,3] int, w[19]) in the oracle's own direction order."""
    L = lib()
    c = np.zeros((Q, 3), dtype=np.int64)
    w = np.zeros(Q)
    ci = (ctypes.c_int * 3)()
    wd = ctypes.c_double()
    for i in range(Q):
        L.or_velocity(i, ci, ctypes.byref(wd))
        c[i] = list(ci)
        w[i] = wd.value
    return c, w


def equilibrium(rho, u):
    out = np.zeros(Q)
    lib().or_equilibrium(float(rho), _dp(_vec(u)), _dp(out))
    return out


def collide_cell(f, F, omega_plus, omega_minus):
    f = _vec(f, Q)
    out = np.zeros(Q)
    rho = ctypes.c_double()
    u = np.zeros(3)
    lib().or_collide_cell(_dp(f), _dp(_vec(F)), float(omega_plus), float(omega_minus), _dp(out),
                          ctypes.cast(ctypes.pointer(rho), ctypes.POINTER(ctypes.c_double)),
                          _dp(u))
    return out, rho.value, u


def rates(eta, beta, magic):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().or_rates(float(eta), float(beta), float(magic),
                   ctypes.cast(ctypes.pointer(a), ctypes.POINTER(ctypes.c_double)),
                   ctypes.cast(ctypes.pointer(b), ctypes.POINTER(ctypes.c_double)))
    return a.value, b.value


def fv_apply(mask, tau, u, eta_p, lambda_p, alpha=0.0, L2=0.0):
    """One finite-volume stress update with a prescribed velocity field
    (alpha > 0: Giesekus source term).

    mask: uint8 [nz, ny, nx]; tau: [6, nz, ny, nx]; u: [3, nz, ny, nx]."""
    nz, ny, nx = mask.shape
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    t = np.ascontiguousarray(tau, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(t)
    lib().or_fv_apply(nx, ny, nz, m.tobytes(), _dp(t), _dp(uu), float(eta_p), float(lambda_p),
                      float(alpha), float(L2), _dp(out))
    return out


def polymer_force(mask, tau, order=0):
    """Discrete polymer force; `order` of the extrapolation into solid face
    neighbours (0 constant, 1 linear, 2 quadratic)."""
    nz, ny, nx = mask.shape
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    t = np.ascontiguousarray(tau, dtype=np.float64)
    out = np.zeros((3,) + mask.shape)
    lib().or_polymer_force_ext(nx, ny, nz, m.tobytes(), _dp(t), int(order), _dp(out))
    return out


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


class Lattice:
    """FP64 reference lattice.  Fields are numpy arrays shaped [k, nz, ny, nx]."""

    def __init__(self, shape, mask=None, periodic=(1, 1, 1), wall_velocity=None):
        nx, ny, nz = shape
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        if mask is None:
            mask = np.zeros((nz, ny, nx), dtype=np.uint8)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == (nz, ny, nx)
        per = (ctypes.c_int * 3)(*[int(bool(p)) for p in periodic])
        wv = np.zeros(3) if wall_velocity is None else np.ascontiguousarray(
            wall_velocity, dtype=np.float64).reshape(-1)
        nw = 0 if wall_velocity is None else wv.size // 3
        self._h = lib().or_create(nx, ny, nz, per, mask.tobytes(), _dp(wv), nw)
        if not self._h:
            raise ValueError("oracle: invalid lattice")

    def close(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    __del__ = close

    def _f(self, k):
        nx, ny, nz = self.shape
        return np.zeros((k, nz, ny, nx))

    def set_params(self, eta=1.0 / 3.0, beta=0.0, lambda_p=1.0, magic=3.0 / 16.0,
                   body_force=(0.0, 0.0, 0.0)):
        rc = lib().or_set_params(self._h, eta, beta, lambda_p, magic, _dp(_vec(body_force)))
        if rc != 0:
            raise ValueError("oracle: invalid parameters")

    def set_counter_force(self, on=True):
        lib().or_set_counter_force(self._h, 1 if on else 0)

    def set_giesekus(self, alpha):
        if lib().or_set_giesekus(self._h, float(alpha)) != 0:
            raise ValueError("oracle: Giesekus mobility must lie in [0, 1/2]")

    def set_force_field(self, F):
        """Per-cell force density added to the body force, shape
        (3, nz, ny, nx); None removes it."""
        if F is None:
            lib().or_set_force_field(self._h, None)
        else:
            F = np.ascontiguousarray(F, dtype=np.float64)
            nx, ny, nz = self.shape
            assert F.shape == (3, nz, ny, nx)
            lib().or_set_force_field(self._h, _dp(F))

    def set_wall_velocity_field(self, u):
        """Per-cell wall velocity, shape (3, nz, ny, nx); None returns to
        the per-id table."""
        if u is None:
            lib().or_set_wall_velocity_field(self._h, None)
        else:
            u = np.ascontiguousarray(u, dtype=np.float64)
            nx, ny, nz = self.shape
            assert u.shape == (3, nz, ny, nx)
            lib().or_set_wall_velocity_field(self._h, _dp(u))

    def set_extrapolation(self, order):
        if lib().or_set_extrapolation(self._h, int(order)) != 0:
            raise ValueError("oracle: extrapolation order must be 0, 1 or 2")

    def set_fene_p(self, L2):
        if lib().or_set_fene_p(self._h, float(L2)) != 0:
            raise ValueError("oracle: FENE-P needs L^2 > 3 (or 0 for off)")

    def set_conversion_smoothing(self, samples):
        """Overlap-fraction smoothing of conversions with samples^3
        sub-samples per cell (0: binary conversion)."""
        if lib().or_set_conversion_smoothing(self._h, int(samples)) != 0:
            raise ValueError("oracle: smoothing samples must lie in 0..8")

    def overlap_fraction(self, pid, x, y, z, samples):
        return float(lib().or_overlap_fraction(self._h, int(pid), int(x), int(y), int(z),
                                               int(samples)))

    def init_equilibrium(self, u=None):
        if u is None:
            lib().or_init_equilibrium(self._h, None)
        else:
            lib().or_init_equilibrium(self._h, _dp(np.ascontiguousarray(u, dtype=np.float64)))

    def set_populations(self, f):
        lib().or_set_populations(self._h, _dp(np.ascontiguousarray(f, dtype=np.float64)))

    def set_stress(self, tau):
        lib().or_set_stress(self._h, _dp(np.ascontiguousarray(tau, dtype=np.float64)))

    def add_sphere(self, center, radius, density_ratio=1.0, movable=False, f_ext=(0, 0, 0),
                   t_ext=(0, 0, 0)):
        pid = lib().or_add_sphere(self._h, _dp(_vec(center)), float(radius),
                                  float(density_ratio), int(bool(movable)), _dp(_vec(f_ext)),
                                  _dp(_vec(t_ext)))
        if pid < 0:
            raise ValueError("oracle: sphere overlaps a non-fluid cell")
        return pid

    def step(self, n=1):
        lib().or_step(self._h, int(n))

    def populations(self):
        out = self._f(Q)
        lib().or_read_populations(self._h, _dp(out))
        return out

    def stress(self):
        out = self._f(6)
        lib().or_read_stress(self._h, _dp(out))
        return out

    def density(self):
        out = self._f(1)
        lib().or_read_density(self._h, _dp(out))
        return out[0]

    def velocity(self):
        out = self._f(3)
        lib().or_read_velocity(self._h, _dp(out))
        return out

    def mask(self):
        nx, ny, nz = self.shape
        buf = ctypes.create_string_buffer(self.N)
        lib().or_read_mask(self._h, buf)
        return np.frombuffer(buf.raw, dtype=np.uint8).reshape(nz, ny, nx).copy()

    def particle(self, pid):
        arrs = [np.zeros(3) for _ in range(5)]
        lib().or_read_particle(self._h, int(pid), *[_dp(a) for a in arrs])
        return dict(zip(("pos", "vel", "omega", "force", "torque"), arrs))

    def particle_parts(self, pid):
        arrs = [np.zeros(3) for _ in range(3)]
        lib().or_read_particle_parts(self._h, int(pid), *[_dp(a) for a in arrs])
        return dict(zip(("mex", "traction", "conversion"), arrs))

    def sums(self):
        m = np.zeros(1)
        p = np.zeros(3)
        lib().or_read_sums(self._h, _dp(m), _dp(p))
        return float(m[0]), p

    def wall_force(self):
        out = np.zeros(3)
        lib().or_read_wall_force(self._h, _dp(out))
        return out

    def pending_conversion(self):
        out = np.zeros(3)
        lib().or_read_pending_conversion(self._h, _dp(out))
        return out

    def dropped_stress(self):
        out = np.zeros(6)
        lib().or_read_dropped_stress(self._h, _dp(out))
        return out

    def conversion_stats(self):
        counts = (ctypes.c_int * 2)()
        before = np.zeros(6)
        after = np.zeros(6)
        lib().or_read_conversion_stats(self._h, counts, _dp(before), _dp(after))
        return (counts[0], counts[1]), before, after

    @property
    def step_count(self):
        return int(lib().or_step_count(self._h))
