"""Thin ctypes binding of libvlb (include/vlb.h).

Module-level functions carry the C names and only marshal arguments; every
step of the method runs in the gfx950 kernels of ``libvlb.so``.  ``Lattice``
is a small convenience wrapper over them.  There is no fallback: if the
library is missing or no HIP device is present the calls raise.

Fields are numpy float64 arrays shaped [k, nz, ny, nx] (x fastest), masks
uint8 [nz, ny, nx].  Populations use the order of ``vlb_velocity``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VLB_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("VLB_LIBRARY") or os.path.join(_HERE, "libvlb.so")
Q = 19

VLB_OK, VLB_EINVAL, VLB_ENOMEM, VLB_EDEVICE, VLB_EUNSTABLE, VLB_ESTATE, VLB_EBUSY, \
    VLB_ENOTFOUND = range(8)
STATUS_NAMES = {0: "VLB_OK", 1: "VLB_EINVAL", 2: "VLB_ENOMEM", 3: "VLB_EDEVICE",
                4: "VLB_EUNSTABLE", 5: "VLB_ESTATE", 6: "VLB_EBUSY", 7: "VLB_ENOTFOUND"}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}


class VlbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class vlb_dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic", ctypes.c_uint8 * 3), ("reserved", ctypes.c_uint8)]


class vlb_params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("beta", ctypes.c_double),
                ("lambda_p", ctypes.c_double), ("magic", ctypes.c_double),
                ("body_force", ctypes.c_double * 3)]


class vlb_request(ctypes.Structure):
    _fields_ = [("dims", vlb_dims), ("mask", ctypes.c_char_p), ("params", vlb_params),
                ("n_spheres", ctypes.c_int32), ("spheres", ctypes.POINTER(ctypes.c_double)),
                ("n_steps", ctypes.c_int64), ("seed", ctypes.c_uint32),
                ("giesekus_alpha", ctypes.c_double), ("n_walls", ctypes.c_int32),
                ("wall_velocity", ctypes.POINTER(ctypes.c_double))]


class vlb_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("graph_captures", ctypes.c_int64),
                ("graph_updates", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_uint64), ("cell_steps_launched", ctypes.c_uint64)]


REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "cancelled", 4: "failed"}

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_P = ctypes.c_void_p

# (name, restype, argtypes) of every exported function of include/vlb.h
SIGNATURES = [
    ("vlb_velocity", ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _D]),
    ("vlb_required_bytes", ctypes.c_size_t, [ctypes.POINTER(vlb_dims), ctypes.c_int, ctypes.c_int32]),
    ("vlb_create", ctypes.c_int, [ctypes.POINTER(vlb_dims), ctypes.c_char_p, _D, ctypes.c_int32,
                                  ctypes.c_int, _P, ctypes.POINTER(_P)]),
    ("vlb_buffer_sizes", ctypes.c_int, [ctypes.POINTER(vlb_dims), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    ("vlb_create_with_buffers", ctypes.c_int, [ctypes.POINTER(vlb_dims), ctypes.c_char_p, _D,
                                               ctypes.c_int32, ctypes.c_int, _P,
                                               ctypes.POINTER(ctypes.c_void_p),
                                               ctypes.POINTER(ctypes.c_size_t),
                                               ctypes.POINTER(_P)]),
    ("vlb_set_params", ctypes.c_int, [_P, ctypes.POINTER(vlb_params)]),
    ("vlb_init_equilibrium", ctypes.c_int, [_P, _D]),
    ("vlb_set_populations", ctypes.c_int, [_P, _D]),
    ("vlb_set_stress", ctypes.c_int, [_P, _D]),
    ("vlb_add_sphere", ctypes.c_int, [_P, _D, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      _D, _D, ctypes.POINTER(ctypes.c_int32)]),
    ("vlb_step", ctypes.c_int, [_P, ctypes.c_int64]),
    ("vlb_sync", ctypes.c_int, [_P]),
    ("vlb_step_count", ctypes.c_int64, [_P]),
    ("vlb_read_density", ctypes.c_int, [_P, _D]),
    ("vlb_read_velocity", ctypes.c_int, [_P, _D]),
    ("vlb_read_velocity_noalloc", ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _D]),
    ("vlb_read_stress", ctypes.c_int, [_P, _D]),
    ("vlb_read_populations", ctypes.c_int, [_P, _D]),
    ("vlb_read_mask", ctypes.c_int, [_P, ctypes.c_char_p]),
    ("vlb_read_particle", ctypes.c_int, [_P, ctypes.c_int32, _D, _D, _D, _D, _D]),
    ("vlb_read_sums", ctypes.c_int, [_P, _D, _D]),
    ("vlb_read_wall_force", ctypes.c_int, [_P, _D]),
    ("vlb_check_health", ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    ("vlb_set_check_interval", ctypes.c_int, [_P, ctypes.c_int64]),
    ("vlb_save", ctypes.c_int, [_P, ctypes.c_char_p]),
    ("vlb_load", ctypes.c_int, [ctypes.c_char_p, _P, ctypes.POINTER(_P)]),
    ("vlb_destroy", None, [_P]),
    ("vlb_last_error", ctypes.c_char_p, [_P]),
    ("vlb_set_timing", ctypes.c_int, [_P, ctypes.c_int32]),
    ("vlb_kernel_time_ms", ctypes.c_double, [_P, ctypes.c_int32]),
    ("vlb_set_rounding", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_uint32]),
    ("vlb_set_velocity_scale", ctypes.c_int, [_P, ctypes.c_double]),
    ("vlb_storage_scale", ctypes.c_double, [_P]),
    ("vlb_set_raw_f32_control", ctypes.c_int, [_P, ctypes.c_int32]),
    ("vlb_set_counter_force", ctypes.c_int, [_P, ctypes.c_int32]),
    ("vlb_set_conversion_smoothing", ctypes.c_int, [_P, ctypes.c_int32]),
    ("vlb_set_giesekus", ctypes.c_int, [_P, ctypes.c_double]),
    ("vlb_set_fene_p", ctypes.c_int, [_P, ctypes.c_double]),
    ("vlb_set_stress_extrapolation", ctypes.c_int, [_P, ctypes.c_int32]),
    ("vlb_set_wall_velocity_field", ctypes.c_int, [_P, _D]),
    ("vlb_set_force_field", ctypes.c_int, [_P, _D]),
    ("vlb_server_create", ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _P,
                                         ctypes.POINTER(_P)]),
    ("vlb_server_set_rounding", ctypes.c_int, [_P, ctypes.c_int]),
    ("vlb_server_request_bytes", ctypes.c_size_t, [ctypes.POINTER(vlb_dims)]),
    ("vlb_server_set_policy", ctypes.c_int, [_P, ctypes.c_int]),
    ("vlb_server_submit", ctypes.c_int, [_P, ctypes.POINTER(vlb_request),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    ("vlb_server_pump", ctypes.c_int, [_P, ctypes.c_int32]),
    ("vlb_server_poll", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    ("vlb_server_result", ctypes.c_int, [_P, ctypes.c_uint64, _D, _D, _D]),
    ("vlb_server_cancel", ctypes.c_int, [_P, ctypes.c_uint64]),
    ("vlb_server_stats_get", ctypes.c_int, [_P, ctypes.POINTER(vlb_server_stats)]),
    ("vlb_server_last_error", ctypes.c_char_p, [_P]),
    ("vlb_server_destroy", None, [_P]),
]


def lib():
    """Load libvlb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libvlb.so not built at {LIB_PATH}; run __graft_entry__.build()")
        # One HIP runtime per process: torch ships its own libamdhip64 under
        # the same soname, so it is loaded first and libvlb binds to it; the
        # other order leaves torch without a usable device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _vec(v, n=3):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))


def _check(status, handle=None):
    if status != VLB_OK:
        msg = lib().vlb_last_error(handle)
        raise VlbError(status, msg.decode() if msg else "")
    return status


# ---- C-named wrappers -------------------------------------------------------

def vlb_velocity(i):
    c = (ctypes.c_int32 * 3)()
    w = ctypes.c_double()
    lib().vlb_velocity(int(i), c, ctypes.byref(w))
    return (c[0], c[1], c[2]), w.value


def make_dims(shape, periodic):
    d = vlb_dims()
    d.nx, d.ny, d.nz = (int(s) for s in shape)
    for a in range(3):
        d.periodic[a] = 1 if periodic[a] else 0
    return d


def vlb_required_bytes(shape, periodic=(1, 1, 1), storage="f32", n_particles=0):
    d = make_dims(shape, periodic)
    return int(lib().vlb_required_bytes(ctypes.byref(d), STORAGE[storage], int(n_particles)))


def vlb_create(shape, mask, periodic=(1, 1, 1), wall_velocity=None, storage="f32", stream=None):
    nx, ny, nz = shape
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.shape != (nz, ny, nx):
        raise ValueError("mask must be shaped [nz, ny, nx]")
    d = make_dims(shape, periodic)
    wv = None
    nw = 0
    if wall_velocity is not None:
        wv = np.ascontiguousarray(wall_velocity, dtype=np.float64).reshape(-1)
        nw = wv.size // 3
    h = _P()
    st = lib().vlb_create(ctypes.byref(d), m.tobytes(), None if wv is None else _dp(wv), nw,
                          STORAGE[storage], None if stream is None else _P(int(stream)),
                          ctypes.byref(h))
    _check(st, None)
    return h


NBUF = 6
NOALLOC_MAX_CELLS = 262144  # staging size of vlb_read_velocity_noalloc, in cells


def vlb_buffer_sizes(shape, periodic=(1, 1, 1), storage="f32"):
    """Bytes of the caller-providable state buffers (mask, 2 x populations,
    2 x stress, velocity)."""
    d = make_dims(shape, periodic)
    sizes = (ctypes.c_size_t * NBUF)()
    _check(lib().vlb_buffer_sizes(ctypes.byref(d), STORAGE[storage], sizes), None)
    return [int(v) for v in sizes]


def vlb_create_with_buffers(shape, mask, buffers, sizes, periodic=(1, 1, 1), wall_velocity=None,
                            storage="f32", stream=None):
    """vlb_create with caller-owned device buffers (pointers as integers)."""
    nx, ny, nz = shape
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.shape != (nz, ny, nx):
        raise ValueError("mask must be shaped [nz, ny, nx]")
    d = make_dims(shape, periodic)
    wv = None
    nw = 0
    if wall_velocity is not None:
        wv = np.ascontiguousarray(wall_velocity, dtype=np.float64).reshape(-1)
        nw = wv.size // 3
    bufs = (ctypes.c_void_p * NBUF)(*[int(b) for b in buffers])
    szs = (ctypes.c_size_t * NBUF)(*[int(v) for v in sizes])
    h = _P()
    st = lib().vlb_create_with_buffers(ctypes.byref(d), m.tobytes(),
                                       None if wv is None else _dp(wv), nw, STORAGE[storage],
                                       None if stream is None else _P(int(stream)), bufs, szs,
                                       ctypes.byref(h))
    _check(st, None)
    return h


def vlb_set_params(h, eta=1.0 / 3.0, beta=0.0, lambda_p=1.0, magic=3.0 / 16.0,
                   body_force=(0.0, 0.0, 0.0)):
    p = vlb_params()
    p.eta, p.beta, p.lambda_p, p.magic = float(eta), float(beta), float(lambda_p), float(magic)
    for a in range(3):
        p.body_force[a] = float(body_force[a])
    return _check(lib().vlb_set_params(h, ctypes.byref(p)), h)


def vlb_init_equilibrium(h, u=None):
    if u is None:
        return _check(lib().vlb_init_equilibrium(h, None), h)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    return _check(lib().vlb_init_equilibrium(h, _dp(uu)), h)


def vlb_set_populations(h, f):
    ff = np.ascontiguousarray(f, dtype=np.float64)
    return _check(lib().vlb_set_populations(h, _dp(ff)), h)


def vlb_set_stress(h, tau):
    t = np.ascontiguousarray(tau, dtype=np.float64)
    return _check(lib().vlb_set_stress(h, _dp(t)), h)


def vlb_add_sphere(h, center, radius, density_ratio=1.0, movable=False, f_ext=(0, 0, 0),
                   t_ext=(0, 0, 0)):
    pid = ctypes.c_int32()
    _check(lib().vlb_add_sphere(h, _dp(_vec(center)), float(radius), float(density_ratio),
                                int(bool(movable)), _dp(_vec(f_ext)), _dp(_vec(t_ext)),
                                ctypes.byref(pid)), h)
    return pid.value


def vlb_step(h, n=1):
    return _check(lib().vlb_step(h, int(n)), h)


def vlb_sync(h):
    return _check(lib().vlb_sync(h), h)


def vlb_step_count(h):
    return int(lib().vlb_step_count(h))


def _read(fn, h, shape_k, shape):
    nx, ny, nz = shape
    out = np.zeros((shape_k, nz, ny, nx))
    _check(fn(h, _dp(out)), h)
    return out


def vlb_read_density(h, shape):
    return _read(lib().vlb_read_density, h, 1, shape)[0]


def vlb_read_velocity(h, shape):
    return _read(lib().vlb_read_velocity, h, 3, shape)


def vlb_read_velocity_noalloc(h, first, count):
    """Velocity of cells first .. first + count - 1 as an array [3, count]."""
    out = np.zeros((3, int(count)))
    _check(lib().vlb_read_velocity_noalloc(h, int(first), int(count), _dp(out)), h)
    return out


def vlb_read_stress(h, shape):
    return _read(lib().vlb_read_stress, h, 6, shape)


def vlb_read_populations(h, shape):
    return _read(lib().vlb_read_populations, h, Q, shape)


def vlb_read_mask(h, shape):
    nx, ny, nz = shape
    buf = ctypes.create_string_buffer(nx * ny * nz)
    _check(lib().vlb_read_mask(h, buf), h)
    return np.frombuffer(buf.raw, dtype=np.uint8).reshape(nz, ny, nx).copy()


def vlb_read_particle(h, pid):
    arrs = [np.zeros(3) for _ in range(5)]
    _check(lib().vlb_read_particle(h, int(pid), *[_dp(a) for a in arrs]), h)
    return dict(zip(("pos", "vel", "omega", "force", "torque"), arrs))


def vlb_read_sums(h):
    m = np.zeros(1)
    p = np.zeros(3)
    _check(lib().vlb_read_sums(h, _dp(m), _dp(p)), h)
    return float(m[0]), p


def vlb_read_wall_force(h):
    out = np.zeros(3)
    _check(lib().vlb_read_wall_force(h, _dp(out)), h)
    return out


def vlb_check_health(h, raise_on_unstable=True):
    sp = np.zeros(1)
    bad = ctypes.c_int64()
    st = lib().vlb_check_health(h, _dp(sp), ctypes.byref(bad))
    if raise_on_unstable:
        _check(st, h)
    return st, float(sp[0]), int(bad.value)


def vlb_set_check_interval(h, steps):
    return _check(lib().vlb_set_check_interval(h, int(steps)), h)


def vlb_save(h, path):
    return _check(lib().vlb_save(h, os.fsencode(path)), h)


def vlb_load(path, stream=None):
    h = _P()
    _check(lib().vlb_load(os.fsencode(path), None if stream is None else _P(int(stream)),
                          ctypes.byref(h)), None)
    return h


def vlb_destroy(h):
    lib().vlb_destroy(h)


def vlb_last_error(h=None):
    return lib().vlb_last_error(h).decode()


def vlb_set_timing(h, on=True):
    return _check(lib().vlb_set_timing(h, int(bool(on))), h)


def vlb_kernel_time_ms(h, which):
    return float(lib().vlb_kernel_time_ms(h, int(which)))


ROUNDING = {"nearest": 0, "stochastic": 1}


def vlb_set_giesekus(h, alpha):
    return _check(lib().vlb_set_giesekus(h, float(alpha)), h)


def vlb_set_fene_p(h, L2):
    return _check(lib().vlb_set_fene_p(h, float(L2)), h)


def vlb_set_conversion_smoothing(h, samples):
    return _check(lib().vlb_set_conversion_smoothing(h, int(samples)), h)


def vlb_set_stress_extrapolation(h, order):
    return _check(lib().vlb_set_stress_extrapolation(h, int(order)), h)


def vlb_set_wall_velocity_field(h, u):
    return _check(lib().vlb_set_wall_velocity_field(h, u), h)


def vlb_set_force_field(h, F):
    return _check(lib().vlb_set_force_field(h, F), h)


def vlb_set_counter_force(h, on=True):
    return _check(lib().vlb_set_counter_force(h, 1 if on else 0), h)


def vlb_set_rounding(h, mode="stochastic", seed=0x2009):
    return _check(lib().vlb_set_rounding(h, ROUNDING[mode], int(seed) & 0xFFFFFFFF), h)


def vlb_set_velocity_scale(h, u_max):
    return _check(lib().vlb_set_velocity_scale(h, float(u_max)), h)


def vlb_storage_scale(h):
    return float(lib().vlb_storage_scale(h))


def vlb_set_raw_f32_control(h, on=True):
    return _check(lib().vlb_set_raw_f32_control(h, 1 if on else 0), h)


# ---- convenience wrapper ------------------------------------------------------

class Lattice:
    """One lattice on the current HIP device (owner of the C handle)."""

    def __init__(self, shape, mask=None, periodic=(1, 1, 1), wall_velocity=None, storage="f32",
                 stream=None, _handle=None, torch_buffers=False):
        """torch_buffers=True keeps the state in torch-allocated device tensors
        (held by this object) instead of library allocations."""
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self._buffers = None
        if _handle is not None:
            self._h = _handle
            return
        if mask is None:
            mask = np.zeros((nz, ny, nx), dtype=np.uint8)
        if torch_buffers:
            import torch

            sizes = vlb_buffer_sizes(self.shape, periodic, storage)
            # torch's caching allocator hands out 512-byte aligned blocks
            self._buffers = [torch.empty(n, dtype=torch.uint8, device="cuda") for n in sizes]
            self._h = vlb_create_with_buffers(self.shape, mask, [b.data_ptr() for b in self._buffers],
                                              sizes, periodic, wall_velocity, storage, stream)
        else:
            self._h = vlb_create(self.shape, mask, periodic, wall_velocity, storage, stream)

    @classmethod
    def load(cls, path, shape, stream=None):
        return cls(shape, _handle=vlb_load(path, stream))

    def close(self):
        if getattr(self, "_h", None):
            vlb_destroy(self._h)
            self._h = None
        self._buffers = None  # caller-owned state goes after the lattice

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def set_params(self, **kw):
        vlb_set_params(self._h, **kw)

    def init_equilibrium(self, u=None):
        vlb_init_equilibrium(self._h, u)

    def set_populations(self, f):
        vlb_set_populations(self._h, f)

    def set_stress(self, tau):
        vlb_set_stress(self._h, tau)

    def add_sphere(self, center, radius, density_ratio=1.0, movable=False, f_ext=(0, 0, 0),
                   t_ext=(0, 0, 0)):
        return vlb_add_sphere(self._h, center, radius, density_ratio, movable, f_ext, t_ext)

    def step(self, n=1):
        vlb_step(self._h, n)

    def sync(self):
        vlb_sync(self._h)

    @property
    def step_count(self):
        return vlb_step_count(self._h)

    def density(self):
        return vlb_read_density(self._h, self.shape)

    def velocity(self):
        return vlb_read_velocity(self._h, self.shape)

    def stress(self):
        return vlb_read_stress(self._h, self.shape)

    def populations(self):
        return vlb_read_populations(self._h, self.shape)

    def mask(self):
        return vlb_read_mask(self._h, self.shape)

    def particle(self, pid):
        return vlb_read_particle(self._h, pid)

    def sums(self):
        return vlb_read_sums(self._h)

    def wall_force(self):
        return vlb_read_wall_force(self._h)

    def check_health(self):
        return vlb_check_health(self._h)

    def set_check_interval(self, steps):
        vlb_set_check_interval(self._h, steps)

    def save(self, path):
        vlb_save(self._h, path)

    def set_timing(self, on=True):
        vlb_set_timing(self._h, on)

    def kernel_time_ms(self, which):
        return vlb_kernel_time_ms(self._h, which)

    def set_rounding(self, mode="stochastic", seed=0x2009):
        vlb_set_rounding(self._h, mode, seed)

    def set_counter_force(self, on=True):
        vlb_set_counter_force(self._h, on)

    def set_velocity_scale(self, u_max):
        """FP16 storage scale from the largest expected flow speed."""
        vlb_set_velocity_scale(self._h, u_max)

    @property
    def storage_scale(self):
        return vlb_storage_scale(self._h)

    def set_raw_f32_control(self, on=True):
        """Control experiment: keep the populations on the FP32 grid of f."""
        vlb_set_raw_f32_control(self._h, on)

    def set_giesekus(self, alpha):
        vlb_set_giesekus(self._h, alpha)

    def set_fene_p(self, L2):
        vlb_set_fene_p(self._h, L2)

    def set_extrapolation(self, order):
        vlb_set_stress_extrapolation(self._h, order)

    def set_conversion_smoothing(self, samples):
        """Overlap-fraction smoothing of conversions with samples^3
        sub-samples per cell (0: binary conversion)."""
        vlb_set_conversion_smoothing(self._h, samples)

    def set_force_field(self, F):
        """Per-cell force density added to the body force, shape
        (3, nz, ny, nx), stored in FP32; None removes it."""
        if F is None:
            vlb_set_force_field(self._h, None)
            return
        nx, ny, nz = self.shape
        F = np.ascontiguousarray(F, dtype=np.float64)
        if F.shape != (3, nz, ny, nx):
            raise ValueError(f"force field must have shape {(3, nz, ny, nx)}")
        vlb_set_force_field(self._h, _dp(F))

    def set_wall_velocity_field(self, u):
        """Per-cell wall velocity, shape (3, nz, ny, nx); None returns to the
        per-id wall table."""
        if u is None:
            vlb_set_wall_velocity_field(self._h, None)
            return
        nx, ny, nz = self.shape
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.shape != (3, nz, ny, nx):
            raise ValueError(f"wall velocity field must have shape {(3, nz, ny, nx)}")
        vlb_set_wall_velocity_field(self._h, _dp(u))


# ---- serving ------------------------------------------------------------------

def _scheck(status, srv):
    if status != VLB_OK:
        msg = lib().vlb_server_last_error(srv) if srv else b""
        raise VlbError(status, msg.decode() if msg else "")
    return status


def vlb_server_create(hbm_budget_bytes, max_slots=64, steps_per_launch=50, stream=None):
    h = _P()
    _scheck(lib().vlb_server_create(int(hbm_budget_bytes), int(max_slots), int(steps_per_launch),
                                    None if stream is None else _P(int(stream)),
                                    ctypes.byref(h)), None)
    return h


def vlb_server_request_bytes(shape, periodic=(1, 1, 1)):
    d = make_dims(shape, periodic)
    return int(lib().vlb_server_request_bytes(ctypes.byref(d)))


POLICIES = {"fifo": 0, "shortest_first": 1}


def vlb_server_set_policy(srv, policy="fifo"):
    return _scheck(lib().vlb_server_set_policy(srv, POLICIES[policy]), srv)


def vlb_server_set_rounding(srv, mode="stochastic"):
    return _scheck(lib().vlb_server_set_rounding(srv, ROUNDING[mode]), srv)


def vlb_server_submit(srv, shape, mask, periodic=(1, 1, 1), params=None, spheres=(), n_steps=1,
                      seed=0x2009, giesekus_alpha=0.0, wall_velocity=None):
    nx, ny, nz = shape
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.shape != (nz, ny, nx):
        raise ValueError("mask must be shaped [nz, ny, nx]")
    req = vlb_request()
    req.dims = make_dims(shape, periodic)
    mb = m.tobytes()
    req.mask = mb
    p = vlb_params()
    pr = dict(eta=1.0 / 3.0, beta=0.0, lambda_p=1.0, magic=3.0 / 16.0, body_force=(0, 0, 0))
    pr.update(params or {})
    p.eta, p.beta, p.lambda_p, p.magic = (float(pr[k]) for k in ("eta", "beta", "lambda_p", "magic"))
    for a in range(3):
        p.body_force[a] = float(pr["body_force"][a])
    req.params = p
    sp = np.ascontiguousarray(np.asarray(spheres, dtype=np.float64).reshape(-1, 4)) if len(spheres) \
        else np.zeros((0, 4))
    req.n_spheres = sp.shape[0]
    req.spheres = _dp(sp) if sp.shape[0] else None
    req.n_steps = int(n_steps)
    req.seed = int(seed) & 0xFFFFFFFF
    req.giesekus_alpha = float(giesekus_alpha)
    wv = None
    if wall_velocity is not None and len(wall_velocity):
        wv = np.ascontiguousarray(np.asarray(wall_velocity, dtype=np.float64).reshape(-1, 3))
        req.n_walls = wv.shape[0]
        req.wall_velocity = _dp(wv)
    ticket = ctypes.c_uint64()
    _scheck(lib().vlb_server_submit(srv, ctypes.byref(req), ctypes.byref(ticket)), srv)
    return ticket.value


def vlb_server_pump(srv, wait=False):
    return _scheck(lib().vlb_server_pump(srv, int(bool(wait))), srv)


def vlb_server_poll(srv, ticket):
    st = ctypes.c_int32()
    _scheck(lib().vlb_server_poll(srv, int(ticket), ctypes.byref(st)), srv)
    return REQ_STATES[st.value]


def vlb_server_result(srv, ticket, shape):
    nx, ny, nz = shape
    u = np.zeros((3, nz, ny, nx))
    tau = np.zeros((6, nz, ny, nx))
    lat = ctypes.c_double()
    _scheck(lib().vlb_server_result(srv, int(ticket), _dp(u), _dp(tau),
                                    ctypes.cast(ctypes.pointer(lat), _D)), srv)
    return u, tau, lat.value


def vlb_server_cancel(srv, ticket):
    return _scheck(lib().vlb_server_cancel(srv, int(ticket)), srv)


def vlb_server_stats_get(srv):
    st = vlb_server_stats()
    _scheck(lib().vlb_server_stats_get(srv, ctypes.byref(st)), srv)
    return {k: getattr(st, k) for k, _ in vlb_server_stats._fields_}


def vlb_server_last_error(srv):
    return lib().vlb_server_last_error(srv).decode()


def vlb_server_destroy(srv):
    lib().vlb_server_destroy(srv)
