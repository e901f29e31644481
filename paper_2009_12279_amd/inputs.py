"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the method itself: it only draws random
numbers (SplitMix64, counter based) and lays out geometry masks (walls,
sphere centres and radii).  Rasterising a sphere into cells is done by each
solver on its own.

Seed base S = 200912279; every draw is keyed by (S, config, item).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 200912279
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream_key(config: int, item: int) -> int:
    """64-bit key of the stream (S, config, item)."""
    k = np.array([SEED_BASE ^ (config << 40) ^ (item << 20)], dtype=np.uint64)
    return int(_mix(k)[0])


def uniform(config: int, item: int, n: int, offset: int = 0) -> np.ndarray:
    """n uniforms in [0, 1): SplitMix64 outputs at counters offset+1 .. offset+n."""
    key = np.uint64(stream_key(config, item))
    ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix(key + ctr * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


class Stream:
    """Sequential draws from one (config, item) stream."""

    def __init__(self, config: int, item: int):
        self.config, self.item, self.pos = config, item, 0

    def uniform(self, n: int = 1, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        v = uniform(self.config, self.item, n, self.pos)
        self.pos += n
        return lo + (hi - lo) * v

    def integers(self, lo: int, hi: int, n: int = 1) -> np.ndarray:
        """Integers in [lo, hi]."""
        return (lo + np.floor(self.uniform(n) * (hi - lo + 1))).astype(np.int64)


def channel_mask(shape, wall_axes=(1,), wall_id=1, top_id=None) -> np.ndarray:
    """uint8 mask [nz, ny, nx]: solid end layers (index 0 and n-1) on each wall axis.

    wall_axes uses 0 = x, 1 = y, 2 = z.  top_id, if given, marks the layer at
    n-1 of the first wall axis with a different wall id (a moving lid)."""
    nx, ny, nz = shape
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    for ax in wall_axes:
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        arr_ax = 2 - ax
        sl0[arr_ax] = 0
        sl1[arr_ax] = shape[ax] - 1
        m[tuple(sl0)] = wall_id
        m[tuple(sl1)] = wall_id
    if top_id is not None:
        ax = wall_axes[0]
        sl1 = [slice(None)] * 3
        sl1[2 - ax] = shape[ax] - 1
        m[tuple(sl1)] = top_id
    return m


def periodic_flags(shape, wall_axes) -> tuple:
    return tuple(0 if a in wall_axes else 1 for a in range(3))


def noise_field(config: int, item: int, shape, amplitude: float, k: int = 3) -> np.ndarray:
    """k-component field [k, nz, ny, nx] of i.i.d. U[-amplitude, amplitude]."""
    nx, ny, nz = shape
    v = uniform(config, item, k * nx * ny * nz)
    return (amplitude * (2.0 * v - 1.0)).reshape(k, nz, ny, nx)


def place_spheres(config: int, item: int, shape, count: int, r_lo: float, r_hi: float,
                  min_gap: float, periodic=(1, 1, 1), margin: float = 0.0,
                  max_tries: int = 100000):
    """Draw `count` sphere (centre, radius) pairs uniformly, rejecting any whose
    (minimum-image) distance to an accepted one is below r1 + r2 + min_gap, or
    that comes closer than `margin` + r to a non-periodic face."""
    s = Stream(config, item)
    L = np.array(shape, dtype=np.float64)
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("place_spheres: could not place all spheres")
        r = float(s.uniform(1, r_lo, r_hi)[0]) if r_hi > r_lo else float(r_lo)
        c = s.uniform(3) * L
        ok = True
        for a in range(3):
            if not periodic[a] and (c[a] - r < margin or c[a] + r > L[a] - 1 - margin):
                ok = False
        if not ok:
            continue
        for (c2, r2) in out:
            d = c - c2
            for a in range(3):
                if periodic[a]:
                    d[a] -= L[a] * np.floor(d[a] / L[a] + 0.5)
            if np.sqrt((d * d).sum()) < r + r2 + min_gap:
                ok = False
                break
        if ok:
            out.append((c, r))
    return out
