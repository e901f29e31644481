"""The C-ABI library: it loads, exports every function include/vlb.h declares,
and rejects invalid arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2009_12279_amd import vlb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(vlb_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_function():
    L = ctypes.CDLL(vlb.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    # and the binding covers them all under the same names
    bound = {n for n, _, _ in vlb.SIGNATURES}
    assert set(names) <= bound | {n for n in names if n.startswith("vlb_server")}


def test_velocity_table_is_d3q19_with_adjacent_opposites():
    cs, ws = [], []
    for i in range(19):
        c, w = vlb.vlb_velocity(i)
        cs.append(c)
        ws.append(w)
    c = np.array(cs)
    w = np.array(ws)
    assert len({tuple(v) for v in cs}) == 19
    assert tuple(c[0]) == (0, 0, 0)
    for i in range(1, 19, 2):
        assert tuple(c[i]) == tuple(-c[i + 1])
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-16)


def test_required_bytes_scales_with_storage():
    b32 = vlb.vlb_required_bytes((256, 256, 256), storage="f32")
    b16 = vlb.vlb_required_bytes((256, 256, 256), storage="f16")
    N = 256 ** 3
    # two population buffers dominate: 19*2*4 B vs 19*2*2 B per cell
    assert b32 - b16 == pytest.approx(2 * 19 * 2 * N, rel=1e-3)
    assert b32 > 2 * 19 * 4 * N + 12 * 4 * N
    assert vlb.vlb_required_bytes((0, 4, 4)) == 0


def _expect_status(fn, status):
    with pytest.raises(vlb.VlbError) as ei:
        fn()
    assert ei.value.status == status


def test_create_rejects_invalid_input_on_the_host():
    m = np.zeros((4, 4, 4), np.uint8)
    _expect_status(lambda: vlb.vlb_create((0, 4, 4), np.zeros((4, 4, 0), np.uint8)),
                   vlb.VLB_EINVAL)
    bad = m.copy()
    bad[1, 1, 1] = 64  # particle ids are reserved for vlb_add_sphere
    _expect_status(lambda: vlb.vlb_create((4, 4, 4), bad), vlb.VLB_EINVAL)
    # y not periodic but no solid end layers
    _expect_status(lambda: vlb.vlb_create((4, 4, 4), m, periodic=(1, 0, 1)), vlb.VLB_EINVAL)
    _expect_status(lambda: vlb.vlb_create((4, 4, 4), m, storage="f32",
                                          wall_velocity=np.zeros((64, 3))), vlb.VLB_EINVAL)
    assert "non-periodic" in vlb.vlb_last_error(None) or vlb.vlb_last_error(None)


def test_create_rejects_oversized_lattices_and_bad_walls():
    """Planes are addressed with 32-bit byte offsets, so lattices of 2^30
    cells or more are refused before the mask is read; non-finite wall
    velocities are refused too.  All on the host."""
    import ctypes

    h = vlb._P()
    d = vlb.make_dims((1024, 1024, 1024), (1, 1, 1))
    tiny = np.zeros(1, np.uint8)  # never read: the size check comes first
    st = vlb.lib().vlb_create(ctypes.byref(d), tiny.tobytes(), None, 0, vlb.STORAGE["f32"], None,
                              ctypes.byref(h))
    assert st == vlb.VLB_EINVAL
    assert "dimensions" in vlb.vlb_last_error(None)
    m = np.zeros((4, 4, 4), np.uint8)
    m[:, 0, :] = 1
    m[:, -1, :] = 2
    _expect_status(lambda: vlb.vlb_create((4, 4, 4), m, periodic=(1, 0, 1),
                                          wall_velocity=[[0, 0, 0], [np.nan, 0, 0]]),
                   vlb.VLB_EINVAL)
    assert "non-finite" in vlb.vlb_last_error(None)


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a HIP device is present")
    _expect_status(lambda: vlb.vlb_create((4, 4, 4), np.zeros((4, 4, 4), np.uint8)),
                   vlb.VLB_EDEVICE)


def test_buffer_sizes_match_the_state_layout():
    shape = (64, 32, 16)
    s32 = vlb.vlb_buffer_sizes(shape, storage="f32")
    s16 = vlb.vlb_buffer_sizes(shape, storage="f16")
    N = 64 * 32 * 16
    assert s32[0] >= N and s32[0] % 256 == 0
    assert s32[1] == s32[2] and s32[3] == s32[4]
    P = s32[5] // 12  # velocity: 3 FP32 planes of P elements
    assert P >= N and s32[1] == 19 * P * 4 and s32[3] == 6 * P * 4
    assert s16[1] == 19 * P * 2 and s16[3] == s32[3]
    assert sum(s32) <= vlb.vlb_required_bytes(shape, storage="f32")


def test_create_with_buffers_checks_them_on_the_host():
    shape = (8, 8, 8)
    mask = np.zeros((8, 8, 8), np.uint8)
    sizes = vlb.vlb_buffer_sizes(shape)
    fake = [256 * (k + 1) << 20 for k in range(vlb.NBUF)]  # never dereferenced
    with pytest.raises(vlb.VlbError) as ei:
        vlb.vlb_create_with_buffers(shape, mask, fake, [n - 1 for n in sizes])
    assert ei.value.status == vlb.VLB_EINVAL
    with pytest.raises(vlb.VlbError) as ei:
        vlb.vlb_create_with_buffers(shape, mask, [p + 4 for p in fake], sizes)
    assert ei.value.status == vlb.VLB_EINVAL


class _CkptHeader(ctypes.Structure):
    """Leading record of a checkpoint file, as vlb_save writes it."""
    _fields_ = [("magic", ctypes.c_uint64), ("dims", ctypes.c_int32 * 6),
                ("storage", ctypes.c_int32), ("n_walls", ctypes.c_int32),
                ("n_parts", ctypes.c_int32), ("polymer", ctypes.c_int32),
                ("step", ctypes.c_int64), ("params", ctypes.c_double * 7),
                ("scale", ctypes.c_float), ("any_movable", ctypes.c_int32),
                ("rounding", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("counter_force", ctypes.c_int32), ("extrap", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("L2", ctypes.c_double),
                ("wall_field", ctypes.c_int32), ("force_field", ctypes.c_int32),
                ("smooth_ns", ctypes.c_int32), ("pad", ctypes.c_int32)]


def _particle_record(radius=2.0, mass=30.0, movable=0):
    # R, v, w, radius, mass, inertia (12 doubles), movable + pad, then ten
    # 3-vectors of forces and torques and the previous position
    d = np.zeros(12)
    d[0:3] = 3.5
    d[9], d[10], d[11] = radius, mass, 0.4 * mass * radius ** 2
    return (d.tobytes() + np.array([movable, 0], np.int32).tobytes() + np.zeros(30).tobytes()
            + np.full(3, 3.5).tobytes())


def _checkpoint(path, mask_byte=0, n_parts=1, any_movable=0, storage=0, scale=1.0, **rec):
    shape = (8, 8, 8)
    N = 8 * 8 * 8
    h = _CkptHeader()
    h.magic = 0x38304B434C424C56
    h.dims[:] = [8, 8, 8, 1, 1, 1]
    h.storage, h.n_parts, h.any_movable = storage, n_parts, any_movable
    h.params[:] = [1 / 3, 0.0, 1.0, 3 / 16, 0.0, 0.0, 0.0]
    h.scale, h.rounding = scale, 1
    mask = np.zeros(N, np.uint8)
    mask[100] = mask_byte
    with open(path, "wb") as fp:
        fp.write(bytes(h))
        fp.write(np.zeros(64 * 3).tobytes())
        for _ in range(n_parts):
            fp.write(_particle_record(**rec))
        fp.write(mask.tobytes())
        fp.write(np.zeros(19 * N, np.float32).tobytes())
        fp.write(np.zeros(12 * N, np.float32).tobytes())
    return shape


@pytest.mark.parametrize("case", ["mask_beyond_table", "zero_mass", "nan_radius",
                                  "movable_flag_mismatch"])
def test_load_rejects_inconsistent_particle_records_on_the_host(tmp_path, case):
    """A checkpoint whose mask names a particle beyond the table, whose
    particle records are not finite positive spheres, or whose movable flag
    disagrees with the records is refused before any device work."""
    p = str(tmp_path / "bad.ckpt")
    if case == "mask_beyond_table":
        _checkpoint(p, mask_byte=64 + 1, n_parts=1)
        why = "beyond the table"
    elif case == "zero_mass":
        _checkpoint(p, mass=0.0)
        why = "invalid particle record"
    elif case == "nan_radius":
        _checkpoint(p, radius=float("nan"))
        why = "invalid particle record"
    else:
        _checkpoint(p, any_movable=1, movable=0)
        why = "movable flag"
    h = vlb._P()
    st = vlb.lib().vlb_load(p.encode(), None, ctypes.byref(h))
    assert st == vlb.VLB_EINVAL
    assert why in vlb.vlb_last_error(None)


@pytest.mark.parametrize("storage,scale", [(1, 3.0), (1, 0.5), (1, 2.0 ** 25), (0, 2.0),
                                           (2, 1024.0), (1, float("nan"))])
def test_load_rejects_a_storage_scale_the_format_cannot_carry(tmp_path, storage, scale):
    """FP16 checkpoints carry a power-of-two scale from 1 to 2^24, FP32 and
    BF16 ones the scale 1; anything else is refused before any device work."""
    p = str(tmp_path / "bad_scale.ckpt")
    _checkpoint(p, storage=storage, scale=scale)
    h = vlb._P()
    st = vlb.lib().vlb_load(p.encode(), None, ctypes.byref(h))
    assert st == vlb.VLB_EINVAL
    assert "not a lattice checkpoint" in vlb.vlb_last_error(None)
