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
