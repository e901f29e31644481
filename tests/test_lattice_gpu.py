"""The lattice handle on the GPU: the health check (speed limit, sticky
instability, reads still allowed), checkpoint restart bit for bit in every
storage precision and with a moving particle, and device-side error paths."""
import numpy as np
import pytest

from paper_2009_12279_amd import inputs, vlb
from parity import log

pytestmark = pytest.mark.gpu


def test_health_check_flags_excess_speed_and_is_sticky():
    shape = (8, 12, 6)
    nx, ny, nz = shape
    mask = inputs.channel_mask(shape, wall_axes=(1,))
    L = vlb.Lattice(shape, mask, (1, 0, 1))
    L.set_params(eta=1 / 3, beta=0.5, lambda_p=50.0)
    u = np.zeros((3, nz, ny, nx))
    u[0, 3, 5, 4] = 0.35
    L.init_equilibrium(u)
    log("[lattice] health check on a state above the speed limit")
    st, speed, bad = vlb.vlb_check_health(L.handle, raise_on_unstable=False)
    assert st == vlb.VLB_EUNSTABLE and speed == pytest.approx(0.35, rel=1e-6) and bad == 0
    with pytest.raises(vlb.VlbError) as ei:
        L.step(1)
    assert ei.value.status == vlb.VLB_EUNSTABLE
    assert L.step_count == 0
    assert np.isfinite(L.velocity()).all()
    L.close()


def test_periodic_check_inside_step_stops_the_run():
    """A uniform flow above the limit stays uniform; with a check every step
    the run stops after the first step and reports the sticky state."""
    shape = (8, 8, 8)
    L = vlb.Lattice(shape, None, (1, 1, 1))
    L.set_params(eta=1 / 3, beta=0.0, lambda_p=1.0)
    u = np.zeros((3, 8, 8, 8))
    u[0] = 0.35
    L.init_equilibrium(u)
    L.set_check_interval(1)
    log("[lattice] check interval 1, uniform u = 0.35")
    with pytest.raises(vlb.VlbError) as ei:
        L.step(5)
    assert ei.value.status == vlb.VLB_EUNSTABLE
    L.sync()
    assert L.step_count == 1
    np.testing.assert_allclose(L.velocity()[0], 0.35, rtol=1e-6)
    L.close()


def _duct_with_moving_sphere(storage):
    shape = (20, 18, 26)
    mask = inputs.channel_mask(shape, wall_axes=(0, 1, 2))
    L = vlb.Lattice(shape, mask, (0, 0, 0), storage=storage)
    L.set_params(eta=1 / 6, beta=0.5, lambda_p=40.0, magic=3 / 16, body_force=(2e-6, 0, 0))
    L.add_sphere(center=(9.5, 8.7, 13.2), radius=3.4, density_ratio=1.5, movable=True,
                 f_ext=(8e-3, 0.0, -2e-2))
    L.set_check_interval(0)
    L.init_equilibrium()
    return L


@pytest.mark.parametrize("storage,smoothing,u_max", [("f32", 0, None), ("f16", 0, None),
                                                     ("bf16", 0, None), ("f32", 4, None),
                                                     ("f16", 0, 2e-3)])
def test_checkpoint_restart_is_bitwise(tmp_path, storage, smoothing, u_max):
    """Save, continue, and load + continue give the same bits; with
    smoothed conversions the sphere's previous position and the sample count
    travel with the checkpoint, and an FP16 scale chosen from the flow speed
    travels with the populations."""
    path = str(tmp_path / f"ck_{storage}.vlb")
    log(f"[lattice] checkpoint restart storage={storage} smoothing={smoothing} u_max={u_max}")
    L = _duct_with_moving_sphere(storage)
    L.set_rounding("stochastic", 77)
    L.set_conversion_smoothing(smoothing)
    if u_max is not None:
        L.set_velocity_scale(u_max)
        assert L.storage_scale == 2.0 ** 14
    L.step(100)
    L.save(path)
    m_saved = L.mask()
    L.step(200)
    ref = (L.populations(), L.stress(), L.mask(), L.particle(0), L.step_count)
    L.close()
    R = vlb.Lattice.load(path, (20, 18, 26))
    assert R.step_count == 100
    if u_max is not None:
        assert R.storage_scale == 2.0 ** 14
    R.step(200)
    got = (R.populations(), R.stress(), R.mask(), R.particle(0), R.step_count)
    R.close()
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1])
    np.testing.assert_array_equal(got[2], ref[2])
    for k in ("pos", "vel", "omega", "force", "torque"):
        np.testing.assert_array_equal(got[3][k], ref[3][k])
    assert got[4] == ref[4] == 300
    # the sphere converted cells after the checkpoint
    assert not np.array_equal(got[2], m_saved)


def test_checkpoint_keeps_wall_velocity_and_force_fields(tmp_path):
    """Per-cell wall velocity and force density survive save/load bit for bit
    (the FP32 force planes included), and clearing them returns to the plain
    lattice."""
    path = str(tmp_path / "ck_fields.vlb")
    shape = (16, 14, 12)
    log("[lattice] checkpoint with wall velocity and force fields")
    mask = inputs.channel_mask(shape, wall_axes=(1, 2))
    wf = inputs.noise_field(51, 0, shape, 1e-3)
    wf[:, mask == 0] = 0.0
    F = inputs.noise_field(52, 0, shape, 1e-4)
    L = vlb.Lattice(shape, mask, (1, 0, 0))
    L.set_params(eta=1 / 3, beta=0.5, lambda_p=30.0, magic=3 / 16)
    L.set_check_interval(0)
    L.set_wall_velocity_field(wf)
    L.set_force_field(F)
    # non-finite entries are refused and leave the fields as they were
    for setter, bad in ((L.set_wall_velocity_field, wf.copy()), (L.set_force_field, F.copy())):
        bad[0, 3, 4, 5] = np.inf
        with pytest.raises(vlb.VlbError) as ei:
            setter(bad)
        assert ei.value.status == vlb.VLB_EINVAL
    L.step(50)
    L.save(path)
    L.step(100)
    ref = (L.populations(), L.stress(), L.velocity())
    R = vlb.Lattice.load(path, shape)
    R.step(100)
    got = (R.populations(), R.stress(), R.velocity())
    R.close()
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    L.close()
    # cleared fields: the same as a lattice that never had them
    runs = []
    for clear in (True, False):
        P = vlb.Lattice(shape, mask, (1, 0, 0))
        P.set_params(eta=1 / 3, beta=0.5, lambda_p=30.0, magic=3 / 16, body_force=(1e-5, 0, 0))
        P.set_check_interval(0)
        if clear:
            P.set_wall_velocity_field(wf)
            P.set_force_field(F)
            P.set_wall_velocity_field(None)
            P.set_force_field(None)
        P.step(50)
        runs.append((P.populations(), P.stress()))
        P.close()
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("storage,tile,moving", [("f32", "4", False), ("f32", "-4", False),
                                                 ("f16", "4", False), ("f32", "4", True)])
def test_graph_replays_give_the_same_bits(monkeypatch, storage, tile, moving):
    """Steps replayed from captured graphs (chunks of 32, 16, ..., 1 steps)
    against the same steps launched one by one: bitwise equal after every
    call of any length, across health checks, a parameter change (a new
    capture) and both starting buffer parities; with a fixed sphere, or with
    a moving sphere under the counter-force (the particle path in the
    graph)."""
    shape = (24, 20, 16)
    mask = inputs.channel_mask(shape, wall_axes=(1,), top_id=2)
    monkeypatch.setenv("VLB_FV_TILE", tile)
    runs = []
    for graph in ("0", "1"):
        monkeypatch.setenv("VLB_GRAPH", graph)
        log(f"[lattice] graph replays {graph} storage={storage} tile={tile} moving={moving}")
        L = vlb.Lattice(shape, mask, (1, 0, 1), [[0, 0, 0], [1e-3, 0, 0]], storage=storage)
        L.set_params(eta=1 / 3, beta=0.5, lambda_p=50.0, magic=3 / 16, body_force=(1e-6, 0, 0))
        if moving:
            L.add_sphere(center=(11.5, 9.7, 8.2), radius=3.0, density_ratio=3.0, movable=True,
                         f_ext=(4e-3, 0.0, -2e-3), t_ext=(0.0, 0.0, 1e-3))
            L.set_counter_force(True)
        else:
            L.add_sphere(center=(11.5, 9.7, 8.2), radius=3.0)
        L.set_check_interval(50)
        L.init_equilibrium()
        out = []
        for n in (100, 37, 5, 20, 64):
            L.step(n)
            out.append((L.populations(), L.stress()))
            if moving:
                p = L.particle(0)
                out.append((p["pos"], p["vel"]))
        L.set_params(eta=1 / 3, beta=0.5, lambda_p=80.0, magic=3 / 16, body_force=(2e-6, 0, 0))
        L.step(65)
        out.append((L.populations(), L.stress()))
        out.append((L.mask(), L.mask()))
        assert L.step_count == 291
        runs.append(out)
        L.close()
    for (fa, ta), (fb, tb) in zip(*runs):
        np.testing.assert_array_equal(fa, fb)
        np.testing.assert_array_equal(ta, tb)


def test_largest_lattice_accelerates_uniformly():
    """The largest lattice the 32-bit plane offsets allow (the FP32 planes
    just under 4 GiB): 1024 x 1024 x 1000 cells, about 224 GB of state held
    in torch tensors.  From rest under a uniform body force g every cell
    carries u = (n + 1/2) g in step n (Guo's half force) and the stress stays
    zero up to rounding noise; checked on every cell through the device
    buffers."""
    import torch

    shape = (1024, 1024, 1000)
    N = shape[0] * shape[1] * shape[2]
    sizes = vlb.vlb_buffer_sizes(shape)
    free, _ = torch.cuda.mem_get_info()
    if sum(sizes) + (8 << 30) > free:
        pytest.skip(f"needs {sum(sizes) / 2**30:.0f} GiB of free device memory")
    log(f"[lattice] largest lattice {shape}, {sum(sizes) / 2**30:.0f} GiB, 3 steps")
    g = 1e-5
    L = vlb.Lattice(shape, np.zeros(shape[::-1], np.uint8), (1, 1, 1), torch_buffers=True)
    L.set_params(eta=1 / 3, beta=0.5, lambda_p=100.0, magic=3 / 16, body_force=(g, 0, 0))
    L.set_check_interval(0)
    L.init_equilibrium()
    L.step(3)
    L.sync()
    P = sizes[5] // 12
    u = L._buffers[5].view(torch.float32)
    ux = u[:N]
    assert float((ux - 2.5 * g).abs().max()) < 1e-5 * 2.5 * g
    # the other components and the stress only carry the rounding noise of
    # the stochastically rounded populations: half a unit in the last place
    # of deviations of a few 1e-6, summed over the directions, is ~1e-12
    assert float(u[P:P + N].abs().max()) < 1e-6 * g
    assert float(u[2 * P:2 * P + N].abs().max()) < 1e-6 * g
    for b in (3, 4):
        t = L._buffers[b].view(torch.float32)
        for c in range(6):
            assert float(t[c * P:c * P + N].abs().max()) < 1e-10
    L.close()
    del u, ux
    torch.cuda.empty_cache()


def test_load_rejects_a_file_that_is_not_a_checkpoint(tmp_path):
    p = tmp_path / "junk.vlb"
    p.write_bytes(b"not a checkpoint" * 8)
    with pytest.raises(vlb.VlbError) as ei:
        vlb.Lattice.load(str(p), (4, 4, 4))
    assert ei.value.status == vlb.VLB_EINVAL


def test_stepping_an_unset_lattice_and_bad_particle_ids():
    L = vlb.Lattice((6, 6, 6), None, (1, 1, 1))
    L.set_params(eta=1 / 3)
    L.init_equilibrium()
    with pytest.raises(vlb.VlbError) as ei:
        L.particle(3)
    assert ei.value.status in (vlb.VLB_EINVAL, vlb.VLB_ENOTFOUND)
    with pytest.raises(vlb.VlbError):
        L.step(-1)
    L.step(2)
    assert L.step_count == 2
    L.close()


def test_torch_owned_state_gives_the_same_bits():
    """The state in torch-allocated device tensors (vlb_create_with_buffers)
    evolves exactly as in library allocations."""
    out = []
    for tb in (False, True):
        log(f"[lattice] torch buffers={tb}")
        shape = (20, 18, 26)
        mask = inputs.channel_mask(shape, wall_axes=(0, 1, 2))
        L = vlb.Lattice(shape, mask, (0, 0, 0), torch_buffers=tb)
        L.set_params(eta=1 / 6, beta=0.5, lambda_p=40.0, magic=3 / 16, body_force=(2e-6, 0, 0))
        L.add_sphere(center=(9.5, 8.7, 13.2), radius=3.4, density_ratio=5.0, movable=True,
                     f_ext=(8e-3, 0.0, -2e-2))
        L.set_check_interval(0)
        L.init_equilibrium()
        L.step(150)
        out.append((L.populations(), L.stress(), L.mask(), L.particle(0)["pos"]))
        L.close()
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
