"""vlb_read_velocity_noalloc, the velocity readout that allocates nothing,
against vlb_read_velocity on the same state: the same bits, on two calls in a
row (the second over a smaller range), with size checks on the host."""
import numpy as np
import pytest

from paper_2009_12279_amd import inputs, vlb

from parity import log

pytestmark = pytest.mark.gpu


def _lattice():
    shape = (40, 30, 24)
    mask = inputs.channel_mask(shape, wall_axes=(1,), top_id=2)
    L = vlb.Lattice(shape, mask, (1, 0, 1), [[0, 0, 0], [1e-3, 0, 0]])
    L.set_params(eta=1 / 3, beta=0.5, lambda_p=60.0, magic=3 / 16, body_force=(1e-6, 0, 0))
    L.add_sphere(center=(19.5, 14.5, 11.5), radius=4.0, density_ratio=3.0, movable=True,
                 f_ext=(2e-3, 0.0, 0.0))
    u0 = inputs.noise_field(9, 0, shape, 1e-3)
    u0[:, L.mask() != 0] = 0
    L.init_equilibrium(u0)
    return L, shape


def test_noalloc_readout_matches_the_allocating_one():
    L, shape = _lattice()
    N = int(np.prod(shape))
    for calls, (first, count) in enumerate(((1000, 20000), (5, 333))):
        log(f"[noalloc] call {calls}: step 25, then cells {first}..{first + count - 1}")
        L.step(25)
        full = L.velocity().reshape(3, N)
        part = vlb.vlb_read_velocity_noalloc(L._h, first, count)
        np.testing.assert_array_equal(part, full[:, first:first + count])
    # the whole lattice in pieces of at most the staging size
    full = L.velocity().reshape(3, N)
    got = np.concatenate([vlb.vlb_read_velocity_noalloc(L._h, a, min(7000, N - a))
                          for a in range(0, N, 7000)], axis=1)
    np.testing.assert_array_equal(got, full)
    L.close()


def test_noalloc_readout_rejects_sizes_beyond_its_staging_array():
    L, shape = _lattice()
    N = int(np.prod(shape))
    for first, count in ((0, 0), (0, vlb.NOALLOC_MAX_CELLS + 1), (-1, 10), (N - 5, 6)):
        with pytest.raises(vlb.VlbError) as ei:
            vlb.vlb_read_velocity_noalloc(L._h, first, count)
        assert ei.value.status == vlb.VLB_EINVAL
    assert "staging" in vlb.vlb_last_error(L._h) or "range" in vlb.vlb_last_error(L._h)
    L.close()
