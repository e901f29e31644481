"""Serving (continuous batching): a solve gives bit-identical results alone,
in a mix it joined while others were running, and through a plain lattice;
admission respects the memory budget and the slot count; cancellation; and
one served solve against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2009_12279_amd import inputs, vlb
from parity import log

pytestmark = pytest.mark.gpu

GB = 1 << 30


def make_request(seed, shape, n_steps, n_spheres=1, wi=0.5):
    """A channel (walls in y, periodic x, z) with fixed spheres, driven by a
    body force; lambda from the Weissenberg number at the wall shear rate."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    mask = inputs.channel_mask(shape, wall_axes=(1,))
    eta, g = 1 / 3, 1e-5
    beta = float(rng.uniform(0.1, 0.9))
    lam = max(1.0, wi / (g * (ny - 2) / (2 * eta)))
    spheres = []
    for _ in range(n_spheres):
        r = float(rng.uniform(2.0, 3.5))
        c = [rng.uniform(0, nx), rng.uniform(r + 2, ny - 3 - r), rng.uniform(0, nz)]
        spheres.append(c + [r])
    params = dict(eta=eta, beta=beta, lambda_p=lam, magic=3 / 16, body_force=(g, 0, 0))
    return dict(shape=shape, mask=mask, periodic=(1, 0, 1), params=params, spheres=spheres,
                n_steps=n_steps, seed=1000 + seed)


# solves 32 or more cells wide take the tiled stress update (32: half the
# tile's lanes past the row; 64 x 14 x 40: ragged y tiles and z chunks), the
# narrower ones the per-cell one, in the same batch
REQS = [
    (1, (16, 18, 12), 120, 1),
    (2, (24, 14, 20), 200, 2),
    (3, (20, 20, 20), 90, 0),
    (4, (32, 12, 8), 160, 1),
    (5, (64, 14, 40), 80, 1),
]


def submit(srv, r):
    return vlb.vlb_server_submit(srv, **{k: r[k] for k in (
        "shape", "mask", "periodic", "params", "spheres", "n_steps", "seed", "giesekus_alpha")
        if k in r})


def serve(reqs, budget=4 * GB, slots=16, k=10, stagger=True):
    srv = vlb.vlb_server_create(budget, slots, k)
    try:
        tickets = {}
        pending = list(reqs)
        # submit the first one, then the others while it runs
        first = pending.pop(0)
        tickets[first["seed"]] = (submit(srv, first), first)
        out = {}
        rounds = 0
        while len(out) < len(reqs):
            vlb.vlb_server_pump(srv, wait=True)
            rounds += 1
            if pending and (not stagger or rounds % 2 == 0):
                r = pending.pop(0)
                tickets[r["seed"]] = (submit(srv, r), r)
            for seed, (t, r) in tickets.items():
                if seed not in out and vlb.vlb_server_poll(srv, t) == "done":
                    out[seed] = vlb.vlb_server_result(srv, t, r["shape"])
            assert rounds < 10000
        return out, vlb.vlb_server_stats_get(srv)
    finally:
        vlb.vlb_server_destroy(srv)


def test_results_identical_alone_and_in_the_mix():
    reqs = [make_request(*r) for r in REQS]
    # two Giesekus solves (per-cell and tiled) among the Oldroyd-B ones
    reqs[1]["giesekus_alpha"] = 0.25
    reqs[4]["giesekus_alpha"] = 0.4
    log("[serving] mix of 4 requests, staggered submission")
    mixed, stats = serve(reqs)
    log(f"[serving]   stats {stats}")
    assert stats["completed"] == len(reqs) and stats["launches"] > 0
    for r in reqs:
        log(f"[serving] alone seed={r['seed']} shape={r['shape']}")
        alone, _ = serve([r], slots=1)
        ua, ta, _ = alone[r["seed"]]
        um, tm, lat = mixed[r["seed"]]
        assert lat > 0
        np.testing.assert_array_equal(ua, um)
        np.testing.assert_array_equal(ta, tm)


def test_result_buffer_grows_between_readouts():
    """A larger solve that finishes after a smaller one has been read out
    makes the server grow its device result buffer (in stream order, while
    replays may be in flight); both results must equal those of solves run
    alone."""
    small = make_request(11, (12, 10, 8), 20, 0)
    large = make_request(12, (40, 30, 24), 90, 2)
    log("[serving] small then large: result buffer growth")
    mixed, stats = serve([small, large], k=10, stagger=False)
    assert stats["completed"] == 2
    for r in (small, large):
        alone, _ = serve([r], slots=1, k=10)
        for a, b in zip(alone[r["seed"]][:2], mixed[r["seed"]][:2]):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("shape,alpha", [((18, 16, 14), 0.0), ((64, 16, 12), 0.0),
                                         ((128, 13, 37), 0.0), ((18, 16, 14), 0.3),
                                         ((64, 16, 12), 0.3)])
def test_served_solve_equals_plain_lattice(shape, alpha):
    """Per-cell (18 wide) and tiled (64 and 128 wide; ragged y tiles and
    z chunks) stress updates in the batch give the bits of the lattice's own
    step, for Oldroyd-B and for the Giesekus law."""
    r = make_request(7, shape, 150, 1)
    r["giesekus_alpha"] = alpha
    log(f"[serving] served vs plain lattice {shape} alpha={alpha}")
    out, _ = serve([r], slots=2, k=7)
    us, ts, _ = out[r["seed"]]
    L = vlb.Lattice(r["shape"], r["mask"], r["periodic"])
    L.set_params(**r["params"])
    if alpha:
        L.set_giesekus(alpha)
    for (cx, cy, cz, rad) in r["spheres"]:
        L.add_sphere(center=(cx, cy, cz), radius=rad)
    L.set_rounding("stochastic", r["seed"])
    L.set_check_interval(0)
    L.init_equilibrium()
    L.step(r["n_steps"])
    np.testing.assert_array_equal(L.velocity(), us)
    np.testing.assert_array_equal(L.stress(), ts)
    L.close()


def test_admission_respects_budget_and_slots():
    reqs = [make_request(10 + i, (16, 16, 16), 40, 0) for i in range(5)]
    one = vlb.vlb_server_request_bytes((16, 16, 16))
    log("[serving] budget for ~2 requests, 3 slots")
    srv = vlb.vlb_server_create(int(2.5 * one), 3, 5)
    try:
        # a request that can never fit is refused at submission
        big = make_request(99, (64, 64, 64), 10, 0)
        with pytest.raises(vlb.VlbError) as ei:
            vlb.vlb_server_submit(srv, **{k: big[k] for k in (
                "shape", "mask", "periodic", "params", "spheres", "n_steps", "seed")})
        assert ei.value.status == vlb.VLB_EBUSY
        ts = [vlb.vlb_server_submit(srv, **{k: r[k] for k in (
            "shape", "mask", "periodic", "params", "spheres", "n_steps", "seed")}) for r in reqs]
        max_running = 0
        for _ in range(200):
            vlb.vlb_server_pump(srv, wait=True)
            st = vlb.vlb_server_stats_get(srv)
            max_running = max(max_running, st["running"])
            assert st["bytes_in_use"] <= 2.5 * one
            if st["completed"] == len(reqs):
                break
        assert st["completed"] == len(reqs)
        assert max_running == 2
        for t in ts:
            assert vlb.vlb_server_poll(srv, t) == "done"
    finally:
        vlb.vlb_server_destroy(srv)


def test_cancel_queued_and_running():
    reqs = [make_request(20 + i, (16, 12, 10), 400, 0) for i in range(3)]
    srv = vlb.vlb_server_create(4 * GB, 1, 5)
    try:
        ts = [vlb.vlb_server_submit(srv, **{k: r[k] for k in (
            "shape", "mask", "periodic", "params", "spheres", "n_steps", "seed")}) for r in reqs]
        vlb.vlb_server_pump(srv, wait=True)
        assert vlb.vlb_server_poll(srv, ts[0]) == "running"
        vlb.vlb_server_cancel(srv, ts[0])
        vlb.vlb_server_cancel(srv, ts[2])
        for _ in range(500):
            vlb.vlb_server_pump(srv, wait=True)
            if vlb.vlb_server_poll(srv, ts[1]) == "done":
                break
        assert vlb.vlb_server_poll(srv, ts[0]) == "cancelled"
        assert vlb.vlb_server_poll(srv, ts[2]) == "cancelled"
        assert vlb.vlb_server_poll(srv, ts[1]) == "done"
    finally:
        vlb.vlb_server_destroy(srv)


def test_served_solve_matches_oracle():
    r = make_request(30, (12, 14, 10), 300, 1)
    out, _ = serve([r], slots=4, k=25)
    us, ts, _ = out[r["seed"]]
    o = oracle.Lattice(r["shape"], r["mask"], r["periodic"])
    o.set_params(**r["params"])
    for (cx, cy, cz, rad) in r["spheres"]:
        o.add_sphere((cx, cy, cz), rad)
    o.init_equilibrium()
    o.step(r["n_steps"])
    fl = o.mask() == 0
    uo, to = o.velocity(), o.stress()
    eu = np.max(np.abs(us[:, fl] - uo[:, fl])) / np.max(np.abs(uo[:, fl]))
    et = np.max(np.abs(ts[:, fl] - to[:, fl])) / np.max(np.abs(to[:, fl]))
    log(f"[serving] vs oracle: u {eu:.2e} tau {et:.2e}")
    assert eu < 1e-5 and et < 1e-5


def test_submit_refuses_a_giesekus_alpha_outside_its_range():
    r = make_request(40, (12, 10, 8), 10, 0)
    srv = vlb.vlb_server_create(GB, 2, 5)
    try:
        for bad in (-0.1, 0.7, float("nan")):
            r["giesekus_alpha"] = bad
            with pytest.raises(vlb.VlbError) as ei:
                submit(srv, r)
            assert ei.value.status == vlb.VLB_EINVAL
    finally:
        vlb.vlb_server_destroy(srv)


@pytest.mark.parametrize("shape", [(20, 18, 14), (64, 18, 20)])
def test_served_solve_with_a_moving_wall_equals_plain_lattice(shape):
    """A channel whose top wall (id 2) slides in x and z, served per cell
    (20 wide) and tiled (64 wide), alone and beside a solve with walls at
    rest: the bits of a plain lattice created with the same wall velocities."""
    nx, ny, nz = shape
    mask = inputs.channel_mask(shape, wall_axes=(1,), top_id=2)
    walls = [[0.0, 0.0, 0.0], [3e-3, 0.0, -1e-3]]
    r = dict(shape=shape, mask=mask, periodic=(1, 0, 1),
             params=dict(eta=1 / 3, beta=0.4, lambda_p=80.0, magic=3 / 16, body_force=(0, 0, 0)),
             spheres=[[nx / 2 - 0.3, ny / 2 + 0.2, nz / 2, 3.0]], n_steps=120, seed=4242)
    other = make_request(8, (16, 18, 12), 90, 1)
    log(f"[serving] moving lid {shape}")
    srv = vlb.vlb_server_create(GB, 4, 10)
    try:
        t = vlb.vlb_server_submit(srv, shape, mask, (1, 0, 1), r["params"], r["spheres"],
                                  r["n_steps"], r["seed"], wall_velocity=walls)
        t2 = submit(srv, other)
        for _ in range(1000):
            vlb.vlb_server_pump(srv, wait=True)
            if vlb.vlb_server_poll(srv, t) == "done" and vlb.vlb_server_poll(srv, t2) == "done":
                break
        us, ts, _ = vlb.vlb_server_result(srv, t, shape)
        with pytest.raises(vlb.VlbError) as ei:
            vlb.vlb_server_submit(srv, shape, mask, (1, 0, 1), r["params"], (), 10, 1,
                                  wall_velocity=[[np.nan, 0, 0]])
        assert ei.value.status == vlb.VLB_EINVAL
    finally:
        vlb.vlb_server_destroy(srv)
    L = vlb.Lattice(shape, mask, (1, 0, 1), walls)
    L.set_params(**r["params"])
    L.add_sphere(center=tuple(r["spheres"][0][:3]), radius=r["spheres"][0][3])
    L.set_rounding("stochastic", r["seed"])
    L.set_check_interval(0)
    L.init_equilibrium()
    L.step(r["n_steps"])
    np.testing.assert_array_equal(L.velocity(), us)
    np.testing.assert_array_equal(L.stress(), ts)
    # the lid drags the fluid next to it
    assert us[0, :, ny - 2, :].mean() > 0
    L.close()


@pytest.mark.parametrize("policy", ["fifo", "shortest_first"])
def test_admission_order_follows_the_policy(policy):
    """One slot, four requests queued before the first pump: FIFO admits them
    in submission order, shortest-first by cell-steps (large ones last), and
    every result equals the solve run alone."""
    reqs = [make_request(50, (20, 16, 14), 60, 1), make_request(51, (12, 10, 8), 30, 0),
            make_request(52, (16, 12, 10), 40, 0), make_request(53, (12, 10, 8), 20, 0)]
    log(f"[serving] admission order, policy {policy}")
    srv = vlb.vlb_server_create(GB, 1, 10)
    order = []
    try:
        vlb.vlb_server_set_policy(srv, policy)
        tickets = [submit(srv, r) for r in reqs]
        done = {}
        for _ in range(1000):
            vlb.vlb_server_pump(srv, wait=True)
            for i, t in enumerate(tickets):
                if i not in done and vlb.vlb_server_poll(srv, t) == "done":
                    done[i] = vlb.vlb_server_result(srv, t, reqs[i]["shape"])
                    order.append(i)
            if len(done) == len(reqs):
                break
        with pytest.raises(KeyError):
            vlb.vlb_server_set_policy(srv, "longest_first")
    finally:
        vlb.vlb_server_destroy(srv)
    work = [np.prod(r["shape"]) * r["n_steps"] for r in reqs]
    expect = list(range(4)) if policy == "fifo" else sorted(range(4), key=lambda i: (work[i], i))
    assert order == expect, (order, expect)
    for i, r in enumerate(reqs):
        alone, _ = serve([r], slots=1)
        np.testing.assert_array_equal(alone[r["seed"]][0], done[i][0])
        np.testing.assert_array_equal(alone[r["seed"]][1], done[i][1])
