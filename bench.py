#!/usr/bin/env python3
"""Throughput of the coupled LB + Oldroyd-B step on one MI355X.

Workload (default): 256^3 periodic box with 64 fixed spheres of radius 6
placed uniformly at random (seeded, non-overlapping), body force 1e-6 along x,
polymer fraction beta drawn once from U[0.1, 0.9], lambda_p = 1000, FP32
deviation storage.  A step is one pass of the whole per-cell path
(stream-collide with bounce-back and polymer force, then the stress update).

Prints one JSON line with MLUPS, the HBM roofline of the whole step (its
algorithmic bytes over the step time, HIP events on the lattice's stream),
the same for each kernel of the step, and the FP64 CPU oracle timed on a
bounded sample of the same workload with one thread and with every host
core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LB+Oldroyd-B MLUPS & % HBM roofline; p50/p99 batched-solve latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per fluid-or-solid cell and step, by kernel and storage:
# populations are read once and written once (19 each), the stress is read
# once by the stream-collide (for the polymer force) and written once by the
# stress update, the mask byte is read once.
POP_BYTES = {"f32": 4, "f16": 2, "bf16": 2}


def algorithmic_bytes(storage):
    p = POP_BYTES[storage]
    return {
        "fused_step": 2 * 19 * p + 2 * 6 * 4 + 1,    # the whole step in one kernel
        "stream_collide": 2 * 19 * p + 6 * 4 + 1,   # populations r+w, stress read, mask
        "stress_update": 6 * 4,                      # stress write
        "step": 2 * 19 * p + 2 * 6 * 4 + 1,          # whole step (201 B for FP32)
    }


def kernel_times(lat, particles=False):
    """Per-launch device times (ms) the library measured with HIP events on
    its stream: the fused step kernel, or stream-collide and stress update
    when the step ran as two kernels."""
    t0, t1 = lat.kernel_time_ms(0), lat.kernel_time_ms(1)
    k = {"fused_step": t0} if t1 < 0 else {"stream_collide": t0, "stress_update": t1}
    if particles:
        k["particles"] = lat.kernel_time_ms(2)
    return k


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "step_256cubed_hbm_traffic.md")
KERNEL_SOURCES = ("paper_2009_12279_amd/csrc/vlb_kernels.hip", "paper_2009_12279_amd/csrc/vlb_internal.h")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE / WRITE_SIZE scaled against a copy of known size), or
    None when the kernel sources have changed since the counters were taken."""
    import hashlib

    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    recorded, value = None, None
    for line in text.splitlines():
        if line.startswith("source_sha256:"):
            recorded = line.split(":", 1)[1].strip()
        if line.startswith(f"traffic_bytes_per_launch {kernel}:"):
            value = float(line.split(":", 1)[1])
    if recorded != h.hexdigest():
        return None
    return value


def build_workload(storage, steps_hint=0):
    from paper_2009_12279_amd import inputs

    shape = (256, 256, 256)
    spheres = inputs.place_spheres(4, 0, shape, 64, 6.0, 6.0, min_gap=2.0, periodic=(1, 1, 1))
    beta = float(inputs.Stream(4, 1).uniform(1, 0.1, 0.9)[0])
    params = dict(eta=1.0 / 3.0, beta=beta, lambda_p=1000.0, magic=3.0 / 16.0,
                  body_force=(1e-6, 0.0, 0.0))
    return shape, spheres, params


SETTLE_S = 0.1


def settle_gpu(seconds=SETTLE_S):
    """Keep the GPU busy with device copies for `seconds` before the warm-up
    steps: its clocks ramp up under load, and a fresh lattice's first 20
    steps after 5 warm-up steps otherwise run about 5 % slower than the steady
    state.  No step of the workload runs here."""
    import torch

    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
    del src, dst


def run_gpu(args, law=None, repeats=0):
    import torch

    from paper_2009_12279_amd import vlb

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    shape, spheres, params = build_workload(args.storage)
    nx, ny, nz = shape
    N = nx * ny * nz
    mask = np.zeros((nz, ny, nx), np.uint8)
    lat = vlb.Lattice(shape, mask, (1, 1, 1), storage=args.storage, stream=stream.cuda_stream)
    lat.set_params(**params)
    for c, r in spheres:
        lat.add_sphere(center=c, radius=r)
    lat.init_equilibrium()
    lat.set_check_interval(0)
    if args.rounding:
        lat.set_rounding(args.rounding)
    if law == "giesekus":
        lat.set_giesekus(0.2)
    elif law == "fene_p":
        lat.set_fene_p(100.0)
    fluid = int((lat.mask() == 0).sum())

    settle_gpu()
    lat.step(args.warmup)
    torch.cuda.synchronize()
    # timed region: K steps, bracketed by device synchronisation
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    mlups = N * args.steps / (gpu_ms / 1e3) / 1e6
    # further repetitions of the same K steps, after the timed region
    reps = []
    for _ in range(repeats):
        ev0.record(stream)
        lat.step(args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        reps.append(ev0.elapsed_time(ev1) / args.steps)

    # per-kernel durations: HIP events recorded by the library on the same
    # stream around every launch, averaged over a second timed pass
    lat.set_timing(True)
    lat.step(args.steps)
    torch.cuda.synchronize()
    k_ms = kernel_times(lat)
    lat.set_timing(False)
    health = lat.check_health()
    alg = algorithmic_bytes(args.storage)
    dom = max(k_ms, key=lambda k: k_ms[k])
    per_kernel = {k: alg[k] * N / (v * 1e-3) / 1e9 for k, v in k_ms.items() if v > 0}
    # the step's bytes over the step's kernel time (the events around each
    # kernel of the step, summed), so that the figure is the kernels' own
    step_achieved = alg["step"] * N / (sum(k_ms.values()) * 1e-3) / 1e9
    lat.close()
    return dict(N=N, fluid=fluid, shape=shape, params=params, ms_per_step=ms_per_step, mlups=mlups,
                repeats=reps, wall_s=wall, kernels=k_ms, dominant=dom, per_kernel=per_kernel,
                step_achieved=step_achieved, alg=alg, health=health)


def _time_lattice(lat, args, stream, particles=True):
    """ms per step (HIP events on the lattice's stream) and per-kernel-family
    times of a second timed pass."""
    import torch

    settle_gpu()
    lat.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    lat.set_timing(True)
    lat.step(args.steps)
    torch.cuda.synchronize()
    k_ms = kernel_times(lat, particles=particles)
    lat.set_timing(False)
    return ms, {k: round(v, 5) for k, v in k_ms.items()}


def run_fixed_configs(args):
    """The smaller fixed-geometry workloads, timed like the others: the
    4 x 64 x 4 Oldroyd-B channel (walls in y, g = 1e-6, lambda_p = 1000,
    BGK) and the 128 x 64 x 64 duct (walls in y and z, fixed sphere r = 8 at
    the centre, g = 1e-6, beta = 0.5) at lambda_p = 100, 1000 and 5000."""
    import torch

    from paper_2009_12279_amd import inputs, vlb

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    out = {}
    shape = (4, 64, 4)
    lat = vlb.Lattice(shape, inputs.channel_mask(shape, wall_axes=(1,)), (1, 0, 1),
                      stream=stream.cuda_stream)
    lat.set_params(eta=1.0 / 3.0, beta=0.5, lambda_p=1000.0, magic=-1.0,
                   body_force=(1e-6, 0.0, 0.0))
    lat.set_check_interval(0)
    lat.init_equilibrium()
    ms, k_ms = _time_lattice(lat, args, stream, particles=False)
    lat.close()
    out["channel_4x64x4"] = dict(ms_per_step=round(ms, 4),
                                 mlups=round(1024 / (ms * 1e-3) / 1e6, 1), kernel_ms=k_ms)
    shape = (128, 64, 64)
    N = int(np.prod(shape))
    for lam in (100.0, 1000.0, 5000.0):
        lat = vlb.Lattice(shape, inputs.channel_mask(shape, wall_axes=(1, 2)), (1, 0, 0),
                          stream=stream.cuda_stream)
        lat.set_params(eta=1.0 / 3.0, beta=0.5, lambda_p=lam, magic=3.0 / 16.0,
                       body_force=(1e-6, 0.0, 0.0))
        lat.add_sphere(center=(63.5, 31.5, 31.5), radius=8.0)
        lat.set_check_interval(0)
        lat.init_equilibrium()
        ms, k_ms = _time_lattice(lat, args, stream, particles=False)
        lat.close()
        out[f"duct_128x64x64_lambda{lam:.0f}"] = dict(
            ms_per_step=round(ms, 4), mlups=round(N / (ms * 1e-3) / 1e6, 1), kernel_ms=k_ms)
    return out


def run_moving(args):
    """Moving boundaries: (1) the settling-sphere box (64x64x256, walls on
    every axis, one movable sphere r = 6 of density ratio 1.5 under an
    external force -0.004 along z, beta = 0.5, Wi = 1); (2) the paper's
    rotating settling sphere at its largest box (periodic L = 240 = 30 R,
    R = 8, eta_n = 1/6, eta_p = eta_n, lambda_p = 6000, F_z = -0.008 taken back
    from the fluid, torque M_z = 0.07).  Momentum exchange, the rigid-body
    update and the fluid/solid conversion run every step."""
    import torch

    from paper_2009_12279_amd import inputs, vlb

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    out = {}
    # (1) closed box
    shape = (64, 64, 256)
    eta, r, F = 1.0 / 3.0, 6.0, 0.004
    lam = r / (F / (6 * np.pi * eta * r))
    mask = inputs.channel_mask(shape, wall_axes=(0, 1, 2))
    lat = vlb.Lattice(shape, mask, (0, 0, 0), stream=stream.cuda_stream)
    lat.set_params(eta=eta, beta=0.5, lambda_p=lam, magic=3.0 / 16.0)
    lat.add_sphere(center=(31.5, 31.5, 191.5), radius=r, density_ratio=1.5, movable=True,
                   f_ext=(0.0, 0.0, -F))
    lat.set_check_interval(0)
    lat.init_equilibrium()
    ms, k_ms = _time_lattice(lat, args, stream)
    p = lat.particle(0)
    lat.close()
    N = int(np.prod(shape))
    out["closed_box"] = dict(
        workload="settling sphere: 64x64x256 closed box, movable sphere r=6, density ratio 1.5, "
                 "F_z=-0.004, beta=0.5, Wi=1 (lambda_p=%.0f)" % lam,
        ms_per_step=round(ms, 4), mlups=round(N / (ms * 1e-3) / 1e6, 1), kernel_ms=k_ms,
        sphere_z=round(float(p["pos"][2]), 4), sphere_vz=float(p["vel"][2]))
    # (2) periodic rotating settling sphere, counter-force
    L = 240
    shape = (L, L, L)
    lat = vlb.Lattice(shape, None, (1, 1, 1), stream=stream.cuda_stream)
    lat.set_params(eta=1.0 / 3.0, beta=0.5, lambda_p=6000.0, magic=3.0 / 16.0)
    lat.add_sphere(center=(119.5, 119.7, 120.2), radius=8.0, density_ratio=1.0, movable=True,
                   f_ext=(0.0, 0.0, -0.008), t_ext=(0.0, 0.0, 0.07))
    lat.set_counter_force(True)
    lat.set_check_interval(0)
    lat.init_equilibrium()
    ms, k_ms = _time_lattice(lat, args, stream)
    p = lat.particle(0)
    lat.close()
    N = L ** 3
    out["periodic_rotating_sphere"] = dict(
        workload="rotating settling sphere: periodic 240^3 (L = 30 R), R=8, beta=0.5, "
                 "lambda_p=6000, F_z=-0.008 with counter-force, M_z=0.07",
        ms_per_step=round(ms, 4), mlups=round(N / (ms * 1e-3) / 1e6, 1), kernel_ms=k_ms,
        sphere_vz=float(p["vel"][2]), sphere_wz=float(p["omega"][2]))
    return out


def run_cpu_baseline(args):
    """The oracle on the same 256^3 workload: args.cpu_steps steps with every
    host thread, then args.cpu_steps_single steps with one thread (each after
    an untimed step that first touches every array)."""
    import oracle

    shape, spheres, params = build_workload("f32")
    nx, ny, nz = shape
    threads = oracle.get_threads()
    mask = np.zeros((nz, ny, nx), np.uint8)
    L = oracle.Lattice(shape, mask, (1, 1, 1))
    L.set_params(**params)
    for c, r in spheres:
        L.add_sphere(c, r)
    L.init_equilibrium()

    def timed(n):
        L.step(1)
        t0 = time.perf_counter()
        L.step(n)
        return nx * ny * nz * n / (time.perf_counter() - t0) / 1e6

    all_cores = timed(args.cpu_steps)
    single = None
    if args.cpu_steps_single > 0:
        oracle.set_threads(1)
        single = timed(args.cpu_steps_single)
        oracle.set_threads(0)
    L.close()
    from paper_2009_12279_amd import inputs

    def duct_rates(dshape, r, n_all, n_single):
        """The fixed-sphere duct (walls in y and z, periodic x, sphere at the
        centre, lambda_p = 1000): n_all steps on every thread, n_single on 1."""
        D = oracle.Lattice(dshape, inputs.channel_mask(dshape, wall_axes=(1, 2)), (1, 0, 0))
        D.set_params(eta=1.0 / 3.0, beta=0.5, lambda_p=1000.0, magic=3.0 / 16.0,
                     body_force=(1e-6, 0.0, 0.0))
        D.add_sphere(tuple((n - 1) / 2.0 for n in dshape), r)
        D.init_equilibrium()
        ncell = dshape[0] * dshape[1] * dshape[2]

        def dtimed(n):
            D.step(1)
            t0 = time.perf_counter()
            D.step(n)
            return ncell * n / (time.perf_counter() - t0) / 1e6

        out = dict(all_cores=round(dtimed(n_all), 3))
        oracle.set_threads(1)
        out["single_thread"] = round(dtimed(n_single), 3)
        oracle.set_threads(0)
        D.close()
        return dict(out, unit="MLUPS", sample=f"{n_all} steps on {threads} threads, "
                                              f"{n_single} steps on 1, after 1 untimed step")

    duct = duct_rates((128, 64, 64), 8.0, 40, 10)
    duct_copy = duct_rates((64, 32, 32), 4.0, 200, 50)
    # the serving list solved one after another by the oracle: the first 4
    # requests, 10 steps each (each after 1 untimed step)
    reqs = serving_requests(4, 1.0)
    cells = 0
    secs = 0.0
    for r in reqs:
        S = oracle.Lattice(r["shape"], r["mask"], r["periodic"])
        S.set_params(**r["params"])
        for c in r["spheres"]:
            S.add_sphere(tuple(c[:3]), c[3])
        S.init_equilibrium()
        S.step(1)
        t0 = time.perf_counter()
        S.step(10)
        secs += time.perf_counter() - t0
        cells += int(np.prod(r["shape"])) * 10
        S.close()
    serving_seq = dict(all_cores=round(cells / secs / 1e6, 3), unit="MLUPS",
                       sample=f"the first 4 serving requests, 10 steps each, {threads} threads")
    return dict(value=all_cores, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"the same 256^3 workload, {args.cpu_steps} steps after 1 untimed step "
                       f"(FP64 oracle, OpenMP {threads} threads)",
                single_thread=None if single is None else dict(
                    value=single, unit="MLUPS", cores=1,
                    sample=f"{args.cpu_steps_single} steps after 1 untimed step, 1 thread"),
                duct_128x64x64=duct, duct_64x32x32=duct_copy, serving_sequential=serving_seq)


def serving_requests(n, steps_scale):
    """Seeded request list of the serving workload: edges drawn from
    {32, 48, 64, 96, 128} per axis, walls at y = 0 and n_y - 1 (periodic x, z),
    0-8 fixed spheres of radius 4-8 at least one cell clear of the walls and
    of each other, Weissenberg number log-uniform in [0.05, 2] converted to
    lambda_p with the wall shear rate of the empty channel, beta uniform in
    [0.1, 0.9], 2000-20000 steps (times steps_scale)."""
    from paper_2009_12279_amd import inputs

    edges = [32, 48, 64, 96, 128]
    eta, g = 1.0 / 3.0, 1e-6
    out = []
    for k in range(n):
        st = inputs.Stream(5, k)
        shape = tuple(int(edges[i]) for i in st.integers(0, 4, 3))
        nx, ny, nz = shape
        wi = float(np.exp(st.uniform(1, np.log(0.05), np.log(2.0))[0]))
        beta = float(st.uniform(1, 0.1, 0.9)[0])
        steps = int(st.integers(2000, 20000, 1)[0] * steps_scale)
        count = int(st.integers(0, 8, 1)[0])
        spheres = []
        while count > 0:
            try:
                spheres = inputs.place_spheres(5, 1000 + k, shape, count, 4.0, 8.0, min_gap=1.0,
                                               periodic=(1, 0, 1), margin=2.0, max_tries=2000)
                break
            except RuntimeError:
                count -= 1
        gamma = g * (ny - 2) / (2 * eta)
        lam = max(1.0, wi / gamma)
        out.append(dict(shape=shape, mask=inputs.channel_mask(shape, wall_axes=(1,)),
                        periodic=(1, 0, 1), spheres=[list(c) + [r] for c, r in spheres],
                        params=dict(eta=eta, beta=beta, lambda_p=lam, magic=3.0 / 16.0,
                                    body_force=(g, 0.0, 0.0)),
                        n_steps=steps, seed=0x2009 + k))
    return out


def run_serving(args):
    """Sequential plain solves, then the same requests through the server with
    Poisson arrivals at 1.5x the sequential service rate."""
    import torch

    from paper_2009_12279_amd import vlb

    torch.cuda.set_device(0)
    reqs = serving_requests(args.serving_requests, args.serving_steps_scale)
    cell_steps = sum(int(np.prod(r["shape"])) * r["n_steps"] for r in reqs)
    # sequential baseline: one plain lattice after another
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for i, r in enumerate(reqs):
        if time.perf_counter() - last > 30.0:
            last = time.perf_counter()
            print(f"[serving] sequential {i}/{len(reqs)}", file=sys.stderr, flush=True)
        L = vlb.Lattice(r["shape"], r["mask"], r["periodic"])
        L.set_params(**r["params"])
        for c in r["spheres"]:
            L.add_sphere(center=c[:3], radius=c[3])
        L.set_rounding("stochastic", r["seed"])
        L.set_check_interval(0)
        L.init_equilibrium()
        L.step(r["n_steps"])
        L.velocity()
        L.stress()
        L.close()
    seq_s = time.perf_counter() - t0
    rate = 1.5 * len(reqs) / seq_s
    budget = int(args.serving_budget_gb * (1 << 30))

    def serve(arrivals, policy="fifo"):
        srv = vlb.vlb_server_create(budget, args.serving_slots, args.serving_k)
        lat = []
        try:
            vlb.vlb_server_set_policy(srv, policy)
            tickets = {}
            nxt = 0
            t0 = time.perf_counter()
            last = t0
            while len(lat) < len(reqs):
                if time.perf_counter() - last > 30.0:
                    last = time.perf_counter()
                    print(f"[serving] {len(lat)}/{len(reqs)} done, {nxt} submitted",
                          file=sys.stderr, flush=True)
                now = time.perf_counter() - t0
                while nxt < len(reqs) and arrivals[nxt] <= now:
                    r = reqs[nxt]
                    tickets[nxt] = vlb.vlb_server_submit(srv, **{k: r[k] for k in (
                        "shape", "mask", "periodic", "params", "spheres", "n_steps", "seed")})
                    nxt += 1
                vlb.vlb_server_pump(srv, wait=False)
                for i, t in list(tickets.items()):
                    if vlb.vlb_server_poll(srv, t) == "done":
                        _, _, ms = vlb.vlb_server_result(srv, t, reqs[i]["shape"])
                        lat.append(ms)
                        del tickets[i]
                if not tickets and nxt < len(reqs):
                    time.sleep(max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t0))))
            wall = time.perf_counter() - t0
            stats = vlb.vlb_server_stats_get(srv)
        finally:
            vlb.vlb_server_destroy(srv)
        return np.array(lat), wall, stats

    # throughput with every request queued at t = 0, then latency under
    # Poisson arrivals at 1.5x the sequential service rate
    _, sat_s, sat_stats = serve(np.zeros(len(reqs)))
    rng = np.random.default_rng(args.serving_requests)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
    lat, bat_s, stats = serve(arrivals)
    lat = np.array(lat)
    # the same arrivals admitted shortest first
    lat_sf, sf_s, _ = serve(arrivals, "shortest_first")
    return dict(
        requests=len(reqs), steps_scale=args.serving_steps_scale,
        cell_steps=cell_steps, arrival_rate_hz=round(rate, 3),
        budget_gb=args.serving_budget_gb, slots=args.serving_slots,
        steps_per_launch=args.serving_k,
        p50_ms=round(float(np.percentile(lat, 50)), 2),
        p99_ms=round(float(np.percentile(lat, 99)), 2),
        policy="fifo",
        shortest_first=dict(p50_ms=round(float(np.percentile(lat_sf, 50)), 2),
                            p99_ms=round(float(np.percentile(lat_sf, 99)), 2),
                            poisson_wall_s=round(sf_s, 3)),
        poisson_wall_s=round(bat_s, 3), saturated_wall_s=round(sat_s, 3),
        sequential_wall_s=round(seq_s, 3),
        batched_mlups=round(cell_steps / sat_s / 1e6, 1),
        sequential_mlups=round(cell_steps / seq_s / 1e6, 1),
        speedup=round(seq_s / sat_s, 3),
        launches=stats["launches"], graph_captures=stats["graph_captures"],
        graph_updates=stats["graph_updates"],
    )


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--rounding", default=None, choices=[None, "nearest", "stochastic"])
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-steps-single", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=48)
    ap.add_argument("--serving-steps-scale", type=float, default=0.1)
    ap.add_argument("--serving-budget-gb", type=float, default=8.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-k", type=int, default=50)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-moving", action="store_true",
                    help="skip the moving-boundary (settling sphere) and the smaller "
                         "fixed-geometry (channel, duct) measurements")
    ap.add_argument("--no-storage-variants", action="store_true",
                    help="skip timing the same workload with FP16 and BF16 population storage")
    ap.add_argument("--no-law-variants", action="store_true",
                    help="skip timing the same workload with the Giesekus and FENE-P laws")
    ap.add_argument("--no-fused-prototype", action="store_true",
                    help="skip timing the fused single-pass step (same bits, slower, opt-in)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (torch) so that hardware byte "
                         "counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    g = run_gpu(args, repeats=5)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fused = None
    if not args.no_fused_prototype:
        # the fused single-pass step the library runs only when asked
        os.environ["VLB_FUSED"] = "1"
        try:
            v = run_gpu(args)
        finally:
            del os.environ["VLB_FUSED"]
        fused = dict(ms_per_step=round(v["ms_per_step"], 4), mlups=round(v["mlups"], 1),
                     kernel_ms={k: round(x, 5) for k, x in v["kernels"].items()},
                     step_hbm_frac=round(v["step_achieved"] / HBM_PEAK_GBS, 4),
                     note="same bits as the default two-kernel step; opt-in (VLB_FUSED=1)")
    variants = None
    if not args.no_storage_variants:
        # the precision pattern: the same workload with 16-bit population storage
        variants = {}
        for st in ("f16", "bf16"):
            if st == args.storage:
                continue
            v = run_gpu(argparse.Namespace(**{**vars(args), "storage": st}))
            variants[st] = dict(
                ms_per_step=round(v["ms_per_step"], 4), mlups=round(v["mlups"], 1),
                kernel_ms={k: round(x, 5) for k, x in v["kernels"].items()},
                algorithmic_bytes_per_cell=v["alg"],
                step_hbm_frac=round(v["step_achieved"] / HBM_PEAK_GBS, 4))
    laws = None
    if not args.no_law_variants:
        # the other constitutive laws through the same stress update
        laws = {}
        for law, what in (("giesekus", "alpha = 0.2"), ("fene_p", "L^2 = 100")):
            v = run_gpu(args, law)
            laws[law] = dict(parameter=what, ms_per_step=round(v["ms_per_step"], 4),
                             mlups=round(v["mlups"], 1),
                             kernel_ms={k: round(x, 5) for k, x in v["kernels"].items()})
    moving = None if args.no_moving else run_moving(args)
    fixed = None if args.no_moving else run_fixed_configs(args)
    serving = None if args.no_serving else run_serving(args)
    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu = run_cpu_baseline(args)
    if rank != 0:
        return
    dtype = "f64" if args.storage == "f32" else "f32"
    # counters were taken for the default configuration only
    traffic = None
    if args.storage == "f32" and args.rounding in (None, "stochastic"):
        parts = [measured_traffic(k) for k in g["kernels"]]
        traffic = None if any(t is None for t in parts) else sum(parts)
    line = {
        "metric": METRIC,
        "value": round(g["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": "precision at scale: 256^3 periodic box, 64 fixed spheres r=6 "
                        "(seeded, non-overlapping), g=1e-6 x, lambda_p=1000, "
                        f"beta={g['params']['beta']:.4f}",
            "cells": g["N"],
            "fluid_cells": g["fluid"],
            "fluid_mflups": round(g["fluid"] / (g["ms_per_step"] * 1e-3) / 1e6, 1),
            "repeats_ms_per_step": [round(x, 4) for x in g["repeats"]],
            "repeats_median_ms_per_step": (round(float(np.median(g["repeats"])), 4)
                                           if g["repeats"] else None),
            "clock_settle_ms": round(SETTLE_S * 1e3),
            "storage": args.storage,
            "arithmetic": dtype,
            "parallelism": "single GPU",
            "kernel_ms": {k: round(v, 5) for k, v in g["kernels"].items()},
            "algorithmic_bytes_per_cell": g["alg"],
            "fixed_obstacle_forces": "summed on read from the state the last step left "
                                     "(same bits as summing them every step); no obstacle "
                                     "moves, so no step needs them",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "step: " + " + ".join(g["kernels"]),
            "achieved": round(g["step_achieved"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(g["step_achieved"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "per_kernel": {k: dict(ms=round(g["kernels"][k], 5), achieved=round(v, 1),
                                   frac=round(v / HBM_PEAK_GBS, 4),
                                   bytes_per_cell=g["alg"][k])
                           for k, v in g["per_kernel"].items()},
        },
        "cpu_baseline": cpu,
        "fused_step_prototype": fused,
        "storage_variants": variants,
        "law_variants": laws,
        "moving_particle": moving,
        "fixed_geometry": fixed,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
