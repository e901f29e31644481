#!/usr/bin/env python3
"""Throughput of the coupled LB + Oldroyd-B step on one MI355X.

Workload (default): 256^3 periodic box with 64 fixed spheres of radius 6
placed uniformly at random (seeded, non-overlapping), body force 1e-6 along x,
polymer fraction beta drawn once from U[0.1, 0.9], lambda_p = 1000, FP32
deviation storage.  A step is one pass of the whole per-cell path
(stream-collide with bounce-back and polymer force, then the stress update).

Prints one JSON line with MLUPS, the HBM roofline of the dominant kernel
(HIP-event timed on the lattice's stream) and the FP64 CPU oracle timed on
a bounded sample of the same workload.
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
        "stream_collide": 2 * 19 * p + 6 * 4 + 1,   # populations r+w, stress read, mask
        "stress_update": 6 * 4,                      # stress write
        "step": 2 * 19 * p + 2 * 6 * 4 + 1,          # whole step (201 B for FP32)
    }


def build_workload(storage, steps_hint=0):
    from paper_2009_12279_amd import inputs

    shape = (256, 256, 256)
    spheres = inputs.place_spheres(4, 0, shape, 64, 6.0, 6.0, min_gap=2.0, periodic=(1, 1, 1))
    beta = float(inputs.Stream(4, 1).uniform(1, 0.1, 0.9)[0])
    params = dict(eta=1.0 / 3.0, beta=beta, lambda_p=1000.0, magic=3.0 / 16.0,
                  body_force=(1e-6, 0.0, 0.0))
    return shape, spheres, params


def run_gpu(args):
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
    fluid = int((lat.mask() == 0).sum())

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

    # per-kernel durations: HIP events recorded by the library on the same
    # stream around every launch, averaged over a second timed pass
    lat.set_timing(True)
    lat.step(args.steps)
    torch.cuda.synchronize()
    k_ms = {"stream_collide": lat.kernel_time_ms(0), "stress_update": lat.kernel_time_ms(1)}
    lat.set_timing(False)
    health = lat.check_health()
    alg = algorithmic_bytes(args.storage)
    dom = max(k_ms, key=lambda k: k_ms[k])
    achieved = alg[dom] * N / (k_ms[dom] * 1e-3) / 1e9
    step_achieved = alg["step"] * N / (ms_per_step * 1e-3) / 1e9
    lat.close()
    return dict(N=N, fluid=fluid, shape=shape, params=params, ms_per_step=ms_per_step, mlups=mlups,
                wall_s=wall, kernels=k_ms, dominant=dom, achieved=achieved,
                step_achieved=step_achieved, alg=alg, health=health)


def run_cpu_baseline(args):
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
    L.step(1)  # first touch of every array
    t0 = time.perf_counter()
    L.step(args.cpu_steps)
    dt = time.perf_counter() - t0
    L.close()
    return dict(value=nx * ny * nz * args.cpu_steps / dt / 1e6, unit="MLUPS", cores=threads,
                kind="oracle",
                sample=f"the same 256^3 workload, {args.cpu_steps} steps after 1 untimed step "
                       f"(FP64 oracle, OpenMP {threads} threads)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--rounding", default=None, choices=[None, "nearest", "stochastic"])
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (torch) so that hardware byte "
                         "counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    g = run_gpu(args)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu = run_cpu_baseline(args)
    if rank != 0:
        return
    dtype = "f64" if args.storage == "f32" else "f32"
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
            "storage": args.storage,
            "arithmetic": dtype,
            "parallelism": "single GPU",
            "step_hbm_frac": round(g["step_achieved"] / HBM_PEAK_GBS, 4),
            "kernel_ms": {k: round(v, 5) for k, v in g["kernels"].items()},
            "algorithmic_bytes_per_cell": g["alg"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": g["dominant"],
            "achieved": round(g["achieved"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(g["achieved"] / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
