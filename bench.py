#!/usr/bin/env python
"""Throughput of the spin-2 QLG step on one MI355X (site-updates per second).

Workload (the paper's 1D scattering runs, Sec. IV): a periodic 1D lattice of
L = 16384 sites with two bright solitons at L/2 -+ L/8 (width 48 sites,
momenta -+0.05 pi rad/site, seeded spinor weights), couplings
(g0, g1, g2) = (1, -0.5, 0.5), eps = 0.1, interleaved split; observables
(norms, populations, energy, overlap energy) every 100 steps.  One bench step
is one QLG time step of the whole lattice; `value` is sites * steps / wall
time of the timed region, inputs resident in HBM.

Prints one JSON line with the roofline of the fused step kernel (it is bound
by the vector ALUs: see `roofline`) and the FP64 CPU oracle's rate on a
bounded sample of the same workload (`cpu_baseline`).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per site-update (derivation in DESIGN.md, "Work per site-update").
# Flops count add/sub/mul as 1 and fma as 2 in the per-site formulas of
# qlg_math.hpp; the three sincos, two square roots and five divisions of each
# self-interaction are not counted.
FLOPS_U = 894          # one application of U (coefficients 190 + 2 x 352 per 5-vector)
FLOPS_IPRIME = 100     # one I' (two collides 2 x 40 + the exact 1/4 scaling 20)
FLOPS_PER_SITE_STEP = {1: 4 * (FLOPS_U + FLOPS_IPRIME), 2: 8 * (FLOPS_U + FLOPS_IPRIME)}
# HBM bytes per site per pass: read + write of 10 complex amplitudes
BYTES_PER_SITE_PASS = {"c64": 2 * 10 * 8, "c128": 2 * 10 * 16}
# MI355X published peaks
PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}     # fp32 vector (packed), fp64 vector
PEAK_HBM_GBS = 8000.0
OBS_EVERY = 100


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c64")
    ap.add_argument("--cpu-steps", type=int, default=120,
                    help="steps of the oracle sample for cpu_baseline (0 = skip)")
    ap.add_argument("--no-graph", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import qlg_inputs as qi
    from paper_1907_12834_amd.qlg import Lattice

    w = qi.c2_two_solitons(nsteps=args.steps)
    L = w.nx[0]
    lat = Lattice(1, [L], g=w.g, eps=w.eps, dtype=args.dtype)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    tuning = lat.autotune()
    if not args.no_graph:
        lat.set_tuning(use_graph=True)
    tuning = lat.tuning()

    def run(nsteps):
        done = 0
        while done < nsteps:
            k = min(OBS_EVERY, nsteps - done)
            lat.step(k)
            done += k
            if done % OBS_EVERY == 0:
                lat.observables()

    run(args.warmup)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    obs0 = lat.observables()[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs1 = lat.observables()[0]
    wall = t1 - t0
    value = L * args.steps / wall

    # Average device time of one fused-step launch, from HIP events recorded
    # around every launch on the library's stream (graphs off while measuring).
    lat.set_tuning(use_graph=False)
    lat.set_timing(True)
    meas_steps = min(args.steps, 2000)
    lat.step(meas_steps)
    kern_ms, launches = lat.last_kernel_ms()
    lat.set_timing(False)
    S = tuning["steps_per_pass"]
    sites_per_launch = L * S
    flops_launch = FLOPS_PER_SITE_STEP[1] * sites_per_launch
    achieved_tflops = flops_launch / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    bytes_launch = BYTES_PER_SITE_PASS[args.dtype] * L
    hbm_gbs = bytes_launch / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None

    cpu = None
    if args.cpu_steps > 0:
        cpu = cpu_baseline(w, args.cpu_steps)

    drift = obs1["norm_q"] / obs0["norm_q"] - 1.0
    out = {
        "metric": "QLG site-updates/s + % HBM roofline; batched and fwd+adjoint vs plain step",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "c64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "1d_two_soliton_scattering",
            "lattice": [L],
            "storage": args.dtype,
            "split": "interleaved",
            "g": list(w.g),
            "eps": w.eps,
            "observables_every": OBS_EVERY,
            "plan": tuning,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": PEAK_TFLOPS[args.dtype],
            "unit": "TFLOP/s",
            "frac": (achieved_tflops / PEAK_TFLOPS[args.dtype]) if achieved_tflops else None,
            "traffic": None,
            "kernel": "k_step1d",
            "kernel_ms_avg": kern_ms,
            "launches_timed": launches,
            "flops_per_site_update": FLOPS_PER_SITE_STEP[1],
            "hbm_algorithmic_gbs": hbm_gbs,
            "hbm_frac": (hbm_gbs / PEAK_HBM_GBS) if hbm_gbs else None,
        },
        "norm_drift": drift,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_baseline(w, nsteps):
    """The FP64 oracle, as it stands, on the first `nsteps` steps of the same workload."""
    import torch
    from oracle import qlg_oracle as O
    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    O.run_psi(w.psi[0], nsteps, w.eps, w.g)
    dt = time.perf_counter() - t0
    L = w.nx[0]
    return {"value": L * nsteps / dt, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": "same 1D L=%d workload, first %d steps (FP64 torch CPU, %d threads), %.1f s"
                      % (L, nsteps, threads, dt)}


if __name__ == "__main__":
    main()
