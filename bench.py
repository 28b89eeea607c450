#!/usr/bin/env python
"""Throughput of the spin-2 QLG step on one MI355X (site-updates per second).

Default workload (the paper's 2D vortex runs, Sec. V and VI; its runs use double
precision, Sec. VII): a periodic 2048 x 2048 lattice, a uniform background
n0 = 1 shared by m_f = +2, 0, -2 with a Pade-profile vortex pair 128 sites
apart (winding +1 in m_f = +-2, -1 in m_f = 0), couplings (g0, g1, g2) =
(1, -0.3, 0.2), eps = 0.1, interleaved split (Lie product n = 8), complex128
storage and FP64 arithmetic; observables (norms, populations, energy, overlap
energy) every 100 steps.  One bench step is one QLG time step of the whole
lattice; `value` is sites * steps / wall time of the timed region, inputs
resident in HBM.  The observables are recorded on the device every 100 steps
and read back and decoded once, at the end of the timed region.  Every
hipGraph the timed region replays is captured before the clock starts.
`secondary` repeats the run in complex64, `spin_texture` on the field plus a
seeded random spinor (F != 0 at every site).  Other workloads (`--workload`):
the 1D two-soliton scattering lattice (L = 16384) and the 3D vortex-line
cubes.

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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per site-update, counted from the per-site formulas.
# Flops count add/sub/mul as 1 and fma as 2 in the per-site formulas of
# qlg_math.hpp; the three sincos, two reciprocal square roots and two
# reciprocals of each self-interaction are not counted.  One U: coefficients 178
# (psi, n, F, the phases and the rotation's blocks), then 288 per 5-vector a and b
# (singlet 84, frame phases 24, d^T 58, diagonal 30, d 58, recombination 34), the count of
# the FP64 form; the FP32 form adds the singlet correction to x in a separate step (10 more
# per 5-vector, not counted).
FLOPS_U = 754          # one application of U (coefficients 178 + 2 x 288 per 5-vector)
FLOPS_IPRIME = 85      # one I' (two collides 2 x 40 + its share of the exact 1/256 per step, 5)
FLOPS_PER_SITE_STEP = {d: 4 * d * (FLOPS_U + FLOPS_IPRIME) for d in (1, 2, 3)}
# plain split: one U (theta = eps^2) and the 4 d I' of a step
FLOPS_PER_SITE_STEP_PLAIN = {d: FLOPS_U + 4 * d * FLOPS_IPRIME for d in (1, 2, 3)}
# HBM passes per step: 1D and 2D one fused pass, 3D a z pass and a y-x pass
PASSES_PER_STEP = {1: 1, 2: 1, 3: 2}
# HBM bytes per site per pass: read + write of 10 complex amplitudes
BYTES_PER_SITE_PASS = {"c64": 2 * 10 * 8, "c128": 2 * 10 * 16}
# MI355X published peaks
PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}     # fp32 vector (packed), fp64 vector
PEAK_HBM_GBS = 8000.0
OBS_EVERY = 100
PREROLL_S = 0.2        # untimed steps right before each clock start, at least this long

# HBM traffic of one launch of the fused step, by (workload, storage, split) and by kernel and
# plan (steps per pass in 1D, band height in 2D and 3D), from rocprofv3 --pmc FETCH_SIZE and
# --pmc WRITE_SIZE runs (KiB per dispatch, median over the dispatches of that plan), each scaled
# by what the same counter reads for a 256 MiB device copy in the same run (FETCH_SIZE: x2.000,
# WRITE_SIZE: x1.000).  Valid only for the kernel sources it was measured on.
KERNEL_SOURCES = ["paper_1907_12834_amd/csrc/qlg_math.hpp", "paper_1907_12834_amd/csrc/qlg_kernels.hip",
                  "paper_1907_12834_amd/csrc/qlg_internal.hpp"]
TRAFFIC = {"sources_sha256_16": "6983e25ef22ca4b8", "fetch_scale": 262144.0 / 131088.5, "write_scale": 1.0,
           "kib": {
               # 1D two-soliton lattice, L = 16384: the two-lane kernel at 2 steps per pass
               "1d_two_soliton_scattering/c64/interleaved": {"k_step1d_lanes/S2": (740.5, 1280.0)},
               # 2D 2048^2 vortex pair (bands of rows, the autotuned plan of each)
               "2d_vortex_pair/c128/interleaved": {"k_step2d/rows76": (365694.0, 655360.0)},
               # the y half over two launches (sums of the two)
               "2d_vortex_pair/c64/interleaved": {"k_step2d/rows25/ysplit": (199636.0 + 193654.0,
                                                                         333441.0 + 330875.0)},
               "2d_vortex_pair/c64/plain": {"k_step2d/rows38": (201067.0, 330155.0)},
               # 3D cubes: one step = z pass + y-x pass (sums of the two)
               "3d_vortex_lines/c64/interleaved": {"k_step3d/rows64": (737418.8 + 743753.5,
                                                                       1310720.0 + 1312845.1)},
               "3d_vortex_lines_512/c128/interleaved": {"k_step3d/rows128": (11141332.2 + 11250320.8,
                                                                             20971520.0 + 20971520.0)}}}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="2d_vortex_pair",
                    help="the 2D 2048^2 vortex pair (default), the 1D two-soliton lattice or a 3D cube")
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c128",
                    help="storage precision; complex128 (FP64 arithmetic, the paper's) by default")
    ap.add_argument("--plan", default=None,
                    help="fix the launch plan instead of autotuning it (for profiler runs, where the "
                         "tracer's per-launch overhead would steer the autotuner): 1D 'S:qubit_split', "
                         "2D and 3D the band height in rows, or 'rows:1' for the y half over two launches")
    ap.add_argument("--split", choices=["interleaved", "plain"], default="interleaved",
                    help="operator splitting of the step (the benchmark uses the interleaved one)")
    ap.add_argument("--secondary", choices=["c64", "c128", "none"], default="c64",
                    help="also time the other storage precision of the same workload")
    ap.add_argument("--cpu-steps", type=int, default=500,
                    help="steps of the oracle sample for cpu_baseline (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=500,
                    help="steps of the batched-vs-one-at-a-time comparison (0 = skip)")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the forward+adjoint vs forward comparison (0 = skip)")
    ap.add_argument("--trap-steps", type=int, default=4000,
                    help="steps of the same workload with a harmonic trap and chemical potential (0 = skip)")
    ap.add_argument("--texture-steps", type=int, default=2000,
                    help="2D and 3D: steps of the same workload with a seeded random spinor of amplitude "
                         "0.05 added to every component, so that F != 0 at every site (0 = skip)")
    ap.add_argument("--diag-reps", type=int, default=50,
                    help="launches of the per-site field and vorticity kernels timed on the workload's "
                         "lattice (0 = skip)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="before timing, copy this many MiB device-to-device (a plain copy kernel of known "
                         "size that rocprofv3 --pmc FETCH_SIZE/WRITE_SIZE runs use to scale their counters)")
    return ap.parse_args()


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


WORKLOADS = {
    # name: (ndim, description)
    "1d_two_soliton_scattering": (1, "1D L = 16384 two bright solitons, w = 48, k = -+0.05 pi"),
    "2d_vortex_pair": (2, "2D 2048^2 uniform background with a Pade vortex pair 128 sites apart"),
    "3d_vortex_lines": (3, "3D 256^3 uniform background with two wavy Pade vortex lines 64 sites apart"),
    "3d_vortex_lines_512": (3, "3D 512^3 uniform background with two wavy Pade vortex lines 128 sites apart"),
}


def workload_input(name, steps):
    import qlg_inputs as qi
    if name == "1d_two_soliton_scattering":
        return qi.two_solitons_1d_L16384(nsteps=steps)
    if name == "2d_vortex_pair":
        return qi.vortex_pair_2d_2048(nsteps=steps)
    if name == "3d_vortex_lines_512":
        return qi.vortex_lines_3d_512(nsteps=steps)
    return qi.vortex_lines_3d_256(nsteps=steps)


def workload_lattice(w, ndim, dtype, split="interleaved"):
    from paper_1907_12834_amd.qlg import Lattice
    return Lattice(ndim, w.nx, w.ny if ndim >= 2 else None, w.nz if ndim == 3 else None, g=w.g, eps=w.eps,
                   dtype=dtype, split=split)


def workload_shape(w, ndim):
    return [w.nx[0]] if ndim == 1 else [w.ny[0], w.nx[0]] if ndim == 2 else [w.nz[0], w.ny[0], w.nx[0]]


def trap_potential(w, ndim):
    """A weak harmonic trap V = omega^2 r^2 / 4 centred on the lattice (m = 1/2), with omega chosen
    so that V reaches 1/2 at the edge midpoints, plus mu = 0.5."""
    shape = workload_shape(w, ndim)
    half = [0.5 * w.eps * n for n in shape]
    omega = math.sqrt(2.0) / max(half)
    axes = [w.eps * (np.arange(n) - n / 2) for n in shape]
    r2 = sum(np.expand_dims(a ** 2, [k for k in range(ndim) if k != i]) for i, a in enumerate(axes))
    return omega ** 2 * r2 / 4, 0.5


def spin_texture(w, ndim):
    """The workload's field plus a seeded complex Gaussian spinor of amplitude 0.05 in every
    component: m = +-1 are populated and F != 0 at every site, so the spin rotation of the
    self-interaction acts everywhere (the vortex states keep F = 0 for the whole run)."""
    import qlg_inputs as qi
    return w.psi[0] + qi.random_field(tuple(workload_shape(w, ndim)), seed=79, scale=0.05)


def measure(dtype, steps, warmup, workload="1d_two_soliton_scattering", split="interleaved", trap=False,
            plan=None, texture=False):
    """Run the workload (with a harmonic trap and mu if `trap`, on the spin texture if `texture`);
    return rate, wall time, per-launch kernel time and plan."""
    import torch

    w = workload_input(workload, steps)
    if texture:
        w.psi[0] = spin_texture(w, WORKLOADS[workload][0])
    ndim = WORKLOADS[workload][0]
    L = int(np.prod(workload_shape(w, ndim)))   # sites
    lat = workload_lattice(w, ndim, dtype, split)
    if trap:
        lat.set_potential(*trap_potential(w, ndim))
    lat.set_psi([torch.from_numpy(w.psi[0])])
    if plan:
        if ndim == 1:
            S, qs = (int(v) for v in plan.split(":"))
            lat.set_tuning(steps_per_pass=S, qubit_split=qs)
        else:
            rows, _, ys = plan.partition(":")
            lat.set_tuning(tile_rows=int(rows), qubit_split=int(ys or 0))
    else:
        lat.autotune()
    lat.set_tuning(use_graph=True)
    tuning = lat.tuning()

    # observables every OBS_EVERY steps are recorded on the device (no host round trip)
    # and decoded once at the end of the run, inside the timed region
    recs = {"buf": lat.new_records(max(steps, warmup) // OBS_EVERY + 1)}

    def run(nsteps):
        rec = recs["buf"]
        done, k = 0, 0
        while done < nsteps:
            n = min(OBS_EVERY, nsteps - done)
            lat.step(n)
            done += n
            if done % OBS_EVERY == 0:
                lat.record_observables(rec, k)
                k += 1
        return lat.decode_records(rec[:k])

    run(warmup)
    # Capture, before the clock starts, every graph the warm-up and timed runs replay: graphs
    # are keyed by (steps, starting copy), and those runs advance in chunks of OBS_EVERY steps
    # plus one remainder.  Each chunk size runs, then one single step (which moves to the other
    # copy wherever a step changes copies), then the chunk size again: both starting copies.
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    sizes = sorted({OBS_EVERY, steps % OBS_EVERY, warmup % OBS_EVERY} - {0})
    for n in sizes:
        lat.step(n)
        lat.step(1)
        lat.step(n)
    torch.cuda.synchronize()
    per_step = (time.perf_counter() - c0) / sum(2 * n + 1 for n in sizes)   # upper bound (captures)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    obs0 = lat.observables()[0]
    # The warm-up again, on the state the timed run continues, so that the GPU is busy up to the
    # start of the clock: after the host-side work above its clock has dropped, and it takes a
    # few tens of milliseconds of work to return to the steady state.  W steps, and at least
    # PREROLL_S seconds of them.
    preroll = max(warmup, int(math.ceil(PREROLL_S / per_step)) if per_step > 0 else 0)
    if preroll // OBS_EVERY + 1 > recs["buf"].shape[0]:
        recs["buf"] = lat.new_records(preroll // OBS_EVERY + 1)
    run(preroll)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trace = run(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs1 = trace[-1][0] if trace else lat.observables()[0]
    wall = t1 - t0
    # run-to-run spread: five more timed runs of about 0.2 s each (whole multiples of the
    # observables interval), continuing the evolution
    each = max(OBS_EVERY, min(steps, int(0.2 * steps / wall)) // OBS_EVERY * OBS_EVERY) if steps else 0
    rates = []
    for _ in range(5 if each else 0):
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        run(each)
        torch.cuda.synchronize()
        rates.append(L * each / (time.perf_counter() - r0))
    repeats = {"runs": len(rates), "steps_each": each, "median": float(np.median(rates)), "min": min(rates),
               "max": max(rates), "unit": "site-updates/s"} if rates else None
    # Kernel time: the same run again, now with a pair of HIP events on every fused-step
    # launch that its dispatch packet stamps at kernel start and end (library stream).
    # Those events add ~9 us of dispatch gap per launch, so they stay out of the
    # throughput region above.
    lat.set_psi([torch.from_numpy(w.psi[0])])
    run(preroll)
    lat.set_timing(True)
    run(min(steps, 4000))
    kern_ms, launches = lat.last_kernel_ms()
    lat.set_timing(False)
    return {"w": w, "L": L, "value": L * steps / wall, "wall": wall, "kern_ms": kern_ms, "launches": launches,
            "tuning": tuning, "drift": obs1["norm_q"] / obs0["norm_q"] - 1.0, "repeats": repeats,
            "preroll": preroll}


def diagnostics(workload, dtype, reps):
    """Per-site fields (Sec. III) and, in 2D and 3D, the vorticity of m = +2 (Sec. VI; in 3D
    its three plane families, fused in one kernel) on the workload's lattice after 20 steps:
    average time per call over `reps` back-to-back calls, from HIP events on the library's
    stream, against the algorithmic HBM bytes of each kernel."""
    import torch
    from paper_1907_12834_amd.qlg import lib

    w = workload_input(workload, 20)
    ndim = WORKLOADS[workload][0]
    lat = workload_lattice(w, ndim, dtype)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.step(20)
    n = lat.sites
    ncomp = 3 if ndim == 3 else 1
    outs = [torch.empty(ncomp * n if k == 0 else n, dtype=torch.float64, device=lat.device) for k in range(4)]
    wind = torch.empty(ncomp * n, dtype=torch.int32, device=lat.device)
    elem = 8 if dtype == "c64" else 16
    L = lib()
    # bytes per site: the 10 qubit amplitudes read and 4 doubles written; a_m, b_m read
    # and one double and one int32 written per plane family (three in 3D, from one pass)
    calls = {"k_fields": (lambda: L.qlg_fields(lat.ctx, *[t.data_ptr() for t in outs]), 10 * elem + 32)}
    if ndim >= 2:
        calls["k_vorticity"] = (lambda: L.qlg_vorticity(lat.ctx, 0, outs[0].data_ptr(), wind.data_ptr()),
                                2 * elem + 12 * ncomp)
    res = {"lattice_sites": n, "storage": dtype}
    for name, (fn, bsite) in calls.items():
        for _ in range(5):
            assert fn() == 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        for _ in range(reps):
            fn()
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = bsite * n / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "bytes_per_site": bsite, "achieved_gbs": gbs, "frac_hbm": gbs / PEAK_HBM_GBS}
    lat.close()
    return res


def batched_ratio(steps):
    """256 uneven 1D two-soliton runs in one batched context vs the same runs one at a time."""
    import torch
    import qlg_inputs as qi
    from paper_1907_12834_amd.qlg import Lattice

    wb = qi.batched_two_solitons_1d_256(nsteps=steps)
    psis = [torch.from_numpy(p) for p in wb.psi]
    lat = Lattice(1, wb.nx, g=wb.g, eps=wb.eps, dtype="c64")
    lat.set_psi(psis)
    lat.autotune()
    lat.set_tuning(use_graph=True)
    plan = lat.tuning()
    # both runs replay captured graphs of `steps` steps: two untimed calls capture the graphs
    # for either starting copy, so the timed call only replays
    lat.step(steps)
    lat.step(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    singles = []
    for i in range(wb.nbatch):
        one = Lattice(1, [wb.nx[i]], g=wb.g, eps=wb.eps, dtype="c64")
        one.set_psi([psis[i]])
        one.autotune()
        one.set_tuning(use_graph=True)
        one.step(steps)
        one.step(steps)
        singles.append(one)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for one in singles:
        one.step(steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    su = wb.sites * steps
    return {"workload": "256 1D two-soliton runs, L = 1024..16384 (sum %d sites), c64, %d steps, hipGraph "
                        "replay for the batch and for each single run" % (wb.sites, steps),
            "batched_site_updates_per_s": su / tb, "one_at_a_time_site_updates_per_s": su / ts,
            "speedup": ts / tb, "plan": plan}


def adjoint_ratio(steps, K, spin_texture=False):
    """(forward with checkpoints + reverse sweep) vs the plain forward, 2D 512^2 vortex pair, c64
    (with spin_texture: plus a seeded random spinor, so that F != 0 at every site)."""
    import torch
    import qlg_inputs as qi
    from paper_1907_12834_amd.qlg import Lattice

    w = (qi.adjoint_spin_texture_2d_512 if spin_texture else qi.adjoint_vortex_pair_2d_512)(
        nsteps=steps, checkpoint_every=K)
    psi = torch.from_numpy(w.psi[0])
    lat = Lattice(2, w.nx, w.ny, g=w.g, eps=w.eps, dtype="c64")
    lat.set_psi([psi])
    lat.autotune()
    lat.step(10)
    lat.set_psi([psi])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    lat.set_psi([psi])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ck = lat.forward_record(steps, K)
    val, lam, dg0 = lat.objective_grad("energy")
    dg = lat.adjoint_step(steps, K, ck, lam)
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    return {"workload": "2D %dx%d vortex pair%s, c64 forward, FP64 self-interaction Jacobian, %d steps, "
                        "checkpoint every %d, gradient of the final energy" %
                        (w.nx[0], w.ny[0], " with a random spinor of amplitude %g added (F != 0 everywhere)" %
                         w.meta["noise"] if spin_texture else "", steps, K),
            "forward_s": tf, "forward_plus_adjoint_s": ta, "ratio": ta / tf,
            "dL_dg": [a + b for a, b in zip(dg, dg0)]}


def progress(what):
    """One line on stderr as each leg of the benchmark ends (stdout carries only the JSON line)."""
    print("bench: %s" % what, file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    m = measure(args.dtype, args.steps, args.warmup, args.workload, args.split, plan=args.plan)
    progress("%s %s: %.4g site-updates/s, kernel %.4g ms per launch" % (args.workload, args.dtype, m["value"],
                                                                       m["kern_ms"]))
    w, L = m["w"], m["L"]
    ndim = WORKLOADS[args.workload][0]
    S = m["tuning"]["steps_per_pass"]
    kern_ms = m["kern_ms"]
    sites_per_launch = L * S
    flops_site = (FLOPS_PER_SITE_STEP if args.split == "interleaved" else FLOPS_PER_SITE_STEP_PLAIN)[ndim]
    flops_launch = flops_site * sites_per_launch
    achieved_tflops = flops_launch / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    # 2D and 3D plans with qubit_split 1 run the y (and z) half over two launches: twice the passes
    ysplit = ndim >= 2 and m["tuning"]["qubit_split"] == 1
    bytes_launch = BYTES_PER_SITE_PASS[args.dtype] * L * PASSES_PER_STEP[ndim] * (2 if ysplit else 1)
    hbm_gbs = bytes_launch / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    # the roofline that bounds this launch: flops per algorithmic byte against the ridge point
    intensity = flops_launch / bytes_launch
    bound = "alu" if intensity >= PEAK_TFLOPS[args.dtype] * 1e12 / (PEAK_HBM_GBS * 1e9) else "hbm"
    if ndim == 1:
        kernel = ("k_step1d", "k_step1d_pair", "k_step1d_lanes")[m["tuning"]["qubit_split"]]
        key = "%s/S%d" % (kernel, S)
    elif ndim == 2:
        kernel = "k_step2d (the two halves of the y half)" if ysplit else "k_step2d"
        key = "k_step2d/rows%d%s" % (m["tuning"]["tile_rows"], "/ysplit" if ysplit else "")
    else:   # a launch here is one step: the z pass and the y-x pass of the same kernel
        kernel = "k_step2d (z pass + y-x pass%s)" % (", each over two launches" if ysplit else "")
        key = "k_step3d/rows%d%s" % (m["tuning"]["tile_rows"], "/ysplit" if ysplit else "")
    traffic = None
    measured = TRAFFIC["kib"].get("%s/%s/%s" % (args.workload, args.dtype, args.split), {})
    if key in measured and kernel_sources_sha() == TRAFFIC["sources_sha256_16"]:
        fk, wk = measured[key]
        traffic = 1024.0 * (fk * TRAFFIC["fetch_scale"] + wk * TRAFFIC["write_scale"])

    secondary = None
    if args.secondary not in ("none", args.dtype):
        m2 = measure(args.secondary, args.steps, min(args.warmup, 200), args.workload, args.split, plan=args.plan)
        secondary = {"storage": args.secondary, "value": m2["value"], "unit": "site-updates/s",
                     "kernel_ms_avg": m2["kern_ms"], "plan": m2["tuning"], "norm_drift": m2["drift"]}
        progress("secondary %s: %.4g site-updates/s" % (args.secondary, m2["value"]))
    batched = batched_ratio(args.batched_steps) if args.batched_steps > 0 else None
    if batched:
        progress("batched: speedup %.3g" % batched["speedup"])
    adjoint = adjoint_ratio(args.adjoint_steps, 64) if args.adjoint_steps > 0 else None
    if adjoint:
        progress("adjoint: ratio %.3g" % adjoint["ratio"])
        adjoint["spin_texture"] = adjoint_ratio(args.adjoint_steps, 64, spin_texture=True)
        progress("adjoint, spin texture: ratio %.3g" % adjoint["spin_texture"]["ratio"])
    diag = diagnostics(args.workload, args.dtype, args.diag_reps) if args.diag_reps > 0 else None
    if diag:
        progress("diagnostics done")
    potential = None
    if args.trap_steps > 0:
        mt = measure(args.dtype, args.trap_steps, min(args.warmup, 200), args.workload, args.split, trap=True,
                     plan=args.plan)
        potential = {"what": "the same workload in a harmonic trap V = omega^2 r^2/4 (V = 1/2 at the edge "
                             "midpoints) with mu = 0.5", "steps": args.trap_steps, "value": mt["value"],
                     "unit": "site-updates/s", "kernel_ms_avg": mt["kern_ms"], "plan": mt["tuning"],
                     # per step: the two runs may choose plans with different steps per pass
                     "kernel_time_vs_no_potential": (mt["kern_ms"] / mt["tuning"]["steps_per_pass"]) /
                     (kern_ms / S) if kern_ms > 0 and mt["kern_ms"] > 0 else None,
                     "norm_drift": mt["drift"]}
        progress("potential: %.4g site-updates/s" % mt["value"])
    texture = None
    if args.texture_steps > 0 and ndim >= 2:
        mx = measure(args.dtype, args.texture_steps, min(args.warmup, 200), args.workload, args.split,
                     plan=args.plan, texture=True)
        texture = {"what": "the same workload plus a seeded random spinor of amplitude 0.05 in every "
                           "component (F != 0 at every site: the spin rotation acts everywhere)",
                   "steps": args.texture_steps, "value": mx["value"], "unit": "site-updates/s",
                   "kernel_ms_avg": mx["kern_ms"], "plan": mx["tuning"],
                   "kernel_time_vs_workload": mx["kern_ms"] / kern_ms if kern_ms > 0 and mx["kern_ms"] > 0
                   else None, "norm_drift": mx["drift"]}
        progress("spin texture: %.4g site-updates/s" % mx["value"])
    cpu = cpu_baseline(w, args.cpu_steps if ndim == 1 else max(1, args.cpu_steps // 500), ndim) \
        if args.cpu_steps > 0 else None

    out = {
        "metric": "QLG site-updates/s + % HBM roofline; batched and fwd+adjoint vs plain step",
        "value": m["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "c64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "lattice": workload_shape(w, ndim),
            "storage": args.dtype,
            "split": args.split,
            "g": list(w.g),
            "eps": w.eps,
            "observables_every": OBS_EVERY,
            "plan": m["tuning"],
            "plan_source": "fixed by --plan" if args.plan else "autotuned",
            "preroll_steps": m["preroll"],
        },
        "roofline": {
            "bound": bound,
            "achieved": achieved_tflops if bound == "alu" else hbm_gbs,
            "peak": PEAK_TFLOPS[args.dtype] if bound == "alu" else PEAK_HBM_GBS,
            "unit": "TFLOP/s" if bound == "alu" else "GB/s",
            "frac": ((achieved_tflops / PEAK_TFLOPS[args.dtype]) if bound == "alu" else hbm_gbs / PEAK_HBM_GBS)
            if kern_ms > 0 else None,
            "flop_per_byte": intensity,
            "traffic": traffic,
            "traffic_unit": "bytes per launch",
            "kernel": kernel,
            "kernel_ms_avg": kern_ms,
            "launches_timed": m["launches"],
            "flops_per_site_update": flops_site,
            "hbm_algorithmic_gbs": hbm_gbs,
            "hbm_frac": (hbm_gbs / PEAK_HBM_GBS) if hbm_gbs else None,
        },
        "norm_drift": m["drift"],
        "repeats": m["repeats"],
        "value_over_repeats_median": m["value"] / m["repeats"]["median"] if m["repeats"] else None,
        "secondary": secondary,
        "spin_texture": texture,
        "batched": batched,
        "adjoint": adjoint,
        "diagnostics": diag,
        "potential": potential,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, nsteps, ndim=1, box3d=96):
    """The FP64 oracle, as it stands, on the first `nsteps` steps of the same workload (3D: of a
    box3d^3 corner of its state, the whole 256^3 lattice being far beyond a bounded sample), on
    all the threads torch uses; then the per-core rate, one thread on a tenth of that sample (1D:
    a tenth of the steps; 2D and 3D: one step on a corner with about a tenth of the sites)."""
    import torch
    from oracle import qlg_oracle as O
    threads = torch.get_num_threads()
    psi = w.psi[0] if ndim < 3 else np.ascontiguousarray(w.psi[0][:, :box3d, :box3d, :box3d])
    t0 = time.perf_counter()
    O.run_psi(psi, nsteps, w.eps, w.g)
    dt = time.perf_counter() - t0
    sites = int(np.prod(psi.shape[1:]))
    shape = "x".join(str(v) for v in psi.shape[1:]) if ndim > 1 else "L=%d" % w.nx[0]
    what = "same %dD %s workload" % (ndim, shape) if ndim < 3 else \
        "a %s corner of the 3D %s workload" % (shape, "x".join(str(v) for v in workload_shape(w, ndim)))
    if ndim == 1:
        psi1, steps1 = psi, max(1, nsteps // 10)
    else:
        side = max(1, int(round(psi.shape[-1] * 0.1 ** (1.0 / ndim))))
        psi1, steps1 = np.ascontiguousarray(psi[(slice(None),) + (slice(0, side),) * ndim]), 1
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.run_psi(psi1, steps1, w.eps, w.g)
        dt1 = time.perf_counter() - t0
    finally:
        torch.set_num_threads(threads)
    sites1 = int(np.prod(psi1.shape[1:]))
    shape1 = "x".join(str(v) for v in psi1.shape[1:])
    return {"value": sites * nsteps / dt, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%s, first %d steps (FP64 torch CPU, %d threads), %.1f s" % (what, nsteps, threads, dt),
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "per_core": {"value": sites1 * steps1 / dt1, "unit": "site-updates/s", "cores": 1,
                         "sample": "%s sites, first %d steps, 1 thread, %.1f s" % (shape1, steps1, dt1)}}


if __name__ == "__main__":
    main()
