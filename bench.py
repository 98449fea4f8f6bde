"""Benchmark of the EM-PIC step on one MI355X.

Workload (the benchmark configuration): periodic 128^3 grid, dx = 1 (c/omega_p),
dt at Courant 0.5, 8 electrons + 8 protons per cell (33.55M particles),
thermal v_th = 0.05c, equal temperatures.  One step is the whole PIC cycle:
Faraday + centring of B, gather + Boris + move + ZigZag for both species,
Ampere-Maxwell, and the counting sort whenever the library's adaptive policy
calls for it (particles leaving their tile windows faster than 2e-5 of the
slots per step, at most 64 steps apart; about every 25 steps here).  Inputs
are generated once (seeded) and resident in HBM before timing.  The plain
FP64 step keeps its particles unsorted.

Prints one JSON line.  value = FP32 cell-relative particle-pushes/s; the plain
FP64 step on the same workload is reported beside it.  The dominant kernel is
the fused FP32 particle kernel; its roofline entry uses the algorithmic bytes
56 per particle (28 read + 28 written) + 36 per cell (E and centred B read,
J written) per launch over its HIP-event-timed average duration.  It reaches
about 41 % of the 8 TB/s peak, short of a 50 % target: the kernel is
co-limited by VALU issue (~411 instructions per particle) and its LDS
atomics rather than by HBM (its traffic is within 9 % of the algorithmic
bytes).  The "adjoint" entry times a 50-step forward + adjoint on a 128^3 anisotropic
plasma (see adjoint_leg); "shape_order_2" the same plasma stepped with
second-order shapes (b_2 weighting, EZ current).  cpu_baseline: the FP64
oracle on one core, 5 steps of a 64^3 box of the same plasma.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-pushes/s (gather+push+deposit+Yee) FP32 vs FP64; adjoint step ms"
COUNTERS = os.path.join(ROOT, "profiles", "push_fused_thermal_ep_128_counters.json")
# the fused kernel's source: its file and the headers it is built from
KERNEL_SRC = [os.path.join(ROOT, "paper_2609_16575_amd", "csrc", f)
              for f in ("push_f32.hip", "pic_math.hpp", "internal.hpp")]


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def time_steps(sim, steps, warmup, torch, events="all"):
    """Wall time of `steps` steps after `warmup` untimed ones, and the HIP
    event times of the kernels over the same steps.  events: "all" kernel
    groups; "push", only the fused particle kernel, timed by events attached
    to its own dispatch (no event marker sits between the other kernels of
    the step); None, no events."""
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.kernel_times()  # discard warm-up timing
    sim.enable_timing(events is not None, push_only=events == "push")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = sim.kernel_times()
    sim.enable_timing(False)
    sim.sync()
    return (t1 - t0), kt


def traffic_from_counters(nbytes_alg):
    """HBM bytes per launch of the fused kernel from committed rocprofv3 PMC
    summaries, or None when they are missing or older than the kernel."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("kernel_source_sha") != kernel_sha():
        return None
    return (c["fetch_kib_per_dispatch"] * c["copy_scale_fetch"] +
            c["write_kib_per_dispatch"] * c["copy_scale_write"]) * 1024.0


def cpu_baseline(n=(64, 64, 64), steps=5):
    """The FP64 oracle (single thread) on a 64^3 box of the same plasma (same
    density, temperatures and cell size), 5 steps: about 15 s of CPU work.
    One step of the whole 128^3 box takes about a minute on one core."""
    from oracle import oracle as O
    from paper_2609_16575_amd import workloads as W
    w = W.thermal_two_species(n=n)
    o = O.OracleSim(w.n, w.d, w.dt)
    for s in w.species:
        o.add_species(s.q, s.m, s.w, s.pos, s.u)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": w.n_particles * steps / dt, "unit": "particle-pushes/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d steps of the same plasma on a %dx%dx%d box (%d particles), "
                      "single-threaded FP64 C, %.1f s" % (steps, *w.n, w.n_particles, dt)}


def adjoint_leg(torch, n=128, steps=50, K=10):
    """Forward + adjoint on a 128^3 periodic slice of the anisotropic
    (T_x/T_perp = 25) electron plasma, 16 per cell (33.55M particles), 50
    steps, checkpoints and sorts every 10 steps; loss = 1/2 dV sum |B|^2 of
    the final step.  Reports the plain FP32 step on the same workload (sort
    every 10) beside the differentiable forward and the adjoint step
    (backward wall time over the steps: segment recompute + step VJPs)."""
    from paper_2609_16575_amd import autograd as AG
    from paper_2609_16575_amd import workloads as W
    from paper_2609_16575_amd.sim import Sim
    w = W.weibel_bimaxwellian(n=(n,) * 3, steps=steps, sort_every=K)
    sim = Sim(w, precision="fp32")
    wall, _ = time_steps(sim, steps, 5, torch, events=None)  # as the adjoint: no events
    fwd_ms = 1e3 * wall / steps
    sim.close()
    del sim
    torch.cuda.empty_cache()
    sim = Sim(w, precision="fp32", sort_every=0)
    sim.sort()
    st0 = sim.save_state()
    U = sim.current_buffers(0)["u"].clone()
    dV = float(w.d[0] * w.d[1] * w.d[2])
    rec = {}
    for rep in range(2):  # the first run warms up
        sim.load_state(st0)
        U0 = U.clone().requires_grad_(True)
        E0 = torch.zeros_like(sim.E).requires_grad_(True)
        B0 = torch.zeros_like(sim.B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, BN = AG.run(sim, steps, K, E0, B0, [U0], sort=True)
        loss = 0.5 * dV * (BN * BN).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rec = {"fwd": t1 - t0, "bwd": t2 - t1, "loss": float(loss.item()),
               "gU_norm": sim.dot_f64(U0.grad, U0.grad) ** 0.5,
               "finite": bool(torch.isfinite(U0.grad).all().item() and torch.isfinite(E0.grad).all().item())}
        _log("adjoint rep %d: fwd %.3f s bwd %.3f s" % (rep, rec["fwd"], rec["bwd"]))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    adj_ms = 1e3 * rec["bwd"] / steps
    return {"workload": "anisotropic electron plasma (T_x/T_perp=25, v_th,x=0.25c), periodic "
                        "%dx%dx%d, 16 per cell (%d particles), %d steps, checkpoints and sorts "
                        "every %d, loss 1/2 dV sum |B|^2" % (n, n, n, w.n_particles, steps, K),
            "forward_step_ms": fwd_ms,
            "diff_forward_ms_per_step": 1e3 * rec["fwd"] / steps,
            "adjoint_step_ms": adj_ms,
            "adjoint_over_forward": adj_ms / fwd_ms,
            "loss": rec["loss"], "grad_u_norm": rec["gU_norm"], "grad_finite": rec["finite"]}


def field_only_leg(torch, n=256, steps=50):
    """The Yee update alone (Faraday + centring of B, Ampere-Maxwell) on a
    periodic vacuum grid of n^3 cells: field cell-updates/s and the HBM
    rate of the two curl kernels (60 + 48 algorithmic bytes per cell in
    FP32: Faraday reads E, B and writes B, B-bar and the zeroed J; Ampere
    reads E, B, J and writes E)."""
    from paper_2609_16575_amd import workloads as W
    from paper_2609_16575_amd.sim import Sim
    w = W.Workload("vacuum", (n,) * 3, (1.0,) * 3, W.courant_dt((1.0,) * 3), (0, 0, 0), [])
    w.E0, w.B0 = W.random_fields(w.n, scale=1.0, seed=3)
    sim = Sim(w, precision="fp32")
    wall, kt = time_steps(sim, steps, 5, torch)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    cells = w.n_cells
    field_ms = kt["field_ms"] / steps
    gbs = 108.0 * cells / (field_ms * 1e-3) / 1e9
    return {"workload": "vacuum, periodic %d^3, FP32" % n, "cell_updates_per_s": cells * steps / wall,
            "ms_per_step": 1e3 * wall / steps, "curl_kernels_ms_per_step": field_ms,
            "achieved_GBps": gbs, "frac_of_hbm": gbs / HBM_PEAK_GBS,
            "algorithmic_bytes_per_cell": 108}


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def other_workload(args, torch):
    """FP32 step time of the other workloads at their full sizes (not the
    headline line): the static-window wakefield box, the 256^3 anisotropic
    plasma, and the two-dimensional wakefield run with its moving window."""
    from paper_2609_16575_amd import workloads as W
    from paper_2609_16575_amd.sim import Sim
    sort_every = None
    if args.workload == "lwfa":
        w = W.lwfa_slab()
        sort_every = -1
        desc = ("laser-wakefield box 1024x128x128, Mur faces, laser a0=2, cold slab with ramp, "
                "2 per cell, per-particle weights (%d particles), adaptive sort" % w.n_particles)
    elif args.workload == "weibel256":
        w = W.weibel_bimaxwellian()
        desc = ("anisotropic electron plasma T_x/T_perp=25, periodic 256^3, 16 per cell "
                "(%d particles), sort every 10" % w.n_particles)
    else:
        w = W.lwfa_2d(per=(4, 2, 4))
        w.laser.t0 = 0.0
        w.window.t_start = 0.0
        desc = ("two-dimensional wakefield 1400x2x300, ppc 32, a0=3, window moving from the start "
                "(%d particles), 16x2x8 tiles, adaptive sort" % w.n_particles)
    sim = Sim(w, precision="fp32", sort_every=sort_every)
    wall, kt = time_steps(sim, args.steps, args.warmup, torch, events="push")
    _, kb = time_steps(sim, args.steps, 0, torch)  # breakdown: every kernel group timed
    push_ms = kt["push_ms"] / max(kt["push_n"], 1)
    wpp = any(s.wpp is not None for s in w.species)
    nbytes = (60.0 if wpp else 56.0) * w.n_particles + 36.0 * w.n_cells
    achieved = nbytes / (push_ms * 1e-3) / 1e9
    d = sim.diagnostics()
    out = {"metric": METRIC, "value": w.n_particles * args.steps / wall, "unit": "particle-pushes/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": desc, "particles": w.n_particles, "cells": w.n_cells},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_push_fused",
                        "avg_ms": push_ms, "algorithmic_bytes_per_launch": nbytes},
           "breakdown_ms_per_step": {"push_fused": kb["push_ms"] / args.steps,
                                     "fields": kb["field_ms"] / args.steps,
                                     "sort": kb["sort_ms"] / args.steps},
           "fp32_checks": {"fault_word": d["fault_word"],
                           "fallback_particles": d["fallback_particles"]}}
    sim.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--only", choices=["fp32", "order2", "fp64", "adjoint", "fields"],
                    default=None)
    ap.add_argument("--workload", choices=["thermal", "lwfa", "weibel256", "lwfa2d"],
                    default="thermal", help="thermal (the benchmark) or another workload's FP32 step")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.workload != "thermal":
        other_workload(args, torch)
        return
    from paper_2609_16575_amd import workloads as W
    from paper_2609_16575_amd.sim import Sim

    if args.calibrate_copy:
        copy_calibration(torch)
    n = (args.n,) * 3
    t0 = time.perf_counter()
    w = W.thermal_two_species(n=n)
    _log("generated %d particles in %.1f s" % (w.n_particles, time.perf_counter() - t0))
    npart, ncell = w.n_particles, w.n_cells
    out = {"metric": METRIC, "value": None, "unit": "particle-pushes/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "thermal e+p plasma, periodic %dx%dx%d, dx=1, Courant 0.5, "
                                  "8 e- + 8 p+ per cell (%d particles), v_th=0.05c, adaptive sort"
                                  % (*n, npart),
                      "particles": npart, "cells": ncell, "sort": "adaptive"}}

    if args.only in (None, "fp32"):
        sim = Sim(w, precision="fp32", sort_every=-1)
        _log("fp32 sim ready")
        wall, kt = time_steps(sim, args.steps, args.warmup, torch, events="push")
        # breakdown over as many further steps, every kernel group timed
        _, kb = time_steps(sim, args.steps, 0, torch)
        d = sim.diagnostics()
        ms = 1e3 * wall / args.steps
        out["value"] = npart * args.steps / wall
        out["ms_per_step"] = ms
        out["cell_updates_per_s"] = ncell * args.steps / wall
        push_ms = kt["push_ms"] / max(kt["push_n"], 1)
        nbytes = 56.0 * npart + 36.0 * ncell
        achieved = nbytes / (push_ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": traffic_from_counters(nbytes),
                           "kernel": "k_push_fused", "avg_ms": push_ms,
                           "algorithmic_bytes_per_launch": nbytes}
        out["breakdown_ms_per_step"] = {
            "push_fused": kb["push_ms"] / args.steps, "fields": kb["field_ms"] / args.steps,
            "sort": kb["sort_ms"] / args.steps}
        out["fp32_checks"] = {"fault_word": d["fault_word"],
                              "fallback_particles": d["fallback_particles"],
                              "U_tot": d["U_tot"]}
        sim.close()
        del sim
        torch.cuda.empty_cache()

    if args.only in (None, "order2"):
        # the same plasma with second-order shapes (b_2 weighting, EZ current)
        sim = Sim(w, precision="fp32", sort_every=-1, shape_order=2)
        _log("order-2 sim ready")
        wall, kt = time_steps(sim, args.steps, args.warmup, torch, events="push")
        d = sim.diagnostics()
        push_ms = kt["push_ms"] / max(kt["push_n"], 1)
        nbytes = 56.0 * npart + 36.0 * ncell
        achieved = nbytes / (push_ms * 1e-3) / 1e9
        out["shape_order_2"] = {
            "value": npart * args.steps / wall, "unit": "particle-pushes/s",
            "ms_per_step": 1e3 * wall / args.steps,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_push_fused (order 2)", "avg_ms": push_ms,
                         "algorithmic_bytes_per_launch": nbytes},
            "fault_word": d["fault_word"], "fallback_particles": d["fallback_particles"]}
        sim.close()
        del sim
        torch.cuda.empty_cache()

    if not args.no_fp64 and args.only in (None, "fp64"):
        sim = Sim(w, precision="fp64")
        _log("fp64 sim ready")
        wall, kt = time_steps(sim, args.steps, args.warmup, torch)
        out["fp64_plain"] = {"value": npart * args.steps / wall, "unit": "particle-pushes/s",
                             "ms_per_step": 1e3 * wall / args.steps,
                             "push_ms_per_step": kt["push_ms"] / args.steps,
                             "field_ms_per_step": kt["field_ms"] / args.steps}
        if out["value"]:
            out["speedup_fp32_vs_fp64"] = out["value"] / out["fp64_plain"]["value"]
        sim.close()
        del sim
        torch.cuda.empty_cache()

    if args.only in (None, "fields"):
        out["fields_only"] = field_only_leg(torch)

    out["adjoint"] = None
    if not args.no_adjoint and args.only in (None, "adjoint"):
        out["adjoint"] = adjoint_leg(torch)
    if not args.no_cpu_baseline and args.only is None:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
