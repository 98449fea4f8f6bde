"""Write ``langmuir32_gradients.json``: FP64 oracle gradients of the
differentiable cold-plasma run, the reference of the GPU adjoint's test at
full size.

The run: periodic 32^3 cells, 16 electrons per cell on a (4, 2, 2) quiet
lattice, u_x = eps sin(2 pi x / L_x) with eps = 1e-2, 500 steps; loss
L = 1/2 dV sum over the probe cells [12, 20)^3 of |E^N|^2 + |B^{N-1/2}|^2.
What is computed, all with the FP64 CPU oracle only:

* the chained discrete adjoint (the oracle's one-step VJPs taken backwards
  through the stored trajectory, re-computed from checkpoints every 50
  steps): dL/d eps and the projection of dL/du^{-1/2} on a seeded smooth
  random direction of all initial momenta;
* central differences of the FP64 forward, h = 1e-4, on eps and along that
  direction;
* the same adjoint along a trajectory whose state is rounded after every
  step to what FP32 cell-relative storage can hold (fields and momenta to
  FP32, in-cell offsets to FP32): how far the storage precision alone moves
  the loss and the gradients.

Inputs come from the seeded generator module; nothing here runs the HIP
path.  Run from the repository root:
    python tests/golden/make_langmuir32_gradients.py
(about 35 minutes on 6 cores).
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2609_16575_amd import workloads as W  # noqa: E402

EPS, H, STEPS, K = 1e-2, 1e-4, 500, 50
PROBE = (12, 20)
DIR_SEED = 3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "langmuir32_gradients.json")


def _workload(eps):
    return W.cold_langmuir_lattice(eps=eps, steps=STEPS)


def _direction():
    w = _workload(EPS)
    box = np.asarray(w.n) * np.asarray(w.d)
    return W.smooth_random_direction(w.species[0].pos, box, DIR_SEED)


def _mask(shape):
    m = np.zeros(shape[1:], bool)
    lo, hi = PROBE
    m[lo:hi, lo:hi, lo:hi] = True
    return m


def _sim(eps, dirU=None, h=0.0):
    w = _workload(eps)
    o = O.OracleSim(w.n, w.d, w.dt)
    s = w.species[0]
    u = s.u if dirU is None else s.u + h * dirU
    o.add_species(s.q, s.m, s.w, s.pos, u)
    o.rho_bg = w.rho_bg
    return o, w


def _loss(o, m):
    return 0.5 * o.dV * (np.sum(o.E[:, m] ** 2) + np.sum(o.B[:, m] ** 2))


def _round_fp32(o):
    """The state as FP32 cell-relative storage holds it: E, B, u rounded to
    FP32; positions as cell index + FP32 offset in [0, 1) (an offset that
    rounds up to 1 moves to offset 0 of the next cell, periodic)."""
    o.E[...] = o.E.astype(np.float32)
    o.B[...] = o.B.astype(np.float32)
    n = np.asarray(o.n, float)
    d = np.asarray(o.d, float)
    for s in o.species:
        xi = s.pos / d
        i = np.floor(xi)
        off = (xi - i).astype(np.float32).astype(np.float64)
        up = off >= 1.0
        i = np.where(up, i + 1.0, i)
        off = np.where(up, 0.0, off)
        i = np.mod(i, n)
        s.pos[...] = (i + off) * d
        s.u[...] = s.u.astype(np.float32)


def forward_loss(args):
    eps, use_dir, h = args
    dirU = _direction() if use_dir else None
    o, _ = _sim(eps, dirU, h)
    o.step(STEPS)
    return _loss(o, _mask(o.E.shape))


def adjoint(rnd=None):
    """Loss and chained-adjoint gradients of the run; rnd(o), if given, is
    applied to the state at the start and after every step (True: the
    FP32 storage rounding of _round_fp32)."""
    if rnd is True:
        rnd = _round_fp32
    t0 = time.time()
    o, w = _sim(EPS)
    m = _mask(o.E.shape)
    if rnd:
        rnd(o)
    x0 = o.species[0].pos.copy()
    ckpt = {}
    trace = []
    for n in range(STEPS):
        if n % K == 0:
            ckpt[n] = o.state()
        o.step(1)
        if rnd:
            rnd(o)
        trace.append(_loss(o, m))
    L = trace[-1]
    lE = np.where(m[None], o.dV * o.E, 0.0)
    lB = np.where(m[None], o.dV * o.B, 0.0)
    lX = [np.zeros_like(x0)]
    lU = [np.zeros_like(x0)]
    for seg in reversed(range(0, STEPS, K)):
        o.set_state(ckpt[seg])
        states = []
        for _ in range(min(K, STEPS - seg)):
            states.append(o.state())
            o.step(1)
            if rnd:
                rnd(o)
        for st in reversed(states):
            o.set_state(st)
            lE, lB, lX, lU = o.step_vjp(lE, lB, lX, lU)
        print("rounded=%d segment %d done, %.0f s" % (bool(rnd), seg, time.time() - t0), flush=True)
    S = np.sin(2 * np.pi * x0[:, 0] / (w.n[0] * w.d[0]))
    g_eps = float(np.sum(lU[0][:, 0] * S))
    g_dir = float(np.sum(lU[0] * _direction()))
    return {"L": float(L), "L_peak": float(max(trace)), "dL_deps": g_eps, "dL_ddir": g_dir,
            "trace": [float(x) for x in trace], "seconds": time.time() - t0}


def _task(t):
    kind, arg = t
    if kind == "adj":
        return adjoint(arg)
    return forward_loss(arg)


def main():
    tasks = [("adj", False), ("adj", True),
             ("fwd", (EPS + H, False, 0.0)), ("fwd", (EPS - H, False, 0.0)),
             ("fwd", (EPS, True, H)), ("fwd", (EPS, True, -H))]
    with mp.get_context("fork").Pool(len(tasks)) as pool:
        res = pool.map(_task, tasks, chunksize=1)
    a64, a32 = res[0], res[1]
    fd_eps = (res[2] - res[3]) / (2 * H)
    fd_dir = (res[4] - res[5]) / (2 * H)
    out = {
        "what": "FP64 oracle gradients of the differentiable cold-plasma run (32^3, 16 per "
                "cell on a (4,2,2) lattice, eps=1e-2, 500 steps, probe [12,20)^3); written by "
                "make_langmuir32_gradients.py from oracle/ alone",
        "eps": EPS, "h": H, "steps": STEPS, "checkpoint_every": K, "probe": list(PROBE),
        "direction_seed": DIR_SEED,
        "L": a64["L"], "L_peak": a64["L_peak"],
        "adjoint_dL_deps": a64["dL_deps"], "adjoint_dL_ddir": a64["dL_ddir"],
        "fd_dL_deps": fd_eps, "fd_dL_ddir": fd_dir,
        "fp32_state": {"L": a32["L"], "dL_deps": a32["dL_deps"], "dL_ddir": a32["dL_ddir"]},
        "loss_trace_fp64": a64["trace"],
        "loss_trace_fp32_state": a32["trace"],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if "trace" not in k}, indent=1))


if __name__ == "__main__":
    main()
