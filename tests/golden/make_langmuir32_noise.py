"""Write ``langmuir32_fp32_noise.json``: how much FP32-sized rounding noise
alone moves the loss and the gradients of the differentiable cold-plasma run
(the run of ``make_langmuir32_gradients.py``: 32^3, 16 per cell, eps = 1e-2,
500 steps, probe [12, 20)^3).

Each sample repeats the FP64 oracle's forward and chained adjoint with the
state stochastically rounded to FP32 after every step: every field value,
momentum and in-cell offset goes to one of its two neighbouring FP32 values,
the upper one with probability equal to the fraction of the gap the value
has covered (an unbiased rounding with a seeded generator, so each sample is
one draw of FP32-sized rounding errors with no systematic part).  At step
500 the probe energy is near a node of the oscillation, where a phase error
is amplified into the energy; the spread over the samples is the size of the
difference between two FP32 computations of the same run that round in
different places.

Inputs come from the seeded generator module; nothing here runs the HIP
path.  Run from the repository root:
    python tests/golden/make_langmuir32_noise.py
(about 35 minutes on 5 cores).
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import make_langmuir32_gradients as G  # noqa: E402

SEEDS = (11, 12, 13, 14, 15)
OUT = os.path.join(HERE, "langmuir32_fp32_noise.json")


def _sr32(x, rng):
    """x (float64 array) rounded stochastically to a neighbouring FP32 value."""
    f = x.astype(np.float32)
    below = f.astype(np.float64) <= x
    lo = np.where(below, f, np.nextafter(f, np.float32(-np.inf)))
    hi = np.nextafter(lo, np.float32(np.inf))
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    gap = hi64 - lo64
    p = np.where(gap > 0, (x - lo64) / np.where(gap > 0, gap, 1.0), 0.0)
    return np.where(rng.random(x.shape) < p, hi64, lo64)


def _rounder(seed):
    rng = np.random.default_rng(seed)

    def rnd(o):
        o.E[...] = _sr32(o.E, rng)
        o.B[...] = _sr32(o.B, rng)
        n = np.asarray(o.n, float)
        d = np.asarray(o.d, float)
        for s in o.species:
            xi = s.pos / d
            i = np.floor(xi)
            off = _sr32(xi - i, rng)
            up = off >= 1.0
            i = np.where(up, i + 1.0, i)
            off = np.where(up, 0.0, off)
            i = np.mod(i, n)
            s.pos[...] = (i + off) * d
            s.u[...] = _sr32(s.u, rng)
    return rnd


def _forward_rounding_all(kind, seed=0):
    """Loss of the FP64 forward with every array the FP32 path stores rounded
    to FP32 where the step writes it: B-bar after Faraday, J after the
    deposit, E and B after Ampere, positions (cell + FP32 offset) and
    momenta after the push.  kind "rn": round to nearest even (what FP32
    storage does); "sr": the seeded stochastic rounding above."""
    rng = np.random.default_rng(seed)
    r = (lambda x: x.astype(np.float32).astype(np.float64)) if kind == "rn" else (lambda x: _sr32(x, rng))
    state = G._round_fp32 if kind == "rn" else _rounder(seed)
    o, _ = G._sim(G.EPS)
    m = G._mask(o.E.shape)
    state(o)
    L = G.O.lib()
    g = G.O.C.byref(o.g)
    P = G.O._p
    for _ in range(G.STEPS):
        L.orc_faraday(g, P(o.E), P(o.B), P(o.Bbar))
        o.Bbar[...] = r(o.Bbar)
        o.J[...] = 0.0
        for sp in o.species:
            L.orc_push_deposit(g, P(o.E), P(o.Bbar), P(o.J), sp.np, P(sp.pos), P(sp.u),
                               G.O._p8(sp.alive), P(sp.wpp), sp.q, sp.m, sp.w, 0, 0, None)
        o.J[...] = r(o.J)
        L.orc_ampere(g, P(o.E), P(o.B), P(o.J))
        o.nstep += 1
        state(o)
    return {"kind": kind, "seed": seed, "L": float(G._loss(o, m))}


def _sample(seed):
    r = G.adjoint(_rounder(seed))
    return {"seed": seed, "L": r["L"], "dL_deps": r["dL_deps"], "dL_ddir": r["dL_ddir"]}


def _all_arrays():
    tasks = [("rn", 0)] + [("sr", sd) for sd in SEEDS[:3]]
    with mp.get_context("fork").Pool(len(tasks)) as pool:
        res = pool.starmap(_forward_rounding_all, tasks, chunksize=1)
    return res


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--all-arrays":
        res = _all_arrays()
        out = json.load(open(OUT))
        ref = json.load(open(G.OUT))
        for r in res:
            r["L_rel_dev_from_fp64"] = (r["L"] - ref["L"]) / ref["L"]
        out["all_arrays_rounded"] = res
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(res, indent=1))
        return
    with mp.get_context("fork").Pool(len(SEEDS)) as pool:
        res = pool.map(_sample, SEEDS, chunksize=1)
    ref = json.load(open(G.OUT))
    spread = {}
    for k, rk in (("L", "L"), ("dL_deps", "adjoint_dL_deps"), ("dL_ddir", "adjoint_dL_ddir")):
        dev = [abs(r[k] - ref[rk]) / abs(ref[rk]) for r in res]
        spread[k] = {"max_rel_dev_from_fp64": max(dev),
                     "rms_rel_dev_from_fp64": float(np.sqrt(np.mean(np.square(dev))))}
    out = {
        "what": "FP64 oracle run of the 32^3 500-step differentiable workload with the state "
                "stochastically rounded to FP32 after every step (seeded); written by "
                "make_langmuir32_noise.py from oracle/ alone",
        "seeds": list(SEEDS), "samples": res, "spread": spread,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
