"""Write ``weibel16_current_noise.json``: how much FP32-sized rounding noise
in the current moves the gradients of the small anisotropic (Weibel) run.

The run: periodic 16^3 cells, 4 electrons per cell, T_x/T_perp = 25
(v_th,x = 0.25 c), immobile ions, 40 steps from E = B = 0; loss
L = 1/2 dV sum over the box of |B^{N-1/2}|^2; gradients along a seeded
smooth random direction of all initial momenta and along a seeded random
initial E (the directions of the GPU test of sorted against unsorted runs).

Two FP32 GPU runs of the same plasma that add the tile windows' currents
to J in different orders differ, every step, by about one FP32 rounding of
J.  Here the FP64 oracle's forward and chained adjoint (checkpoint every 10
steps) run once as they are and then with J multiplied after every deposit
by (1 + delta), delta uniform in [-2^-24, 2^-24] per entry (seeded): the
relative change of the gradients over the 40 steps of instability growth
is the size of the difference such rounding makes.

A second set of samples instead rounds the state (E, B, momenta, in-cell
offsets) stochastically to FP32 after every step, each sample with its own
seed (the rounding of make_langmuir32_noise.py): two such runs differ by
FP32 rounding everywhere, as two FP32 runs do once any one value has
rounded differently.

Inputs come from the seeded generator module; nothing here runs the HIP
path.  Run from the repository root:
    python tests/golden/make_weibel16_noise.py
(about a minute).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2609_16575_amd import workloads as W  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import make_langmuir32_noise as N  # noqa: E402

STEPS, K = 40, 10
SEEDS = (1, 2, 3, 4, 5, 6)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weibel16_current_noise.json")


def _workload():
    return W.weibel_bimaxwellian(n=(16, 16, 16), ppc=4, steps=STEPS, sort_every=0)


def _directions(w):
    box = np.asarray(w.n) * np.asarray(w.d)
    dirU = W.smooth_random_direction(w.species[0].pos, box, 21)
    dirE = 1e-3 * np.random.default_rng(22).standard_normal((3,) + tuple(w.n[::-1]))
    return dirU, dirE


def _state_sr(o, rng):
    """The state stochastically rounded to FP32 (cell + FP32 offset)."""
    o.E[...] = N._sr32(o.E, rng)
    o.B[...] = N._sr32(o.B, rng)
    n = np.asarray(o.n, float)
    d = np.asarray(o.d, float)
    for s in o.species:
        xi = s.pos / d
        i = np.floor(xi)
        off = N._sr32(xi - i, rng)
        up = off >= 1.0
        i = np.mod(np.where(up, i + 1.0, i), n)
        s.pos[...] = (i + np.where(up, 0.0, off)) * d
        s.u[...] = N._sr32(s.u, rng)


def _step(o, rng, mode="J"):
    """One periodic step of the oracle; with rng, mode "J": J multiplied by
    (1 + delta) after the deposit, mode "state": the state stochastically
    rounded to FP32 after the step."""
    L = O.lib()
    g = O.C.byref(o.g)
    L.orc_faraday(g, O._p(o.E), O._p(o.B), O._p(o.Bbar))
    o.J[...] = 0.0
    for s in o.species:
        L.orc_push_deposit(g, O._p(o.E), O._p(o.Bbar), O._p(o.J), s.np, O._p(s.pos), O._p(s.u),
                           O._p8(s.alive), O._p(s.wpp), s.q, s.m, s.w, 0, 0, None)
    if rng is not None and mode == "J":
        o.J *= 1.0 + rng.uniform(-2.0 ** -24, 2.0 ** -24, o.J.shape)
    L.orc_ampere(g, O._p(o.E), O._p(o.B), O._p(o.J))
    o.nstep += 1
    if rng is not None and mode == "state":
        _state_sr(o, rng)


def run(seed, mode="J"):
    """(L, <dL/dU0, dirU>, <dL/dE0, dirE>) of the oracle run; seed None: no
    perturbation."""
    w = _workload()
    dirU, dirE = _directions(w)
    rng = None if seed is None else np.random.default_rng(seed)
    o = O.OracleSim(w.n, w.d, w.dt)
    s = w.species[0]
    o.add_species(s.q, s.m, s.w, s.pos, s.u)
    ckpt, trace_rng = {}, {}
    for n in range(STEPS):
        if n % K == 0:
            ckpt[n] = o.state()
            # the generator's state, so that the recomputation draws the same deltas
            trace_rng[n] = None if rng is None else rng.bit_generator.state
        _step(o, rng, mode)
    dV = w.d[0] * w.d[1] * w.d[2]
    Lv = 0.5 * dV * float(np.sum(o.B ** 2))
    lE = np.zeros_like(o.E)
    lB = dV * o.B.copy()
    lX = [np.zeros_like(s.pos)]
    lU = [np.zeros_like(s.pos)]
    for seg in reversed(range(0, STEPS, K)):
        o.set_state(ckpt[seg])
        r2 = None
        if rng is not None:
            r2 = np.random.default_rng()
            r2.bit_generator.state = trace_rng[seg]
        states = []
        for _ in range(K):
            states.append(o.state())
            _step(o, r2, mode)
        for st in reversed(states):
            o.set_state(st)
            lE, lB, lX, lU = o.step_vjp(lE, lB, lX, lU)
    return Lv, float(np.sum(lU[0] * dirU)), float(np.sum(lE * dirE))


def main():
    L0, gU0, gE0 = run(None)
    out = {
        "what": "FP64 oracle gradients of the 16^3 Weibel run (4 per cell, 40 steps, checkpoints "
                "every 10) without and with J multiplied by (1 + U[-2^-24, 2^-24]) after every "
                "deposit (J_noise), and with the state stochastically rounded to FP32 after "
                "every step (state_rounding); written by make_weibel16_noise.py from oracle/ "
                "alone",
        "L": L0, "gU": gU0, "gE": gE0,
    }
    for mode, key in (("J", "J_noise"), ("state", "state_rounding")):
        samples = []
        for sd in SEEDS:
            Lp, gU, gE = run(sd, mode)
            samples.append({"seed": sd, "L": Lp, "gU": gU, "gE": gE,
                            "gU_rel_change": abs(gU - gU0) / abs(gU0),
                            "gE_rel_change": abs(gE - gE0) / abs(gE0)})
            print(mode, json.dumps(samples[-1]), flush=True)
        out[key] = {"samples": samples,
                    "max_gU_rel_change": max(s["gU_rel_change"] for s in samples),
                    "max_gE_rel_change": max(s["gE_rel_change"] for s in samples)}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: (v if not isinstance(v, dict) else {a: b for a, b in v.items() if a != "samples"})
                      for k, v in out.items()}, indent=1))


if __name__ == "__main__":
    main()
