"""Pins of the oracle's adjoint (vector-Jacobian product) of one step.

The adjoint is not in the paper; it is checked against what mathematics
fixes independently of its code: the transpose identity of the two discrete
curls, and central finite differences of the forward step (itself pinned by
the other oracle tests) along random directions, for one step and for the
probe-energy gradient of a cold Langmuir run with respect to the amplitude.
"""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16575_amd import workloads as W


def test_curl_transpose_identity():
    n, d = (5, 4, 6), (1.0, 0.7, 1.3)
    g = O.make_grid(n, d, 0.3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 6, 4, 5))   # E-located
    y = rng.standard_normal((3, 6, 4, 5))   # B-located
    L = O.lib()
    Bx = np.zeros_like(x)
    L.orc_faraday(ctypes.byref(g), O._p(x), O._p(Bx), None)
    cf_x = -Bx / 0.3                          # curl_f(x)
    Ey = np.zeros_like(y)
    L.orc_ampere(ctypes.byref(g), O._p(Ey), O._p(np.ascontiguousarray(y)), None)
    cb_y = Ey / 0.3                           # curl_b(y)
    lhs, rhs = np.sum(cf_x * y), np.sum(x * cb_y)
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def _random_sim(seed, n=(5, 4, 6), d=(1.0, 0.8, 1.2), npart=12):
    rng = np.random.default_rng(seed)
    sim = O.OracleSim(n, d, O.courant_dt(d))
    sim.E[...] = 0.2 * rng.standard_normal(sim.E.shape)
    sim.B[...] = 0.2 * rng.standard_normal(sim.B.shape)
    L = np.asarray(n) * np.asarray(d)
    for q, m in ((-1.0, 1.0), (1.0, 5.0)):
        pos = rng.random((npart, 3)) * L
        u = 0.4 * rng.standard_normal((npart, 3))
        sim.add_species(q, m, 0.3, pos, u)
    return sim, rng


def _outputs(sim):
    return sim.E.copy(), sim.B.copy(), [s.pos.copy() for s in sim.species], [s.u.copy() for s in sim.species]


def _dot(a, b, L):
    """<a, b> over (E, B, X[], U[]) with minimal-image position differences."""
    tot = np.sum(a[0] * b[0]) + np.sum(a[1] * b[1])
    for xa, xb in zip(a[2], b[2]):
        tot += np.sum(xa * xb)
    for ua, ub in zip(a[3], b[3]):
        tot += np.sum(ua * ub)
    return tot


@pytest.mark.parametrize("seed,filt", [(0, (0, 0)), (1, (0, 0)), (2, (0, 0)), (0, (1, 1)), (1, (2, 0))])
def test_one_step_vjp_matches_central_differences(seed, filt):
    """filt: current filter (binomial passes, compensate) inside the step."""
    sim, rng = _random_sim(seed)
    sim.filter = filt
    Lbox = np.asarray(sim.n) * np.asarray(sim.d)
    s0 = sim.state()
    lam = (rng.standard_normal(sim.E.shape), rng.standard_normal(sim.B.shape),
           [rng.standard_normal(s.pos.shape) for s in sim.species],
           [rng.standard_normal(s.u.shape) for s in sim.species])
    vjp = sim.step_vjp(*lam)
    for trial in range(3):
        dirn = (rng.standard_normal(sim.E.shape), rng.standard_normal(sim.B.shape),
                [rng.standard_normal(s.pos.shape) for s in sim.species],
                [rng.standard_normal(s.u.shape) for s in sim.species])
        h = 1e-6
        outs = []
        for sgn in (1.0, -1.0):
            E, B, X, U = s0
            sim.set_state((E + sgn * h * dirn[0], B + sgn * h * dirn[1],
                           [np.mod(x + sgn * h * dx, Lbox) for x, dx in zip(X, dirn[2])],
                           [u + sgn * h * du for u, du in zip(U, dirn[3])]))
            sim.step(1)
            outs.append(_outputs(sim))
        diff = [(outs[0][0] - outs[1][0]) / (2 * h), (outs[0][1] - outs[1][1]) / (2 * h), [], []]
        for xp, xm in zip(outs[0][2], outs[1][2]):
            dx = xp - xm
            dx -= Lbox * np.round(dx / Lbox)
            diff[2].append(dx / (2 * h))
        for up, um in zip(outs[0][3], outs[1][3]):
            diff[3].append((up - um) / (2 * h))
        fd = _dot(lam, diff, Lbox)
        an = _dot(vjp, dirn, Lbox)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (seed, trial, fd, an)
    sim.set_state(s0)


def _probe_loss(sim, lo, hi):
    m = np.zeros(sim.E.shape[1:], bool)
    m[lo:hi, lo:hi, lo:hi] = True
    return 0.5 * sim.dV * (np.sum(sim.E[:, m] ** 2) + np.sum(sim.B[:, m] ** 2)), m


def _cold_run(eps, n=8, steps=40):
    w = W.cold_langmuir_lattice(n=(n, n, n), per_axis=(2, 2, 2), eps=eps)
    sim = O.OracleSim(w.n, w.d, w.dt)
    s = w.species[0]
    sim.add_species(s.q, s.m, s.w, s.pos, s.u)
    return sim, w


def test_multistep_eps_gradient_matches_central_differences():
    """Cold Langmuir lattice (8^3, 8 per cell), 40 steps, probe energy in
    cells [2, 6)^3; dL/d eps from the chained step adjoints vs central FD."""
    eps, steps, lo, hi = 1e-2, 40, 2, 6
    sim, w = _cold_run(eps, steps=steps)
    states = []
    for _ in range(steps):
        states.append(sim.state())
        sim.step(1)
    Lval, m = _probe_loss(sim, lo, hi)
    lE = np.where(m[None], sim.dV * sim.E, 0.0)
    lB = np.where(m[None], sim.dV * sim.B, 0.0)
    lX = [np.zeros_like(sim.species[0].pos)]
    lU = [np.zeros_like(sim.species[0].u)]
    for st in reversed(states):
        sim.set_state(st)
        lE, lB, lX, lU = sim.step_vjp(lE, lB, lX, lU)
    x0 = w.species[0].pos[:, 0]
    grad = np.sum(lU[0][:, 0] * np.sin(2 * np.pi * x0 / (w.n[0] * w.d[0])))
    h = 1e-4
    vals = []
    for e in (eps + h, eps - h):
        s2, _ = _cold_run(e, steps=steps)
        s2.step(steps)
        vals.append(_probe_loss(s2, lo, hi)[0])
    fd = (vals[0] - vals[1]) / (2 * h)
    assert Lval > 0 and abs(grad) > 0
    assert abs(grad - fd) <= 1e-5 * abs(fd), (grad, fd)
