"""Pins of the Esirkepov and EZ currents of the oracle (the charge-conserving
alternatives the paper names beside ZigZag, Sec. 2.5).

* Esirkepov's current conserves charge to round-off for general 3D moves.
* In one dimension (moves along x only) it is the exact CIC flux, so it
  equals the ZigZag current, crossings included.
* For a move inside one cell it equals the ZigZag current.
* For a move that crosses a face in 3D it differs from ZigZag by a loop
  current (divergence-free), since the two take different paths.
* EZ (Esirkepov on each ZigZag segment) equals the ZigZag current of the
  step's deposit to round-off: at first order the step's segment weights
  are Esirkepov's decomposition.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import esirkepov as EZ
from oracle import oracle as O

N, D = (5, 4, 6), (1.0, 0.8, 1.2)


def _setup():
    dt = O.courant_dt(D)
    sim = O.OracleSim(N, D, dt)
    return sim, dt


def _rho(sim, xi, q):
    out = np.zeros(sim.E.shape[1:])
    pos = np.ascontiguousarray(np.mod(np.asarray(xi), np.asarray(N, float)).reshape(-1, 3) * np.asarray(D))
    O.lib().orc_rho(C.byref(sim.g), pos.shape[0], O._p(pos), None, None, float(q), 1.0, O._p(out))
    return out


def _moves(seed, P=150, span=0.9):
    rng = np.random.default_rng(seed)
    xi0 = rng.random((P, 3)) * np.asarray(N)
    return xi0, xi0 + rng.uniform(-span, span, size=(P, 3))


@pytest.mark.parametrize("seed", [0, 1])
def test_esirkepov_conserves_charge(seed):
    sim, dt = _setup()
    xi0, xi1 = _moves(seed)
    q = 0.61
    J = np.zeros(sim.E.shape)
    for p in range(len(xi0)):
        EZ.esirkepov(N, D, dt, xi0[p], xi1[p], q, J)
    r0, r1 = _rho(sim, xi0, q), _rho(sim, xi1, q)
    res = (r1 - r0) / dt + sim.div(J)
    assert np.max(np.abs(res)) * dt < 1e-13 * np.max(np.abs(r0))
    assert np.sum(np.floor(xi0) != np.floor(xi1)) > 50


def test_one_dimensional_moves_equal_zigzag():
    sim, dt = _setup()
    rng = np.random.default_rng(5)
    q = -0.4
    for _ in range(40):
        xi0 = rng.random(3) * np.asarray(N)
        xi1 = xi0.copy()
        xi1[0] += rng.uniform(-0.95, 0.95)
        Je = EZ.esirkepov(N, D, dt, xi0, xi1, q, np.zeros(sim.E.shape))
        Jz = O.zigzag(sim.g, sim.E.shape, xi0, xi1, q)
        assert np.max(np.abs(Je - Jz)) <= 1e-14 * np.max(np.abs(Jz))


def test_moves_inside_one_cell_equal_zigzag():
    sim, dt = _setup()
    rng = np.random.default_rng(6)
    q = 1.3
    for _ in range(40):
        c = np.floor(rng.random(3) * np.asarray(N))
        a, b = c + rng.random(3), c + rng.random(3)
        Je = EZ.esirkepov(N, D, dt, a, b, q, np.zeros(sim.E.shape))
        Jz = O.zigzag(sim.g, sim.E.shape, a, b, q)
        assert np.max(np.abs(Je - Jz)) <= 1e-13 * np.max(np.abs(Jz))


def test_crossing_moves_differ_from_zigzag_by_a_loop_current():
    sim, dt = _setup()
    xi0 = np.array([1.7, 2.2, 3.9])
    xi1 = np.array([2.3, 1.8, 4.4])  # crosses a face on every axis
    q = 1.0
    Je = EZ.esirkepov(N, D, dt, xi0, xi1, q, np.zeros(sim.E.shape))
    Jz = O.zigzag(sim.g, sim.E.shape, xi0, xi1, q)
    dJ = Je - Jz
    assert np.max(np.abs(dJ)) > 1e-3 * np.max(np.abs(Jz))
    assert np.max(np.abs(sim.div(dJ))) < 1e-13 * np.max(np.abs(Jz)) / min(D)


@pytest.mark.parametrize("seed", [2, 3])
def test_ez_equals_zigzag_segment_weights(seed):
    sim, dt = _setup()
    xi0, xi1 = _moves(seed)
    q = -0.83
    Jez = np.zeros(sim.E.shape)
    Jz = np.zeros(sim.E.shape)
    for p in range(len(xi0)):
        EZ.ez(N, D, dt, xi0[p], xi1[p], q, Jez)
        O.zigzag(sim.g, sim.E.shape, xi0[p], xi1[p], q, J=Jz)
    assert np.max(np.abs(Jez - Jz)) <= 1e-13 * np.max(np.abs(Jz))
    assert np.sum(np.floor(xi0) != np.floor(xi1)) > 50
