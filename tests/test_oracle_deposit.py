"""Pins of the oracle's particle-mesh operators (Sec. 2.5 of the paper).

ZigZag deposit: discrete continuity at every node to round-off for general
3D moves with and without cell crossings (the property the paper relies on,
~1e-13 in its test); the literal midpoint-product weights fail it in 3D but
pass when one displacement component is zero (why the exact line-integral
weights are the reading taken); brute-force quadrature of the CIC weights
along the straight path; total current = q * displacement / dt; a crossing
move deposits only on edges of its two cells.

Gather: uniform and linear fields are reproduced exactly on every staggered
sub-grid (a wrong stagger shifts the linear field and fails).

CIC rho: the total charge is exact.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O


def _rho(g, shape, xi, d, qsp):
    out = np.zeros(shape)
    pos = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(-1, 3) * np.asarray(d))
    O.lib().orc_rho(C.byref(g), pos.shape[0], O._p(pos), None, None, float(qsp), 1.0, O._p(out))
    return out


def _wrap(xi, n):
    return np.mod(xi, np.asarray(n, dtype=np.float64))


def _div(sim, J):
    return sim.div(J)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zigzag_continuity_roundoff(seed):
    n, d = (4, 5, 3), (1.0, 0.7, 1.3)
    dt = O.courant_dt(d)
    sim = O.OracleSim(n, d, dt)
    rng = np.random.default_rng(seed)
    P = 200
    xi1 = rng.random((P, 3)) * np.asarray(n)
    dxi = rng.uniform(-0.9, 0.9, size=(P, 3))
    xi2 = xi1 + dxi
    q = -0.37
    J = np.zeros(sim.E.shape)
    for p in range(P):
        O.zigzag(sim.g, sim.E.shape, xi1[p], xi2[p], q, J=J)
    shape = sim.E.shape[1:]
    r1 = _rho(sim.g, shape, xi1, d, q)
    r2 = _rho(sim.g, shape, _wrap(xi2, n), d, q)
    res = (r2 - r1) / dt + _div(sim, J)
    assert np.max(np.abs(res)) * dt < 1e-13 * np.max(np.abs(r1))
    # crossings were exercised
    assert np.sum(np.floor(xi1) != np.floor(xi2)) > 50


def test_midpoint_only_weights_fail_3d_but_pass_2d():
    n, d = (4, 4, 4), (1.0, 1.0, 1.0)
    dt = O.courant_dt(d)
    sim = O.OracleSim(n, d, dt)
    rng = np.random.default_rng(11)
    P = 100
    xi1 = rng.random((P, 3)) * 4
    dxi = rng.uniform(-0.6, 0.6, size=(P, 3))
    q = 1.0
    shape = sim.E.shape[1:]
    for zero_z, should_pass in ((False, False), (True, True)):
        dx = dxi.copy()
        if zero_z:
            dx[:, 2] = 0.0
        xi2 = xi1 + dx
        J = np.zeros(sim.E.shape)
        for p in range(P):
            O.zigzag(sim.g, sim.E.shape, xi1[p], xi2[p], q, midpoint_only=True, J=J)
        r1 = _rho(sim.g, shape, xi1, d, q)
        r2 = _rho(sim.g, shape, _wrap(xi2, n), d, q)
        err = np.max(np.abs((r2 - r1) / dt + _div(sim, J))) * dt / np.max(np.abs(r1))
        if should_pass:
            assert err < 1e-13
        else:
            assert err > 1e-4


def test_weights_match_bruteforce_line_integral():
    """Non-crossing moves: integrate the CIC edge weights along the straight
    path with M midpoint sub-steps; converges to the exact weights at O(1/M^2)."""
    n, d = (3, 3, 3), (1.0, 1.0, 1.0)
    dt = 0.3
    g = O.make_grid(n, d, dt)
    rng = np.random.default_rng(4)
    shape = (3, 3, 3, 3)
    for _ in range(5):
        cell = rng.integers(0, 3, size=3).astype(float)
        s = cell + rng.uniform(0.05, 0.95, size=3)
        e = np.clip(s + rng.uniform(-0.5, 0.5, size=3), cell + 0.01, cell + 0.99)
        J = O.zigzag(g, shape, s, e, 1.0)
        M = 4000
        Jb = np.zeros(shape)
        ts = (np.arange(M) + 0.5) / M
        pts = s[None, :] + ts[:, None] * (e - s)[None, :]
        dseg = (e - s) / M
        ci = cell.astype(int)
        W = pts - cell[None, :]
        for c in range(3):
            b1, b2 = (c + 1) % 3, (c + 2) % 3
            for o1 in (0, 1):
                for o2 in (0, 1):
                    w = (W[:, b1] if o1 else 1 - W[:, b1]) * (W[:, b2] if o2 else 1 - W[:, b2])
                    idx = ci.copy()
                    idx[b1] += o1
                    idx[b2] += o2
                    idx %= 3
                    Jb[c, idx[2], idx[1], idx[0]] += np.sum(w) * dseg[c] * d[c] / dt
        assert np.max(np.abs(J - Jb)) < 1e-6 * np.max(np.abs(J))


def test_total_current_and_footprint():
    n, d = (5, 5, 5), (1.0, 0.5, 2.0)
    dt = 0.2
    g = O.make_grid(n, d, dt)
    shape = (3, 5, 5, 5)
    dV = d[0] * d[1] * d[2]
    xi1 = np.array([2.3, 1.95, 3.05])
    xi2 = np.array([2.6, 2.1, 2.97])   # crosses in y (up) and z (down)
    q = -2.0
    J = O.zigzag(g, shape, xi1, xi2, q)
    for c in range(3):
        assert abs(J[c].sum() * dV - q * (xi2[c] - xi1[c]) * d[c] / dt) < 1e-12
    # nonzero only on edges of cells (2,1,3) and (2,2,2)
    allowed = np.zeros(shape, dtype=bool)
    for cell in ((2, 1, 3), (2, 2, 2)):
        for c in range(3):
            b1, b2 = (c + 1) % 3, (c + 2) % 3
            for o1 in (0, 1):
                for o2 in (0, 1):
                    idx = list(cell)
                    idx[b1] += o1
                    idx[b2] += o2
                    allowed[c, idx[2] % 5, idx[1] % 5, idx[0] % 5] = True
    assert np.all(J[~allowed] == 0.0)
    assert np.count_nonzero(J) > 12


def test_one_dimensional_limit_is_cic_flux():
    """A move along x only gives J_x = q v_x times the fixed y, z CIC weights."""
    n, d = (4, 4, 4), (1.0, 1.0, 1.0)
    dt = 0.25
    g = O.make_grid(n, d, dt)
    xi1 = np.array([1.2, 2.3, 0.6])
    xi2 = np.array([1.45, 2.3, 0.6])
    J = O.zigzag(g, (3, 4, 4, 4), xi1, xi2, 1.0)
    vx = (xi2[0] - xi1[0]) / dt
    wy, wz = 0.3, 0.6
    expect = {(2, 0): (1 - wy) * (1 - wz), (3, 0): wy * (1 - wz), (2, 1): (1 - wy) * wz,
              (3, 1): wy * wz}
    for (j, k), w in expect.items():
        assert abs(J[0, k, j, 1] - vx * w) < 1e-14
    assert np.all(J[1:] == 0.0)


def test_gather_uniform_and_linear_exact():
    n, d = (6, 5, 4), (1.0, 0.8, 1.25)
    g = O.make_grid(n, d, 0.1)
    shape = (3, 4, 5, 6)
    rng = np.random.default_rng(9)
    a = rng.standard_normal(6)
    b = rng.standard_normal((6, 3))
    E = np.zeros(shape)
    B = np.zeros(shape)
    z, y, x = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    for c in range(3):
        se = [0.5 if q == c else 0.0 for q in range(3)]
        sb = [0.0 if q == c else 0.5 for q in range(3)]
        XE = [(x + se[0]) * d[0], (y + se[1]) * d[1], (z + se[2]) * d[2]]
        XB = [(x + sb[0]) * d[0], (y + sb[1]) * d[1], (z + sb[2]) * d[2]]
        E[c] = a[c] + b[c, 0] * XE[0] + b[c, 1] * XE[1] + b[c, 2] * XE[2]
        B[c] = a[3 + c] + b[3 + c, 0] * XB[0] + b[3 + c, 1] * XB[1] + b[3 + c, 2] * XB[2]
    for _ in range(50):
        # keep away from the periodic seam, where a linear field is not periodic
        pos = (1.0 + rng.random(3) * (np.array([6, 5, 4]) - 2.5)) * np.asarray(d)
        Ep, Bp = O.gather(g, E, B, pos)
        for c in range(3):
            assert abs(Ep[c] - (a[c] + b[c] @ pos)) < 1e-12
            assert abs(Bp[c] - (a[3 + c] + b[3 + c] @ pos)) < 1e-12
    Eu = np.ones(shape) * np.array([1.5, -2.0, 0.25])[:, None, None, None]
    for _ in range(20):
        pos = rng.random(3) * np.array([6, 5, 4]) * np.asarray(d)
        Ep, Bp = O.gather(g, Eu, Eu, pos)
        assert np.allclose(Ep, [1.5, -2.0, 0.25], atol=1e-14, rtol=0)


def test_rho_total_charge():
    n, d = (5, 4, 3), (1.0, 0.5, 2.0)
    g = O.make_grid(n, d, 0.1)
    rng = np.random.default_rng(2)
    xi = rng.random((300, 3)) * np.asarray(n)
    q = -0.125
    r = _rho(g, (3, 4, 5), xi, d, q)
    assert abs(r.sum() * d[0] * d[1] * d[2] - q * 300) < 1e-12
