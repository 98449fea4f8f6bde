"""Pins of the oracle's perfectly conducting walls and waveguide port (the
field-solver benchmark of Sec. 3.2), against what the mathematics fixes:

* the vacuum Yee energy 1/2 sum |E|^2 + 1/2 sum B^{n-1/2}.B^{n+1/2} is
  conserved exactly in a closed PEC cavity (the discrete curls stay adjoint
  when tangential E vanishes on the walls), tangential E stays zero and
  div B keeps its initial value;
* a TE101 cavity mode obeys the leapfrog recurrence
  E^{n+1} + E^{n-1} = 2 cos(w dt) E^n with w from the closed-form discrete
  Yee dispersion relation;
* the driven TE10 waveguide carries e0 sin(pi x/a) sin(w t - beta z) with
  beta from the same dispersion relation (k_x = pi/a exact on nodes).
"""
import ctypes as C

import numpy as np

from oracle import oracle as O


def _pec_state(n, d, rng):
    sim = O.OracleSim(n, d, O.courant_dt(d), bc=(O.PEC,) * 3)
    E = rng.standard_normal(sim.E.shape)
    B = rng.standard_normal(sim.B.shape)
    # padding: a half-staggered component stops at index n-1 along a walled axis
    for c in range(3):
        for a in range(3):
            sl = [slice(None)] * 3
            sl[2 - a] = n[a]
            if a == c:
                E[c][tuple(sl)] = 0.0
            else:
                B[c][tuple(sl)] = 0.0
    sim.E[...] = E
    sim.B[...] = B
    O.lib().orc_pec(C.byref(sim.g), O._p(sim.E))
    return sim


def _energy(sim):
    Bh = sim.B.copy()
    O.lib().orc_faraday(C.byref(sim.g), O._p(sim.E.copy()), O._p(Bh), None)
    return 0.5 * np.sum(sim.E ** 2) + 0.5 * np.sum(sim.B * Bh)


def _tangential_face_values(sim):
    """Largest |tangential E| on the faces of the walled axes (padding is zero)."""
    vals = []
    for a in range(3):
        for c in range(3):
            if c == a:
                continue
            for side in (0, sim.n[a]):
                sl = [slice(None)] * 3
                sl[2 - a] = side
                vals.append(np.abs(sim.E[c][tuple(sl)]).max())
    return max(vals)


def test_pec_cavity_conserves_vacuum_energy():
    rng = np.random.default_rng(1)
    n, d = (6, 5, 7), (1.0, 0.8, 1.2)
    sim = _pec_state(n, d, rng)
    u0 = _energy(sim)
    divb0 = _div_nodes_B(sim)
    for _ in range(100):
        sim.step(1)
    u1 = _energy(sim)
    assert abs(u1 - u0) <= 1e-12 * u0, (u0, u1)
    assert _tangential_face_values(sim) == 0.0
    assert np.abs(_div_nodes_B(sim) - divb0).max() <= 1e-11


def _div_nodes_B(sim):
    """div B at cell centres (forward differences of the face-normal components)."""
    n = sim.n
    B = sim.B
    d = sim.d
    bx = (B[0][:n[2], :n[1], 1:n[0] + 1] - B[0][:n[2], :n[1], :n[0]]) / d[0]
    by = (B[1][:n[2], 1:n[1] + 1, :n[0]] - B[1][:n[2], :n[1], :n[0]]) / d[1]
    bz = (B[2][1:n[2] + 1, :n[1], :n[0]] - B[2][:n[2], :n[1], :n[0]]) / d[2]
    return bx + by + bz


def test_te101_cavity_mode_follows_discrete_dispersion():
    n, d = (8, 3, 6), (1.0, 1.1, 0.9)
    dt = O.courant_dt(d)
    sim = O.OracleSim(n, d, dt, bc=(O.PEC,) * 3)
    i = np.arange(n[0] + 1)
    k = np.arange(n[2] + 1)
    prof = np.sin(np.pi * k / n[2])[:, None, None] * np.sin(np.pi * i / n[0])[None, None, :]
    sim.E[1][:, :n[1], :] = prof  # E_y nodal in x and z, half in y
    kx, kz = np.pi / (n[0] * d[0]), np.pi / (n[2] * d[2])
    s2 = (dt / d[0] * np.sin(kx * d[0] / 2)) ** 2 + (dt / d[2] * np.sin(kz * d[2] / 2)) ** 2
    cos_wdt = 1.0 - 2.0 * s2
    probe = (n[2] // 2, 1, n[0] // 2)
    series = []
    for _ in range(300):
        series.append(sim.E[1][probe])
        sim.step(1)
    e = np.asarray(series)
    ok = np.abs(e[1:-1]) > 0.2 * np.abs(e).max()
    ratio = (e[2:] + e[:-2])[ok] / (2.0 * e[1:-1][ok])
    assert np.abs(ratio - cos_wdt).max() <= 1e-11, np.abs(ratio - cos_wdt).max()
    # the mode keeps its shape: E_x, E_z stay zero, E_y stays proportional to the profile
    assert np.abs(sim.E[0]).max() <= 1e-12 and np.abs(sim.E[2]).max() <= 1e-12
    ey = sim.E[1][:, :n[1], :]
    c = np.sum(ey * prof[:, :1, :]) / np.sum(prof[:, :1, :] ** 2 * n[1])
    assert np.abs(ey - c * prof).max() <= 1e-11


def _fit_sine(t, y, w):
    A = np.stack([np.sin(w * t), np.cos(w * t)], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    return np.hypot(a, b), np.arctan2(b, a)


def test_te10_port_drives_the_discrete_guided_mode():
    a_cells, b_cells, nz = 6, 3, 240
    d = (1.0, 1.0, 1.0)
    dt = O.courant_dt(d)
    sim = O.OracleSim((a_cells, b_cells, nz), d, dt, bc=(O.PEC, O.PEC, O.ABSORBING))
    w, e0 = 0.9, 1.0
    sim.set_port(axis=2, plane=0, comp=1, prof_axis=0, e0=e0, omega=w, tau=2 * 2 * np.pi / w)
    z1, z2 = 40, 60
    ts, s1, s2 = [], [], []
    for _ in range(800):
        sim.step(1)
        ts.append(sim.nstep * dt)
        s1.append(sim.E[1][z1, 1, a_cells // 2])
        s2.append(sim.E[1][z2, 1, a_cells // 2])
    ts, s1, s2 = map(np.asarray, (ts, s1, s2))
    win = ts >= 160.0  # envelope settled (e^-11), far-end reflection not yet back
    A1, p1 = _fit_sine(ts[win], s1[win], w)
    A2, p2 = _fit_sine(ts[win], s2[win], w)
    s2w = (np.sin(w * dt / 2) / dt) ** 2 - (np.sin(np.pi * d[0] / (2 * a_cells * d[0])) / d[0]) ** 2
    beta = 2.0 / d[2] * np.arcsin(d[2] * np.sqrt(s2w))
    dphase = np.mod(p1 - p2, 2 * np.pi)
    assert abs(dphase - np.mod(beta * (z2 - z1) * d[2], 2 * np.pi)) <= 2e-3 * beta * (z2 - z1), (dphase, beta)
    assert abs(A1 - e0) <= 1e-3 and abs(A2 - e0) <= 1e-3, (A1, A2)
    # the continuous guide's beta differs at second order in the cell size
    beta_c = np.sqrt(w ** 2 - (np.pi / a_cells) ** 2)
    assert abs(beta - beta_c) > 1e-3 * beta_c


def test_convergence_table_fixture_matches_the_papers_fit():
    """The transcribed table reproduces the paper's own fit: slope 2.136 and
    R^2 0.972 of log eps against log dh (Sec. 3.2), and its dh column follows
    from the node counts (a = 3 cm, b = 1.5 cm, L_z = 100 cm, n nodes)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "te10_convergence.json")))
    rows = gold["rows"]
    dh = np.array([r["dh"] for r in rows])
    eps = np.array([r["eps_E0"] for r in rows])
    x, y = np.log(dh), np.log(eps)
    slope, icpt = np.polyfit(x, y, 1)
    r2 = 1.0 - np.sum((y - (slope * x + icpt)) ** 2) / np.sum((y - y.mean()) ** 2)
    assert abs(slope - gold["fit"]["rate"]) < 5e-3 and abs(r2 - gold["fit"]["r2"]) < 5e-3, (slope, r2)
    for k, r in enumerate(rows):
        nx, ny, nz = r["nodes"]
        h = np.sqrt((3.0 / (nx - 1)) ** 2 + (1.5 / (ny - 1)) ** 2 + (100.0 / (nz - 1)) ** 2) / 100.0
        assert abs(h - r["dh"]) <= 2e-3 * r["dh"], (r, h)
        # the time step halves with every refinement: n_t - 1 = 1250 * 2^k
        assert r["nt"] - 1 == 1250 * 2 ** k
    # the coarsest run covers 30 periods of 9 GHz at Courant 0.5
    nx, ny, nz = rows[0]["nodes"]
    dt = 0.5 / np.sqrt((((nx - 1) / 3.0) ** 2 + ((ny - 1) / 1.5) ** 2 + ((nz - 1) / 100.0) ** 2))
    periods = (rows[0]["nt"] - 1) * dt / (29.9792458 / 9.0)
    assert abs(periods - 30.0) < 0.3, periods
