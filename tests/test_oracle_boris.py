"""Pins of the oracle's relativistic Boris push against closed forms and the
numbers printed in Sec. 3.1 of the paper (tests/golden/paper_values.json).

A dropped term, a wrong sign or a swapped cross product in the oracle's
push fails at least one of: exact |u| conservation, the polygon circumradius
and rotation angle of the discrete gyration, the exact half-step momenta and
midpoint-rule positions of the electric benchmark, the E x B drift.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _circle_radius(pts):
    """Algebraic least-squares circle through 2D points."""
    c = pts.mean(axis=0)
    p = pts - c
    A = np.column_stack([p[:, 0], p[:, 1], np.ones(len(p))])
    b = -(p[:, 0] ** 2 + p[:, 1] ** 2)
    (D, E, F), *_ = np.linalg.lstsq(A, b, rcond=None)
    return np.sqrt(D * D / 4 + E * E / 4 - F)


def _fit(x, y):
    X, Y = np.log(x), np.log(y)
    slope, icpt = np.polyfit(X, Y, 1)
    pred = slope * X + icpt
    r2 = 1 - np.sum((Y - pred) ** 2) / np.sum((Y - Y.mean()) ** 2)
    return slope, r2


def _magnetic_run(npt, periods, record_last=True):
    g = GOLD["boris_magnetic"]
    v = g["v_over_c"]
    gam = 1.0 / np.sqrt(1.0 - v * v)
    q, m, B = -1.0, 1.0, g["B"]
    dt = 2.0 * np.pi * gam / (npt - 1)
    r = q * dt / (2.0 * m)
    u0 = np.array([0.0, gam * v, 0.0])
    x, u, _ = O.particle_uniform(r, [0, 0, 0], [0, 0, B], dt, (periods - 1) * (npt - 1),
                                 [0, 0, 0], u0)
    x, u, traj = O.particle_uniform(r, [0, 0, 0], [0, 0, B], dt, npt - 1, x, u, record=True)
    return gam, v, dt, u0, u, traj


def test_gamma_printed():
    g = GOLD["boris_magnetic"]
    gam = 1.0 / np.sqrt(1.0 - g["v_over_c"] ** 2)
    assert abs(gam - g["gamma_printed"]) < 0.005


def test_magnetic_speed_conserved_to_roundoff():
    """Sec. 3.1: speed, energy and gamma stay constant at double round-off."""
    gam, v, dt, u0, u, _ = _magnetic_run(1281, 1000)
    rel = abs(np.linalg.norm(u) - np.linalg.norm(u0)) / np.linalg.norm(u0)
    assert rel < 1e-13, rel


@pytest.mark.parametrize("npt", [11, 41, 321])
def test_magnetic_rotation_angle_closed_form(npt):
    """The Boris rotation turns u by 2 atan(Omega dt / 2) each step."""
    g = GOLD["boris_magnetic"]
    v = g["v_over_c"]
    gam = 1.0 / np.sqrt(1.0 - v * v)
    dt = 2.0 * np.pi * gam / (npt - 1)
    u0 = np.array([0.0, gam * v, 0.0])
    u1 = O.boris(u0, [0, 0, 0], [0, 0, 1.0], -dt / 2.0)
    ang = np.arctan2(np.cross(u0, u1)[2], np.dot(u0, u1))
    omega = 1.0 / gam  # |q| B / (gamma m)
    expect = 2.0 * np.arctan(omega * dt / 2.0)
    assert abs(abs(ang) - expect) < 1e-14
    # an electron (q < 0) in +z B gyrates counter-clockwise in the x-y plane
    assert ang > 0


def test_magnetic_larmor_radius_convergence():
    """Sec. 3.1, Fig. 'Boris convergence': relative Larmor-radius error vs dt.

    The discrete orbit is a regular polygon whose circumradius is
    R sqrt(1 + (Omega dt / 2)^2) (chord dt v, turning angle 2 atan(Omega dt/2)),
    so the relative error is sqrt(1 + (pi/(N_pt-1))^2) - 1 for the paper's
    dt = 2 pi gamma/(N_pt - 1).  The least-squares slope over the paper's
    resolutions is compared with the printed 1.998 (R^2 = 0.999995).
    """
    g = GOLD["boris_magnetic"]
    errs, dts = [], []
    for npt in g["points_per_period"]:
        gam, v, dt, u0, u, traj = _magnetic_run(npt, g["periods"])
        R = gam * v  # u_perp / (|q| B / m)
        Rnum = _circle_radius(traj[:, :2])
        closed = np.sqrt(1.0 + (np.pi / (npt - 1)) ** 2) - 1.0
        err = (Rnum - R) / R
        assert abs(err - closed) <= 1e-9 * max(1.0, closed) + 1e-12, (npt, err, closed)
        errs.append(err)
        dts.append(dt)
    slope, r2 = _fit(np.array(dts), np.array(errs))
    assert abs(slope - g["larmor_error_slope"]) < 0.01, slope
    assert r2 > 0.9999, r2


def _electric_run(N):
    g = GOLD["boris_electric"]
    q, m, E = -1.0, 1.0, g["E"]
    dt = g["t_end"] / (N - 1)
    r = q * dt / (2.0 * m)
    # centred start: u^{-1/2} = u(0) - (q/m) E dt/2
    u0 = [-(q / m) * E * dt / 2.0, 0.0, 0.0]
    x, u, _ = O.particle_uniform(r, [E, 0, 0], [0, 0, 0], dt, N - 1, [0, 0, 0], u0)
    return dt, x, u


def test_electric_position_convergence_and_exact_momenta():
    """Sec. 3.1, Fig. 'Boris electric': electron from rest in E = x.

    Analytic: u(t) = (q/m) E t, x(t) = (m/(qE)) (sqrt(1 + (qEt/m)^2) - 1).
    With the centred start the half-step momenta are exact, so the momentum
    error stays at round-off (paper: 1e-16 .. 1e-13), and the position is the
    midpoint rule of the exact velocity, error O(dt^2) (paper slope 2.002).
    """
    g = GOLD["boris_electric"]
    errs, dts = [], []
    for N in g["samples"]:
        dt, x, u = _electric_run(N)
        t_last_half = (N - 1 - 0.5) * dt
        u_exact = -t_last_half
        assert abs(u[0] - u_exact) / abs(u_exact) < 5e-13
        assert u[1] == 0.0 and u[2] == 0.0
        x_exact = -(np.sqrt(1.0 + g["t_end"] ** 2) - 1.0)
        # midpoint rule of v(t) = u/sqrt(1+u^2) with the exact half-step u
        th = (np.arange(N - 1) + 0.5) * dt
        mid = np.sum(dt * (-th) / np.sqrt(1.0 + th * th))
        assert abs(x[0] - mid) / abs(mid) < 1e-12
        errs.append(abs(x[0] - x_exact) / abs(x_exact))
        dts.append(dt)
    slope, r2 = _fit(np.array(dts), np.array(errs))
    assert abs(slope - g["position_error_slope"]) < 0.01, slope
    assert r2 > 0.99999, r2


def test_exb_drift():
    """E perpendicular to B with |E| = 0.1 |B|: the mean velocity is E x B / B^2."""
    E = np.array([0.0, 0.1, 0.0])
    B = np.array([0.0, 0.0, 1.0])
    dt = 0.05
    nsteps = 20000
    for q in (-1.0, 1.0):
        r = q * dt / 2.0
        x, u, traj = O.particle_uniform(r, E, B, dt, nsteps, [0, 0, 0], [0, 0, 0], record=True)
        t = (np.arange(nsteps) + 1) * dt
        vx = np.polyfit(t, traj[:, 0], 1)[0]
        vy = np.polyfit(t, traj[:, 1], 1)[0]
        vd = np.cross(E, B) / np.dot(B, B)
        assert abs(vx - vd[0]) < 2e-3 * abs(vd[0]), (q, vx)
        assert abs(vy) < 2e-4, (q, vy)
        assert np.all(traj[:, 2] == 0.0)
