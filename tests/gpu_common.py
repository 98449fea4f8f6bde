"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np

from oracle import oracle as O


def oracle_from(w, E0=None, B0=None, order=1):
    sim = O.OracleSim(w.n, w.d, w.dt, w.bc)
    sim.shape_order = order
    if E0 is not None:
        sim.E[...] = E0
    if B0 is not None:
        sim.B[...] = B0
    for s in w.species:
        sim.add_species(s.q, s.m, s.w, s.pos, s.u, s.wpp)
    sim.rho_bg = w.rho_bg
    if w.laser is not None:
        L = w.laser
        sim.set_laser(L.a0, L.w0, L.tau, L.t0, L.omega0, L.yc, L.zc, L.i_s, L.slab)
    if getattr(w, "filter", None):
        sim.filter = tuple(w.filter)
    if getattr(w, "port", None) is not None:
        P = w.port
        sim.set_port(P.axis, P.plane, P.comp, P.prof_axis, P.e0, P.omega, P.tau)
    if getattr(w, "window", None) is not None:
        Wn = w.window
        sim.set_window(Wn.axis, Wn.cells, Wn.velocity, Wn.t_start, Wn.inject)
    return sim


def rel(a, b):
    """||a - b||_inf / ||b||_inf."""
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (den if den > 0 else 1.0)


def pos_err_cells(P, Pref, w):
    """Largest position difference in cells, minimal image on periodic axes."""
    d = np.asarray(w.d)
    L = np.asarray(w.n, dtype=float) * d
    dx = P - Pref
    for a in range(3):
        if w.bc[a] == 0:
            dx[:, a] -= L[a] * np.round(dx[:, a] / L[a])
    return float(np.max(np.abs(dx) / d)) if len(dx) else 0.0


def compare_state(gpu, orc, w, sp_tol, f_tol, label=""):
    """Compare fields and every species by id; returns the error dict."""
    E, B, J = gpu.fields()
    errs = {"E": rel(E, orc.E), "B": rel(B, orc.B), "J": rel(J, orc.J)}
    for i, s in enumerate(orc.species):
        P, U, I = gpu.particles_by_id(i)
        alive = np.ones(s.np, bool) if s.alive is None else s.alive.astype(bool)
        ref_ids = np.nonzero(alive)[0]
        assert np.array_equal(I, ref_ids), (label, i, len(I), len(ref_ids))
        errs["x%d" % i] = pos_err_cells(P, s.pos[ref_ids], w)
        errs["u%d" % i] = rel(U, s.u[ref_ids])
    for k, v in errs.items():
        tol = f_tol if k in ("E", "B", "J") else sp_tol
        assert v <= tol, (label, k, v, tol, errs)
    return errs


def check_box_currents(g, w, boxes, tol, margin=2, order=1):
    """One step of the GPU run `g`, with J compared element-wise with the
    oracle's inside each box (lo, hi) of cells: the oracle takes the GPU's
    fields and every particle within `margin` cells of the box (a particle
    moves at most one cell, so these are all that deposit inside it; a
    second-order stencil reaches one cell further: margin 3) and steps once
    with the given shape order.  Returns the largest relative difference (to
    max |J| over the box)."""
    E, B, _ = g.fields()
    parts = []
    for i in range(len(w.species)):
        got = {}
        for lo, hi in boxes:
            lo_m = [lo[a] - margin for a in range(3)]
            hi_m = [hi[a] + margin for a in range(3)]
            P, U, I = g.particles_in_box(i, lo_m, hi_m)
            for k in range(len(I)):
                got[int(I[k])] = (P[k], U[k])
        ids = np.array(sorted(got), dtype=np.int64)
        P = np.array([got[k][0] for k in ids]).reshape(-1, 3)
        U = np.array([got[k][1] for k in ids]).reshape(-1, 3)
        parts.append((P, U, ids))
    g.step(1)
    _, _, Jg = g.fields()
    o = O.OracleSim(w.n, w.d, w.dt, w.bc)
    o.shape_order = order
    o.E[...] = E
    o.B[...] = B
    for i, (P, U, I) in enumerate(parts):
        s = w.species[i]
        wpp = None if s.wpp is None else s.wpp[I]
        o.add_species(s.q, s.m, s.w, P, U, wpp=wpp, ids=I)
    o.step(1)
    worst = 0.0
    for lo, hi in boxes:
        sl = (slice(None), slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        a, b = Jg[sl], o.J[sl]
        den = float(np.max(np.abs(a)))
        assert den > 0, (lo, hi)
        err = float(np.max(np.abs(a - b))) / den
        assert err <= tol, (lo, hi, err)
        worst = max(worst, err)
    return worst
