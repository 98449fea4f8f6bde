"""Pins of the oracle's moving window (a module of Sec. 2.2, used by the
wakefield run of Sec. 4; its algorithm is a reading).

Nothing behind a window that moves at c can reach its interior, so a run in
the moving window must reproduce, to round-off, the same region of a run in
a static box long enough to hold everything, except a thin layer at the
window's back edge.  The static box's extra plasma is laid out in the order
the window injects it, so particle ids correspond.
"""
import numpy as np

from oracle import oracle as O

N_WIN, NY, NZ = 64, 2, 16
D = (0.5, 1.0, 0.5)
PER = (2, 1, 2)
X_PLASMA = 16          # plasma fills x >= 16 cells
CELLS = 8              # window shift
N0 = 0.05              # density
W = N0 * D[0] * D[1] * D[2] / (PER[0] * PER[1] * PER[2])


def _lattice(x0, x1, n):
    axes = []
    lo, hi = [x0, 0, 0], [x1, n[1], n[2]]
    for b in range(3):
        cells = np.arange(lo[b], hi[b])
        offs = (np.arange(PER[b]) + 0.5) / PER[b]
        axes.append((cells[:, None] + offs[None, :]).reshape(-1) * D[b])
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], axis=1)


def _sim(nx, extra_shifts=0):
    n = (nx, NY, NZ)
    dt = O.courant_dt(D)
    sim = O.OracleSim(n, D, dt, bc=(O.ABSORBING, O.PERIODIC, O.ABSORBING))
    pos = [_lattice(X_PLASMA, N_WIN, n)]
    for s in range(extra_shifts):  # what the window will inject, in its order
        pos.append(_lattice(N_WIN + s * CELLS, N_WIN + (s + 1) * CELLS, n))
    pos = np.concatenate(pos)
    sim.add_species(-1.0, 1.0, W, pos, np.zeros_like(pos))
    sim.set_laser(a0=0.3, w0=3.0, tau=4.0, t0=10.0, omega0=2.0, yc=0.5 * NY * D[1],
                  zc=0.5 * NZ * D[2], i_s=1)
    return sim


def test_window_run_equals_the_static_run_inside_the_window():
    steps, t_start = 240, 22.0
    win = _sim(N_WIN)
    win.set_window(axis=0, cells=CELLS, velocity=1.0, t_start=t_start,
                   inject=[(0, PER, W)])
    n_shift = int(np.floor((steps - 1) * win.dt - t_start) / (CELLS * D[0]))  # shifts made
    big = _sim(N_WIN + (n_shift + 1) * CELLS, extra_shifts=n_shift + 1)
    win.step(steps)
    big.step(steps)
    shifts = win.window["shifts"]
    assert shifts >= 3
    off = shifts * CELLS
    # cells next to the back edge that feel the Mur face: the Yee stencil reaches
    # one cell per step, so its influence decays through a layer there
    back = 16
    # fields on the common planes (x nodes back .. N_WIN - 1)
    for name in ("E", "B", "J"):
        a = getattr(win, name)[..., back:N_WIN]
        b = getattr(big, name)[..., off + back:off + N_WIN]
        scale = max(np.abs(b).max(), 1e-30)
        assert np.abs(a - b).max() <= 1e-10 * scale, (name, np.abs(a - b).max() / scale)
    assert np.abs(win.E[1]).max() > 0.05  # the pulse is in the window
    # particles by id: those inside the compared region
    sw, sb = win.species[0], big.species[0]
    alive = sw.alive.astype(bool)
    x = sw.pos[:, 0]
    sel = alive & (x >= (back + 1) * D[0])
    ids = sw.ids[sel]
    assert len(ids) > 1000
    pw = sw.pos[sel]
    pb = sb.pos[ids]
    pb = pb - np.array([off * D[0], 0.0, 0.0])
    assert np.abs(pw - pb).max() <= 1e-10, np.abs(pw - pb).max()
    assert np.abs(sw.u[sel] - sb.u[ids]).max() <= 1e-11
    # particles that left through the back are removed; none appear ahead
    assert (~alive).sum() > 0 and np.all(sw.pos[alive, 0] < N_WIN * D[0])
    # particle count: initial + injected - removed
    inj = shifts * CELLS * NY * NZ * PER[0] * PER[1] * PER[2]
    n_init = (N_WIN - X_PLASMA) * NY * NZ * PER[0] * PER[1] * PER[2]
    assert sw.np == n_init + inj
