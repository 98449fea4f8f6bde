"""Python face of the FP64 CPU oracle of the EM-PIC step (KEMPIC-3D).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; the product path never imports
it.  It shares no code with the HIP library: the arithmetic is in
``oracle.c``; this module only owns numpy arrays and calls the C loops in the
order of the paper's PIC cycle (Sec. 2.2): Faraday + centring of B ->
gather/Boris/move/ZigZag per species -> Ampere-Maxwell -> external source ->
absorbing faces.

State convention: ``E`` holds E^n, ``B`` holds B^{n-1/2}, particle positions
are global x^n in [0, L) (FP64), momenta u^{n-1/2} = gamma v (c = 1).
Arrays are ``[3][ext_z][ext_y][ext_x]`` with ``ext = n + (absorbing)``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB may name another build of oracle.c (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
_lib = None

PERIODIC = 0
ABSORBING = 1
PEC = 2


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("bc", C.c_int32 * 3), ("d", C.c_double * 3),
                ("dt", C.c_double)]


class _Laser(C.Structure):
    _fields_ = [("a0", C.c_double), ("w0", C.c_double), ("tau", C.c_double),
                ("t0", C.c_double), ("omega0", C.c_double), ("yc", C.c_double),
                ("zc", C.c_double), ("i_s", C.c_int32), ("slab", C.c_int32)]


class _Port(C.Structure):
    _fields_ = [("axis", C.c_int32), ("plane", C.c_int32), ("comp", C.c_int32),
                ("prof_axis", C.c_int32), ("e0", C.c_double), ("omega", C.c_double),
                ("tau", C.c_double)]


_D = C.POINTER(C.c_double)
_I8 = C.POINTER(C.c_int8)


def lib():
    """Load liboracle.so, building it first when it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433
        _b.build()
    L = C.CDLL(_LIB_PATH)
    G = C.POINTER(_Grid)
    L.orc_faraday.argtypes = [G, _D, _D, _D]
    L.orc_ampere.argtypes = [G, _D, _D, _D]
    L.orc_mur.argtypes = [G, _D, _D]
    L.orc_pec.argtypes = [G, _D]
    L.orc_filter_J.argtypes = [G, _D, C.c_int32, C.c_int32]
    L.orc_window_shift.argtypes = [G, _D, _D, C.c_int32, C.c_int32]
    L.orc_port_apply.argtypes = [G, _D, C.POINTER(_Port), C.c_double]
    L.orc_laser_apply.argtypes = [G, _D, C.POINTER(_Laser), C.c_double]
    L.orc_laser_field.argtypes = [C.POINTER(_Laser), C.c_double, C.c_double, C.c_double]
    L.orc_laser_field.restype = C.c_double
    L.orc_gather.argtypes = [G, _D, _D, _D, _D, _D]
    L.orc_boris.argtypes = [_D, _D, _D, C.c_double]
    L.orc_particle_uniform.argtypes = [C.c_double, _D, _D, C.c_double, C.c_int64, _D, _D, _D]
    L.orc_zigzag.argtypes = [G, _D, _D, _D, C.c_double, C.c_int]
    L.orc_push_deposit.argtypes = [G, _D, _D, _D, C.c_int64, _D, _D, _I8, _D, C.c_double,
                                   C.c_double, C.c_double, C.c_int, C.c_int, _D]
    L.orc_rho.argtypes = [G, C.c_int64, _D, _I8, _D, C.c_double, C.c_double, _D]
    L.orc_gather2.argtypes = [G, _D, _D, _D, _D, _D]
    L.orc_ez2.argtypes = [G, _D, _D, _D, C.c_double]
    L.orc_push_deposit2.argtypes = [G, _D, _D, _D, C.c_int64, _D, _D, _I8, _D, C.c_double,
                                    C.c_double, C.c_double, C.c_int, _D]
    L.orc_rho2.argtypes = [G, C.c_int64, _D, _I8, _D, C.c_double, C.c_double, _D]
    L.orc_div_nodes.argtypes = [G, _D, _D]
    L.orc_energy_E.argtypes = [G, _D]
    L.orc_energy_E.restype = C.c_double
    L.orc_energy_B.argtypes = [G, _D, _D]
    L.orc_energy_B.restype = C.c_double
    L.orc_kinetic.argtypes = [C.c_int64, _D, _I8, _D, C.c_double, C.c_double]
    L.orc_kinetic.restype = C.c_double
    L.orc_particles_vjp.argtypes = [G, _D, _D, _D, C.c_int64, _D, _D, _D, C.c_double, C.c_double,
                                    C.c_double, _D, _D, _D, _D]
    L.orc_fields_vjp.argtypes = [G, _D, _D, _D, _D]
    _lib = L
    return L


def _p(a):
    """Pointer to a C-contiguous float64 array (None -> NULL)."""
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_D)


def _p8(a):
    if a is None:
        return None
    assert a.dtype == np.int8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I8)


def make_grid(n, d, dt, bc=(PERIODIC, PERIODIC, PERIODIC)) -> _Grid:
    g = _Grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.bc[a] = int(bc[a])
        g.d[a] = float(d[a])
    g.dt = float(dt)
    return g


def courant_dt(d, courant=0.5):
    """Time step at a given Courant number, from the 3D CFL bound (Sec. 2.3)."""
    return courant / np.sqrt(sum(1.0 / float(x) ** 2 for x in d))


class Species:
    def __init__(self, q, m, w, pos, u, wpp=None, ids=None, absorbing=False):
        self.q, self.m, self.w = float(q), float(m), float(w)
        self.pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3).copy()
        self.u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3).copy()
        self.np = self.pos.shape[0]
        self.wpp = None if wpp is None else np.ascontiguousarray(wpp, dtype=np.float64).copy()
        self.ids = np.arange(self.np, dtype=np.int64) if ids is None else np.asarray(ids).copy()
        self.alive = np.ones(self.np, dtype=np.int8) if absorbing else None


class OracleSim:
    """FP64 single-threaded reference simulation."""

    def __init__(self, n, d, dt, bc=(PERIODIC, PERIODIC, PERIODIC)):
        self.n = tuple(int(x) for x in n)
        self.d = tuple(float(x) for x in d)
        self.dt = float(dt)
        self.bc = tuple(int(x) for x in bc)
        self.g = make_grid(self.n, self.d, self.dt, self.bc)
        # walled (absorbing or PEC) axes hold n+1 node planes
        self.ext = tuple(self.n[a] + (1 if self.bc[a] != PERIODIC else 0) for a in range(3))
        shape = (3, self.ext[2], self.ext[1], self.ext[0])
        self.E = np.zeros(shape)
        self.B = np.zeros(shape)
        self.J = np.zeros(shape)
        self.Bbar = np.zeros(shape)
        self.species: list[Species] = []
        self.laser = None
        self.port = None
        self.filter = (0, 0)  # (binomial passes, compensate)
        self.window = None    # moving window (see set_window)
        self.rho_bg = 0.0
        self.nstep = 0
        self.midpoint_only = False
        self.shape_order = 1  # 2: b_2 weighting (triangular clouds), EZ deposit

    # -- set-up --------------------------------------------------------------
    @property
    def dV(self):
        return self.d[0] * self.d[1] * self.d[2]

    def add_species(self, q, m, w, pos, u, wpp=None, ids=None) -> int:
        absorbing = any(b != PERIODIC for b in self.bc)  # particles leave through walls
        self.species.append(Species(q, m, w, pos, u, wpp, ids, absorbing))
        return len(self.species) - 1

    def set_laser(self, a0, w0, tau, t0, omega0, yc, zc, i_s=1, slab=False):
        L = _Laser()
        L.a0, L.w0, L.tau, L.t0, L.omega0 = a0, w0, tau, t0, omega0
        L.yc, L.zc, L.i_s, L.slab = yc, zc, int(i_s), int(bool(slab))
        self.laser = L

    def set_port(self, axis, plane, comp, prof_axis, e0, omega, tau):
        """Hard TE10-like source on a node plane (Sec. 3.2; see orc_port_apply)."""
        P = _Port()
        P.axis, P.plane, P.comp, P.prof_axis = int(axis), int(plane), int(comp), int(prof_axis)
        P.e0, P.omega, P.tau = float(e0), float(omega), float(tau)
        self.port = P

    def set_window(self, axis, cells, velocity, t_start, inject=()):
        """Moving window along walled axis `axis` (READING of the module of
        Sec. 2.2 used in Sec. 4): at the start of a step, whenever the window
        has travelled (t - t_start) * velocity >= (shifts + 1) * cells * d,
        fields move `cells` planes back (zeros enter at the front), particles
        move by -cells * d, those behind the window are removed, and cold
        particles are injected into the new cells on a quiet lattice:
        inject = [(species, (px, py, pz), w), ...], offsets (m + 1/2)/p."""
        self.window = dict(axis=int(axis), cells=int(cells), v=float(velocity),
                           t0=float(t_start), shifts=0, inject=list(inject))

    def _window_step(self):
        W_ = self.window
        a, cells = W_["axis"], W_["cells"]
        t = self.nstep * self.dt
        if (t - W_["t0"]) * W_["v"] < (W_["shifts"] + 1) * cells * self.d[a]:
            return False
        W_["shifts"] += 1
        lib().orc_window_shift(C.byref(self.g), _p(self.E), _p(self.B), a, cells)
        shift = cells * self.d[a]
        for s in self.species:
            s.pos[:, a] -= shift
            out = s.pos[:, a] < 0.0
            s.alive[out] = 0
        for sp, per, w in W_["inject"]:
            s = self.species[sp]
            lo = [0] * 3
            hi = list(self.n)
            lo[a] = self.n[a] - cells
            axes = []
            for b in range(3):
                cellsb = np.arange(lo[b], hi[b])
                offs = (np.arange(per[b]) + 0.5) / per[b]
                axes.append(((cellsb[:, None] + offs[None, :]).reshape(-1)) * self.d[b])
            zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
            pos = np.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], axis=1)
            m = pos.shape[0]
            s.pos = np.concatenate([s.pos, pos])
            s.u = np.concatenate([s.u, np.zeros((m, 3))])
            wpp_new = np.full(m, float(w))
            if s.wpp is None:
                if abs(float(w) - s.w) > 0:
                    raise ValueError("injected weight differs from the species weight")
            else:
                s.wpp = np.concatenate([s.wpp, wpp_new])
            start = int(s.ids.max()) + 1 if len(s.ids) else 0
            s.ids = np.concatenate([s.ids, start + np.arange(m)])
            s.alive = np.concatenate([s.alive, np.ones(m, dtype=np.int8)])
            s.np = s.pos.shape[0]
        return True

    # -- the PIC cycle (Sec. 2.2) --------------------------------------------
    def step(self, nsteps: int = 1):
        L = lib()
        g = C.byref(self.g)
        absorbing = any(b == ABSORBING for b in self.bc)
        for _ in range(int(nsteps)):
            if self.window is not None:
                self._window_step()
            L.orc_faraday(g, _p(self.E), _p(self.B), _p(self.Bbar))
            self.J[...] = 0.0
            for s in self.species:
                if self.shape_order == 2:
                    L.orc_push_deposit2(g, _p(self.E), _p(self.Bbar), _p(self.J), s.np,
                                        _p(s.pos), _p(s.u), _p8(s.alive), _p(s.wpp), s.q, s.m,
                                        s.w, 0, None)
                    continue
                L.orc_push_deposit(g, _p(self.E), _p(self.Bbar), _p(self.J), s.np, _p(s.pos),
                                   _p(s.u), _p8(s.alive), _p(s.wpp), s.q, s.m, s.w,
                                   int(self.midpoint_only), 0, None)
            if self.filter[0] or self.filter[1]:
                L.orc_filter_J(g, _p(self.J), int(self.filter[0]), int(self.filter[1]))
            E_old = self.E.copy() if absorbing else None
            L.orc_ampere(g, _p(self.E), _p(self.B), _p(self.J))
            if self.laser is not None:
                L.orc_laser_apply(g, _p(self.E), C.byref(self.laser),
                                  (self.nstep + 0.5) * self.dt)
            if absorbing:
                L.orc_mur(g, _p(self.E), _p(E_old))
            if any(b == PEC for b in self.bc):
                L.orc_pec(g, _p(self.E))
            if self.port is not None:
                L.orc_port_apply(g, _p(self.E), C.byref(self.port), (self.nstep + 1) * self.dt)
            self.nstep += 1

    # -- adjoint of one step (periodic grids) ----------------------------------
    def step_vjp(self, lamE, lamB, lamX, lamU):
        """Vector-Jacobian product of one step taken from the current state.

        lamE, lamB: adjoints of E^{n+1}, B^{n+1/2}; lamX[s], lamU[s]: adjoints
        of x^{n+1}, u^{n+1/2} of species s ((N,3) arrays).  Returns the adjoints
        of E^n, B^{n-1/2}, x^n, u^{n-1/2}.  The state is not changed.
        """
        assert all(b == PERIODIC for b in self.bc), "adjoint needs a periodic grid"
        assert self.shape_order == 1, "adjoint of the first-order step only"
        L = lib()
        g = C.byref(self.g)
        Bh = self.B.copy()
        Bbar = np.zeros_like(self.B)
        L.orc_faraday(g, _p(self.E), _p(Bh), _p(Bbar))
        lJ = np.ascontiguousarray(-self.dt * lamE)
        if self.filter[0] or self.filter[1]:
            # E^{n+1} takes F J with F the (symmetric) filter: the deposit's
            # adjoint is F^T lam_J = F lam_J
            L.orc_filter_J(g, _p(lJ), int(self.filter[0]), int(self.filter[1]))
        lE = np.ascontiguousarray(lamE, dtype=np.float64).copy()
        lB = np.ascontiguousarray(lamB, dtype=np.float64).copy()
        lEg = np.zeros_like(lE)
        lBbar = np.zeros_like(lB)
        outX, outU = [], []
        for s, lx, lu in zip(self.species, lamX, lamU):
            lx = np.ascontiguousarray(lx, dtype=np.float64).copy()
            lu = np.ascontiguousarray(lu, dtype=np.float64).copy()
            L.orc_particles_vjp(g, _p(self.E), _p(Bbar), _p(lJ), s.np, _p(s.pos), _p(s.u),
                                _p(s.wpp), s.q, s.m, s.w, _p(lx), _p(lu), _p(lEg), _p(lBbar))
            outX.append(lx)
            outU.append(lu)
        L.orc_fields_vjp(g, _p(lE), _p(lB), _p(lEg), _p(lBbar))
        return lE, lB, outX, outU

    def state(self):
        return (self.E.copy(), self.B.copy(), [s.pos.copy() for s in self.species],
                [s.u.copy() for s in self.species])

    def set_state(self, st):
        E, B, X, U = st
        self.E[...] = E
        self.B[...] = B
        for s, x, u in zip(self.species, X, U):
            s.pos[...] = x
            s.u[...] = u

    # -- moments and diagnostics ---------------------------------------------
    def rho(self, species=None, with_background=False):
        L = lib()
        out = np.zeros(self.E.shape[1:])
        sel = range(len(self.species)) if species is None else [species]
        for i in sel:
            s = self.species[i]
            f = L.orc_rho2 if self.shape_order == 2 else L.orc_rho
            f(C.byref(self.g), s.np, _p(s.pos), _p8(s.alive), _p(s.wpp), s.q, s.w, _p(out))
        if with_background:
            out += self.rho_bg
        return out

    def div(self, F):
        out = np.zeros(F.shape[1:])
        lib().orc_div_nodes(C.byref(self.g), _p(np.ascontiguousarray(F)), _p(out))
        return out

    def gauss_residual(self):
        return self.div(self.E) - self.rho(with_background=True)

    def kinetic_plus(self):
        """K^{n+1/2} per species from a dry push of the current state."""
        L = lib()
        Bbar = self.B.copy()
        Bh = self.B.copy()
        L.orc_faraday(C.byref(self.g), _p(self.E), _p(Bh), _p(Bbar))
        out = []
        for s in self.species:
            k = C.c_double(0.0)
            u = s.u.copy()
            pos = s.pos.copy()
            alive = _p8(None if s.alive is None else s.alive.copy())
            if self.shape_order == 2:
                L.orc_push_deposit2(C.byref(self.g), _p(self.E), _p(Bbar), None, s.np, _p(pos),
                                    _p(u), alive, _p(s.wpp), s.q, s.m, s.w, 1, C.byref(k))
            else:
                L.orc_push_deposit(C.byref(self.g), _p(self.E), _p(Bbar), None, s.np, _p(pos),
                                   _p(u), alive, _p(s.wpp), s.q, s.m, s.w, 0, 1, C.byref(k))
            out.append(k.value)
        return out

    def diagnostics(self):
        L = lib()
        g = C.byref(self.g)
        UE = L.orc_energy_E(g, _p(self.E))
        UB = L.orc_energy_B(g, _p(self.E), _p(self.B))
        km = [L.orc_kinetic(s.np, _p(s.u), _p8(s.alive), _p(s.wpp), s.m, s.w)
              for s in self.species]
        kp = self.kinetic_plus()
        K = [0.5 * (a + b) for a, b in zip(km, kp)]
        r = self.gauss_residual()
        return {"step": self.nstep, "t": self.nstep * self.dt, "U_E": UE, "U_B": UB,
                "K_minus": km, "K_plus": kp, "K": K, "U_tot": UE + UB + sum(K),
                "gauss_max": float(np.max(np.abs(r))),
                "gauss_l2": float(np.sqrt(np.mean(r * r))),
                "n_particles": [int(s.np if s.alive is None else s.alive.sum())
                                for s in self.species]}


# -- single-particle helpers for the Sec. 3.1 benchmarks ----------------------
def boris(u, Ep, Bp, r):
    u = np.array(u, dtype=np.float64)
    lib().orc_boris(_p(u), _p(np.asarray(Ep, dtype=np.float64)),
                    _p(np.asarray(Bp, dtype=np.float64)), float(r))
    return u


def particle_uniform(r, E, B, dt, nsteps, x0, u0, record=False):
    x = np.array(x0, dtype=np.float64)
    u = np.array(u0, dtype=np.float64)
    traj = np.zeros((int(nsteps), 3)) if record else None
    lib().orc_particle_uniform(float(r), _p(np.asarray(E, dtype=np.float64)),
                               _p(np.asarray(B, dtype=np.float64)), float(dt), int(nsteps),
                               _p(x), _p(u), _p(traj))
    return x, u, traj


def zigzag(grid: _Grid, shape, xi1, xi2, qsp, midpoint_only=False, J=None):
    J = np.zeros(shape) if J is None else J
    lib().orc_zigzag(C.byref(grid), _p(J), _p(np.asarray(xi1, dtype=np.float64)),
                     _p(np.asarray(xi2, dtype=np.float64)), float(qsp), int(midpoint_only))
    return J


def gather2(grid: _Grid, E, Bbar, pos):
    Ep = np.zeros(3)
    Bp = np.zeros(3)
    lib().orc_gather2(C.byref(grid), _p(E), _p(Bbar), _p(np.asarray(pos, dtype=np.float64)),
                      _p(Ep), _p(Bp))
    return Ep, Bp


def ez2(grid: _Grid, shape, xi1, xi2, qsp, J=None):
    J = np.zeros(shape) if J is None else J
    lib().orc_ez2(C.byref(grid), _p(J), _p(np.asarray(xi1, dtype=np.float64)),
                  _p(np.asarray(xi2, dtype=np.float64)), float(qsp))
    return J


def gather(grid: _Grid, E, Bbar, pos):
    Ep = np.zeros(3)
    Bp = np.zeros(3)
    lib().orc_gather(C.byref(grid), _p(E), _p(Bbar), _p(np.asarray(pos, dtype=np.float64)),
                     _p(Ep), _p(Bp))
    return Ep, Bp
