"""Seeded synthetic plasmas and set-ups of the workloads of this project
(the five benchmark configurations, the waveguide and PEC cases, and the
two-dimensional wakefield run of Sec. 4).

This module only draws random numbers and lays out initial conditions; it
holds none of the PIC step's arithmetic, so both the FP64 oracle and the HIP
path can take their inputs from it.  Every array is FP64 with *global*
positions in [0, L) and momenta u = gamma v (c = 1); the HIP path converts to
its own storage on the device.

Units: c = eps0 = mu0 = 1.  Plasma workloads take n0 = 1, so omega_p = 1 and
the cell size is one skin depth; electrons have q = -1, m = 1, protons q = +1,
m = 1836.  A macro-particle of weight w carries q w and m w (Sec. 2.1 of the
paper).  The time step is the paper's Courant number 0.5 (Sec. 3.2, 3.3).

Generator: numpy PCG64 seeded with 1000 + workload number.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PERIODIC = 0
ABSORBING = 1
PEC = 2
M_PROTON = 1836.0


@dataclass
class SpeciesInit:
    name: str
    q: float
    m: float
    w: float
    pos: np.ndarray            # (N, 3) float64 global positions
    u: np.ndarray              # (N, 3) float64, u^{-1/2}
    wpp: Optional[np.ndarray] = None   # (N,) per-particle weight, replaces w


@dataclass
class LaserInit:
    a0: float
    w0: float
    tau: float
    t0: float
    omega0: float
    yc: float
    zc: float
    i_s: int = 1
    slab: bool = False        # spot Gaussian in z only (two-dimensional runs)


@dataclass
class PortInit:
    """Hard source E_comp = e0 sin(pi s/L) (1 - exp(-t/tau)) sin(omega t) on a node plane."""
    axis: int
    plane: int
    comp: int
    prof_axis: int
    e0: float
    omega: float
    tau: float


@dataclass
class WindowInit:
    """Moving window along a walled axis: shifts of `cells` cells once the
    window has travelled (t - t_start) velocity; cold plasma injected into the
    new cells: inject = [(species, (px, py, pz) per cell, weight), ...]."""
    axis: int
    cells: int
    velocity: float
    t_start: float
    inject: list = field(default_factory=list)


@dataclass
class Workload:
    name: str
    n: tuple
    d: tuple
    dt: float
    bc: tuple
    species: list = field(default_factory=list)
    rho_bg: float = 0.0
    laser: Optional[LaserInit] = None
    port: Optional[PortInit] = None
    filter: Optional[tuple] = None    # (binomial passes, compensate) of the current filter
    window: Optional[WindowInit] = None
    steps: int = 1
    sort_every: int = 10
    E0: Optional[np.ndarray] = None   # (3, ext_z, ext_y, ext_x) or None -> zero
    B0: Optional[np.ndarray] = None

    @property
    def n_particles(self) -> int:
        return int(sum(s.pos.shape[0] for s in self.species))

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.n))


def courant_dt(d, courant: float = 0.5) -> float:
    return float(courant / np.sqrt(sum(1.0 / float(x) ** 2 for x in d)))


def _uniform_in_cells(rng, n, d, ppc, cell_mask=None):
    """ppc positions uniformly random inside every cell, cell-ordered (x fastest)."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    if cell_mask is not None:
        cells = cells[cell_mask.ravel()]
    cells = np.repeat(cells, ppc, axis=0)
    frac = rng.random(cells.shape)
    pos = (cells + frac) * np.asarray(d, dtype=np.float64)
    L = np.asarray(n, dtype=np.float64) * np.asarray(d, dtype=np.float64)
    # (i + frac) * d can round up to L for the last cell: keep positions in [0, L)
    pos = np.where(pos >= L, np.nextafter(L, 0.0), pos)
    return pos


def _quiet_lattice(n, d, per_axis):
    """Regular lattice with per-axis counts at offsets (m + 1/2)/n_m in every cell."""
    offs = [(np.arange(c) + 0.5) / c for c in per_axis]
    oz, oy, ox = np.meshgrid(offs[2], offs[1], offs[0], indexing="ij")
    local = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    pos = (cells[:, None, :] + local[None, :, :]).reshape(-1, 3)
    return pos * np.asarray(d, dtype=np.float64)


def langmuir_thermal(n=(16, 16, 16), ppc=8, vth=0.01, amp=1e-3, mode=1, steps=200, seed=1001):
    """Periodic thermal plasma with a Langmuir perturbation.

    16^3 cells of size 1, 8 electrons per cell uniformly random in the cell,
    u ~ N(0, vth^2) per component plus u_x += amp sin(2 pi mode x / L_x),
    immobile neutralising background rho_bg = +1, 200 steps, FP64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d = (1.0, 1.0, 1.0)
    pos = _uniform_in_cells(rng, n, d, ppc)
    u = rng.normal(0.0, vth, size=pos.shape)
    u[:, 0] += amp * np.sin(2.0 * np.pi * mode * pos[:, 0] / (n[0] * d[0]))
    sp = SpeciesInit("electron", -1.0, 1.0, 1.0 / ppc, pos, u)
    return Workload("langmuir_thermal_%dx%dx%d_ppc%d" % (*n, ppc), tuple(n), d, courant_dt(d),
                    (PERIODIC,) * 3, [sp], rho_bg=1.0, steps=steps, sort_every=10)


def thermal_two_species(n=(128, 128, 128), ppc=8, vth=0.05, steps=100, seed=1002,
                        sort_every=10):
    """Periodic thermal electron-proton plasma (the benchmark).

    128^3 cells of size 1, 8 electrons and 8 protons per cell; protons sit on
    the electron positions (exact initial neutrality, E^0 = 0 satisfies
    Gauss's law).  u_e ~ N(0, 0.05^2), u_p ~ N(0, (0.05/sqrt(1836))^2) per
    component (equal temperatures).  Weight 1/ppc each (n0 = 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d = (1.0, 1.0, 1.0)
    pos = _uniform_in_cells(rng, n, d, ppc)
    ue = rng.normal(0.0, vth, size=pos.shape)
    up = rng.normal(0.0, vth / np.sqrt(M_PROTON), size=pos.shape)
    e = SpeciesInit("electron", -1.0, 1.0, 1.0 / ppc, pos, ue)
    p = SpeciesInit("proton", 1.0, M_PROTON, 1.0 / ppc, pos.copy(), up)
    return Workload("thermal_ep_%dx%dx%d_ppc%d" % (*n, ppc), tuple(n), d, courant_dt(d),
                    (PERIODIC,) * 3, [e, p], rho_bg=0.0, steps=steps, sort_every=sort_every)


def lwfa_slab(n=(1024, 128, 128), d=(0.05, 0.2, 0.2), ppc=2, x_start=128, ramp=40,
              n_plasma=0.01, a0=2.0, w0=8.0, tau=10.0, steps=2000, seed=1003,
              sort_every=10):
    """Laser-wakefield-like box with absorbing faces (laser units).

    c = omega0 = 1, densities in units of n_c.  Cold electron slab filling
    x >= x_start cells with a linear up-ramp over `ramp` cells to n_plasma,
    `ppc` particles per cell along a (ppc, 1, 1) regular lattice with
    per-particle weight n(x) dV / ppc.  Linearly (y) polarised Gaussian pulse
    of peak amplitude a0, waist w0, intensity FWHM tau, injected at x node 1.
    """
    nx, ny, nz = n
    dV = d[0] * d[1] * d[2]
    offs = (np.arange(ppc) + 0.5) / ppc
    xs = np.arange(x_start, nx)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), xs, indexing="ij")
    cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    cells = np.repeat(cells, ppc, axis=0)
    local = np.zeros_like(cells)
    local[:, 0] = np.tile(offs, cells.shape[0] // ppc)
    local[:, 1] = 0.5
    local[:, 2] = 0.5
    rng = np.random.Generator(np.random.PCG64(seed))
    # small seeded jitter in the transverse offsets breaks the exact lattice symmetry
    local[:, 1:] += 0.25 * (rng.random((cells.shape[0], 2)) - 0.5)
    pos = (cells + local) * np.asarray(d)
    xc = pos[:, 0] / d[0]
    dens = n_plasma * np.clip((xc - x_start) / ramp, 0.0, 1.0)
    wpp = dens * dV / ppc
    u = np.zeros_like(pos)
    sp = SpeciesInit("electron", -1.0, 1.0, n_plasma * dV / ppc, pos, u, wpp=wpp)
    Ly, Lz = ny * d[1], nz * d[2]
    laser = LaserInit(a0=a0, w0=w0, tau=tau, t0=2.5 * tau, omega0=1.0, yc=0.5 * Ly,
                      zc=0.5 * Lz, i_s=1)
    return Workload("lwfa_%dx%dx%d_ppc%d" % (nx, ny, nz, ppc), tuple(n), tuple(d),
                    courant_dt(d), (ABSORBING,) * 3, [sp], rho_bg=0.0, laser=laser,
                    steps=steps, sort_every=sort_every)


def cold_langmuir_lattice(n=(32, 32, 32), per_axis=(4, 2, 2), eps=1e-2, mode=1, steps=500):
    """Cold quiet-start plasma for the differentiable run.

    32^3 cells, 16 particles per cell on a (4, 2, 2) lattice at offsets
    (m + 1/2)/n_m, u_x = eps sin(2 pi mode x / L_x), background rho_bg = +1.
    Deterministic (no random draws).
    """
    d = (1.0, 1.0, 1.0)
    pos = _quiet_lattice(n, d, per_axis)
    ppc = int(np.prod(per_axis))
    u = np.zeros_like(pos)
    u[:, 0] = eps * np.sin(2.0 * np.pi * mode * pos[:, 0] / (n[0] * d[0]))
    sp = SpeciesInit("electron", -1.0, 1.0, 1.0 / ppc, pos, u)
    return Workload("cold_langmuir_%dx%dx%d_ppc%d" % (*n, ppc), tuple(n), d, courant_dt(d),
                    (PERIODIC,) * 3, [sp], rho_bg=1.0, steps=steps, sort_every=0)


def smooth_random_direction(pos, box, seed, scale=1e-2):
    """A random direction in the space of all initial momenta of a species:
    a smooth random momentum field (four Fourier modes per component with
    integer wave numbers 0..2 along each axis and random phases) sampled at
    each particle's position, normalised to unit RMS, plus white noise of the
    same RMS, times `scale`.  A pure white-noise direction would be nearly
    orthogonal to the modes a field loss responds to.  Seeded, draws only."""
    rng = np.random.default_rng(seed)
    out = np.zeros_like(pos)
    for c in range(3):
        for _ in range(4):
            k = rng.integers(0, 3, size=3) / np.asarray(box)
            out[:, c] += rng.standard_normal() * np.cos(2 * np.pi * (pos @ k) + 2 * np.pi * rng.random())
    out /= np.sqrt(np.mean(out ** 2))
    out += rng.standard_normal(pos.shape)
    return scale * out


def weibel_bimaxwellian(n=(256, 256, 256), ppc=16, vth_x=0.25, vth_perp=0.05, steps=50,
                        seed=1005, sort_every=10):
    """Anisotropic (T_x/T_perp = 25) electrons over immobile ions.

    u_x ~ N(0, 0.25^2), u_y, u_z ~ N(0, 0.05^2); 16 electrons per cell
    uniformly random in the cell; background rho_bg = +1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d = (1.0, 1.0, 1.0)
    pos = _uniform_in_cells(rng, n, d, ppc)
    u = np.empty_like(pos)
    u[:, 0] = rng.normal(0.0, vth_x, size=pos.shape[0])
    u[:, 1:] = rng.normal(0.0, vth_perp, size=(pos.shape[0], 2))
    sp = SpeciesInit("electron", -1.0, 1.0, 1.0 / ppc, pos, u)
    return Workload("weibel_%dx%dx%d_ppc%d" % (*n, ppc), tuple(n), d, courant_dt(d),
                    (PERIODIC,) * 3, [sp], rho_bg=1.0, steps=steps, sort_every=sort_every)


def random_fields(n, bc=(PERIODIC,) * 3, scale=1e-2, seed=7):
    """Random E and B arrays (valid entries only; walled-axis padding left zero)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = [n[a] + (1 if bc[a] != PERIODIC else 0) for a in range(3)]
    E = scale * rng.standard_normal((3, ext[2], ext[1], ext[0]))
    B = scale * rng.standard_normal((3, ext[2], ext[1], ext[0]))
    for c in range(3):
        for a in range(3):
            if bc[a] == PERIODIC:
                continue
            # E_c is half-staggered along a == c; B_c along a != c: index n is padding
            sl = [slice(None)] * 3
            sl[2 - a] = n[a]
            if a == c:
                E[c][tuple(sl)] = 0.0
            else:
                B[c][tuple(sl)] = 0.0
    return E, B


# speed of light in cm/ns: lengths in cm, c = 1
C_CM_PER_NS = 29.9792458


def waveguide_te10(nodes=(12, 6, 376), a=3.0, b=1.5, Lz=100.0, f0_ghz=9.0, e0=1.0,
                   tau_periods=2.0, steps=None):
    """The field-solver benchmark of Sec. 3.2: a PEC rectangular guide a x b x Lz
    (cm; a = 3, b = a/2, Lz = 1 m) driven at z = 0 by the TE10 field
    E_y = e0 sin(pi x/a) (1 - exp(-t/tau)) sin(2 pi f0 t), f0 = 9 GHz, tau = 2
    periods; Courant 0.5.  `nodes` counts grid points per axis as the paper's
    convergence table does (cells = nodes - 1).  Units: c = 1, lengths in cm.
    x and y are PEC walls; the far end z = Lz is absorbing (Mur).  No
    particles.  steps defaults to 30 periods (the table's n_t)."""
    n = tuple(int(v) - 1 for v in nodes)
    d = (a / n[0], b / n[1], Lz / n[2])
    dt = courant_dt(d)
    omega = 2.0 * np.pi * f0_ghz / C_CM_PER_NS
    T0 = 2.0 * np.pi / omega
    port = PortInit(axis=2, plane=0, comp=1, prof_axis=0, e0=e0, omega=omega,
                    tau=tau_periods * T0)
    nsteps = int(round(30.0 * T0 / dt)) if steps is None else int(steps)
    return Workload("waveguide_te10_%dx%dx%d" % tuple(nodes), n, d, dt, (PEC, PEC, ABSORBING),
                    [], rho_bg=0.0, port=port, steps=nsteps, sort_every=0)


def pec_cavity_plasma(n=(16, 12, 8), d=(1.0, 0.9, 1.1), ppc=4, vth=0.3, seed=1006):
    """Hot electrons with per-particle weights in a closed PEC box: particles
    reach the walls (and are removed) within a few steps; for parity of the
    wall treatment.  Random initial fields with tangential E zero on the
    walls."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = _uniform_in_cells(rng, n, d, ppc)
    u = vth * rng.standard_normal(pos.shape)
    wpp = 0.5 + rng.random(pos.shape[0])
    sp = SpeciesInit("electron", -1.0, 1.0, 1.0, pos, u, wpp=wpp / ppc)
    w = Workload("pec_cavity_%dx%dx%d" % tuple(n), tuple(n), tuple(d), courant_dt(d), (PEC,) * 3,
                 [sp], rho_bg=0.0, steps=20, sort_every=5)
    E, B = random_fields(n, bc=(PEC,) * 3, scale=0.05, seed=seed + 1)
    for a in range(3):  # tangential E is zero on the walls
        for c in range(3):
            if c == a:
                continue
            for side in (0, n[a]):
                sl = [slice(None)] * 3
                sl[2 - a] = side
                E[c][tuple(sl)] = 0.0
    w.E0, w.B0 = E, B
    return w



# SI constants (CODATA 2018) for the unit conversions of the wakefield run
C_SI = 299792458.0
E_SI = 1.602176634e-19
ME_SI = 9.1093837015e-31
EPS0_SI = 8.8541878128e-12


@dataclass
class LaserUnits:
    """Laser units of a run: c = omega0 = 1, lengths in c/omega0, densities in
    n_c = eps0 m omega0^2 / e^2, fields in m c omega0 / e."""
    lambda0_m: float

    @property
    def omega0(self) -> float:            # rad/s
        return 2.0 * np.pi * C_SI / self.lambda0_m

    @property
    def length_m(self) -> float:          # c / omega0
        return C_SI / self.omega0

    @property
    def time_s(self) -> float:            # 1 / omega0
        return 1.0 / self.omega0

    @property
    def n_crit_cm3(self) -> float:
        return EPS0_SI * ME_SI * self.omega0 ** 2 / E_SI ** 2 * 1e-6

    @property
    def field_v_per_m(self) -> float:     # m c omega0 / e
        return ME_SI * C_SI * self.omega0 / E_SI


def lwfa_2d(per=(4, 2, 4), cells=(1400, 2, 300), n0_cm3=3.0e18, lambda0_um=0.8,
            fwhm_fs=28.0, w0_um=12.0, a0=3.0, window_lp=(3.0, 1.0, 3.0), travel_lp=6.0,
            window_start=0.75, shift_cells=8, sort_every=-1, steps=None):
    """The two-dimensional laser-wakefield run of Sec. 4 (its parameter table).

    Our x is the paper's propagation axis z, our z its transverse x, y is the
    periodic axis two cells wide; the pulse is polarised along y.  Cell sizes
    come from the paper's window (L_x, L_y, L_z) = (3, 1, 3) lambda_p over
    (1400, 2, 300) cells, i.e. its (301 x 2 x 1401) counts of grid nodes;
    `cells` may shrink the box at those cell sizes (parity runs).  Laser
    units (LaserUnits); Courant 0.5.  A cold homogeneous electron plasma of
    density n0 fills the box on a quiet `per` lattice (offsets (m + 1/2)/p)
    over an immobile neutralising background; the window moves at c once
    the pulse peak has crossed `window_start` of the box, in shifts of
    `shift_cells` cells, injecting the same lattice.  The laser sheet sits
    at x node 1: E_inc = a0 exp(-(z - zc)^2/w0^2) exp(-2 ln2 (t-t0)^2/tau^2)
    sin(t - t0), tau = the intensity FWHM, t0 = 2.5 tau.  `steps` defaults to
    the pulse peak travelling `travel_lp` plasma wavelengths past the sheet.
    Sorting is adaptive (every window shift sorts as well).  Deterministic
    (no random draws).
    """
    U = LaserUnits(lambda0_um * 1e-6)
    n_pl = n0_cm3 / U.n_crit_cm3
    lam_p = 2.0 * np.pi / np.sqrt(n_pl)
    d = (float(window_lp[2] * lam_p / 1400.0), float(window_lp[1] * lam_p / 2.0),
         float(window_lp[0] * lam_p / 300.0))
    n = tuple(int(c) for c in cells)
    dt = courant_dt(d)
    ppc = int(np.prod(per))
    dV = d[0] * d[1] * d[2]
    w = n_pl * dV / ppc
    pos = _quiet_lattice(n, d, per)
    sp = SpeciesInit("electron", -1.0, 1.0, w, pos, np.zeros_like(pos))
    tau = fwhm_fs * 1e-15 / U.time_s
    t0 = 2.5 * tau
    Lx, Ly, Lz = (float(n[a] * d[a]) for a in range(3))
    laser = LaserInit(a0=a0, w0=w0_um * 1e-6 / U.length_m, tau=tau, t0=t0, omega0=1.0,
                      yc=0.5 * Ly, zc=0.5 * Lz, i_s=1, slab=True)
    window = WindowInit(axis=0, cells=shift_cells, velocity=1.0, t_start=t0 + window_start * Lx,
                        inject=[(0, tuple(per), w)])
    nsteps = int(np.ceil((t0 + travel_lp * lam_p) / dt)) if steps is None else int(steps)
    wl = Workload("lwfa2d_%dx%dx%d_ppc%d" % (*n, ppc), n, d, dt, (ABSORBING, PERIODIC, ABSORBING),
                  [sp], rho_bg=n_pl, laser=laser, window=window, steps=nsteps,
                  sort_every=sort_every)
    wl.units = U
    wl.n_plasma = n_pl
    wl.lambda_p = lam_p
    return wl
