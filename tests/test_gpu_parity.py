"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (relative, ||a - b||_inf / ||b||_inf; positions in cells):
  FP64 plain step   <= 1e-12 after one step, <= 1e-9 after 50 steps (the
                    only difference is the order of the FP64 atomic adds);
  FP32 fused step   <= 2e-5 after one step from a common FP64 state rounded
                    to FP32; continuity residual <= 1e-5 max|rho|.
"""
import numpy as np
import pytest

from gpu_common import check_box_currents, compare_state, oracle_from, pos_err_cells, rel
from oracle import oracle as O
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, prec, **kw):
    from paper_2609_16575_amd.sim import Sim
    return Sim(w, precision=prec, **kw)


def _thermal(n=(16, 16, 16), ppc=8, vth=0.05, field_scale=0.05, seed=11):
    w = W.langmuir_thermal(n=n, ppc=ppc, vth=vth)
    if field_scale:
        w.E0, w.B0 = W.random_fields(w.n, w.bc, scale=field_scale, seed=seed)
    return w


@pytest.mark.parametrize("prec,tol1,tol20", [("fp64", 1e-12, 1e-11), ("fp32", 2e-5, 2e-4)])
def test_vacuum_yee(prec, tol1, tol20):
    w = W.Workload("vacuum", (24, 16, 12), (1.0, 0.8, 1.2), W.courant_dt((1.0, 0.8, 1.2)),
                   (0, 0, 0), [], steps=20)
    w.E0, w.B0 = W.random_fields(w.n, scale=1.0, seed=3)
    g, o = _sim(w, prec), oracle_from(w, w.E0, w.B0)
    g.step(1)
    o.step(1)
    E, B, _ = g.fields()
    assert rel(E, o.E) <= tol1 and rel(B, o.B) <= tol1, (rel(E, o.E), rel(B, o.B))
    g.step(19)
    o.step(19)
    E, B, _ = g.fields()
    assert rel(E, o.E) <= tol20 and rel(B, o.B) <= tol20, (rel(E, o.E), rel(B, o.B))


def test_fp64_one_step_thermal_with_fields():
    w = _thermal()
    g, o = _sim(w, "fp64"), oracle_from(w, w.E0, w.B0)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=1e-12, f_tol=1e-12, label="fp64 1 step")


def test_fp64_langmuir_workload_50_steps():
    """The Langmuir thermal plasma as specified (16^3, 8 ppc, v_th = 0.01c, E = B = 0)."""
    w = W.langmuir_thermal()
    g, o = _sim(w, "fp64"), oracle_from(w)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=1e-12, f_tol=1e-12, label="fp64 step 1")
    g.step(49)
    o.step(49)
    compare_state(g, o, w, sp_tol=1e-9, f_tol=1e-9, label="fp64 step 50")


def test_fp32_one_step_thermal_with_fields():
    w = _thermal()
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    # common state: the oracle starts from the FP32-rounded state of the GPU
    E, B, _ = g.fields()
    o.E[...] = E
    o.B[...] = B
    P, U, _ = g.particles_by_id(0)
    o.species[0].pos[...] = P
    o.species[0].u[...] = U
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="fp32 1 step")


def _common_fp32_state(g, o):
    E, B, _ = g.fields()
    o.E[...] = E
    o.B[...] = B
    for i in range(len(o.species)):
        P, U, I = g.particles_by_id(i)
        o.species[i].pos[...] = P
        o.species[i].u[...] = U


def test_fp32_two_species_one_step():
    w = W.thermal_two_species(n=(16, 16, 16), ppc=8)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=5)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="fp32 e+p")


def test_fp32_dense_tiles_two_species():
    """20 electrons + 20 protons per cell on 16^3: 5120 particles of each
    species per 256-cell tile, so every tile takes three batches of 2048
    (four per thread) per species and the sort moves tiles larger than its
    LDS staging; fields, currents and particles by id after one step from a
    common state (2e-5) and after ten more (2e-4)."""
    w = W.thermal_two_species(n=(16, 16, 16), ppc=20, vth=0.05)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=8)
    g, o = _sim(w, "fp32", sort_every=5), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="dense 1 step")
    g.diagnostics()  # rho of this step, for the continuity of the next
    for _ in range(10):
        g.step(1)
        d = g.diagnostics()
        assert d["cont_valid"] and d["cont_max"] <= 1e-5 * d["rho_max"], d
        assert d["fault_word"] & ~16 == 0, d
    o.step(10)
    compare_state(g, o, w, sp_tol=2e-4, f_tol=2e-4, label="dense 11 steps")


def test_fp32_multistep_tracks_oracle_and_conserves_charge():
    """20 steps of the Langmuir thermal plasma (sort every 10): stays near the FP64 run and the
    continuity residual of every step is at FP32 round-off."""
    w = W.langmuir_thermal(steps=20)
    g, o = _sim(w, "fp32"), oracle_from(w)
    _common_fp32_state(g, o)
    g.diagnostics()
    for k in range(20):
        g.step(1)
        d = g.diagnostics()
        assert d["cont_valid"]
        assert d["cont_max"] <= 1e-5 * d["rho_max"], (k, d["cont_max"], d["rho_max"])
        assert d["fault_word"] & ~16 == 0
    o.step(20)
    compare_state(g, o, w, sp_tol=2e-4, f_tol=2e-3, label="fp32 20 steps")


def test_gauss_drift_gpu():
    w = W.langmuir_thermal()
    for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        g = _sim(w, prec)
        o = oracle_from(w)
        E, _, _ = g.fields()
        r0 = o.div(E) - g.rho() - w.rho_bg
        g.step(30)
        E, _, _ = g.fields()
        r1 = o.div(E) - g.rho() - w.rho_bg
        assert np.max(np.abs(r1 - r0)) <= tol * np.max(np.abs(g.rho())), prec


def test_diagnostics_match_oracle_fp64():
    w = _thermal(field_scale=0.02)
    g, o = _sim(w, "fp64"), oracle_from(w, w.E0, w.B0)
    g.step(5)
    o.step(5)
    dg, do = g.diagnostics(), o.diagnostics()
    for k in ("U_E", "U_B", "U_tot", "gauss_max"):
        assert abs(dg[k] - do[k]) <= 1e-11 * abs(do[k]), (k, dg[k], do[k])
    for k in ("K_minus", "K_plus", "K"):
        assert abs(dg[k][0] - do[k][0]) <= 1e-11 * abs(do[k][0]), (k, dg[k], do[k])


def test_diagnostics_fp32_close_to_oracle():
    w = _thermal(field_scale=0.02)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    dg, do = g.diagnostics(), o.diagnostics()
    for k in ("U_E", "U_B", "U_tot"):
        assert abs(dg[k] - do[k]) <= 1e-5 * abs(do[k]), (k, dg[k], do[k])
    assert abs(dg["K_plus"][0] - do["K_plus"][0]) <= 1e-5 * do["K_plus"][0]


def test_fp32_edge_offsets_and_seams():
    """Particles on cell faces, just below 1, across the periodic seam, in all
    crossing directions; one step from a common state."""
    n = (8, 8, 8)
    rng = np.random.default_rng(21)
    base = np.array([[0.0, 0.0, 0.0], [7.0, 7.0, 7.0], [3.0, 4.0, 5.0], [7.999999, 0.0, 3.5],
                     [0.0, 7.9999999, 0.5], [4.5, 4.5, 4.5], [1.0, 2.0, 3.0], [6.0, 0.0, 7.0]])
    jitter = np.array([0.0, 1 - 2 ** -24, 0.5, 2 ** -20])
    pos = []
    for b in base:
        for j in jitter:
            pos.append(np.mod(b + j, 8.0))
    pos = np.array(pos)
    u = rng.choice([-0.6, 0.6], size=pos.shape) + rng.normal(0, 0.01, pos.shape)
    w = W.Workload("edges", n, (1.0, 1.0, 1.0), W.courant_dt((1.0, 1.0, 1.0)), (0, 0, 0),
                   [W.SpeciesInit("e", -1.0, 1.0, 0.5, pos, u)], steps=1, sort_every=1)
    w.E0, w.B0 = W.random_fields(n, scale=0.1, seed=2)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    for _ in range(3):
        g.step(1)
        o.step(1)
        compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="edges")
        _common_fp32_state(g, o)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 2)])
def test_fp32_ragged_grid(bc):
    """A grid that is a multiple of the 8 x 8 x 4 tile on no axis (13 x 11 x 7),
    periodic, and absorbing / periodic / PEC: hot electrons with per-particle
    weights, one step from a common state, then five more."""
    n, d = (13, 11, 7), (1.0, 0.9, 1.1)
    rng = np.random.default_rng(31)
    pos = W._uniform_in_cells(rng, n, d, 6)
    u = rng.normal(0.0, 0.2, pos.shape)
    wpp = 0.05 + 0.1 * rng.random(len(pos))
    w = W.Workload("ragged", n, d, W.courant_dt(d), bc,
                   [W.SpeciesInit("e", -1.0, 1.0, 0.1, pos, u, wpp=wpp)], sort_every=2)
    w.E0, w.B0 = W.random_fields(n, bc, scale=0.05, seed=6)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="ragged 1 step")
    g.step(5)
    o.step(5)
    compare_state(g, o, w, sp_tol=2e-4, f_tol=2e-4, label="ragged 6 steps")


def test_fp32_largest_packed_cell_indices():
    """The largest grid the packed FP32 cell index holds (2047 x 3 x 1023
    cells, periodic): particles in the last cells and across the seams of
    the long axes, one step against the oracle."""
    n = (2047, 3, 1023)
    d = (1.0, 1.0, 1.0)
    rng = np.random.default_rng(41)
    corners = np.array([[2046.5, 1.5, 1022.5], [0.2, 0.5, 1022.9], [2046.95, 2.9, 0.05],
                        [1023.5, 1.5, 511.5], [0.01, 0.01, 0.01]])
    pos = np.mod(np.repeat(corners, 16, axis=0) + rng.uniform(-0.4, 0.4, (80, 3)),
                 np.array(n, dtype=float))
    u = rng.choice([-0.5, 0.5], size=pos.shape) + rng.normal(0, 0.05, pos.shape)
    w = W.Workload("largest", n, d, W.courant_dt(d), (0, 0, 0),
                   [W.SpeciesInit("e", -1.0, 1.0, 0.5, pos, u)], sort_every=1)
    w.E0, w.B0 = W.random_fields(n, scale=0.02, seed=12)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    for _ in range(2):
        g.step(1)
        o.step(1)
        compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="largest")
        _common_fp32_state(g, o)


def test_fp32_out_of_window_fallback():
    """No re-sort and fast particles: many leave their tile's LDS window and go
    through the global-memory path; results still match the oracle."""
    w = W.langmuir_thermal(n=(16, 16, 16), ppc=4, vth=1.5)
    w.sort_every = 0
    w.E0, w.B0 = W.random_fields(w.n, scale=0.02, seed=8)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    for k in range(12):
        g.step(1)
        o.step(1)
        if k >= 6:
            compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="fallback %d" % k)
        _common_fp32_state(g, o)
    d = g.diagnostics()
    assert d["fallback_particles"] > 0
    assert d["fault_word"] & 16


@pytest.mark.parametrize("n,ppc", [((16, 16, 16), 4), ((40, 2, 20), 4), ((16, 16, 16), 20)])
def test_sort_is_a_permutation(n, ppc):
    """Also on a grid two cells thick along y, which gets the 16 x 2 x 8 tiles,
    and with 20 per cell: 5120 particles of a species per tile, more than the
    sort's per-tile register and LDS staging holds (4608), so that its
    direct paths run."""
    w = W.thermal_two_species(n=n, ppc=ppc)
    g = _sim(w, "fp32")
    g.step(3)
    before = [g.particles_by_id(i) for i in range(2)]
    g.sort()
    after = [g.particles_by_id(i) for i in range(2)]
    for (P0, U0, I0), (P1, U1, I1) in zip(before, after):
        assert np.array_equal(I0, I1)
        assert np.array_equal(P0, P1) and np.array_equal(U0, U1)
    # storage order is by tile, then by cell inside the tile
    from paper_2609_16575_amd import _lib
    T = np.array(_lib.tile_shape(g.desc))
    assert tuple(T) == ((16, 2, 8) if n[1] <= 3 else (8, 8, 4))
    nt = -(-np.array(w.n) // T)
    P, _, _ = g.particles(0)
    c = np.floor(P).astype(int)
    t = c // T
    loc = c - t * T
    key = ((t[:, 0] + nt[0] * (t[:, 1] + nt[1] * t[:, 2])) * T.prod()
           + loc[:, 0] + T[0] * (loc[:, 1] + T[1] * loc[:, 2]))
    assert np.all(np.diff(key) >= 0)


def test_empty_species_and_no_species():
    w = W.Workload("empty", (8, 8, 8), (1.0, 1.0, 1.0), W.courant_dt((1.0, 1.0, 1.0)), (0, 0, 0),
                   [W.SpeciesInit("e", -1.0, 1.0, 1.0, np.zeros((0, 3)), np.zeros((0, 3)))])
    w.E0, w.B0 = W.random_fields(w.n, scale=1.0, seed=4)
    for prec in ("fp32", "fp64"):
        g, o = _sim(w, prec), oracle_from(w, w.E0, w.B0)
        g.step(4)
        o.step(4)
        E, B, J = g.fields()
        assert rel(E, o.E) < 1e-4 and rel(B, o.B) < 1e-4 and np.all(J == 0)
        assert g.count(0) == 0


def test_absorbing_laser_fp32():
    """Reduced laser-wakefield box: Mur faces on all axes, laser sheet, cold
    slab with per-particle weights; one step from a common state, then 40."""
    w = W.lwfa_slab(n=(64, 16, 16), x_start=24, ramp=8, n_plasma=0.05, w0=1.5, tau=2.0)
    w.laser.t0 = 0.0
    w.E0, w.B0 = W.random_fields(w.n, w.bc, scale=0.02, seed=9)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="lwfa 1 step")
    _common_fp32_state(g, o)
    g.step(39)
    o.step(39)
    compare_state(g, o, w, sp_tol=2e-4, f_tol=2e-4, label="lwfa 40 steps")


def test_particles_leave_through_absorbing_faces():
    n = (16, 8, 8)
    pos = np.array([[0.2, 4.0, 4.0], [15.8, 4.0, 4.0], [8.0, 0.1, 4.0], [8.0, 4.0, 7.9],
                    [8.0, 4.0, 4.0]])
    u = np.array([[-3.0, 0, 0], [3.0, 0, 0], [0, -3.0, 0], [0, 0, 3.0], [0.1, 0.1, 0.1]])
    w = W.Workload("leave", n, (1.0, 1.0, 1.0), W.courant_dt((1.0, 1.0, 1.0)), (1, 1, 1),
                   [W.SpeciesInit("e", -1.0, 1.0, 0.1, pos, u)], sort_every=2)
    g, o = _sim(w, "fp32"), oracle_from(w)
    g.step(4)
    o.step(4)
    g.sort()  # removed particles are dropped by the next sort
    assert g.count(0) == 1 and int(o.species[0].alive.sum()) == 1
    compare_state(g, o, w, sp_tol=1e-5, f_tol=1e-4, label="leave")


def test_full_size_thermal_ep_sampled():
    """The thermal e+p benchmark plasma at its full size (128^3, 8 e + 8 p per cell, 33.5M particles),
    in the configuration the benchmark times (adaptive sorting): continuity
    per step from the GPU's FP64 diagnostics, and sampled particles pushed
    one by one by the oracle with the GPU's fields, for both arithmetic
    paths."""
    w = W.thermal_two_species()
    rng = np.random.default_rng(0)
    for prec, tol in (("fp32", 2e-5), ("fp64", 1e-12)):
        g = _sim(w, prec, sort_every=-1)
        g.step(2)
        g.diagnostics()
        E, B, _ = g.fields()
        st = []
        for i in range(2):
            P, U, I = g.particles_by_id(i)
            sel = rng.choice(len(I), 4000, replace=False)
            st.append((P[sel], U[sel], I[sel]))
        g.step(1)
        d = g.diagnostics()
        assert d["cont_valid"] and d["cont_max"] <= 1e-5 * d["rho_max"], d
        assert d["fault_word"] & ~16 == 0
        o = O.OracleSim(w.n, w.d, w.dt)
        o.E[...] = E
        o.B[...] = B
        for i, (P, U, I) in enumerate(st):
            s = w.species[i]
            o.add_species(s.q, s.m, s.w, P, U, ids=I)
        o.step(1)
        for i in range(2):
            Pg, Ug, Ig = g.particles_by_id(i)
            idx = np.searchsorted(Ig, o.species[i].ids)
            assert np.array_equal(Ig[idx], o.species[i].ids)
            assert pos_err_cells(Pg[idx], o.species[i].pos, w) <= tol
            assert rel(Ug[idx], o.species[i].u) <= tol
        # J element by element in boxes of cells
        check_box_currents(g, w, [((10, 20, 30), (18, 28, 38)), ((64, 64, 64), (72, 72, 72)),
                                  ((100, 4, 110), (108, 12, 118))], tol)
        g.close()
