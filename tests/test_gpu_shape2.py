"""Second-order shapes on the GPU (b_2 weighting, EZ current: the
shape-function equation of Sec. 2.4 with l = 1 and the EZ deposit of Sec.
2.5) against the FP64 oracle's second-order step, through the C ABI.

Tolerances as for the first-order FP32 step: 2e-5 relative after one step
from a common state, 2e-4 after ten more; continuity of the b_2 charge to
1e-5 max|rho| every step."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import check_box_currents, compare_state, oracle_from, pos_err_cells, rel
from oracle import oracle as O
from paper_2609_16575_amd import _lib as LB
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, **kw):
    from paper_2609_16575_amd.sim import Sim
    return Sim(w, precision="fp32", shape_order=2, **kw)


def _common(g, o):
    E, B, _ = g.fields()
    o.E[...] = E
    o.B[...] = B
    for i in range(len(o.species)):
        P, U, _ = g.particles_by_id(i)
        o.species[i].pos[...] = P
        o.species[i].u[...] = U


def test_order2_one_step_two_species():
    w = W.thermal_two_species(n=(16, 16, 16), ppc=8, vth=0.05)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=51)
    g, o = _sim(w), oracle_from(w, w.E0, w.B0, order=2)
    _common(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="order 2, 1 step")


def test_order2_dense_tiles_and_continuity():
    """20 + 20 per cell on 16^3 (three batches of 2048 per species and tile):
    one step from a common state, then ten more with the continuity of the
    b_2 charge checked every step, then against the oracle again."""
    w = W.thermal_two_species(n=(16, 16, 16), ppc=20, vth=0.05)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=52)
    g, o = _sim(w, sort_every=5), oracle_from(w, w.E0, w.B0, order=2)
    _common(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="order 2 dense, 1 step")
    g.diagnostics()
    for _ in range(10):
        g.step(1)
        d = g.diagnostics()
        assert d["cont_valid"] and d["cont_max"] <= 1e-5 * d["rho_max"], d
        assert d["fault_word"] & ~16 == 0, d
    o.step(10)
    compare_state(g, o, w, sp_tol=2e-4, f_tol=2e-4, label="order 2 dense, 11 steps")


def test_order2_particles_outside_their_tile():
    """No re-sort and a hot plasma: particles leave their tiles and take the
    global path (b_2 gather and EZ current from global memory)."""
    w = W.langmuir_thermal(n=(16, 16, 16), ppc=4, vth=1.5)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.02, seed=53)
    g, o = _sim(w, sort_every=0), oracle_from(w, w.E0, w.B0, order=2)
    _common(g, o)
    for k in range(8):
        g.step(1)
        o.step(1)
        if k >= 3:
            compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="order 2 global %d" % k)
        _common(g, o)
    d = g.diagnostics()
    assert d["fallback_particles"] > 0 and d["fault_word"] & 16


def test_order2_gauss_drift_and_determinism():
    w = W.langmuir_thermal(n=(16, 16, 16), ppc=8, vth=0.1)
    g = _sim(w, sort_every=10)
    o = oracle_from(w, order=2)
    E, _, _ = g.fields()
    rho0 = g.rho()
    r0 = o.div(E) - rho0 - w.rho_bg
    g.step(30)
    E1, B1, J1 = g.fields()
    rho1 = g.rho()
    r1 = o.div(E1) - rho1 - w.rho_bg
    assert np.max(np.abs(r1 - r0)) <= 2e-5 * np.max(np.abs(rho1))
    # the b_2 charge: oracle's rho_2 of the GPU's particles
    P, U, I = g.particles_by_id(0)
    o.species[0].pos[...] = P
    assert rel(rho1, o.rho()) < 1e-6
    g.close()
    g2 = _sim(w, sort_every=10)
    g2.step(30)
    E2, B2, J2 = g2.fields()
    assert np.array_equal(E1, E2) and np.array_equal(B1, B2) and np.array_equal(J1, J2)
    g2.close()


def test_order2_refusals():
    from paper_2609_16575_amd.sim import Sim
    w = W.langmuir_thermal(n=(8, 8, 8), ppc=2)
    g = Sim(w, precision="fp32")
    assert g.L.empic_set_shape_order(g.h, 3) == LB.E_ARG
    assert g.L.empic_set_shape_order(g.h, 2) == LB.OK
    assert g.L.empic_set_shape_order(g.h, 1) == LB.OK
    g.close()
    g = Sim(w, precision="fp64")
    assert g.L.empic_set_shape_order(g.h, 2) == LB.E_UNSUPPORTED
    g.close()
    wa = W.langmuir_thermal(n=(8, 8, 8), ppc=2)
    wa.bc = (LB.BC_ABSORBING, 0, 0)
    g = Sim(wa, precision="fp32")
    assert g.L.empic_set_shape_order(g.h, 2) == LB.E_UNSUPPORTED
    g.close()


def test_order2_full_size_thermal_sampled():
    """The thermal e+p benchmark plasma at full size (128^3, 33.5M
    particles) with second-order shapes: continuity every step, sampled
    particles pushed one by one by the oracle, J element by element in
    boxes."""
    w = W.thermal_two_species()
    rng = np.random.default_rng(5)
    g = _sim(w, sort_every=-1)
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
    o.shape_order = 2
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
        assert pos_err_cells(Pg[idx], o.species[i].pos, w) <= 2e-5
        assert rel(Ug[idx], o.species[i].u) <= 2e-5
    check_box_currents(g, w, [((10, 20, 30), (18, 28, 38)), ((64, 64, 64), (72, 72, 72))], 2e-5,
                       margin=3, order=2)
    g.close()
