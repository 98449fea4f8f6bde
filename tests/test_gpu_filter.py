"""The current filter (compensated binomial passes) on the GPU, through the
C ABI, against the FP64 oracle: one step of the plain FP64 path (1e-12) and
of the FP32 path from a common state (2e-5), periodic and walled grids, and
the step adjoint with the filter inside the step."""
import numpy as np
import pytest

from gpu_common import compare_state, oracle_from, rel
from oracle import oracle as O
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, prec, **kw):
    from paper_2609_16575_amd.sim import Sim
    return Sim(w, precision=prec, **kw)


def _common_fp32_state(g, o):
    E, B, _ = g.fields()
    o.E[...] = E
    o.B[...] = B
    for i in range(len(o.species)):
        P, U, I = g.particles_by_id(i)
        o.species[i].pos[...] = P
        o.species[i].u[...] = U


@pytest.mark.parametrize("filt", [(1, 1), (2, 0)])
def test_filter_fp64_one_step(filt):
    w = W.langmuir_thermal(n=(16, 16, 16), ppc=4, vth=0.1)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=3)
    w.filter = filt
    g, o = _sim(w, "fp64"), oracle_from(w, w.E0, w.B0)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=1e-12, f_tol=1e-12, label="filter fp64 %s" % (filt,))
    # the filter did act: J differs from an unfiltered step's
    w2 = W.langmuir_thermal(n=(16, 16, 16), ppc=4, vth=0.1)
    w2.E0, w2.B0 = w.E0, w.B0
    o2 = oracle_from(w2, w2.E0, w2.B0)
    o2.step(1)
    assert rel(o.J, o2.J) > 1e-2


@pytest.mark.parametrize("filt", [(1, 1), (3, 1)])
def test_filter_fp32_one_step_and_twenty(filt):
    w = W.thermal_two_species(n=(16, 16, 16), ppc=4)
    w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=5)
    w.filter = filt
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="filter fp32 1")
    g.step(19)
    o.step(19)
    compare_state(g, o, w, sp_tol=2e-4, f_tol=2e-4, label="filter fp32 20")


def test_filter_on_walled_axes_fp32():
    w = W.pec_cavity_plasma()
    w.filter = (1, 1)
    g, o = _sim(w, "fp32"), oracle_from(w, w.E0, w.B0)
    _common_fp32_state(g, o)
    g.step(1)
    o.step(1)
    compare_state(g, o, w, sp_tol=2e-5, f_tol=2e-5, label="filter pec")


def test_step_vjp_with_filter_matches_oracle():
    import torch
    n, d = (8, 8, 8), (1.0, 0.9, 1.1)
    rng = np.random.default_rng(15)
    L = np.asarray(n) * np.asarray(d)
    sp = [W.SpeciesInit("s", -1.0, 1.0, 0.3, rng.random((600, 3)) * L,
                        0.3 * rng.standard_normal((600, 3)))]
    w = W.Workload("vjpf", n, d, W.courant_dt(d), (0, 0, 0), sp, sort_every=0, filter=(1, 1))
    w.E0, w.B0 = W.random_fields(n, scale=0.1, seed=16)
    g = _sim(w, "fp32")
    g.sort()
    st = g.save_state()
    o = O.OracleSim(w.n, w.d, w.dt)
    o.filter = (1, 1)
    E, B, _ = g.fields()
    o.E[...] = E
    o.B[...] = B
    P, U, I = g.particles(0)
    o.add_species(-1.0, 1.0, 0.3, P, U)
    lam = g.alloc_adjoint()
    lamE = rng.standard_normal(o.E.shape).astype(np.float32)
    lamB = rng.standard_normal(o.B.shape).astype(np.float32)
    lam["E"].copy_(torch.from_numpy(lamE))
    lam["B"].copy_(torch.from_numpy(lamB))
    N = len(I)
    x = rng.standard_normal((N, 3)).astype(np.float32)
    u = rng.standard_normal((N, 3)).astype(np.float32)
    lam["pos"][0][:, :N].copy_(torch.from_numpy(x.T.copy()))
    lam["u"][0][:, :N].copy_(torch.from_numpy(u.T.copy()))
    g.step_vjp(st, lam)
    oE, oB, oX, oU = o.step_vjp(lamE.astype(np.float64), lamB.astype(np.float64),
                                [x.astype(np.float64)], [u.astype(np.float64)])
    errs = {"E": rel(lam["E"].double().cpu().numpy(), oE),
            "B": rel(lam["B"].double().cpu().numpy(), oB),
            "x": rel(lam["pos"][0][:, :N].double().cpu().numpy().T, oX[0]),
            "u": rel(lam["u"][0][:, :N].double().cpu().numpy().T, oU[0])}
    for k, v in errs.items():
        assert v <= 1e-4, (k, v, errs)
