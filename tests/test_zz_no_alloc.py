"""empic_create_static (the library's own per-device workspace, for callers
that cannot allocate device memory) against empic_create with a caller's
workspace: the same runs through the C ABI, two handles in a row on the
static workspace, the second on a smaller grid; the refusals of the call."""
import ctypes as C

import numpy as np
import pytest

from paper_2609_16575_amd import _lib as LB
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 2e-5  # the FP32 step's per-step bar (the step itself is deterministic; the bar is the contract)


def _rel(a, b):
    s = float(np.abs(b).max())
    return float(np.abs(a - b).max()) / (s if s > 0 else 1.0)


def _run(w, static, steps, sort_every):
    from paper_2609_16575_amd.sim import Sim
    g = Sim(w, precision="fp32", sort_every=sort_every, static_workspace=static)
    g.step(steps)
    d = g.diagnostics()
    E, B, J = g.fields()
    parts = [g.particles_by_id(i) for i in range(len(w.species))]
    return g, d, (E, B, J), parts


def _compare(w, steps, sort_every):
    gs, ds, Fs, Ps = _run(w, True, steps, sort_every)
    gs.close()
    gw, dw, Fw, Pw = _run(w, False, steps, sort_every)
    gw.close()
    assert ds["fault_word"] == 0 and dw["fault_word"] == 0
    for a, b in zip(Fs, Fw):
        assert _rel(a, b) <= TOL, _rel(a, b)
    L = np.asarray(w.n) * np.asarray(w.d)
    for (P, U, I), (Q, V, K) in zip(Ps, Pw):
        assert np.array_equal(I, K)
        dx = P - Q
        dx -= L * np.round(dx / L)
        assert float(np.abs(dx).max()) <= TOL, float(np.abs(dx).max())
        assert _rel(U, V) <= TOL, _rel(U, V)
    for k in ("U_E", "U_B", "U_tot"):
        assert abs(ds[k] - dw[k]) <= TOL * max(abs(dw[k]), 1e-300), (k, ds[k], dw[k])


def _desc(n, sort_every, prec=LB.FP32_CELLREL):
    d = LB.GridDesc()
    for a in range(3):
        d.n[a], d.bc[a], d.d[a] = int(n[a]), LB.BC_PERIODIC, 1.0
    d.dt = W.courant_dt((1.0, 1.0, 1.0))
    d.precision = prec
    d.sort_every = sort_every
    return d


def test_static_workspace_matches_caller_workspace_twice():
    import torch
    L = LB.lib()
    # first handle: two species on a 32 x 24 x 16 grid (ragged tiles), random fields
    w = W.thermal_two_species(n=(32, 24, 16), ppc=8, vth=0.05)
    w.E0, w.B0 = W.random_fields(w.n, w.bc, scale=0.05, seed=21)
    print("no-alloc: thermal e+p 32x24x16, 8 steps, sort every 4", flush=True)
    _compare(w, 8, 4)
    # second handle on the same workspace, a smaller grid (one species)
    w2 = W.langmuir_thermal(n=(16, 16, 16), ppc=8, vth=0.05)
    w2.E0, w2.B0 = W.random_fields(w2.n, w2.bc, scale=0.05, seed=22)
    print("no-alloc: langmuir 16^3, 10 steps, sort every 5", flush=True)
    _compare(w2, 10, 5)
    torch.cuda.synchronize()


def test_static_workspace_refusals():
    import torch
    from paper_2609_16575_amd.sim import Sim
    L = LB.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    h = C.c_void_p()
    # more than the static workspace holds
    big = _desc((256, 256, 256), 10)
    assert L.empic_workspace_bytes(C.byref(big), 1, 1 << 24) > LB.STATIC_SCRATCH_BYTES
    assert L.empic_create_static(C.byref(big), 1, 1 << 24, stream, C.byref(h)) == LB.E_CAPACITY
    assert not h.value
    # the adaptive sort needs pinned host memory
    ad = _desc((16, 16, 16), -1)
    assert L.empic_create_static(C.byref(ad), 1, 4096, stream, C.byref(h)) == LB.E_UNSUPPORTED
    # one live handle per device
    w = W.langmuir_thermal(n=(16, 16, 16), ppc=2, vth=0.05)
    g = Sim(w, precision="fp32", sort_every=5, static_workspace=True)
    ok = _desc((16, 16, 16), 5)
    assert L.empic_create_static(C.byref(ok), 1, 4096, stream, C.byref(h)) == LB.E_ARG
    g.close()
    assert L.empic_create_static(C.byref(ok), 1, 4096, stream, C.byref(h)) == LB.OK
    L.empic_destroy(h)
    torch.cuda.synchronize()
