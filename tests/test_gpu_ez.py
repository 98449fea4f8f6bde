"""The GPU's current against the oracle's EZ current (Esirkepov's
decomposition on each ZigZag segment, the scheme the paper names beside
ZigZag in Sec. 2.5).  At first order the two are the same current, so one
step of free streaming (E = B = 0) must give the EZ current of the moves to
the FP32 bar.  The EZ code is oracle/esirkepov.py: numpy, independent of
the step's deposit (pinned in tests/test_oracle_ez.py)."""
import numpy as np
import pytest

from oracle import esirkepov as EZ
from paper_2609_16575_amd import workloads as W

from gpu_common import rel

pytestmark = pytest.mark.gpu


def test_gpu_current_is_the_ez_current():
    from paper_2609_16575_amd.sim import Sim
    w = W.langmuir_thermal(n=(16, 16, 16), ppc=2, vth=0.3, amp=0.0)
    w.rho_bg = 0.0
    g = Sim(w, precision="fp32")
    P0, U0, I0 = g.particles_by_id(0)
    g.step(1)
    _, _, J = g.fields()
    P1, U1, I1 = g.particles_by_id(0)
    assert np.array_equal(I0, I1) and np.array_equal(U0, U1)  # no fields: no push
    d = np.asarray(w.d)
    L = np.asarray(w.n) * d
    xi0 = P0 / d
    step = P1 - P0
    step -= L * np.round(step / L)  # minimal image across the periodic seams
    xi1 = xi0 + step / d
    assert np.sum(np.floor(xi0) != np.floor(xi1)) > 300  # crossings exercised
    q = w.species[0].q * w.species[0].w
    Jez = np.zeros(J.shape)
    for p in range(len(xi0)):
        EZ.ez(w.n, w.d, w.dt, xi0[p], xi1[p], q, Jez)
    assert rel(J, Jez) <= 2e-5, rel(J, Jez)
