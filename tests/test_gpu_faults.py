"""Failure detection through the C ABI: the kernels' fault word surfaces as
a status at empic_sync (and empic_diagnostics).

A non-finite momentum gives EMPIC_E_NONFINITE, an in-cell offset outside
[0, 1) EMPIC_E_STATE.  Both are ordinary values for the kernels: a NaN
momentum makes every comparison of the move false, so the cell step is 0 and
every window and array index stays what the cell index gives; an offset of
1.0 selects the upper interpolation corner and a step of at most one cell.
The handle is destroyed afterwards.  Also: a state-to-state step leaves the
handle's clock alone and refuses time-dependent sources.
"""
import numpy as np
import pytest

from paper_2609_16575_amd import _lib as LB
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, prec="fp32", **kw):
    from paper_2609_16575_amd.sim import Sim
    return Sim(w, precision=prec, **kw)


def _plasma():
    return W.thermal_two_species(n=(16, 16, 16), ppc=2, vth=0.05)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_nan_momentum_loaded_raises_nonfinite(prec):
    w = _plasma()
    w.species[0].u[17, 1] = np.nan
    g = _sim(w, prec)
    g.step(1)
    with pytest.raises(LB.EmpicError) as e:
        g.sync()
    assert e.value.status == 6, e.value  # EMPIC_E_NONFINITE
    g.close()


def test_nan_written_into_momentum_buffer_raises_nonfinite():
    g = _sim(_plasma())
    g.sort()
    g.step(1)
    g.sync()
    u = g.current_buffers(1)["u"]
    u[2, 33] = float("nan")
    g.step(1)
    with pytest.raises(LB.EmpicError) as e:
        g.sync()
    assert e.value.status == 6, e.value
    g.close()


def test_offset_of_one_in_a_loaded_state_raises_state():
    g = _sim(_plasma(), sort_every=0)
    g.sort()
    g.step(2)
    g.sync()
    st = g.save_state()
    N = int(st["tiles"][0][-1].item())
    assert N > 100
    st["pos"][0][0, N // 2] = 1.0
    g.load_state(st)
    g.step(1)
    with pytest.raises(LB.EmpicError) as e:
        g.sync()
    assert e.value.status == 2, e.value  # EMPIC_E_STATE
    assert "fault word" in str(e.value)
    g.close()


def test_clean_run_has_no_fault():
    g = _sim(_plasma())
    g.step(5)
    d = g.diagnostics()
    assert d["fault_word"] & ~16 == 0, d
    g.sync()
    g.close()


def test_step_state_leaves_the_clock_alone():
    g = _sim(_plasma(), sort_every=0)
    g.sort()
    g.step(3)
    st = g.save_state()
    d0 = g.diagnostics()
    a, b = g.save_state(), g.alloc_state()
    g.step_state(a, b)
    g.step_state(b, a)
    g.load_state(st)
    d1 = g.diagnostics()
    assert d1["step"] == d0["step"] == 3 and d1["t"] == d0["t"], (d0["step"], d1["step"])
    g.close()


def test_step_state_refuses_a_laser():
    w = W.lwfa_slab(n=(64, 16, 16), x_start=40, ramp=8)
    g = _sim(w, sort_every=0)
    g.sort()
    a, b = g.save_state(), g.alloc_state()
    with pytest.raises(LB.EmpicError) as e:
        g.step_state(a, b)
    assert e.value.status == 7, e.value  # EMPIC_E_UNSUPPORTED
    g.close()
