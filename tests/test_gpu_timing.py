"""Kernel timing modes of the library (HIP events on the handle's stream),
through the C ABI: mode 1 times every kernel group, mode 2 only the particle
kernel (events attached to its own dispatch), 0 none; other modes are
refused and leave the handle usable."""
import pytest

from paper_2609_16575_amd import _lib as LB
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_timing_modes(prec):
    from paper_2609_16575_amd.sim import Sim
    w = W.thermal_two_species(n=(16, 16, 16), ppc=2)
    g = Sim(w, precision=prec, **({"sort_every": 0} if prec == "fp32" else {}))
    g.step(2)
    g.kernel_times()  # nothing recorded while off
    g.enable_timing(True)
    g.step(3)
    kt = g.kernel_times()
    # one timed particle entry per step (the fused kernel; the species' FP64
    # kernels under one event pair), two field groups per step
    assert kt["push_n"] == 3, kt
    assert kt["field_n"] == 6 and kt["push_ms"] > 0 and kt["field_ms"] > 0, kt
    g.enable_timing(True, push_only=True)
    g.step(4)
    kt = g.kernel_times()
    assert kt["push_n"] == 4 and kt["push_ms"] > 0, kt
    assert kt["field_n"] == 0 and kt["sort_n"] == 0, kt
    g.enable_timing(False)
    g.step(1)
    kt = g.kernel_times()
    assert kt["push_n"] == 0 and kt["field_n"] == 0, kt
    for bad in (-1, 3):
        assert g.L.empic_enable_timing(g.h, bad) == 1  # EMPIC_E_ARG
    g.step(1)
    d = g.diagnostics()
    assert d["fault_word"] & ~LB.FAULT_FALLBACK == 0, d["fault_word"]
    g.close()
