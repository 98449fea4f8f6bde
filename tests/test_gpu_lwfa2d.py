"""The two-dimensional laser-wakefield run of Sec. 4 at its full size.

1400 x 2 x 300 cells with the moving window, the paper's a0 = 3 pulse and
its ppc 2 and ppc 8 lattices (1.7M and 6.7M particles, 6767 steps each, a
few seconds on the GPU).  The paper gives no data to compare with element
by element, so the checks are the features it reports: a nonlinear wake
with a depleted first bucket behind the pulse and a density spike at its
back, a peak accelerating field of the order of the cold wave-breaking
field, and results that barely change with the number of particles per
cell.  The peak field is held to this code's own value, 1.44 m c omega_p / e
at ppc 8 and 1.49 at ppc 2, within 10 %, so that a change in the result
shows; the paper quotes about 0.169 TV/m, i.e. 1.01 m c omega_p / e, for a
set-up whose injection, envelope and read-out time it leaves open.  Parity
of the same set-up with the oracle is tested in a reduced box
(test_gpu_window).
"""
PEAK_E0 = {2: 1.49, 8: 1.44}   # this code's peak accelerating field, m c omega_p / e
import numpy as np
import pytest

from paper_2609_16575_amd import _lib as LB

pytestmark = pytest.mark.gpu


def _bins(x, v, lam, width=0.1):
    """(bin start in lambda_p, mean, max) over bins of `width` lambda_p."""
    out = []
    for a in np.arange(0.0, x[-1] / lam, width):
        m = (x / lam >= a) & (x / lam < a + width)
        if m.any():
            out.append((a, float(v[m].mean()), float(v[m].max())))
    return out


def test_lwfa2d_full_size_wake():
    from paper_2609_16575_amd import lwfa2d
    from paper_2609_16575_amd import workloads as W
    res = {}
    for ppc in (2, 8):
        out, prof = lwfa2d.run(ppc=ppc)
        assert out["fault_word"] & ~LB.FAULT_FALLBACK == 0, out
        assert abs(out["particles_end"] / out["particles"] - 1.0) < 0.02, out
        res[ppc] = (out, prof)
    w = W.lwfa_2d(per=(1, 2, 1))
    lam = w.lambda_p
    for ppc, (out, prof) in res.items():
        assert abs(out["peak_accel_field_E0"] / PEAK_E0[ppc] - 1.0) <= 0.1, (ppc, out)
        # the pulse sits in the front third; behind it the first bucket is
        # depleted on axis and ends in a density spike
        x_n = np.arange(prof["ne"].shape[0]) * w.d[0]
        b = _bins(x_n, prof["ne"], lam)
        first = [m for a, m, _ in b if 1.3 <= a < 1.9]
        assert max(first) < 0.6, (ppc, first)
        assert max(mx for a, _, mx in b if 0.8 <= a < 1.3) > 4.0, ppc
        # the accelerating field peaks at the back of that bucket
        assert 0.8 <= out["peak_position_lambda_p"] <= 1.5, out
    p2, p8 = res[2][0]["peak_accel_field_E0"], res[8][0]["peak_accel_field_E0"]
    assert abs(p2 / p8 - 1.0) < 0.1, (p2, p8)
