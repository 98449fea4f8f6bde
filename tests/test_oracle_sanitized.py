"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(a separate build, liboracle_san.so, with -fno-sanitize-recover): a child
process preloads libasan and runs every oracle path once (periodic, Mur +
laser, PEC + port, filter, moving window, the step's adjoint, second-order
shapes, diagnostics).  Any out-of-bounds access or undefined behaviour
aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
from oracle import oracle as O
from paper_2609_16575_amd import workloads as W
sys.path.insert(0, %r)
from gpu_common import oracle_from

def run(w, steps, order=1, vjp=False):
    o = oracle_from(w, w.E0, w.B0, order=order)
    o.step(steps)
    o.diagnostics()
    if vjp:
        lam = [np.ones_like(s.pos) for s in o.species]
        o.step_vjp(np.ones_like(o.E), np.ones_like(o.B), lam, lam)

w = W.thermal_two_species(n=(8, 8, 8), ppc=2, vth=0.3)
w.E0, w.B0 = W.random_fields(w.n, scale=0.05, seed=1)
run(w, 3, vjp=True)
run(w, 3, order=2)
w.filter = (2, 1)
run(w, 2)
run(W.lwfa_2d(per=(1, 1, 1), cells=(64, 2, 24)), 3)
run(W.pec_cavity_plasma(n=(8, 6, 5), ppc=2), 3)
run(W.waveguide_te10(nodes=(6, 4, 24)), 3)
wl = W.lwfa_slab(n=(48, 8, 8), ppc=1, x_start=8, ramp=4)
run(wl, 3)
print("sanitized oracle ok", flush=True)
"""


def test_oracle_under_asan_and_ubsan():
    from oracle import build
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no libasan here")
    lib = build.build(sanitize=True)
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    code = CHILD % (ROOT, os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:],
                                                                    r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
