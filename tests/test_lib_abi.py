"""CPU-only checks of the C-ABI library: it loads, exports every function
declared in include/empic.h, and its host-side validation (CFL bound, grid
limits, argument checks) answers before any device work."""
import ctypes as C
import os
import re

import pytest

from paper_2609_16575_amd import _lib as LB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "empic.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LB.LIB_PATH):
        from paper_2609_16575_amd import build
        build.build()
    return LB.lib()


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(empic_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(LB.SIGNATURES), set(names) ^ set(LB.SIGNATURES)


def _desc(n=(16, 16, 16), d=(1.0, 1.0, 1.0), dt=None, bc=(0, 0, 0), prec=0, sort_every=10):
    g = LB.GridDesc()
    for a in range(3):
        g.n[a], g.d[a], g.bc[a] = n[a], d[a], bc[a]
    g.dt = 0.5 / (sum(1 / x ** 2 for x in d)) ** 0.5 if dt is None else dt
    g.precision = prec
    g.sort_every = sort_every
    return g


def _create(L, g, species=1, cap=64, ws=256):
    h = C.c_void_p()
    st = L.empic_create(C.byref(g), species, cap, None, C.c_void_p(ws), 1 << 40, C.byref(h))
    return st, h


def test_workspace_bytes_scales(L):
    small = L.empic_workspace_bytes(C.byref(_desc()), 1, 1024)
    big = L.empic_workspace_bytes(C.byref(_desc(n=(32, 32, 32))), 1, 1024)
    assert 0 < small < big
    assert L.empic_workspace_bytes(C.byref(_desc(n=(0, 4, 4))), 1, 64) == 0
    assert L.empic_workspace_bytes(C.byref(_desc()), 5, 64) == 0


def test_cfl_rejected(L):
    g = _desc(d=(1.0, 0.5, 2.0))
    limit = 1.0 / (1 + 4 + 0.25) ** 0.5
    g.dt = limit * 1.01
    assert _create(L, g)[0] == 4  # EMPIC_E_CFL


def test_argument_checks(L):
    assert _create(L, _desc(n=(4, 0, 4)))[0] == 1
    assert _create(L, _desc(bc=(1, 0, 0), n=(1, 4, 4)))[0] == 1   # absorbing axis needs n >= 2
    assert _create(L, _desc(prec=2))[0] == 1
    assert _create(L, _desc(sort_every=-2))[0] == 1   # -1 is the adaptive policy
    assert _create(L, _desc(), species=0)[0] == 1
    assert _create(L, _desc(), ws=100)[0] == 1                     # unaligned workspace
    assert _create(L, _desc(n=(2048, 8, 8)))[0] == 7               # packed cell index limit
    assert _create(L, _desc(bc=(1, 0, 0), prec=1))[0] == 7         # FP64 plain is periodic only
    g = _desc()
    h = C.c_void_p()
    small = L.empic_workspace_bytes(C.byref(g), 1, 64)
    assert L.empic_create(C.byref(g), 1, 64, None, C.c_void_p(256), small - 1, C.byref(h)) == 1


def test_null_handle_calls(L):
    assert L.empic_step(None, 1) == 1
    assert L.empic_sync(None) == 1
    assert L.empic_last_error(None) == b"null handle"
    L.empic_destroy(None)


def test_static_create_refusals_before_device_work(L):
    """empic_create_static answers these from the host, before any HIP call."""
    txt = open(HEADER).read()
    m = re.search(r"#define EMPIC_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == LB.STATIC_SCRATCH_BYTES
    h = C.c_void_p()
    big = _desc(n=(256, 256, 256))
    assert L.empic_workspace_bytes(C.byref(big), 1, 1 << 24) > LB.STATIC_SCRATCH_BYTES
    assert L.empic_create_static(C.byref(big), 1, 1 << 24, None, C.byref(h)) == LB.E_CAPACITY
    assert L.empic_create_static(C.byref(_desc(sort_every=-1)), 1, 64, None,
                                 C.byref(h)) == LB.E_UNSUPPORTED
    g = _desc(d=(1.0, 0.5, 2.0))
    g.dt = 1.01 / (1 + 4 + 0.25) ** 0.5
    assert L.empic_create_static(C.byref(g), 1, 64, None, C.byref(h)) == LB.E_CFL
    assert L.empic_create_static(None, 1, 64, None, C.byref(h)) == LB.E_ARG
    assert L.empic_create_static(C.byref(_desc()), 1, 64, None, None) == LB.E_ARG
    assert not h.value
