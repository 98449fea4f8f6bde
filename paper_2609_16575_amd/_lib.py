"""ctypes declarations of libempic (include/empic.h).

Argument marshalling only.  If libempic.so has not been built this raises;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libempic.so")

MAX_SPECIES = 4
BC_PERIODIC, BC_ABSORBING, BC_PEC = 0, 1, 2
FP32_CELLREL, FP64_PLAIN = 0, 1

STATUS = {0: "EMPIC_OK", 1: "EMPIC_E_ARG", 2: "EMPIC_E_STATE", 3: "EMPIC_E_HIP", 4: "EMPIC_E_CFL",
          5: "EMPIC_E_CAPACITY", 6: "EMPIC_E_NONFINITE", 7: "EMPIC_E_UNSUPPORTED"}
OK, E_ARG, E_STATE, E_HIP, E_CFL, E_CAPACITY, E_NONFINITE, E_UNSUPPORTED = range(8)
STATIC_SCRATCH_BYTES = 64 << 20  # EMPIC_STATIC_SCRATCH_BYTES
FAULT_NONFINITE, FAULT_FAST, FAULT_OFFSET, FAULT_CELL, FAULT_FALLBACK = 1, 2, 4, 8, 16


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("bc", C.c_int32 * 3), ("d", C.c_double * 3),
                ("dt", C.c_double), ("precision", C.c_int32), ("sort_every", C.c_int32)]


class SpeciesDesc(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double),
                ("per_particle_w", C.c_int32), ("pad", C.c_int32)]


class ParticleBuffers(C.Structure):
    _fields_ = [("cell", C.c_void_p), ("pos", C.c_void_p * 3), ("u", C.c_void_p * 3),
                ("id", C.c_void_p), ("w", C.c_void_p)]


class LaserDesc(C.Structure):
    _fields_ = [("a0", C.c_double), ("w0", C.c_double), ("tau", C.c_double), ("t0", C.c_double),
                ("omega0", C.c_double), ("yc", C.c_double), ("zc", C.c_double),
                ("i_s", C.c_int32), ("enabled", C.c_int32), ("slab", C.c_int32),
                ("pad", C.c_int32)]


class PortDesc(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("axis", C.c_int32), ("plane", C.c_int32),
                ("comp", C.c_int32), ("prof_axis", C.c_int32), ("pad", C.c_int32),
                ("e0", C.c_double), ("omega", C.c_double), ("tau", C.c_double)]


class WindowDesc(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("axis", C.c_int32), ("cells", C.c_int32),
                ("pad", C.c_int32), ("velocity", C.c_double), ("t_start", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("U_E", C.c_double), ("U_B", C.c_double),
                ("U_tot", C.c_double), ("K", C.c_double * MAX_SPECIES),
                ("K_minus", C.c_double * MAX_SPECIES), ("K_plus", C.c_double * MAX_SPECIES),
                ("gauss_max", C.c_double), ("gauss_l2", C.c_double), ("cont_max", C.c_double),
                ("rho_max", C.c_double), ("cont_valid", C.c_int32), ("fault_word", C.c_uint32),
                ("n_particles", C.c_int64 * MAX_SPECIES), ("fallback_particles", C.c_int64)]


class State(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("cell", C.c_void_p * MAX_SPECIES),
                ("pos", (C.c_void_p * 3) * MAX_SPECIES), ("u", (C.c_void_p * 3) * MAX_SPECIES),
                ("id", C.c_void_p * MAX_SPECIES), ("w", C.c_void_p * MAX_SPECIES),
                ("tiles", C.c_void_p * MAX_SPECIES)]


class Adjoint(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3),
                ("pos", (C.c_void_p * 3) * MAX_SPECIES), ("u", (C.c_void_p * 3) * MAX_SPECIES)]


class EmpicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


# name -> (restype, argtypes)
_P = C.c_void_p
SIGNATURES = {
    "empic_workspace_bytes": (C.c_size_t, [C.POINTER(GridDesc), C.c_int32, C.c_int64]),
    "empic_create": (C.c_int, [C.POINTER(GridDesc), C.c_int32, C.c_int64, _P, _P, C.c_size_t,
                               C.POINTER(_P)]),
    "empic_create_static": (C.c_int, [C.POINTER(GridDesc), C.c_int32, C.c_int64, _P,
                                      C.POINTER(_P)]),
    "empic_bind_fields": (C.c_int, [_P, _P * 3, _P * 3, _P * 3]),
    "empic_set_shape_order": (C.c_int, [_P, C.c_int32]),
    "empic_add_species": (C.c_int, [_P, C.POINTER(SpeciesDesc), C.c_int64,
                                    C.POINTER(ParticleBuffers), C.POINTER(ParticleBuffers),
                                    C.POINTER(C.c_int32)]),
    "empic_load_particles_f64": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, _P, _P]),
    "empic_store_particles_f64": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.POINTER(C.c_int64)]),
    "empic_current_buffer": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "empic_set_background": (C.c_int, [_P, C.c_double]),
    "empic_set_laser": (C.c_int, [_P, C.POINTER(LaserDesc)]),
    "empic_set_port": (C.c_int, [_P, C.POINTER(PortDesc)]),
    "empic_set_filter": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "empic_set_window": (C.c_int, [_P, C.POINTER(WindowDesc)]),
    "empic_set_injection": (C.c_int, [_P, C.c_int32, C.c_int32 * 3, C.c_double]),
    "empic_step": (C.c_int, [_P, C.c_int32]),
    "empic_sort": (C.c_int, [_P]),
    "empic_deposit_rho": (C.c_int, [_P, C.c_int32, _P]),
    "empic_diagnostics": (C.c_int, [_P, C.POINTER(Diag)]),
    "empic_particle_count": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64)]),
    "empic_sync": (C.c_int, [_P]),
    "empic_enable_timing": (C.c_int, [_P, C.c_int32]),
    "empic_kernel_times": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "empic_save_state": (C.c_int, [_P, C.POINTER(State)]),
    "empic_load_state": (C.c_int, [_P, C.POINTER(State)]),
    "empic_step_vjp": (C.c_int, [_P, C.POINTER(State), C.POINTER(Adjoint)]),
    "empic_state_tile_words": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "empic_step_state": (C.c_int, [_P, C.POINTER(State), C.POINTER(State)]),
    "empic_dot_f64": (C.c_int, [_P, _P, _P, C.c_int64, C.POINTER(C.c_double)]),
    "empic_sort_recorded": (C.c_int, [_P, C.c_void_p * MAX_SPECIES]),
    "empic_sort_vjp": (C.c_int, [_P, C.c_void_p * MAX_SPECIES, C.POINTER(Adjoint)]),
    "empic_tile_shape": (None, [C.POINTER(C.c_int32)]),
    "empic_grid_tile_shape": (None, [C.POINTER(GridDesc), C.POINTER(C.c_int32)]),
    "empic_last_error": (C.c_char_p, [_P]),
    "empic_destroy": (None, [_P]),
}

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libempic.so is not built (run __graft_entry__.build() or "
                          "python paper_2609_16575_amd/build.py); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def tile_shape(grid=None):
    """Tile shape of the FP32 path: of three-dimensional grids, or the one
    the grid descriptor `grid` gets."""
    out = (C.c_int32 * 3)()
    if grid is None:
        lib().empic_tile_shape(out)
    else:
        lib().empic_grid_tile_shape(C.byref(grid), out)
    return tuple(out)


def check(handle, status):
    if status != 0:
        msg = lib().empic_last_error(handle) if handle else b""
        raise EmpicError(status, (msg or b"").decode())
    return status
