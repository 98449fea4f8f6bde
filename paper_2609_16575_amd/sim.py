"""Python face of libempic: a simulation whose device memory is torch tensors.

Every step of the PIC cycle runs in the library's HIP kernels; this class
only allocates tensors, passes their pointers and torch's current HIP stream
through the C ABI, and converts results to numpy for inspection.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as LB


def _ptr(t) -> int:
    return t.data_ptr()


def _round_up(x, m):
    return (int(x) + m - 1) // m * m


class Sim:
    """One EM-PIC simulation on one GPU.

    precision: "fp32" (cell-relative FP32, sorted, fused kernel) or "fp64"
    (plain FP64 global positions).  `workload` is a
    paper_2609_16575_amd.workloads.Workload.  static_workspace=True creates
    the handle with empic_create_static (the library's per-device workspace,
    one live handle per device; no device allocation by the library).
    shape_order=2: second-order shapes (b_2 weighting, EZ current).
    """

    def __init__(self, workload, precision: str = "fp32", device: Optional[str] = None,
                 sort_every: Optional[int] = None, capacity_slack: float = 0.0,
                 static_workspace: bool = False, shape_order: int = 1):
        import torch
        self.torch = torch
        self.L = LB.lib()
        self.dev = torch.device(device or "cuda")
        if self.dev.type != "cuda":
            raise ValueError("libempic runs on a GPU device")
        self.w = workload
        self.fp64 = precision == "fp64"
        if precision not in ("fp32", "fp64"):
            raise ValueError(precision)
        self.dtype = torch.float64 if self.fp64 else torch.float32
        n, bc = workload.n, workload.bc
        self.ext = tuple(n[a] + (1 if bc[a] != LB.BC_PERIODIC else 0) for a in range(3))
        shape = (3, self.ext[2], self.ext[1], self.ext[0])
        self.E = torch.zeros(shape, dtype=self.dtype, device=self.dev)
        self.B = torch.zeros(shape, dtype=self.dtype, device=self.dev)
        self.J = torch.zeros(shape, dtype=self.dtype, device=self.dev)
        if workload.E0 is not None:
            self.E.copy_(torch.from_numpy(np.asarray(workload.E0)).to(self.dev, self.dtype))
        if workload.B0 is not None:
            self.B.copy_(torch.from_numpy(np.asarray(workload.B0)).to(self.dev, self.dtype))

        nsp = len(workload.species)
        win = getattr(workload, "window", None)
        extra = [0] * nsp
        if win is not None:
            # room for a full window of injected plasma, a quarter more for plasma
            # compressed by the fields, and one shift in flight (removed
            # particles are compacted by the sort after the injection)
            for sp, per, _w in win.inject:
                ppc = int(np.prod(per))
                full = int(np.prod(n)) * ppc
                m = full // int(n[win.axis]) * int(win.cells)
                extra[sp] = m + max(0, full - workload.species[sp].pos.shape[0]) + full // 4
        self.caps = [_round_up(max(8, int(s.pos.shape[0] * (1.0 + capacity_slack)) + extra[i]), 64)
                     for i, s in enumerate(workload.species)]
        max_cap = max(self.caps) if self.caps else 0
        d = LB.GridDesc()
        for a in range(3):
            d.n[a], d.bc[a], d.d[a] = int(n[a]), int(bc[a]), float(workload.d[a])
        d.dt = float(workload.dt)
        d.precision = LB.FP64_PLAIN if self.fp64 else LB.FP32_CELLREL
        d.sort_every = int(workload.sort_every if sort_every is None else sort_every)
        self.sort_every = d.sort_every
        self.desc = d
        self.stream = torch.cuda.current_stream(self.dev)
        h = C.c_void_p()
        if static_workspace:
            # the library's own per-device workspace (empic_create_static)
            self.ws = None
            with torch.cuda.device(self.dev):
                st = self.L.empic_create_static(C.byref(d), max(nsp, 1), max_cap,
                                                C.c_void_p(self.stream.cuda_stream), C.byref(h))
            if st != 0:
                raise LB.EmpicError(st, "empic_create_static failed")
        else:
            wsb = self.L.empic_workspace_bytes(C.byref(d), max(nsp, 1), max_cap)
            if wsb == 0:
                raise LB.EmpicError(1, "bad grid for the workspace size")
            self.ws = torch.empty(int(wsb), dtype=torch.uint8, device=self.dev)
            st = self.L.empic_create(C.byref(d), max(nsp, 1), max_cap,
                                     C.c_void_p(self.stream.cuda_stream),
                                     C.c_void_p(_ptr(self.ws)), int(wsb), C.byref(h))
            if st != 0:
                raise LB.EmpicError(st, "empic_create failed")
        self.h = h
        arr = C.c_void_p * 3
        LB.check(h, self.L.empic_bind_fields(h, arr(*[_ptr(self.E[a]) for a in range(3)]),
                                             arr(*[_ptr(self.B[a]) for a in range(3)]),
                                             arr(*[_ptr(self.J[a]) for a in range(3)])))
        self.bufs = []
        for i, s in enumerate(workload.species):
            self._add_species(s, self.caps[i])
        LB.check(h, self.L.empic_set_background(h, float(workload.rho_bg)))
        if shape_order != 1:
            LB.check(h, self.L.empic_set_shape_order(h, int(shape_order)))
        if workload.laser is not None:
            Ls = workload.laser
            ld = LB.LaserDesc(Ls.a0, Ls.w0, Ls.tau, Ls.t0, Ls.omega0, Ls.yc, Ls.zc, int(Ls.i_s), 1,
                              int(bool(Ls.slab)), 0)
            LB.check(h, self.L.empic_set_laser(h, C.byref(ld)))
        if getattr(workload, "filter", None):
            LB.check(h, self.L.empic_set_filter(h, int(workload.filter[0]), int(workload.filter[1])))
        if getattr(workload, "port", None) is not None:
            P = workload.port
            pd = LB.PortDesc(1, int(P.axis), int(P.plane), int(P.comp), int(P.prof_axis), 0,
                             float(P.e0), float(P.omega), float(P.tau))
            LB.check(h, self.L.empic_set_port(h, C.byref(pd)))
        if win is not None:
            wd = LB.WindowDesc(1, int(win.axis), int(win.cells), 0, float(win.velocity),
                               float(win.t_start))
            LB.check(h, self.L.empic_set_window(h, C.byref(wd)))
            for sp, per, wi in win.inject:
                LB.check(h, self.L.empic_set_injection(h, int(sp), (C.c_int32 * 3)(*per), float(wi)))
        torch.cuda.synchronize(self.dev)

    # -- set-up -----------------------------------------------------------------
    def _alloc_set(self, cap, wpp):
        t = self.torch
        fd = self.dtype
        cell = t.zeros(cap, dtype=t.int32, device=self.dev)
        pos = t.zeros((3, cap), dtype=fd, device=self.dev)
        u = t.zeros((3, cap), dtype=fd, device=self.dev)
        ids = t.zeros(cap, dtype=t.int32, device=self.dev)
        w = t.zeros(cap, dtype=fd, device=self.dev) if wpp else None
        pb = LB.ParticleBuffers()
        pb.cell = _ptr(cell)
        for a in range(3):
            pb.pos[a] = _ptr(pos[a])
            pb.u[a] = _ptr(u[a])
        pb.id = _ptr(ids)
        pb.w = _ptr(w) if w is not None else None
        return {"cell": cell, "pos": pos, "u": u, "id": ids, "w": w, "pb": pb}

    def _add_species(self, s, cap):
        t = self.torch
        wpp = s.wpp is not None
        b0 = self._alloc_set(cap, wpp)
        b1 = None if self.fp64 else self._alloc_set(cap, wpp)
        sd = LB.SpeciesDesc(float(s.q), float(s.m), float(s.w), 1 if wpp else 0, 0)
        sid = C.c_int32()
        LB.check(self.h, self.L.empic_add_species(self.h, C.byref(sd), cap, C.byref(b0["pb"]),
                                                  C.byref(b1["pb"]) if b1 else None, C.byref(sid)))
        self.bufs.append((b0, b1))
        self.load_particles(sid.value, s.pos, s.u, s.wpp)

    def load_particles(self, sp, pos, u, wpp=None, ids=None):
        t = self.torch
        pos_d = t.from_numpy(np.ascontiguousarray(pos, dtype=np.float64)).to(self.dev)
        u_d = t.from_numpy(np.ascontiguousarray(u, dtype=np.float64)).to(self.dev)
        w_d = None if wpp is None else t.from_numpy(np.ascontiguousarray(wpp, dtype=np.float64)).to(self.dev)
        id_d = None if ids is None else t.from_numpy(np.ascontiguousarray(ids, dtype=np.int32)).to(self.dev)
        LB.check(self.h, self.L.empic_load_particles_f64(
            self.h, sp, int(pos_d.shape[0]), _ptr(pos_d), _ptr(u_d),
            _ptr(w_d) if w_d is not None else None, _ptr(id_d) if id_d is not None else None))
        self.torch.cuda.synchronize(self.dev)

    def set_fields(self, E=None, B=None):
        t = self.torch
        if E is not None:
            self.E.copy_(t.from_numpy(np.asarray(E, dtype=np.float64)).to(self.dev, self.dtype))
        if B is not None:
            self.B.copy_(t.from_numpy(np.asarray(B, dtype=np.float64)).to(self.dev, self.dtype))
        t.cuda.synchronize(self.dev)

    # -- the PIC cycle ------------------------------------------------------------
    def step(self, nsteps: int = 1):
        LB.check(self.h, self.L.empic_step(self.h, int(nsteps)))

    def sort(self):
        LB.check(self.h, self.L.empic_sort(self.h))

    def sync(self):
        LB.check(self.h, self.L.empic_sync(self.h))

    # -- results -------------------------------------------------------------------
    def diagnostics(self) -> dict:
        dg = LB.Diag()
        LB.check(self.h, self.L.empic_diagnostics(self.h, C.byref(dg)))
        nsp = len(self.w.species)
        return {"step": dg.step, "t": dg.t, "U_E": dg.U_E, "U_B": dg.U_B, "U_tot": dg.U_tot,
                "K": list(dg.K)[:nsp], "K_minus": list(dg.K_minus)[:nsp],
                "K_plus": list(dg.K_plus)[:nsp], "gauss_max": dg.gauss_max,
                "gauss_l2": dg.gauss_l2, "cont_max": dg.cont_max, "rho_max": dg.rho_max,
                "cont_valid": bool(dg.cont_valid), "fault_word": dg.fault_word,
                "n_particles": list(dg.n_particles)[:nsp],
                "fallback_particles": dg.fallback_particles}

    def particles(self, sp: int):
        """(positions (N,3) f64, momenta (N,3) f64, ids (N,)) of live particles, storage order."""
        t = self.torch
        cap = self.caps[sp]
        pos = t.empty((cap, 3), dtype=t.float64, device=self.dev)
        u = t.empty((cap, 3), dtype=t.float64, device=self.dev)
        ids = t.empty(cap, dtype=t.int32, device=self.dev)
        cnt = C.c_int64()
        LB.check(self.h, self.L.empic_store_particles_f64(self.h, sp, _ptr(pos), _ptr(u), _ptr(ids),
                                                          C.byref(cnt)))
        n = cnt.value
        P, U, I = pos[:n].cpu().numpy(), u[:n].cpu().numpy(), ids[:n].cpu().numpy()
        keep = I >= 0
        return P[keep], U[keep], I[keep]

    def sample_particles(self, sp: int, ids):
        """(positions, momenta, ids) of the live particles of `sp` whose id is
        in `ids`, sorted by id.  The selection runs on the device, so only the
        sample is copied to the host."""
        t = self.torch
        cap = self.caps[sp]
        pos = t.empty((cap, 3), dtype=t.float64, device=self.dev)
        u = t.empty((cap, 3), dtype=t.float64, device=self.dev)
        idv = t.empty(cap, dtype=t.int32, device=self.dev)
        cnt = C.c_int64()
        LB.check(self.h, self.L.empic_store_particles_f64(self.h, sp, _ptr(pos), _ptr(u), _ptr(idv),
                                                          C.byref(cnt)))
        n = cnt.value
        want = t.as_tensor(np.asarray(ids, dtype=np.int32), device=self.dev)
        m = t.isin(idv[:n], want) & (idv[:n] >= 0)
        I = idv[:n][m]
        order = t.argsort(I)
        return tuple(x.cpu().numpy() for x in (pos[:n][m][order], u[:n][m][order], I[order]))

    def particles_in_box(self, sp: int, lo, hi):
        """(positions, momenta, ids) of the live particles of `sp` whose cell
        coordinate x_a / d_a lies in [lo_a, hi_a) on every axis, sorted by id.
        The selection runs on the device."""
        t = self.torch
        cap = self.caps[sp]
        pos = t.empty((cap, 3), dtype=t.float64, device=self.dev)
        u = t.empty((cap, 3), dtype=t.float64, device=self.dev)
        idv = t.empty(cap, dtype=t.int32, device=self.dev)
        cnt = C.c_int64()
        LB.check(self.h, self.L.empic_store_particles_f64(self.h, sp, _ptr(pos), _ptr(u), _ptr(idv),
                                                          C.byref(cnt)))
        n = cnt.value
        xi = pos[:n] / t.as_tensor(np.asarray(self.w.d, dtype=np.float64), device=self.dev)
        m = idv[:n] >= 0
        for a in range(3):
            m &= (xi[:, a] >= float(lo[a])) & (xi[:, a] < float(hi[a]))
        I = idv[:n][m]
        order = t.argsort(I)
        return tuple(x.cpu().numpy() for x in (pos[:n][m][order], u[:n][m][order], I[order]))

    def particles_by_id(self, sp: int):
        P, U, I = self.particles(sp)
        order = np.argsort(I, kind="stable")
        return P[order], U[order], I[order]

    def fields(self):
        self.torch.cuda.synchronize(self.dev)
        f = lambda x: x.double().cpu().numpy()
        return f(self.E), f(self.B), f(self.J)

    def rho(self, sp: int = -1):
        t = self.torch
        out = t.empty(tuple(reversed(self.ext)), dtype=t.float64, device=self.dev)
        LB.check(self.h, self.L.empic_deposit_rho(self.h, int(sp), _ptr(out)))
        t.cuda.synchronize(self.dev)
        return out.cpu().numpy()

    def count(self, sp: int) -> int:
        n = C.c_int64()
        LB.check(self.h, self.L.empic_particle_count(self.h, sp, C.byref(n)))
        return n.value

    # -- differentiable runs (FP32 path, periodic grid) ----------------------------
    def alloc_state(self, particle_record=True):
        """Device tensors for one saved state (fields + the full particle record).
        particle_record=False leaves out ids and weights (for states that borrow
        another state's, which no step changes)."""
        t = self.torch
        if not hasattr(self, "_tile_words"):
            n = C.c_int64()
            LB.check(self.h, self.L.empic_state_tile_words(self.h, C.byref(n)))
            self._tile_words = n.value
        st = {"E": t.empty_like(self.E), "B": t.empty_like(self.B), "cell": [], "pos": [], "u": [],
              "id": [], "w": [], "tiles": []}
        for i, cap in enumerate(self.caps):
            st["cell"].append(t.empty(cap, dtype=t.int32, device=self.dev))
            st["pos"].append(t.empty((3, cap), dtype=self.dtype, device=self.dev))
            st["u"].append(t.empty((3, cap), dtype=self.dtype, device=self.dev))
            has_w = self.bufs[i][0]["w"] is not None
            rec = particle_record
            st["id"].append(t.empty(cap, dtype=t.int32, device=self.dev) if rec else None)
            st["w"].append(t.empty(cap, dtype=self.dtype, device=self.dev) if has_w and rec else None)
            st["tiles"].append(t.empty(self._tile_words, dtype=t.int32, device=self.dev))
        return st

    def alloc_adjoint(self):
        t = self.torch
        lam = {"E": t.zeros_like(self.E), "B": t.zeros_like(self.B), "pos": [], "u": []}
        for cap in self.caps:
            lam["pos"].append(t.zeros((3, cap), dtype=self.dtype, device=self.dev))
            lam["u"].append(t.zeros((3, cap), dtype=self.dtype, device=self.dev))
        return lam

    def _state_struct(self, st):
        S = LB.State()
        for a in range(3):
            S.E[a] = _ptr(st["E"][a])
            S.B[a] = _ptr(st["B"][a])
        for i in range(len(self.caps)):
            S.cell[i] = _ptr(st["cell"][i])
            S.id[i] = _ptr(st["id"][i]) if st["id"][i] is not None else None
            S.w[i] = _ptr(st["w"][i]) if st["w"][i] is not None else None
            S.tiles[i] = _ptr(st["tiles"][i])
            for a in range(3):
                S.pos[i][a] = _ptr(st["pos"][i][a])
                S.u[i][a] = _ptr(st["u"][i][a])
        return S

    def _adjoint_struct(self, lam):
        A = LB.Adjoint()
        for a in range(3):
            A.E[a] = _ptr(lam["E"][a])
            A.B[a] = _ptr(lam["B"][a])
        for i in range(len(self.caps)):
            for a in range(3):
                A.pos[i][a] = _ptr(lam["pos"][i][a])
                A.u[i][a] = _ptr(lam["u"][i][a])
        return A

    def save_state(self, st=None):
        st = self.alloc_state() if st is None else st
        S = self._state_struct(st)
        LB.check(self.h, self.L.empic_save_state(self.h, C.byref(S)))
        return st

    def load_state(self, st):
        S = self._state_struct(st)
        LB.check(self.h, self.L.empic_load_state(self.h, C.byref(S)))

    def step_state(self, src, dst):
        """One step from state src into state dst (the Sim's particle buffers untouched)."""
        S, D = self._state_struct(src), self._state_struct(dst)
        LB.check(self.h, self.L.empic_step_state(self.h, C.byref(S), C.byref(D)))

    def step_vjp(self, st, lam):
        """In place: lam (adjoint after the step taken from st) -> adjoint of st."""
        S, A = self._state_struct(st), self._adjoint_struct(lam)
        LB.check(self.h, self.L.empic_step_vjp(self.h, C.byref(S), C.byref(A)))

    def dot_f64(self, a, b):
        """FP64 sum of a * b over two FP32 device tensors of equal size (fixed order)."""
        t = self.torch
        if a.dtype != t.float32 or b.dtype != t.float32 or a.numel() != b.numel():
            raise ValueError("dot_f64 takes two float32 tensors of the same size")
        dev = self.E.device
        if not (a.is_contiguous() and b.is_contiguous()) or a.device != dev or b.device != dev:
            raise ValueError("dot_f64 takes contiguous tensors on the Sim's device")
        out = C.c_double()
        LB.check(self.h, self.L.empic_dot_f64(self.h, _ptr(a), _ptr(b), a.numel(), C.byref(out)))
        return out.value

    def alloc_perm(self):
        """One int32 permutation array per species, for sort_recorded."""
        t = self.torch
        return [t.empty(cap, dtype=t.int32, device=self.dev) for cap in self.caps]

    def _perm_array(self, perm):
        P = (C.c_void_p * LB.MAX_SPECIES)()
        for i, p in enumerate(perm):
            P[i] = _ptr(p)
        return P

    def sort_recorded(self, perm):
        """Sort now; perm[i][j] = slot before the sort of what is in slot j."""
        LB.check(self.h, self.L.empic_sort_recorded(self.h, self._perm_array(perm)))

    def sort_vjp(self, perm, lam):
        """In place: particle adjoints after a recorded sort -> before it."""
        A = self._adjoint_struct(lam)
        LB.check(self.h, self.L.empic_sort_vjp(self.h, self._perm_array(perm), C.byref(A)))

    def current_buffers(self, sp):
        """Tensors of species sp's current buffer set (storage order)."""
        w = C.c_int32()
        LB.check(self.h, self.L.empic_current_buffer(self.h, sp, C.byref(w)))
        return self.bufs[sp][w.value]

    def enable_timing(self, on=True, push_only=False):
        """HIP-event timing of the kernels (push_only: the particle kernel
        alone, with no event markers between the other kernels)."""
        mode = (2 if push_only else 1) if on else 0
        LB.check(self.h, self.L.empic_enable_timing(self.h, mode))

    def kernel_times(self):
        v = [C.c_double(), C.c_int64(), C.c_double(), C.c_int64(), C.c_double(), C.c_int64()]
        LB.check(self.h, self.L.empic_kernel_times(self.h, *[C.byref(x) for x in v]))
        return {"push_ms": v[0].value, "push_n": v[1].value, "field_ms": v[2].value,
                "field_n": v[3].value, "sort_ms": v[4].value, "sort_n": v[5].value}

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize(self.dev)
            self.L.empic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
