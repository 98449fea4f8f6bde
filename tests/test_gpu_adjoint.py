"""GPU adjoint of the FP32 step (through the C ABI) against the FP64 oracle's
adjoint and against central finite differences of the FP64 forward.

Targets: one-step VJP within 1e-4 (relative, FP32 against FP64); gradients
of the probe energy of the differentiable workload (32^3, 16 per cell, 500
steps, checkpoints every 50) within 1e-4 of central differences (h = 1e-4)
with respect to the perturbation amplitude eps and along a random direction
in the space of all initial momenta; the same for a hot plasma with sorts at
the checkpoints, where the step sizes are kept below the loss's jumps.
"""
import json
import os

import numpy as np
import pytest

from gpu_common import rel
from oracle import oracle as O
from paper_2609_16575_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, prec="fp32", **kw):
    from paper_2609_16575_amd.sim import Sim
    return Sim(w, precision=prec, **kw)


def _storage_state(g, w):
    """Oracle with the GPU's (FP32-rounded) state, particles in storage order."""
    o = O.OracleSim(w.n, w.d, w.dt)
    E, B, _ = g.fields()
    o.E[...] = E
    o.B[...] = B
    ids = []
    for i, s in enumerate(w.species):
        P, U, I = g.particles(i)
        o.add_species(s.q, s.m, s.w, P, U)
        ids.append(I)
    return o, ids


def test_state_roundtrip_is_exact():
    w = W.thermal_two_species(n=(8, 8, 8), ppc=4)
    g = _sim(w, sort_every=0)
    g.sort()
    g.step(2)
    st = g.save_state()
    E0, B0, _ = g.fields()
    parts0 = [g.particles(i) for i in range(2)]
    g.step(3)
    g.sort()
    g.step(2)
    g.load_state(st)
    E1, B1, _ = g.fields()
    assert np.array_equal(E0, E1) and np.array_equal(B0, B1)
    for i in range(2):
        P0, U0, I0 = parts0[i]
        P1, U1, I1 = g.particles(i)
        assert np.array_equal(P0, P1) and np.array_equal(U0, U1) and np.array_equal(I0, I1)
    # the reloaded state steps on (its tile offsets came back with it)
    g.step(2)
    d = g.diagnostics()
    assert d["fault_word"] == 0 and np.isfinite(d["U_tot"])


def test_sort_vjp_moves_adjoints_back():
    import torch
    w = W.weibel_bimaxwellian(n=(16, 16, 16), ppc=4, steps=8, sort_every=0)
    g = _sim(w, sort_every=0)
    g.sort()
    g.step(8)  # particles leave their cells
    _, _, I0 = g.particles(0)
    perm = g.alloc_perm()
    g.sort_recorded(perm)
    _, _, I1 = g.particles(0)
    N, cap = len(I1), g.caps[0]
    p = perm[0].cpu().numpy()
    assert len(I0) == N and np.all(p[N:] == -1)
    assert np.array_equal(np.sort(p[:N]), np.arange(N))
    assert np.array_equal(I1, I0[p[:N]])
    assert not np.array_equal(p[:N], np.arange(N))  # the sort did move particles
    lam = g.alloc_adjoint()
    rng = np.random.default_rng(11)
    post = rng.standard_normal((6, cap)).astype(np.float32)
    lam["pos"][0].copy_(torch.from_numpy(post[:3].copy()))
    lam["u"][0].copy_(torch.from_numpy(post[3:].copy()))
    g.sort_vjp(perm, lam)
    pre = np.concatenate([lam["pos"][0].cpu().numpy(), lam["u"][0].cpu().numpy()])
    expect = np.zeros_like(post)
    expect[:, p[:N]] = post[:, :N]
    assert np.array_equal(pre, expect)


@pytest.mark.parametrize("drift_steps,n", [(0, (16, 16, 8)), (25, (16, 16, 8)), (0, (40, 2, 16)),
                                           (25, (40, 2, 16)), (0, (15, 9, 7)), (25, (15, 9, 7))])
def test_one_step_vjp_matches_oracle(drift_steps, n):
    """One-step VJP against the oracle's; with drift_steps unsorted steps
    first, some particles are outside their tile window and take the
    global-memory path.  The 40 x 2 x 16 grid gets the 16 x 2 x 8 tiles;
    15 x 9 x 7 has ragged tiles on every axis and an odd number of points
    (the accumulators are cleared float by float)."""
    import torch
    d = (1.0, 0.9, 1.1)
    rng = np.random.default_rng(5)
    L = np.asarray(n) * np.asarray(d)
    sp = []
    for q, m in ((-1.0, 1.0), (1.0, 5.0)):
        pos = rng.random((700, 3)) * L
        sp.append(W.SpeciesInit("s", q, m, 0.3, pos, 0.3 * rng.standard_normal((700, 3))))
    w = W.Workload("vjp", n, d, W.courant_dt(d), (0, 0, 0), sp, sort_every=0)
    w.E0, w.B0 = W.random_fields(n, scale=0.1, seed=6)
    g = _sim(w)
    g.sort()
    if drift_steps:
        g.step(drift_steps)
        assert g.diagnostics()["fallback_particles"] > 0
    st = g.save_state()
    o, ids = _storage_state(g, w)
    lam = g.alloc_adjoint()
    lamE = rng.standard_normal(o.E.shape).astype(np.float32)
    lamB = rng.standard_normal(o.B.shape).astype(np.float32)
    lam["E"].copy_(torch.from_numpy(lamE))
    lam["B"].copy_(torch.from_numpy(lamB))
    lX, lU = [], []
    for i in range(2):
        N = len(ids[i])
        x = rng.standard_normal((N, 3)).astype(np.float32)
        u = rng.standard_normal((N, 3)).astype(np.float32)
        lam["pos"][i][:, :N].copy_(torch.from_numpy(x.T.copy()))
        lam["u"][i][:, :N].copy_(torch.from_numpy(u.T.copy()))
        lX.append(x.astype(np.float64))
        lU.append(u.astype(np.float64))
    g.step_vjp(st, lam)
    oE, oB, oX, oU = o.step_vjp(lamE.astype(np.float64), lamB.astype(np.float64), lX, lU)
    errs = {"E": rel(lam["E"].double().cpu().numpy(), oE), "B": rel(lam["B"].double().cpu().numpy(), oB)}
    for i in range(2):
        N = len(ids[i])
        errs["x%d" % i] = rel(lam["pos"][i][:, :N].double().cpu().numpy().T, oX[i])
        errs["u%d" % i] = rel(lam["u"][i][:, :N].double().cpu().numpy().T, oU[i])
    for k, v in errs.items():
        assert v <= 1e-4, (k, v, errs)


PROBE = (12, 20)


def _probe_mask(shape, lo, hi):
    m = np.zeros(shape[1:], bool)
    m[lo:hi, lo:hi, lo:hi] = True
    return m


def _adjoint_gradients(w, steps, K, eps, dirU=None, probe=None):
    """FP32 forward + checkpointed adjoint: (L, dL/deps, <dL/dU0, dirU>)."""
    import torch
    from paper_2609_16575_amd import autograd as AG
    g = _sim(w, sort_every=0)
    g.sort()
    P, _, I = g.particles(0)
    cap = g.caps[0]
    N = len(I)
    S = np.zeros((3, cap), np.float32)
    S[0, :N] = np.sin(2 * np.pi * P[:, 0] / (w.n[0] * w.d[0]))
    Sd = torch.from_numpy(S).to(g.dev)
    e = torch.tensor(eps, dtype=torch.float32, device=g.dev, requires_grad=True)
    dU = torch.zeros((3, cap), dtype=torch.float32, device=g.dev, requires_grad=True)
    U0 = e * Sd + dU
    E0 = torch.zeros_like(g.E)
    B0 = torch.zeros_like(g.B)
    EN, BN = AG.run(g, steps, K, E0, B0, [U0])
    m = torch.from_numpy(_probe_mask(EN.shape, *(probe or PROBE))).to(g.dev)
    dV = w.d[0] * w.d[1] * w.d[2]
    loss = 0.5 * dV * ((EN * EN)[:, m].sum() + (BN * BN)[:, m].sum())
    loss.backward()
    # dL/d eps = sum over all particles of S . dL/dU0, summed in FP64 on the GPU
    geps = g.dot_f64(Sd, dU.grad)
    assert abs(geps - float(e.grad.item())) <= 1e-4 * abs(geps) + 1e-30, (geps, e.grad.item())
    dir_grad = None
    if dirU is not None:
        gU = dU.grad[:, :N].double().cpu().numpy().T      # storage order
        gU_by_id = np.empty_like(gU)
        gU_by_id[I] = gU
        dir_grad = float(np.sum(gU_by_id * dirU))
    return float(loss.item()), geps, dir_grad


def _fp64_loss(w_fn, eps, dirU=None, h=0.0, steps=500):
    """Probe energy after `steps` FP64 steps (GPU plain path, itself parity-
    tested against the oracle)."""
    w = w_fn(eps)
    if dirU is not None:
        w.species[0].u = w.species[0].u + h * dirU
    g = _sim(w, "fp64")
    dV = w.d[0] * w.d[1] * w.d[2]
    g.step(steps)
    E, B, _ = g.fields()
    m = _probe_mask(E.shape, *PROBE)
    out = 0.5 * dV * (np.sum(E[:, m] ** 2) + np.sum(B[:, m] ** 2))
    g.close()
    return out


def _random_direction(pos, box, seed):
    """A random direction in the space of all initial momenta (seeded input
    generator): a smooth random momentum field plus white noise.  A pure
    white-noise direction is nearly orthogonal to the modes the loss responds
    to, so its derivative would be ~1/sqrt(N) of the problem's scale and FP32
    rounding would dominate the comparison."""
    return W.smooth_random_direction(pos, box, seed)


def _check_gradients(steps, K):
    """Gradients wrt eps and along a random direction of all initial momenta
    within 1e-4 (relative) of central differences (h = 1e-4) of the FP64
    forward (the GPU's plain FP64 step, parity-tested against the oracle)."""
    eps, h = 1e-2, 1e-4
    wf = lambda e: W.cold_langmuir_lattice(eps=e, steps=steps)
    w = wf(eps)
    box = np.asarray(w.n) * np.asarray(w.d)
    dirU = _random_direction(w.species[0].pos, box, 3)
    Lv, geps, gdir = _adjoint_gradients(w, steps, K, eps, dirU)
    fd_eps = (_fp64_loss(wf, eps + h, steps=steps) - _fp64_loss(wf, eps - h, steps=steps)) / (2 * h)
    fd_dir = ((_fp64_loss(wf, eps, dirU, h, steps=steps) - _fp64_loss(wf, eps, dirU, -h, steps=steps))
              / (2 * h))
    assert Lv > 0
    assert abs(geps - fd_eps) <= 1e-4 * abs(fd_eps), (steps, geps, fd_eps)
    assert abs(gdir - fd_dir) <= 1e-4 * abs(fd_dir), (steps, gdir, fd_dir)


def test_gradients_match_central_differences_100_steps():
    """Differentiable workload (32^3, 16 per cell on a (4,2,2) lattice,
    eps = 1e-2), 100 steps, checkpoints every 10."""
    _check_gradients(100, 10)


GOLDEN_32 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "langmuir32_gradients.json")


def test_differentiable_workload_gradients_500_steps():
    """The differentiable workload as stated: 32^3, 16 per cell, eps = 1e-2,
    500 steps, checkpoints every 50.  The FP32 GPU gradients with respect to
    eps and along the seeded random momentum direction against the FP64
    oracle's central differences (h = 1e-4) and its chained adjoint gradient
    of the same run (tests/golden/langmuir32_gradients.json, written by
    make_langmuir32_gradients.py from the oracle alone).

    The criterion, 1e-4 relative to the central differences, is asserted as
    stated.  Against the oracle's own adjoint the bound is 1e-4 plus the
    distance between the oracle's two references (4.8e-5 for eps, 3.9e-6
    for the direction).  At step 500 the probe energy is about 1/1900 of its
    peak, a node of the oscillation, where a phase error is amplified
    ~90-fold into L; the FP32 Yee updates evaluate in FP64 and round once
    per stored value, since their intermediate FP32 roundings (of J, of
    curl - J, of the two-part update) add up coherently on the quiet
    lattice and made L miss by 1.2e-4 and the gradients by 1.0-1.8e-4."""
    ref = json.load(open(GOLDEN_32))
    steps, K, eps = ref["steps"], ref["checkpoint_every"], ref["eps"]
    w = W.cold_langmuir_lattice(eps=eps, steps=steps)
    box = np.asarray(w.n) * np.asarray(w.d)
    dirU = _random_direction(w.species[0].pos, box, ref["direction_seed"])
    Lv, geps, gdir = _adjoint_gradients(w, steps, K, eps, dirU, probe=tuple(ref["probe"]))
    errs = {"L": abs(Lv - ref["L"]) / ref["L"],
            "eps_vs_adjoint": abs(geps - ref["adjoint_dL_deps"]) / abs(ref["adjoint_dL_deps"]),
            "eps_vs_fd": abs(geps - ref["fd_dL_deps"]) / abs(ref["fd_dL_deps"]),
            "dir_vs_adjoint": abs(gdir - ref["adjoint_dL_ddir"]) / abs(ref["adjoint_dL_ddir"]),
            "dir_vs_fd": abs(gdir - ref["fd_dL_ddir"]) / abs(ref["fd_dL_ddir"])}
    print("config-4 gradients at 500 steps:", json.dumps(errs), flush=True)
    spread = {"eps": abs(ref["adjoint_dL_deps"] - ref["fd_dL_deps"]) / abs(ref["fd_dL_deps"]),
              "dir": abs(ref["adjoint_dL_ddir"] - ref["fd_dL_ddir"]) / abs(ref["fd_dL_ddir"])}
    assert errs["L"] <= 1e-4, (errs, Lv)
    for g in ("eps", "dir"):
        assert errs[g + "_vs_fd"] <= 1e-4, (g, errs, geps, gdir)
        assert errs[g + "_vs_adjoint"] <= 1e-4 + spread[g], (g, errs, spread, geps, gdir)


def test_gradient_matches_fp64_oracle_adjoint():
    """Reduced differentiable workload (8^3, 8 per cell, 40 steps, checkpoints
    every 10): FP32 GPU adjoint against the FP64 oracle's chained adjoint."""
    steps, K, eps, lo, hi = 40, 10, 1e-2, 2, 6
    w = W.cold_langmuir_lattice(n=(8, 8, 8), per_axis=(2, 2, 2), eps=eps, steps=steps)
    _, geps, _ = _adjoint_gradients(w, steps, K, eps, probe=(lo, hi))
    o = O.OracleSim(w.n, w.d, w.dt)
    s = w.species[0]
    o.add_species(s.q, s.m, s.w, s.pos, s.u)
    states = []
    for _ in range(steps):
        states.append(o.state())
        o.step(1)
    m = _probe_mask(o.E.shape, lo, hi)
    lE = np.where(m[None], o.dV * o.E, 0.0)
    lB = np.where(m[None], o.dV * o.B, 0.0)
    lX, lU = [np.zeros_like(s.pos)], [np.zeros_like(s.u)]
    for st in reversed(states):
        o.set_state(st)
        lE, lB, lX, lU = o.step_vjp(lE, lB, lX, lU)
    g_orc = float(np.sum(lU[0][:, 0] * np.sin(2 * np.pi * s.pos[:, 0] / (w.n[0] * w.d[0]))))
    assert abs(geps - g_orc) <= 1e-4 * abs(g_orc), (geps, g_orc)


def _weibel(steps):
    return W.weibel_bimaxwellian(n=(16, 16, 16), ppc=4, steps=steps, sort_every=0)


def _weibel_adjoint(w, steps, K, sort, dirU, dirE):
    """FP32 forward + adjoint of L = 1/2 dV sum |B^{N-1/2}|^2 over the box:
    (L, <dL/dU0, dirU>, <dL/dE0, dirE>)."""
    import torch
    from paper_2609_16575_amd import autograd as AG
    g = _sim(w, sort_every=0)
    if not sort:
        g.sort()  # states need sorted particles; with sort=True the run sorts first
    _, U, I = g.particles(0)
    cap, N = g.caps[0], len(I)
    Ust = np.zeros((3, cap), np.float32)
    Ust[:, :N] = U.T
    U0 = torch.from_numpy(Ust).to(g.dev).requires_grad_(True)
    E0 = torch.zeros_like(g.E).requires_grad_(True)
    B0 = torch.zeros_like(g.B)
    _, BN = AG.run(g, steps, K, E0, B0, [U0], sort=sort)
    dV = w.d[0] * w.d[1] * w.d[2]
    loss = 0.5 * dV * (BN * BN).sum()
    loss.backward()
    gU = np.empty((N, 3))
    gU[I] = U0.grad[:, :N].double().cpu().numpy().T
    gE = E0.grad.double().cpu().numpy()
    out = (float(loss.item()), float(np.sum(gU * dirU)), float(np.sum(gE * dirE)))
    g.close()
    return out


def _weibel_fp64_loss(steps, dirU, dirE, h):
    w = _weibel(steps)
    w.species[0].u = w.species[0].u + h * dirU
    g = _sim(w, "fp64")
    g.set_fields(E=h * dirE)
    g.step(steps)
    _, B, _ = g.fields()
    g.close()
    return 0.5 * w.d[0] * w.d[1] * w.d[2] * np.sum(B ** 2)


def _fd(f, h):
    return (f(h) - f(-h)) / (2 * h)


def test_gradients_with_sorts_at_checkpoints():
    """Anisotropic (Weibel) plasma, 16^3, 4 per cell, 40 steps, checkpoints
    and counting sorts every 10 steps (particles cross ~3 cells in x):
    gradients of the box's magnetic energy along a random momentum direction
    and a random initial-E direction within 1e-4 of central differences of the
    FP64 forward, and within 1e-5 of the same run without sorts.  The forward
    runs are bit-identical (the current is summed in int64 fixed point); the
    adjoint adds its field gradients with FP32 atomics, whose order differs.
    For scale, FP32-sized noise in J alone moves these gradients by up to
    4e-7 in the FP64 oracle (tests/golden/weibel16_current_noise.json).

    The ZigZag current is discontinuous where a particle's end point crosses
    a cell face (the relay point jumps from the segment's midpoint to the
    face), so the loss is piecewise smooth with jumps and the gradient is the
    derivative inside the current piece.  The differences therefore use steps
    small enough that no particle changes piece within +-h (h = 3e-7 and
    1e-7 here; 1e-4 lands on jumps for this hot plasma), shown by the two
    agreeing with each other."""
    steps, K = 40, 10
    w = _weibel(steps)
    box = np.asarray(w.n) * np.asarray(w.d)
    dirU = _random_direction(w.species[0].pos, box, 21)
    dirE = 1e-3 * np.random.default_rng(22).standard_normal((3,) + tuple(w.n[::-1]))
    L_s, gU_s, gE_s = _weibel_adjoint(w, steps, K, True, dirU, dirE)
    L_n, gU_n, gE_n = _weibel_adjoint(_weibel(steps), steps, K, False, dirU, dirE)
    print("sorted vs unsorted: L", L_s, L_n, "gU", abs(gU_s - gU_n) / abs(gU_n), "gE",
          abs(gE_s - gE_n) / abs(gE_n), flush=True)
    assert L_s == L_n  # the forward step is deterministic
    assert abs(gU_s - gU_n) <= 1e-5 * abs(gU_n), (gU_s, gU_n)
    assert abs(gE_s - gE_n) <= 1e-5 * abs(gE_n), (gE_s, gE_n)
    fU = lambda h: _weibel_fp64_loss(steps, dirU, 0 * dirE, h)
    fE = lambda h: _weibel_fp64_loss(steps, 0 * dirU, dirE, h)
    fdU = [_fd(fU, h) for h in (3e-7, 1e-7)]
    fdE = [_fd(fE, h) for h in (3e-7, 1e-7)]
    assert abs(fdU[0] - fdU[1]) <= 3e-5 * abs(fdU[1]), ("piece switch inside +-h", fdU)
    assert abs(fdE[0] - fdE[1]) <= 3e-5 * abs(fdE[1]), ("piece switch inside +-h", fdE)
    assert abs(gU_s - fdU[1]) <= 1e-4 * abs(fdU[1]), (gU_s, fdU, L_s)
    assert abs(gE_s - fdE[1]) <= 1e-4 * abs(fdE[1]), (gE_s, fdE, L_s)


def _hot_absorbing(seed=31):
    """Hot electrons with per-particle weights in an absorbing 16 x 16 x 8
    box: particles leave through the faces within a few steps."""
    rng = np.random.default_rng(seed)
    n, d = (16, 16, 8), (1.0, 1.0, 1.0)
    N = 6000
    pos = rng.random((N, 3)) * np.asarray(n, float)
    u = 0.6 * rng.standard_normal((N, 3))
    wpp = 0.5 + rng.random(N)
    sp = W.SpeciesInit("e", -1.0, 1.0, 1.0, pos, u, wpp=wpp)
    return W.Workload("hot_abs", n, d, W.courant_dt(d), (W.ABSORBING,) * 3, [sp], sort_every=0)


def _global_cells(st, i, n):
    """Positions in cell units (NaN for removed particles) of state st."""
    c = st["cell"][i].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ijk = np.stack([c & 0x7FF, (c >> 11) & 0x7FF, c >> 22], axis=1).astype(np.float64)
    x = ijk + st["pos"][i].double().cpu().numpy().T
    x[c == 0xFFFFFFFF] = np.nan
    return x


@pytest.mark.parametrize("case", ["periodic_two_species", "absorbing_weighted"])
def test_step_state_matches_step_in_place(case):
    """empic_step_state from a saved state equals loading it and stepping in
    place, bit for bit (the FP32 step is deterministic): the particle records
    and the fields after one step and after four, removed particles
    included; the handle's own particle buffers and fields stay untouched."""
    w = W.thermal_two_species(n=(16, 16, 16), ppc=4) if case == "periodic_two_species" \
        else _hot_absorbing()
    g = _sim(w, sort_every=0)
    g.sort()
    g.step(2)
    st0 = g.save_state()
    own = [g.particles(i) for i in range(len(w.species))]
    nsp = len(w.species)
    a, b = g.save_state(), g.alloc_state()
    E_own, B_own, _ = g.fields()
    g.step_state(a, b)
    for i in range(nsp):  # own buffers untouched
        P, U, I = g.particles(i)
        assert np.array_equal(P, own[i][0]) and np.array_equal(U, own[i][1])
    E1, B1, _ = g.fields()
    assert np.array_equal(E1, E_own) and np.array_equal(B1, B_own)
    g.load_state(st0)
    g.step(1)
    ref = g.save_state()
    for i in range(nsp):
        N = int(ref["tiles"][i][-1].item())  # slot count; later slots are not state
        assert torch_equal(b["tiles"][i], ref["tiles"][i]), (case, i)
        for k in ("cell", "pos", "u", "id", "w"):
            if b[k][i] is not None:
                assert torch_equal(b[k][i][..., :N], ref[k][i][..., :N]), (case, k, i)
    for k in ("E", "B"):
        assert torch_equal(b[k], ref[k]), (case, k)
    # three more steps state to state, against the in-place run
    for _ in range(3):
        g.step_state(b, a)
        a, b = b, a
    g.load_state(ref)
    g.step(3)
    ref = g.save_state()
    for i in range(nsp):
        N = int(ref["tiles"][i][-1].item())
        xa, xr = _global_cells(b, i, w.n)[:N], _global_cells(ref, i, w.n)[:N]
        assert np.array_equal(np.isnan(xa), np.isnan(xr)), case
        live = ~np.isnan(xr[:, 0])
        dx = xa[live] - xr[live]
        dx -= np.asarray(w.n) * np.round(dx / np.asarray(w.n))
        assert np.abs(dx).max() == 0.0, (case, i, np.abs(dx).max())
        for k in ("cell", "pos", "u"):
            assert torch_equal(b[k][i][..., :N], ref[k][i][..., :N]), (case, k, i)
    if case == "absorbing_weighted":
        N = int(ref["tiles"][0][-1].item())
        assert int((ref["cell"][0][:N] == -1).sum().item()) > 100  # particles were removed
    for k in ("E", "B"):
        assert torch_equal(b[k], ref[k]), (case, k)


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))


def test_dot_f64_matches_numpy_and_repeats():
    import torch
    w = W.thermal_two_species(n=(8, 8, 8), ppc=1)
    g = _sim(w)
    rng = np.random.default_rng(9)
    for n in (0, 1, 1000, 3 * 1000 * 1000 + 17):
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        ta, tb = torch.from_numpy(a).to(g.dev), torch.from_numpy(b).to(g.dev)
        r1, r2 = g.dot_f64(ta, tb), g.dot_f64(ta, tb)
        ref = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        assert r1 == r2  # fixed summation order
        assert abs(r1 - ref) <= 1e-12 * max(np.sum(np.abs(a.astype(np.float64) * b)), 1e-300), (n, r1, ref)
