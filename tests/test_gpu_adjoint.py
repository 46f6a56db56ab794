"""GPU adjoint (hydro_step_vjp) vs the CPU oracle's hand-written adjoint,
element by element, plus linearity, determinism, checkpointed rollouts and
finite differences (needs an MI355X)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W
from paper_2401_03378_amd.adjoint import rollout, rollout_vjp, TorchStepper, hydro_rollout, hydro_step
from parity import assert_parity
from steppers import OracleStepper

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(p, **tune):
    from paper_2401_03378_amd.solver import Solver
    return Solver(p, tuning=tune or None)


def _bench_tuning(p):
    """The autotuner's cached launch configuration for this problem (the one
    bench.py times), or None."""
    import json
    import os
    from paper_2401_03378_amd import autotune
    if not os.path.exists(autotune.CACHE):
        return None
    return json.load(open(autotune.CACHE)).get(autotune.signature(p), {}).get("tuning")


def _rand_cot(p, seed):
    rng = np.random.default_rng(seed)
    return np.where(np.isfinite(p.U0), rng.standard_normal(p.U0.shape), 0.0)


SMALL = [
    (2, 0, 2, 12, 2, "outflow", (2, 2, 1)),
    (2, 0, 2, 16, 2, "periodic", (3, 2, 1)),
    (2, 1, 3, 10, 3, "periodic", (2, 2, 1)),
    (2, 1, 2, 9, 3, "outflow", (2, 3, 1)),
    (3, 0, 2, 10, 2, "periodic", (2, 2, 2)),
    (3, 0, 3, 8, 2, "outflow", (2, 1, 2)),
    (3, 1, 3, 12, 3, "outflow", (2, 2, 2)),
    (3, 1, 3, 8, 3, "periodic", (1, 2, 2)),
    (3, 1, 2, 7, 4, "periodic", (2, 2, 1)),
    # blocks exactly as wide as their guard layers: every guard layer reaches
    # across the whole neighbour interior
    (3, 1, 3, 3, 3, "periodic", (2, 2, 2)),
    (3, 1, 3, 3, 3, "outflow", (2, 1, 2)),
    (3, 0, 2, 2, 2, "outflow", (2, 2, 2)),
    (2, 1, 3, 3, 3, "periodic", (3, 2, 1)),
]


@pytest.mark.parametrize("ndim,recon,rk,n,ng,bc,NB", SMALL)
def test_step_vjp_parity(ndim, recon, rk, n, ng, bc, NB):
    p = W.random_blocks(ndim, n, ng, seed=3, recon=recon, rk=rk, bc=bc, NB=NB)
    dt = O.cfl_dt(p, p.U0)
    g = _rand_cot(p, 11)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p)
    Ug = S.to_device(p.U0)
    got = S.step_vjp(Ug, S.to_device(g), dt)
    S.status()
    out = got.cpu().numpy()
    assert_parity(p, out, ref, "step_vjp")
    assert np.all(out[:, ~W.interior_mask(p.blocks, p.ncell, ndim)] == 0.0)
    # linearity (bitwise) and determinism
    got2 = S.step_vjp(Ug, S.to_device(2.0 * g), dt).cpu().numpy()
    assert np.array_equal(got2, 2.0 * out)
    again = S.step_vjp(Ug, S.to_device(g), dt).cpu().numpy()
    assert np.array_equal(again, out)
    S.close()


def test_step_vjp_batched_uneven_blocks():
    p = W.batched_uneven(nblocks=48, seed=2)
    dt = O.cfl_dt(p, p.U0)
    g = _rand_cot(p, 5)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p)
    got = S.step_vjp(S.to_device(p.U0), S.to_device(g), dt).cpu().numpy()
    assert_parity(p, got, ref, "batched vjp")
    S.close()


UNEVEN = [
    (3, 1, 3, "periodic", ((8, 12, 16), (10, 6), (9, 7))),
    (3, 0, 2, "outflow", ((6, 9, 13), (7, 5), (11, 4))),
    (3, 1, 3, "outflow", ((3, 17, 5), (20, 4), (6, 3))),
    (2, 1, 3, "periodic", ((8, 12, 16), (10, 6))),
    (2, 0, 2, "outflow", ((5, 19, 2), (9, 33))),
]


@pytest.mark.parametrize("ndim,recon,rk,bc,widths", UNEVEN)
def test_step_vjp_uneven_neighbours(ndim, recon, rk, bc, widths):
    """Blocks whose neighbours differ in their extent along the shared
    face's normal: the guard cotangents are summed back into cells of blocks
    of another padded shape (and the x lines' transposed copies span them)."""
    ng = 3 if recon == 1 else 2
    p = W.rectilinear(ndim, widths, ng, seed=19, recon=recon, rk=rk, bc=bc)
    dt = O.cfl_dt(p, p.U0)
    g = _rand_cot(p, 23)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p)
    got = S.step_vjp(S.to_device(p.U0), S.to_device(g), dt).cpu().numpy()
    S.status()
    S.close()
    assert_parity(p, got, ref, "step_vjp uneven neighbours")
    assert np.all(got[:, ~W.interior_mask(p.blocks, p.ncell, ndim)] == 0.0)


def test_kh_rollout_gradient_full_config():
    """50 steps of the 256^2 Kelvin-Helmholtz problem, loss
    sum (rho_T - rho_target)^2 with the target from perturbation seed+1,
    checkpoint every 10 steps; gradient w.r.t. the initial conserved state."""
    p = W.config(3)
    tgt = W.kh2d(seed=1)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    UT_tgt = tgt.U0.copy()
    O.run(tgt, UT_tgt, p.nsteps)
    # oracle: forward, loss gradient, checkpointed reverse
    ost = OracleStepper(p)
    UN_o, tape_o = rollout(ost, p.U0, p.nsteps, 10)
    gN = np.zeros_like(p.U0)
    gN[0, m] = 2.0 * (UN_o[0, m] - UT_tgt[0, m])
    g0_o = rollout_vjp(ost, tape_o, gN)
    # GPU
    S = _solver(p)
    st = TorchStepper(S)
    UN_g, tape_g = rollout(st, S.to_device(p.U0), p.nsteps, 10)
    S.status()
    assert tape_g.dts == tape_o.dts
    assert_parity(p, UN_g.cpu().numpy(), UN_o, "kh forward")
    gN_g = torch.zeros_like(UN_g)
    tgt_d = S.to_device(UT_tgt)
    mask = torch.as_tensor(m, device=UN_g.device)
    gN_g[0, mask] = 2.0 * (UN_g[0, mask] - tgt_d[0, mask])
    g0_g = rollout_vjp(st, tape_g, gN_g)
    S.status()
    errs = assert_parity(p, g0_g.cpu().numpy(), g0_o, "kh gradient")
    print("kh gradient field errors", errs)
    # the autograd.Function gives the same gradient
    U0 = S.to_device(p.U0).requires_grad_(True)
    UN = hydro_rollout(U0, S, p.nsteps, 10)
    loss = ((UN[0, mask] - tgt_d[0, mask]) ** 2).sum()
    loss.backward()
    assert torch.equal(U0.grad, g0_g)
    S.close()


def test_turbulence_step_vjp_full_size():
    p = W.config(4)
    dt = O.cfl_dt(p, p.U0)
    g = _rand_cot(p, 4)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p)
    got = S.step_vjp(S.to_device(p.U0), S.to_device(g), dt).cpu().numpy()
    errs = assert_parity(p, got, ref, "turb vjp 256^3")
    # the observed agreement is ~4e-16; a change of the reverse arithmetic that
    # keeps the tolerance but loses digits against the oracle fails here
    assert max(e for e, _ in errs) <= 1e-14, errs
    S.close()


def test_sedov_step_vjp_full_size_and_rollout():
    """The bench workload: the step VJP at full size (outflow faces, the
    strong shock, positivity fallbacks) and a 4-step checkpointed rollout."""
    p = W.config(1)
    dt = O.cfl_dt(p, p.U0)
    g = _rand_cot(p, 8)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p, **(_bench_tuning(p) or {}))
    got = S.step_vjp(S.to_device(p.U0), S.to_device(g), dt).cpu().numpy()
    errs = assert_parity(p, got, ref, "sedov vjp 128^3")
    assert max(e for e, _ in errs) <= 1e-14, errs      # observed ~3e-15
    ost = OracleStepper(p)
    _, tape_o = rollout(ost, p.U0, 4, 2)
    g_o = rollout_vjp(ost, tape_o, g)
    st = TorchStepper(S)
    _, tape_g = rollout(st, S.to_device(p.U0), 4, 2)
    assert tape_g.dts == tape_o.dts
    g_g = rollout_vjp(st, tape_g, S.to_device(g)).cpu().numpy()
    assert_parity(p, g_g, g_o, "sedov 4-step rollout gradient")
    S.close()


def test_turbulence_rollout_small():
    p = W.turb3d(N=64, n=16, seed=3)
    rng = np.random.default_rng(6)
    w = np.where(np.isfinite(p.U0), rng.standard_normal(p.U0.shape), 0.0)
    ost = OracleStepper(p)
    _, tape_o = rollout(ost, p.U0, 10, 5)
    g_o = rollout_vjp(ost, tape_o, w)
    S = _solver(p)
    st = TorchStepper(S)
    # the forward pass keeps the last segment (CFL dts from hydro_cfl_dt)
    U0 = S.to_device(p.U0)
    UN, tape_g = rollout(st, U0, 10, 5, keep_last=True)
    assert tape_g.dts == tape_o.dts and sorted(tape_g.tail) == list(range(5, 10))
    # U_N has U0's guard cells, as with steps in place
    gm = torch.as_tensor(~W.interior_mask(p.blocks, p.ncell, p.ndim), device=U0.device)
    assert torch.equal(UN[:, gm].isnan(), U0[:, gm].isnan())
    assert torch.equal(torch.nan_to_num(UN[:, gm]), torch.nan_to_num(U0[:, gm]))
    g_g = rollout_vjp(st, tape_g, S.to_device(w)).cpu().numpy()
    assert tape_g.recomputed_steps == 4
    assert_parity(p, g_g, g_o, "turb 64^3 rollout gradient")
    S.close()


def test_step_autograd_function_and_central_differences():
    """Smooth random data (no exactly-flat cells, whose zero slopes are
    limiter kinks that central differences would straddle)."""
    p = W.random_blocks(2, 16, 2, seed=8, amp=0.1, NB=(4, 4, 1))
    S = _solver(p)
    m = np.isfinite(p.U0)
    U0 = S.to_device(p.U0)
    dt = float(S.cfl_dt(U0).item())
    rng = np.random.default_rng(7)
    w = S.to_device(np.where(m, rng.standard_normal(p.U0.shape), 0.0))
    x = U0.clone().requires_grad_(True)
    y = hydro_step(hydro_step(x, dt, S), dt, S)
    (y * w).nansum().backward()
    grad = x.grad
    # the Function's saved stage inputs give hydro_step_vjp's gradient bit for bit
    x1 = U0.clone().requires_grad_(True)
    y1 = hydro_step(x1, dt, S)
    (y1 * w).nansum().backward()
    U1 = U0.clone()
    S.step(U1, dt)
    m1 = torch.as_tensor(W.interior_mask(p.blocks, p.ncell, 2), device=U0.device)
    assert torch.equal(y1.detach()[:, m1], U1[:, m1])
    assert torch.equal(x1.grad, S.step_vjp(U0, torch.nan_to_num(w), dt))
    def grad_at(U):
        # the gradient of <w, step(step(U))> at U, through the two step VJPs
        U1 = U.clone()
        S.step(U1, dt)
        return S.step_vjp(U, S.step_vjp(U1, torch.nan_to_num(w), dt), dt)

    g0 = grad_at(U0)
    assert torch.equal(g0, grad)
    scale = float(g0.abs().max())
    accepted, rejected = 0, []
    for trial in range(30):
        v = S.to_device(np.where(m, rng.standard_normal(p.U0.shape), 0.0))
        h = 1e-7 * float(torch.nan_to_num(U0).abs().max()) / float(v.abs().max())
        up, um = U0 + h * v, U0 - h * v
        # kink check: a direction whose perturbation crosses a branch (a
        # limiter case, the fallback, an HLLC region or a Davis argument)
        # changes the adjoint by O(1) somewhere; without a crossing it moves
        # by O(h).  Such directions are left out, and counted.
        dev = max(float((grad_at(up) - g0).abs().max()), float((grad_at(um) - g0).abs().max())) / scale
        if dev > 1e-5:
            rejected.append(dev)
            continue
        for U in (up, um):
            S.step(U, dt)
            S.step(U, dt)
        fd = float(torch.nansum(w * (up - um))) / (2 * h)
        ad = float(torch.nansum(grad * v))
        # every direction that crosses no branch must agree
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (trial, fd, ad)
        accepted += 1
        if accepted >= 8:
            break
    S.close()
    print(f"central differences: {accepted} directions agree; {len(rejected)} crossed a branch "
          f"(adjoint moved by {rejected} of its maximum)")
    assert accepted >= 8


@pytest.mark.parametrize("k", range(8))
def test_random_problems_step_vjp(k):
    """Step VJPs of seeded random problems (the first eight of the forward
    tests' random cases) against the oracle's adjoint."""
    from test_gpu_forward import RANDOM_CASES
    ndim, recon, rk, n, ng, bc, NB, amp, seed, tune = RANDOM_CASES[k]
    p = W.random_blocks(ndim, n, ng, seed, recon=recon, rk=rk, bc=bc, NB=NB, amp=amp)
    dt = O.cfl_dt(p, p.U0)
    g = _rand_cot(p, seed)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p, **tune)
    got = S.step_vjp(S.to_device(p.U0), S.to_device(g), dt).cpu().numpy()
    assert_parity(p, got, ref, f"random vjp {k}")
    S.close()


def _kept_vs_recomputed(p, S, seed):
    from paper_2401_03378_amd._hip import HydroError
    dt = O.cfl_dt(p, p.U0)
    Ug = S.to_device(p.U0)
    U_before = Ug.clone()
    m = torch.as_tensor(W.interior_mask(p.blocks, p.ncell, p.ndim), device=Ug.device)
    UN, stages = S.step_keep(Ug, dt)
    assert len(stages) == p.rk - 1
    # input left as it was, guard cells included (NaN stays NaN)
    assert torch.equal(Ug.isnan(), U_before.isnan())
    assert torch.equal(torch.nan_to_num(Ug), torch.nan_to_num(U_before))
    Ustep = Ug.clone()
    S.step(Ustep, dt)
    assert torch.equal(UN[:, m], Ustep[:, m])                                # the same step, bit for bit
    g = S.to_device(_rand_cot(p, seed))
    kept = S.step_vjp(Ug, g, dt, stages=stages)
    rec = S.step_vjp(Ug, g, dt)
    S.status()
    assert torch.equal(kept, rec)
    # argument checks of the entry point
    with pytest.raises(HydroError):
        S.step_vjp(Ug, g, dt, gUn=stages[0], stages=stages)
    with pytest.raises(ValueError):
        S.step_vjp(Ug, g, dt, stages=stages + [stages[0]])
    with pytest.raises(ValueError):
        S.step_keep(Ug, dt, out=Ug)


@pytest.mark.parametrize("ndim,recon,rk,n,ng,bc,NB", [SMALL[i] for i in (0, 2, 5, 6, 9)])
@pytest.mark.parametrize("mode", [0, 1, 3])
def test_step_vjp_with_kept_stage_inputs(ndim, recon, rk, n, ng, bc, NB, mode):
    """hydro_step_vjp_stages fed the stage inputs of step_keep (hydro_rk_stage
    stage by stage) gives hydro_step_vjp's result bit for bit, and step_keep
    leaves its input as it was, also in the per-block and materialised modes
    whose stages write the guard cells of their input."""
    p = W.random_blocks(ndim, n, ng, seed=5, recon=recon, rk=rk, bc=bc, NB=NB)
    S = _solver(p, mode=mode)
    _kept_vs_recomputed(p, S, 12)
    S.close()


def test_step_vjp_with_kept_stage_inputs_sedov_full_size():
    p = W.config(1)
    S = _solver(p, **(_bench_tuning(p) or {}))
    _kept_vs_recomputed(p, S, 13)
    S.close()


@pytest.mark.parametrize("mode", [1, 3])
def test_rollout_gradient_in_materialising_modes(mode):
    """Per-block and materialised modes write guard cells into the states the
    rollout keeps; the gradient is the persistent mode's bit for bit."""
    p = W.random_blocks(3, 8, 3, seed=9, recon=1, rk=3, bc="outflow", NB=(2, 2, 1))
    w = _rand_cot(p, 9)
    out = []
    for md in (0, mode):
        S = _solver(p, mode=md)
        st = TorchStepper(S)
        UN, tape = rollout(st, S.to_device(p.U0), 5, 2, keep_last=True)
        g = rollout_vjp(st, tape, S.to_device(w))
        S.status()
        m = torch.as_tensor(W.interior_mask(p.blocks, p.ncell, 3), device=UN.device)
        out.append((tape.dts, UN[:, m].clone(), g.clone()))
        S.close()
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])


@pytest.mark.timeout(1200)
def test_turbulence_rollout_gradient_128():
    """The turbulence workload's adjoint rollout (10 steps, checkpoint every
    5, seeded N(0,1) cotangent on all fields) at 128^3 from the same
    generator: the 256^3 oracle adjoint would take the host tens of minutes."""
    p = W.turb3d(N=128, n=16, seed=0)
    w = _rand_cot(p, 6)
    ost = OracleStepper(p)
    _, tape_o = rollout(ost, p.U0, 10, 5)
    g_o = rollout_vjp(ost, tape_o, w)
    S = _solver(p)
    st = TorchStepper(S)
    UN, tape_g = rollout(st, S.to_device(p.U0), 10, 5, keep_last=True)
    assert tape_g.dts == tape_o.dts
    g_g = rollout_vjp(st, tape_g, S.to_device(w)).cpu().numpy()
    S.status()
    errs = assert_parity(p, g_g, g_o, "turb 128^3 rollout gradient")
    print("turb 128^3 rollout gradient field errors", errs)
    S.close()


def test_second_rollout_after_freeing_the_first_state():
    """A rollout whose final state is freed, then a fresh rollout from a new
    copy of U0 (which the caching allocator may place at the same address):
    the new rollout's first dt comes from its own state, so both runs give
    the same dts and the same final state."""
    p = W.random_blocks(3, 8, 3, seed=14, recon=1, rk=3, NB=(2, 2, 2))
    S = _solver(p)
    st = TorchStepper(S)
    U0 = S.to_device(p.U0)
    UN, tape = rollout(st, U0, 6, 3)
    dts1, addr = list(tape.dts), UN.data_ptr()
    m = torch.as_tensor(W.interior_mask(p.blocks, p.ncell, 3), device=U0.device)
    first = UN[:, m].clone()
    del UN, tape
    UN2, tape2 = rollout(st, U0, 6, 3)
    print("second rollout's state at the first one's address:", UN2.data_ptr() == addr)
    assert tape2.dts == dts1
    assert torch.equal(UN2[:, m], first)
    dto = []
    V = p.U0.copy()
    for _ in range(6):
        dto.append(O.step(p, V))
    assert dts1 == dto
    S.close()


def test_step_vjp_rejects_gUn_aliasing_Un():
    from paper_2401_03378_amd._hip import HydroError
    p = W.random_blocks(2, 12, 2, seed=2, NB=(2, 2, 1))
    S = _solver(p)
    U = S.to_device(p.U0)
    before = U.clone()
    g = S.to_device(_rand_cot(p, 3))
    with pytest.raises(HydroError):
        S.step_vjp(U, g, 1e-3, gUn=U)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(U), torch.nan_to_num(before))
    S.close()
