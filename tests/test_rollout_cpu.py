"""Checkpointed rollout logic (host code of the adjoint), driven by the CPU
oracle as the step implementation (no GPU)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W
from paper_2401_03378_amd.adjoint import rollout, rollout_vjp
from steppers import OracleStepper


def _loss_grad(p, UN, target, m):
    g = np.zeros_like(UN)
    g[0, m] = 2.0 * (UN[0, m] - target[0, m])
    return g


@pytest.mark.parametrize("k", [1, 2, 3, 7, 10])
def test_checkpointing_equals_store_all(k):
    p = W.kh2d(N=32, n=8, nsteps=7)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    st = OracleStepper(p)
    UN1, tape1 = rollout(st, p.U0, 7, 1)
    UNk, tapek = rollout(st, p.U0, 7, k)
    assert np.array_equal(UN1[:, m], UNk[:, m]) and tape1.dts == tapek.dts
    target = p.U0.copy()
    g = _loss_grad(p, UN1, target, m)
    g1 = rollout_vjp(st, tape1, g)
    gk = rollout_vjp(st, tapek, g)
    assert np.array_equal(g1, gk)
    # every segment recomputes all but its last step
    assert tapek.recomputed_steps == sum(min(k, 7 - s) - 1 for s in range(0, 7, k))


def test_rollout_gradient_matches_complex_step():
    p = W.kh2d(N=32, n=8, nsteps=4)
    m = np.isfinite(p.U0)
    st = OracleStepper(p)
    UN, tape = rollout(st, p.U0, 4, 2)
    rng = np.random.default_rng(0)
    w = np.where(m, rng.standard_normal(p.U0.shape), 0.0)
    v = np.where(m, rng.standard_normal(p.U0.shape), 0.0)
    g = rollout_vjp(st, tape, w)
    re, jv = p.U0.copy(), v.copy()
    for dt in tape.dts:
        re, jv = O.step_cs(p, re, jv, dt)
    a = np.sum(w[m] * jv[m])
    b = np.sum(g[m] * v[m])
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


class _KeepingStepper(OracleStepper):
    """A stepper whose step_keep hands back what it was given, so that the
    rollout's pairing of kept data with steps can be checked.  Like the GPU
    solver's step_keep it writes the interior only: a fresh output's guard
    cells hold arbitrary values (here random ones), out's stay as they were."""

    def __init__(self, prob):
        super().__init__(prob)
        self.used = 0
        self.m = W.interior_mask(prob.blocks, prob.ncell, prob.ndim)
        self.rng = np.random.default_rng(99)

    def step_keep(self, Un, dt=None, out=None):
        U = Un.copy()
        dt = O.step(self.p, U, dt)
        res = self.rng.standard_normal(Un.shape) if out is None else out
        res[:, self.m] = U[:, self.m]
        return res, (Un.copy(), dt), dt

    def step_vjp(self, Un, g, dt, kept=None):
        if kept is not None:
            assert np.array_equal(kept[0], Un, equal_nan=True) and kept[1] == dt
            self.used += 1
        return super().step_vjp(Un, g, dt)


@pytest.mark.parametrize("k", [1, 3, 4, 7])
def test_kept_stage_data_reaches_the_vjp_of_its_own_step(k):
    p = W.kh2d(N=32, n=8, nsteps=7)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    plain, keeping = OracleStepper(p), _KeepingStepper(p)
    UN, tape = rollout(plain, p.U0, 7, k)
    UNk, tapek = rollout(keeping, p.U0, 7, k)
    assert np.array_equal(UN[:, m], UNk[:, m])
    g = _loss_grad(p, UN, p.U0.copy(), m)
    ck = {n: c.copy() for n, c in tapek.checkpoints.items()}
    assert np.array_equal(rollout_vjp(plain, tape, g), rollout_vjp(keeping, tapek, g))
    # every recomputed step hands its kept data to its own VJP; the last step
    # of each segment has none; checkpoints are left as they were
    assert keeping.used == tapek.recomputed_steps == sum(min(k, 7 - s) - 1 for s in range(0, 7, k))
    assert all(np.array_equal(ck[n], tapek.checkpoints[n], equal_nan=True) for n in ck)


@pytest.mark.parametrize("k,nsteps", [(1, 7), (3, 7), (4, 8), (7, 7), (10, 7)])
def test_last_segment_kept_by_the_forward_pass(k, nsteps):
    p = W.kh2d(N=32, n=8, nsteps=nsteps)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    plain, keeping = OracleStepper(p), _KeepingStepper(p)
    UN, tape = rollout(plain, p.U0, nsteps, k)
    UNk, tapek = rollout(keeping, p.U0, nsteps, k, keep_last=True)
    assert np.array_equal(UN[:, m], UNk[:, m]) and tape.dts == tapek.dts
    last = ((nsteps - 1) // k) * k
    # U_N's guard cells are those of the state the kept segment starts from
    # (the in-place steps before it), not the arbitrary ones of step_keep's
    # fresh outputs
    assert np.array_equal(UNk[:, ~m], tapek.checkpoints[last][:, ~m], equal_nan=True)
    assert sorted(tapek.tail) == list(range(last, nsteps))
    g = _loss_grad(p, UN, p.U0.copy(), m)
    ref = rollout_vjp(plain, tape, g)
    assert np.array_equal(ref, rollout_vjp(keeping, tapek, g))
    # the last segment is not recomputed and all its steps use kept data
    segs = [(s, min(s + k, nsteps)) for s in range(0, nsteps, k)]
    assert tapek.recomputed_steps == sum(s1 - s0 - 1 for s0, s1 in segs[:-1])
    assert keeping.used == tapek.recomputed_steps + (nsteps - last)
    # the kept segment is used once; a second backward pass recomputes it
    assert tapek.tail == {}
    assert np.array_equal(ref, rollout_vjp(keeping, tapek, g))


def test_cfl_record_gating():
    """The solver takes a step's dt from the maxima the previous step
    recorded only for the tensor that step wrote, alive and unwritten by
    torch since; a fresh copy (even one at a reused address), a tensor
    written in place, or a forgotten record computes the dt from the state."""
    import torch
    from paper_2401_03378_amd import _hip
    from paper_2401_03378_amd.solver import CflRecord
    rec = CflRecord()
    U = torch.zeros(4, 8, dtype=torch.float64)
    assert rec.mode(U) == _hip.HYDRO_DT_RECORD          # nothing recorded yet
    rec.wrote(U)
    assert rec.mode(U) == _hip.HYDRO_DT_FROM_PREVIOUS
    assert rec.mode(U.clone()) == _hip.HYDRO_DT_RECORD  # another tensor
    U.add_(1.0)                                         # written through torch
    assert rec.mode(U) == _hip.HYDRO_DT_RECORD
    rec.wrote(U)
    rec.forget()
    assert rec.mode(U) == _hip.HYDRO_DT_RECORD
    rec.wrote(U)
    del U                                               # freed: the record dies with it
    V = torch.zeros(4, 8, dtype=torch.float64)
    assert rec.mode(V) == _hip.HYDRO_DT_RECORD
