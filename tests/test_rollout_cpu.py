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
