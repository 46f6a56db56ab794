"""Pins of the oracle's hand-written adjoint (no GPU).

The reverse-mode code is checked against the complex-step derivative of the
forward code (an exact linearisation to rounding, with branches decided on
real parts) through the dot-product identity <w, J v> = <J^T w, v>, piece by
piece and for whole steps, and against central finite differences.
"""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W
from test_oracle_pins import P2, _rand_prims


def _dot_rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("ndim", [2, 3])
def test_eos_vjp(ndim):
    rng = np.random.default_rng(0)
    prob = P2(ndim)
    Wp = _rand_prims(rng, 500, ndim)
    U, _, _ = O.state_flux(prob, Wp, 0)
    V = rng.standard_normal(U.shape)
    gW = rng.standard_normal((U.shape[0], 5))
    if ndim == 2:
        gW[:, 3] = 0.0
    _, Jv = O.eos_cs(prob, U, V)
    gU = O.eos_vjp(prob, U, gW)
    assert np.max(np.abs(np.sum(gW * Jv, 1) - np.sum(gU * V, 1)) / np.abs(np.sum(gW * Jv, 1))) < 1e-12


def test_plm_vjp_all_branches():
    rng = np.random.default_rng(1)
    q = rng.standard_normal((4000, 3))
    v = rng.standard_normal(q.shape)
    gm, gp = rng.standard_normal((2, q.shape[0]))
    (m, jm), (p, jp) = O.plm_cs(q, v)
    _, _, code = O.plm(q)
    assert set(code) == {0, 1, 2, 3}
    gq = O.plm_vjp(q, gm, gp)
    lhs = gm * jm + gp * jp
    rhs = np.sum(gq * v, 1)
    scale = np.abs(gm * jm) + np.abs(gp * jp) + np.sum(np.abs(gq * v), 1)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-14


def test_weno5_vjp():
    rng = np.random.default_rng(2)
    q = rng.standard_normal((3000, 5))
    q[:1000] = np.sin(0.1 * np.arange(5))[None, :] + 0.01 * q[:1000]    # smooth-ish rows
    v = rng.standard_normal(q.shape)
    gm, gp = rng.standard_normal((2, q.shape[0]))
    (m, jm), (p, jp) = O.weno5_cs(q, v)
    gq = O.weno5_vjp(q, gm, gp)
    lhs = gm * jm + gp * jp
    rhs = np.sum(gq * v, 1)
    assert np.max(np.abs(lhs - rhs) / (np.abs(gm * jm) + np.abs(gp * jp) + 1e-12)) < 1e-11


@pytest.mark.parametrize("ndim", [2, 3])
def test_hllc_vjp_all_regions(ndim):
    rng = np.random.default_rng(3)
    prob = P2(ndim)
    WL = _rand_prims(rng, 3000, ndim)
    WR = _rand_prims(rng, 3000, ndim)
    VL = rng.standard_normal(WL.shape)
    VR = rng.standard_normal(WR.shape)
    if ndim == 2:
        VL[:, 3] = VR[:, 3] = 0.0
    for n in range(ndim):
        F, tape, _ = O.hllc(prob, WL, WR, n)
        assert set(np.unique(tape)) >= {0, 1, 2, 3}
        assert len(set(np.unique(tape >> 2))) == 4          # all Davis argmin/argmax combos
        gF = rng.standard_normal(F.shape)
        _, Jv = O.hllc_cs(prob, WL, WR, n, VL, VR)
        gL, gR = O.hllc_vjp(prob, WL, WR, n, gF)
        lhs = np.sum(gF * Jv, 1)
        rhs = np.sum(gL * VL, 1) + np.sum(gR * VR, 1)
        assert np.max(np.abs(lhs - rhs) / (np.abs(gF) @ np.ones(F.shape[1]) * np.abs(Jv).max(1) + 1e-12)) < 1e-12


CASES = [(2, 0, 2, 8, "periodic"), (2, 1, 3, 8, "outflow"), (3, 0, 2, 6, "outflow"),
         (3, 1, 3, 6, "periodic")]


@pytest.mark.parametrize("ndim,recon,rk,n,bc", CASES)
def test_step_vjp_dot_product(ndim, recon, rk, n, bc):
    p = W.random_blocks(ndim, n, 3 if recon else 2, seed=4, recon=recon, rk=rk, bc=bc)
    U = p.U0
    dt = O.cfl_dt(p, U)
    rng = np.random.default_rng(5)
    m = np.isfinite(U)
    for trial in range(3):
        V = np.where(m, rng.standard_normal(U.shape), 0.0)
        Wt = np.where(m, rng.standard_normal(U.shape), 0.0)
        _, Jv = O.step_cs(p, U, V, dt)
        g = O.step_vjp(p, U, dt, Wt)
        a = np.sum(Wt[m] * Jv[m])
        b = np.sum(g[m] * V[m])
        assert _dot_rel(a, b) < 1e-12
        assert np.all(g[~m] == 0.0)


def test_step_vjp_linearity_bitwise():
    p = W.random_blocks(3, 6, 3, seed=6, recon=1, rk=3)
    U = p.U0
    dt = O.cfl_dt(p, U)
    g = np.where(np.isfinite(U), np.random.default_rng(7).standard_normal(U.shape), 0.0)
    a = O.step_vjp(p, U, dt, g)
    b = O.step_vjp(p, U, dt, 2.0 * g)
    assert np.array_equal(2.0 * a, b)


@pytest.mark.parametrize("ndim,recon,rk", [(2, 0, 2), (3, 1, 3)])
def test_step_vjp_central_differences(ndim, recon, rk):
    """Central differences at dt fixed along random directions; a direction
    whose +/- perturbation crosses a branch (a limiter kink) is redrawn."""
    p = W.random_blocks(ndim, 8 if ndim == 2 else 6, 3 if recon else 2, seed=8,
                        recon=recon, rk=rk, amp=0.1)
    U = p.U0
    m = np.isfinite(U)
    dt = O.cfl_dt(p, U)
    rng = np.random.default_rng(9)
    Wt = np.where(m, rng.standard_normal(U.shape), 0.0)
    g = O.step_vjp(p, U, dt, Wt)
    good = 0
    for trial in range(40):
        V = np.where(m, rng.standard_normal(U.shape), 0.0)
        h = 1e-7 * np.max(np.abs(U[m])) / np.max(np.abs(V))
        Up, Um = U + h * V, U - h * V
        O.step(p, Up, dt)
        O.step(p, Um, dt)
        fd = np.sum(Wt[m] * (Up[m] - Um[m])) / (2 * h)
        # kink check: the complex-step slopes at U and U +/- hV agree
        _, J0 = O.step_cs(p, U, V, dt)
        _, J1 = O.step_cs(p, U + h * V, V, dt)
        _, J2 = O.step_cs(p, U - h * V, V, dt)
        s0, s1, s2 = (np.sum(Wt[m] * J[m]) for J in (J0, J1, J2))
        if _dot_rel(s1, s0) > 1e-5 or _dot_rel(s2, s0) > 1e-5:
            continue
        ad = np.sum(g[m] * V[m])
        assert _dot_rel(fd, ad) < 1e-6, (fd, ad)
        good += 1
        if good >= 8:
            break
    assert good >= 8
