"""Pins of the oracle's telescoping step (the paper's second RK listing in
Sec. 4.2: one thick guard fill per step, stages updated on the shrinking
extended region).  On a domain without physical boundaries every halo cell
is a copy of a cell some block updates identically, so the telescoping step
must reproduce the per-stage-fill step bit for bit; at outflow boundaries the
two variants differ (halo cells evolve instead of being re-copied)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W

CASES = [(2, 8, 2, 0, 2, (2, 2, 1)), (2, 12, 3, 1, 3, (1, 2, 1)), (3, 8, 2, 0, 2, (1, 1, 1)),
         (3, 8, 2, 0, 3, (2, 2, 2)), (3, 10, 3, 1, 3, (2, 1, 2)), (3, 9, 3, 1, 2, (1, 1, 1))]


@pytest.mark.parametrize("ndim,n,ng,recon,rk,NB", CASES)
def test_telescoping_equals_per_stage_fill_on_periodic_domains(ndim, n, ng, recon, rk, NB):
    p = W.random_blocks(ndim, n, ng, seed=5, recon=recon, rk=rk, bc="periodic", NB=NB)
    m = W.interior_mask(p.blocks, p.ncell, ndim)
    U1, U2 = p.U0.copy(), p.U0.copy()
    for _ in range(3):
        d1 = O.step(p, U1)
        d2 = O.step_telescoping(p, U2)
        assert d1 == d2
    assert np.array_equal(U1[:, m], U2[:, m])


@pytest.mark.parametrize("ndim,recon,rk,widths", [
    (3, 1, 3, ((9, 12, 16), (10, 14), (9, 11))), (3, 0, 2, ((4, 9, 6), (7, 5), (11, 4))),
    (2, 1, 2, ((9, 20, 12), (10, 16)))])
def test_telescoping_equals_per_stage_fill_with_uneven_neighbours(ndim, recon, rk, widths):
    """Thick copies gathered from neighbours of other padded shapes (a block
    grid whose columns, rows and layers have their own widths)."""
    p = W.rectilinear(ndim, widths, 3 if recon == 1 else 2, seed=31, recon=recon, rk=rk, bc="periodic")
    m = W.interior_mask(p.blocks, p.ncell, ndim)
    U1, U2 = p.U0.copy(), p.U0.copy()
    for _ in range(2):
        assert O.step(p, U1) == O.step_telescoping(p, U2)
    assert np.array_equal(U1[:, m], U2[:, m])


def test_telescoping_batched_independent_blocks():
    p = W.batched_uneven(nblocks=24, seed=3)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    U1, U2 = p.U0.copy(), p.U0.copy()
    for _ in range(2):
        O.step(p, U1)
        O.step_telescoping(p, U2)
    assert np.array_equal(U1[:, m], U2[:, m])


def test_telescoping_differs_at_outflow_but_stays_close():
    p = W.sod2d(N=32, n=16)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    U1, U2 = p.U0.copy(), p.U0.copy()
    for _ in range(5):
        O.step(p, U1)
        O.step_telescoping(p, U2)
    G1 = W.gather_global(U1, p.blocks, p.grid, 2)[0, 0]
    G2 = W.gather_global(U2, p.blocks, p.grid, 2)[0, 0]
    # identical away from the outflow boundaries, where waves have not arrived
    assert np.array_equal(G1[:, 4:-4], G2[:, 4:-4])
    assert np.array_equal(G1, G2) or np.max(np.abs(G1 - G2)) < 1e-3


def test_telescoping_rejects_blocks_shallower_than_the_halo():
    p = W.random_blocks(3, 6, 3, seed=0, recon=1, rk=3, bc="periodic")   # needs 9 layers
    with pytest.raises(O.OracleError) as e:
        O.step_telescoping(p, p.U0.copy())
    assert e.value.code == O.ORA_EINVAL
