"""GPU step on meshes with refinement levels (coarse-fine guard fill, flux
registers in the stage kernel, flux correction after every stage) vs the CPU
oracle, element by element (needs an MI355X)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W
from parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(p, level_by_level=False, **tune):
    from paper_2401_03378_amd.solver import Solver
    return Solver(p, tuning=tune or None, level_by_level=level_by_level)


CASES = [
    # ndim, recon, rk, n, ng, NBc
    (2, 0, 2, 8, 2, (4, 4)),
    (2, 1, 3, 16, 3, (4, 4)),
    (3, 0, 2, 8, 2, (4, 4, 4)),
    (3, 1, 3, 8, 3, (4, 4, 4)),
]


@pytest.mark.parametrize("ndim,recon,rk,n,ng,NBc", CASES)
@pytest.mark.parametrize("lbl", [False, True])
def test_amr_parity(ndim, recon, rk, n, ng, NBc, lbl):
    p = W.amr_problem(ndim, NBc=NBc, n=n, ng=ng, recon=recon, rk=rk, flow="random", seed=7)
    Uo = p.U0.copy()
    dto = O.amr_run(p, Uo, 3)
    for tile in (0, 2):
        S = _solver(p, level_by_level=lbl, tile=tile)
        U = S.to_device(p.U0)
        dtg = S.run(U, 3).cpu().numpy()
        S.status()
        Ug = U.cpu().numpy()
        S.close()
        np.testing.assert_array_equal(dtg, np.array(dto))
        assert_parity(p, Ug, Uo, f"amr {ndim}d recon {recon} tile {tile} lbl {lbl}", bitwise=True)
        m = W.interior_mask(p.blocks, p.ncell, ndim)
        assert np.array_equal(Ug[:, m], Uo[:, m])


def test_amr_full_size_weno_3d():
    """16^3 blocks, 56 coarse + 64 fine (central 2^3 coarse blocks refined),
    WENO5 + RK3, the blob crossing the coarse-fine faces."""
    p = W.amr_problem(3, NBc=(4, 4, 4), n=16, ng=3, recon=1, rk=3, flow="blob", seed=0)
    Uo = p.U0.copy()
    dto = O.amr_run(p, Uo, 2)
    S = _solver(p)
    U = S.to_device(p.U0)
    dtg = S.run(U, 2).cpu().numpy()
    S.status()
    np.testing.assert_array_equal(dtg, np.array(dto))
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(U.cpu().numpy()[:, m], Uo[:, m])
    S.close()


def test_amr_conserves_on_gpu():
    p = W.amr_problem(3, NBc=(4, 4, 4), n=8, ng=3, recon=1, rk=3, flow="random", seed=2)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    vol = p.cell_volumes()
    t0 = np.array([np.sum(p.U0[v, m] * vol[m]) for v in range(p.nvar)])
    S = _solver(p)
    U = S.to_device(p.U0)
    S.run(U, 5)
    S.status()
    Ug = U.cpu().numpy()
    t1 = np.array([np.sum(Ug[v, m] * vol[m]) for v in range(p.nvar)])
    assert np.max(np.abs(t1 - t0) / (np.abs(t0) + 1.0)) < 5e-15
    S.close()


def test_amr_fill_guards_matches_oracle():
    for ndim in (2, 3):
        p = W.amr_problem(ndim, n=8, ng=3, recon=1, rk=3, flow="random", seed=5)
        S = _solver(p)
        U = S.to_device(p.U0)
        S.fill_guards(U)
        got = U.cpu().numpy()
        ref = p.U0.copy()
        O.amr_fill_guards(p, ref)
        both_nan = np.isnan(got) & np.isnan(ref)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        assert np.array_equal(got[~both_nan], ref[~both_nan])
        S.close()


def test_amr_refusals():
    from paper_2401_03378_amd._hip import HydroError, HYDRO_EINVAL
    p = W.amr_problem(2, n=8, ng=2)
    S = _solver(p)
    U = S.to_device(p.U0)
    with pytest.raises(HydroError) as e:
        S.step_vjp(U, torch.zeros_like(U), 1e-3)
    assert e.value.code == HYDRO_EINVAL
    for mode in (1, 2):
        with pytest.raises(HydroError) as e:
            S.set_tuning(mode=mode)
        assert e.value.code == HYDRO_EINVAL
    S.close()


@pytest.mark.parametrize("ndim,recon,rk,n,ng", [(2, 0, 2, 8, 2), (3, 1, 3, 8, 3)])
def test_amr_blast_with_outflow_faces(ndim, recon, rk, n, ng):
    """A Sedov-like blast inside the refined patch, outflow on the domain
    faces: the shock crosses the coarse-fine faces (strong jumps, positivity
    fallback) within a few steps."""
    p = W.amr_problem(ndim, NBc=(4, 4, 4), n=n, ng=ng, recon=recon, rk=rk, flow="blast")
    Uo = p.U0.copy()
    dto = O.amr_run(p, Uo, 6)
    for lbl in (False, True):
        S = _solver(p, level_by_level=lbl)
        U = S.to_device(p.U0)
        dtg = S.run(U, 6).cpu().numpy()
        S.status()
        np.testing.assert_array_equal(dtg, np.array(dto))
        m = W.interior_mask(p.blocks, p.ncell, ndim)
        assert np.array_equal(U.cpu().numpy()[:, m], Uo[:, m])
        S.close()
