"""GPU telescoping step vs the oracle's telescoping step, and against the
GPU per-stage-fill step where the two must agree (needs an MI355X)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W
from parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(p, nsteps, **tune):
    from paper_2401_03378_amd.solver import Solver
    S = Solver(p, tuning=tune or None)
    U = S.to_device(p.U0)
    dts = S.run(U, nsteps)
    S.status()
    out = U.cpu().numpy(), dts.cpu().numpy()
    S.close()
    return out


CASES = [(2, 16, 2, 0, 2, "outflow", (2, 2, 1)), (2, 12, 3, 1, 3, "periodic", (2, 1, 1)),
         (3, 8, 2, 0, 2, "periodic", (2, 2, 1)), (3, 10, 3, 1, 3, "outflow", (1, 2, 1)),
         (3, 9, 3, 1, 2, "periodic", (1, 1, 2))]


@pytest.mark.parametrize("ndim,n,ng,recon,rk,bc,NB", CASES)
def test_telescoping_parity(ndim, n, ng, recon, rk, bc, NB):
    p = W.random_blocks(ndim, n, ng, seed=6, recon=recon, rk=rk, bc=bc, NB=NB)
    Uo = p.U0.copy()
    dto = [O.step_telescoping(p, Uo) for _ in range(3)]
    for tile in (0, 1, 2):
        Ug, dtg = _run(p, 3, mode=2, tile=tile)
        assert list(dtg) == dto
        assert_parity(p, Ug, Uo, f"telescoping tile {tile}", bitwise=True)


@pytest.mark.parametrize("ndim,recon,rk,bc,widths", [
    (3, 1, 3, "periodic", ((9, 12, 16), (10, 14), (9, 11))),
    (3, 0, 2, "outflow", ((4, 9, 6), (7, 5), (11, 4))),
    (2, 1, 3, "outflow", ((9, 20, 12), (10, 16))),
])
def test_telescoping_uneven_neighbours(ndim, recon, rk, bc, widths):
    """Thick copies gathered from neighbours of other padded shapes: the
    oracle's telescoping step bit for bit in every tile, and on the periodic
    mesh the per-stage fill's result."""
    ng = 3 if recon == 1 else 2
    p = W.rectilinear(ndim, widths, ng, seed=29, recon=recon, rk=rk, bc=bc)
    Uo = p.U0.copy()
    dto = [O.step_telescoping(p, Uo) for _ in range(2)]
    for tile in (0, 1, 2):
        Ug, dtg = _run(p, 2, mode=2, tile=tile)
        assert list(dtg) == dto
        assert_parity(p, Ug, Uo, f"telescoping uneven tile {tile}", bitwise=True)
    if bc == "periodic":
        m = W.interior_mask(p.blocks, p.ncell, ndim)
        Ua, da = _run(p, 2)
        assert list(da) == dto
        assert np.array_equal(Ua[:, m], Uo[:, m])


def test_telescoping_equals_per_stage_fill_on_periodic_configs():
    for p, n in ((W.batched_uneven(nblocks=64, seed=2), 3), (W.kh2d(N=64, n=16), 4),
                 (W.turb3d(N=32, n=16, seed=1), 2)):
        m = W.interior_mask(p.blocks, p.ncell, p.ndim)
        Ua, da = _run(p, n)
        Ub, db = _run(p, n, mode=2)
        assert np.array_equal(da, db)
        assert np.array_equal(Ua[:, m], Ub[:, m]), p.name


def test_telescoping_sedov_outflow_parity():
    p = W.sedov3d(N=64, n=16)
    Uo = p.U0.copy()
    for _ in range(2):
        O.step_telescoping(p, Uo)
    Ug, _ = _run(p, 2, mode=2)
    assert_parity(p, Ug, Uo, "sedov telescoping", bitwise=True)


def test_telescoping_mode_errors():
    from paper_2401_03378_amd.solver import Solver
    from paper_2401_03378_amd._hip import HydroError, HYDRO_EINVAL
    p = W.random_blocks(3, 6, 3, seed=0, recon=1, rk=3)       # 9 halo layers > 6
    S = Solver(p)
    with pytest.raises(HydroError) as e:
        S.set_tuning(mode=2)
    assert e.value.code == HYDRO_EINVAL
    S.close()
    q = W.random_blocks(2, 16, 2, seed=0)
    S = Solver(q, tuning=dict(mode=2))
    U = S.to_device(q.U0)
    with pytest.raises(HydroError):
        S.rk_stage(1, U, U, U.clone())
    with pytest.raises(HydroError):
        S.step_vjp(U, U.clone(), 1e-3)
    # the per-step autograd Function still steps forward in this mode (the
    # telescoping step); its backward pass is refused like step_vjp
    from paper_2401_03378_amd.adjoint import hydro_step
    ref = U.clone()
    S.step(ref, 1e-3)
    x = U.clone().requires_grad_(True)
    y = hydro_step(x, 1e-3, S)
    m = torch.as_tensor(W.interior_mask(q.blocks, q.ncell, 2), device=U.device)
    assert torch.equal(y.detach()[:, m], ref[:, m])
    with pytest.raises(RuntimeError):        # HydroError, as raised through autograd
        torch.nan_to_num(y).sum().backward()
    S.close()
