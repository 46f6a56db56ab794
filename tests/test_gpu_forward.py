"""GPU forward path vs the CPU oracle, element by element (needs an MI355X).

Every call goes through the C ABI (libhydro.so via ctypes); the oracle runs
the same seeded inputs on the host.
"""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W
from parity import assert_parity, field_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(p, **tune):
    from paper_2401_03378_amd.solver import Solver
    return Solver(p, tuning=tune or None)


def _gpu_run(p, nsteps, **tune):
    S = _solver(p, **tune)
    U = S.to_device(p.U0)
    dts = S.run(U, nsteps)
    S.status()
    out = U.cpu().numpy(), dts.cpu().numpy()
    S.close()
    return out


def _bench_tuning(p):
    """The launch configuration bench.py and the solver use for this problem
    (the autotuner's cached choice), or None if it has none."""
    import json
    import os
    from paper_2401_03378_amd import autotune
    if not os.path.exists(autotune.CACHE):
        return None
    db = json.load(open(autotune.CACHE))
    return db.get(autotune.signature(p), {}).get("tuning")


def _gpu_runs(p, nsteps):
    """The default launch configuration and, if cached, the tuned one; both
    must give the same bits."""
    Ug, dtg = _gpu_run(p, nsteps)
    tuned = _bench_tuning(p)
    if tuned is not None:
        Ut, dtt = _gpu_run(p, nsteps, **tuned)
        m = W.interior_mask(p.blocks, p.ncell, p.ndim)
        assert np.array_equal(dtt, dtg), tuned
        assert np.array_equal(Ut[:, m], Ug[:, m]), tuned
    return Ug, dtg


def _ora_run(p, nsteps):
    U = p.U0.copy()
    dts = O.run(p, U, nsteps)
    return U, np.array(dts)


SMALL = [
    # ndim, recon, rk, n, ng, bc, NB
    (2, 0, 2, 12, 2, "outflow", (2, 2, 1)),
    (2, 0, 2, 16, 2, "periodic", (3, 2, 1)),
    (2, 1, 3, 20, 3, "periodic", (2, 2, 1)),
    (2, 1, 2, 9, 3, "outflow", (2, 3, 1)),
    (3, 0, 2, 10, 2, "periodic", (2, 2, 2)),
    (3, 0, 3, 8, 2, "outflow", (2, 1, 2)),
    (3, 1, 3, 12, 3, "outflow", (2, 2, 2)),
    (3, 1, 3, 16, 3, "periodic", (1, 2, 2)),
    (3, 1, 2, 7, 4, "periodic", (2, 2, 1)),
    # blocks exactly as wide as their guard layers: every guard layer reaches
    # across the whole neighbour interior
    (3, 1, 3, 3, 3, "periodic", (2, 2, 2)),
    (3, 1, 3, 3, 3, "outflow", (2, 1, 2)),
    (3, 0, 2, 2, 2, "outflow", (2, 2, 2)),
    (2, 1, 3, 3, 3, "periodic", (3, 2, 1)),
]


@pytest.mark.parametrize("ndim,recon,rk,n,ng,bc,NB", SMALL)
def test_parity_small_all_tiles(ndim, recon, rk, n, ng, bc, NB):
    """Several tiles and a ragged tail per block; every tile shape, z-chunking
    and kernel schedule gives the oracle's result (and the same bits as each
    other)."""
    p = W.random_blocks(ndim, n, ng, seed=3, recon=recon, rk=rk, bc=bc, NB=NB)
    Uo, dto = _ora_run(p, 3)
    first = None
    combos = [(t, z, v) for t in (0, 1, 2) for z in ((0, 5) if ndim == 3 else (0,)) for v in (0, 1)]
    for tile, zchunk, variant in combos:
        Ug, dtg = _gpu_run(p, 3, tile=tile, zchunk=zchunk, variant=variant)
        assert np.array_equal(dtg, dto), (tile, zchunk, dtg, dto)
        assert_parity(p, Ug, Uo, f"tile {tile} zchunk {zchunk} variant {variant}", bitwise=True)
        if first is None:
            first = Ug
        else:
            m = W.interior_mask(p.blocks, p.ncell, ndim)
            assert np.array_equal(first[:, m], Ug[:, m])


UNEVEN = [
    # ndim, recon, rk, bc, widths
    (3, 1, 3, "periodic", ((8, 12, 16), (10, 6), (9, 7))),
    (3, 0, 2, "outflow", ((6, 9, 13), (7, 5), (11, 4))),
    (3, 1, 3, "outflow", ((3, 17, 5), (20, 4), (6, 3))),
    (2, 1, 3, "periodic", ((8, 12, 16), (10, 6))),
    (2, 0, 2, "outflow", ((5, 19, 2), (9, 33))),
]


@pytest.mark.parametrize("ndim,recon,rk,bc,widths", UNEVEN)
def test_uneven_neighbours_all_launch_forms(ndim, recon, rk, bc, widths):
    """Blocks whose neighbours differ in their extent along the shared
    face's normal, so a halo cell's source block has another padded plane
    (its index steps through the planes by that block's plane size): every
    tile, z-chunking, schedule, grid and launch form gives the oracle's
    states and dts bit for bit."""
    from paper_2401_03378_amd import _hip
    ng = 3 if recon == 1 else 2
    p = W.rectilinear(ndim, widths, ng, seed=17, recon=recon, rk=rk, bc=bc)
    Uo, dto = _ora_run(p, 3)
    tunes = [dict(tile=t, zchunk=z, variant=v) for t in (0, 1, 2) for z in ((0, 5) if ndim == 3 else (0,))
             for v in (0, 1)]
    tunes += [dict(tile=2, grid=16, xcd=1), dict(tile=1, grid=64, xcd=2, zchunk=3 if ndim == 3 else 0),
              dict(mode=_hip.MODE_PERBLOCK), dict(mode=_hip.MODE_MATERIALISED, tile=0)]
    for tune in tunes:
        Ug, dtg = _gpu_run(p, 3, **tune)
        assert np.array_equal(dtg, dto), tune
        assert_parity(p, Ug, Uo, f"uneven {tune}", bitwise=True)


def test_sod_full_config():
    p = W.config(0)
    Uo, dto = _ora_run(p, p.nsteps)
    Ug, dtg = _gpu_runs(p, p.nsteps)
    assert np.array_equal(dtg, dto)
    errs = assert_parity(p, Ug, Uo, "sod2d", bitwise=True)
    print("sod2d field errors", errs)


def test_sedov_full_config():
    p = W.config(1)
    Uo, dto = _ora_run(p, p.nsteps)
    Ug, dtg = _gpu_runs(p, p.nsteps)
    np.testing.assert_array_equal(dtg, dto)
    errs = assert_parity(p, Ug, Uo, "sedov3d", bitwise=True)
    print("sedov3d field errors", errs)


@pytest.mark.timeout(900)
def test_batched_full_size_all_steps():
    """The batched workload at full size (4096 uneven blocks, 21.2 M zones)
    over all 10 of its steps, in the default and the tuned launch."""
    p = W.config(2)
    Uo, dto = _ora_run(p, p.nsteps)
    Ug, dtg = _gpu_runs(p, p.nsteps)
    np.testing.assert_array_equal(dtg, dto)
    errs = assert_parity(p, Ug, Uo, "batched", bitwise=True)
    print("batched field errors", errs)


def test_batched_subset_all_steps():
    p = W.batched_uneven(nblocks=256, seed=1)
    Uo, dto = _ora_run(p, 10)
    Ug, dtg = _gpu_run(p, 10)
    np.testing.assert_array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, "batched-256", bitwise=True)


def test_kh_full_config():
    p = W.config(3)
    Uo, dto = _ora_run(p, p.nsteps)
    Ug, dtg = _gpu_runs(p, p.nsteps)
    np.testing.assert_array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, "kh2d", bitwise=True)


@pytest.mark.timeout(1200)
def test_turbulence_full_size_all_steps():
    """The 256^3 turbulence workload (4096 blocks of 16^3) over all 20 of
    its steps, in the default and the tuned launch."""
    p = W.config(4)
    Uo, dto = _ora_run(p, p.nsteps)
    Ug, dtg = _gpu_runs(p, p.nsteps)
    np.testing.assert_array_equal(dtg, dto)
    errs = assert_parity(p, Ug, Uo, "turb3d", bitwise=True)
    print("turb3d field errors", errs)


def test_weno_epsilon_other_than_the_default():
    """A problem's own WENO5 epsilon reaches the kernels: at eps = 1e-2 the
    GPU steps equal the oracle's at that epsilon bit for bit, and differ from
    the default epsilon's."""
    p = W.random_blocks(3, 10, 3, seed=21, recon=W.WENO5, rk=3, bc="outflow")
    q = p.copy()
    q.weno_eps = 1e-2
    Uo, dto = _ora_run(q, 3)
    Ug, dtg = _gpu_run(q, 3)
    np.testing.assert_array_equal(dtg, dto)
    assert_parity(q, Ug, Uo, "weno eps 1e-2", bitwise=True)
    Ud, _ = _gpu_run(p, 3)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert not np.array_equal(Ud[:, m], Ug[:, m])


def test_turbulence_small_all_steps():
    p = W.turb3d(N=64, n=16, seed=2)
    Uo, dto = _ora_run(p, 5)
    Ug, dtg = _gpu_run(p, 5)
    np.testing.assert_array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, "turb3d-64", bitwise=True)


@pytest.mark.parametrize("mode_kw", [dict(mode=1), dict(use_graph=0), dict(grid=37), dict(grid=256, xcd=1),
                                     dict(xcd=2), dict(grid=512, xcd=2, zchunk=4),
                                     dict(variant=1), dict(mode=1, variant=1),
                                     dict(mode=3), dict(mode=3, use_graph=0, variant=1),
                                     dict(mode=3, tile=0, grid=37)])
def test_launch_forms_bitwise_identical(mode_kw):
    """Per-block launches, one materialised fill per stage, no graph, odd
    persistent grids and the XCD placement all give the persistent
    graph-replayed result bit for bit."""
    p = W.batched_uneven(nblocks=96, seed=4)
    ref, dref = _gpu_run(p, 3)
    Ug, dtg = _gpu_run(p, 3, **mode_kw)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(dtg, dref)
    assert np.array_equal(Ug[:, m], ref[:, m])


def test_stage_and_dt_entry_points():
    p = W.random_blocks(3, 10, 3, seed=5, recon=1, rk=3, bc="outflow")
    S = _solver(p)
    U = S.to_device(p.U0)
    dt = S.cfl_dt(U)
    assert float(dt.item()) == O.cfl_dt(p, p.U0)
    B1 = U.clone()
    B2 = U.clone()
    U3 = U.clone()
    S.rk_stage(1, U, U, B1)
    S.rk_stage(2, U, B1, B2)
    S.rk_stage(3, U, B2, U3)
    ref = p.U0.copy()
    O.step(p, ref, float(dt.item()))
    assert_parity(p, U3.cpu().numpy(), ref, "stages", bitwise=True)
    Ustep = S.to_device(p.U0)
    S.step(Ustep)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(Ustep.cpu().numpy()[:, m], U3.cpu().numpy()[:, m])
    S.close()


def test_fill_guards_matches_oracle():
    p = W.random_blocks(3, 6, 3, seed=6, bc="periodic", NB=(2, 1, 3))
    S = _solver(p)
    U = S.to_device(p.U0)
    S.fill_guards(U)
    ref = p.U0.copy()
    O.fill_guards(p, ref)
    got = U.cpu().numpy()
    both_nan = np.isnan(got) & np.isnan(ref)
    assert np.array_equal(got[~both_nan], ref[~both_nan]) and np.array_equal(np.isnan(got), np.isnan(ref))
    S.close()


def test_materialised_stage_fills_the_input_guards():
    """HYDRO_MODE_MATERIALISED: a stage writes the guard cells of its input
    as the oracle's fill does, and its output is the gathering form's."""
    p = W.random_blocks(3, 6, 3, seed=6, bc="outflow", NB=(2, 1, 3))
    S = _solver(p)
    U = S.to_device(p.U0)
    dt = S.cfl_dt(U)
    ref_out = U.clone()
    S.rk_stage(1, U, U, ref_out)
    S.set_tuning(mode=3)
    out = U.clone()
    S.rk_stage(1, U, U, out)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert torch.equal(out[:, m], ref_out[:, m])
    ref = p.U0.copy()
    O.fill_guards(p, ref)
    got = U.cpu().numpy()
    both_nan = np.isnan(got) & np.isnan(ref)
    assert np.array_equal(got[~both_nan], ref[~both_nan]) and np.array_equal(np.isnan(got), np.isnan(ref))
    S.close()


def test_graph_replays_are_identical():
    p = W.random_blocks(2, 16, 2, seed=7, NB=(3, 3, 1))
    S = _solver(p)
    U1 = S.to_device(p.U0)
    for _ in range(4):
        S.step(U1, 1e-4)
    S.set_tuning(use_graph=0)
    U2 = S.to_device(p.U0)
    for _ in range(4):
        S.step(U2, 1e-4)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    assert np.array_equal(U1.cpu().numpy()[:, m], U2.cpu().numpy()[:, m])
    S.close()


def test_fresh_buffers_and_graph_replay_agree():
    """hydro_step captures a graph only for repeated arguments; steps on a
    fresh buffer each time (direct launches), steps in place (graph replay)
    and alternating fixed and CFL dt all give the same bits."""
    p = W.random_blocks(3, 12, 3, seed=9, recon=1, rk=3, bc="outflow", NB=(2, 2, 1))
    m = W.interior_mask(p.blocks, p.ncell, 3)
    S = _solver(p)
    U1 = S.to_device(p.U0)
    for _ in range(4):
        S.step(U1)
    U2 = S.to_device(p.U0)
    for _ in range(4):
        V = U2.clone()
        S.step(V)
        U2 = V
    assert np.array_equal(U1.cpu().numpy()[:, m], U2.cpu().numpy()[:, m])
    U3 = S.to_device(p.U0)
    U4 = S.to_device(p.U0)
    for n in range(4):
        dt = S.cfl_dt(U3).clone()
        S.step(U3, dt)
        S.step(U4)
    assert np.array_equal(U3.cpu().numpy()[:, m], U1.cpu().numpy()[:, m])
    assert np.array_equal(U4.cpu().numpy()[:, m], U1.cpu().numpy()[:, m])
    S.status()
    S.close()


def test_problem_without_blocks():
    """No blocks: the step, stage and adjoint calls are no-ops that leave
    their arrays untouched; the CFL dt has no cells to bound it (EINVAL)."""
    from paper_2401_03378_amd._hip import HydroError, HYDRO_EINVAL
    p = W.random_blocks(2, 8, 2, seed=1, NB=(1, 1, 1))
    p.blocks = p.blocks[:0]
    p.links = p.links[:0]
    S = _solver(p)
    U = S.to_device(p.U0)
    before = U.clone()
    S.step(U, 1e-3)
    S.rk_stage(1, U, U.clone(), U)
    g = torch.zeros_like(U)
    out = torch.full_like(U, 7.0)
    S.step_vjp(U, g, 1e-3, out)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(U), torch.nan_to_num(before))
    assert torch.all(out == 7.0)
    with pytest.raises(HydroError) as e:
        S.cfl_dt(U)
    assert e.value.code == HYDRO_EINVAL
    S.status()
    S.close()


def test_free_stream_gpu():
    p = W.random_blocks(3, 8, 3, seed=0, recon=1, rk=2)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    for v, val in enumerate([1.3, 0.4, -0.7, 0.2, 2.9]):
        p.U0[v, m] = val
    Ug, _ = _gpu_run(p, 4)
    assert np.array_equal(Ug[:, m], p.U0[:, m])


def test_nonphysical_state_is_reported():
    from paper_2401_03378_amd._hip import HydroError, HYDRO_ENONPHYS
    p = W.random_blocks(3, 8, 2, seed=1)
    m = np.flatnonzero(W.interior_mask(p.blocks, p.ncell, 3))
    p.U0[4, m[11]] = -5.0
    S = _solver(p)
    U = S.to_device(p.U0)
    S.step(U, 1e-4)
    with pytest.raises(HydroError) as e:
        S.status()
    assert e.value.code == HYDRO_ENONPHYS
    S.status()          # the count was reset
    S.close()


@pytest.mark.parametrize("case", ["sedov", "turb", "kh", "batched", "outflow_weno"])
@pytest.mark.parametrize("use_graph,variant", [(1, 0), (0, 0), (1, 1)])
def test_dt_from_previous_step_is_the_same_step(case, use_graph, variant):
    """dt from the maxima the previous step's final stage recorded
    (HYDRO_DT_FROM_PREVIOUS): the same dts and states, bit for bit, as reading
    U for every dt, in the plain and the prefetching schedule; after a stage
    written into U by hydro_rk_stage the recorded maxima are not used."""
    p = {"sedov": lambda: W.sedov3d(N=32, n=16),
         "turb": lambda: W.turb3d(N=32, n=16, seed=4),
         "kh": lambda: W.kh2d(N=64, seed=1),
         "batched": lambda: W.batched_uneven(nblocks=40, seed=5),
         "outflow_weno": lambda: W.random_blocks(3, 10, 3, seed=6, recon=1, rk=3, bc="outflow")}[case]()
    m = W.interior_mask(p.blocks, p.ncell, p.ndim)
    out = {}
    for fused in (False, True):
        S = _solver(p, use_graph=use_graph, variant=variant)
        U = S.to_device(p.U0)
        dts = S.run(U, 5, dt_from_previous=fused).cpu().numpy()
        # a stage of the caller's own into U, then more steps
        dt = torch.tensor([float(dts[-1]) * 0.5], dtype=torch.float64, device=U.device)
        tmp = torch.empty_like(U)
        assert S._L.hydro_rk_stage(S.ctx, 1, dt.data_ptr(), U.data_ptr(), U.data_ptr(), tmp.data_ptr()) == 0
        U[:, m] = tmp[:, m]
        dts2 = S.run(U, 3, dt_from_previous=fused).cpu().numpy()
        S.status()
        out[fused] = (U.cpu().numpy(), dts, dts2)
        S.close()
    (Ua, da, da2), (Ub, db, db2) = out[False], out[True]
    assert np.array_equal(da, db) and np.array_equal(da2, db2)
    assert np.array_equal(Ua[:, m], Ub[:, m])


def test_dt_from_previous_with_two_states_and_levels():
    """Alternating two states, each call finds maxima recorded for the other
    state and reads U; on a mesh with levels the mode reads U every step.
    Both give the dts and states of the plain CFL step bit for bit."""
    p = W.sedov3d(N=32, n=16)
    m = W.interior_mask(p.blocks, p.ncell, p.ndim)
    res = {}
    for fused in (False, True):
        S = _solver(p)
        A, B = S.to_device(p.U0), S.to_device(p.U0)
        B[:, m] = B[:, m] * 1.01
        dts = []
        for n in range(4):
            for X in (A, B):
                S.step(X, dt_from_previous=fused)
                dts.append(float(S.dt.item()))
        S.status()
        res[fused] = (A.cpu().numpy(), B.cpu().numpy(), dts)
        S.close()
    assert res[False][2] == res[True][2]
    assert np.array_equal(res[False][0][:, m], res[True][0][:, m])
    assert np.array_equal(res[False][1][:, m], res[True][1][:, m])
    from paper_2401_03378_amd.solver import Solver
    a = W.amr_problem(3, NBc=(2, 2, 2), n=8, ng=3, recon=W.WENO5, rk=3, flow="blob", refine=[(0, 0, 0)])
    ma = W.interior_mask(a.blocks, a.ncell, 3)
    out = []
    for fused in (False, True):
        S = Solver(a)
        V = S.to_device(a.U0)
        d = S.run(V, 3, dt_from_previous=fused).cpu().numpy()
        S.status()
        out.append((V.cpu().numpy(), d))
        S.close()
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][0][:, ma], out[1][0][:, ma])


# Seeded random problems (dimension, reconstruction, RK order, block size and
# grid, guard width, boundary kind, state amplitude) with random launch
# configurations; drawn once with numpy.random.default_rng(20240106), keeping
# those the oracle steps without a non-physical state.
RANDOM_CASES = [
    (3, 1, 3, 10, 4, 'outflow', (1, 1, 1), 0.3, 527, {'tile': 1, 'zchunk': 3, 'grid': 64, 'xcd': 1, 'variant': 1}),
    (3, 0, 3, 12, 3, 'outflow', (1, 3, 2), 0.6, 944, {'tile': 2, 'zchunk': 3, 'grid': 64, 'xcd': 1, 'variant': 0}),
    (2, 1, 2, 6, 3, 'periodic', (3, 2, 1), 0.6, 174, {'tile': 2, 'zchunk': 3, 'grid': 0, 'xcd': 1, 'variant': 1}),
    (2, 1, 3, 7, 3, 'periodic', (1, 3, 1), 0.3, 909, {'tile': 0, 'zchunk': 3, 'grid': 64, 'xcd': 1, 'variant': 1}),
    (3, 1, 2, 12, 4, 'outflow', (2, 1, 1), 0.6, 47, {'tile': 2, 'zchunk': 0, 'grid': 0, 'xcd': 2, 'variant': 1}),
    (2, 0, 3, 18, 2, 'outflow', (2, 2, 1), 0.6, 445, {'tile': 0, 'zchunk': 0, 'grid': 0, 'xcd': 1, 'variant': 0}),
    (3, 0, 3, 10, 3, 'outflow', (2, 3, 2), 0.6, 183, {'tile': 1, 'zchunk': 5, 'grid': 0, 'xcd': 1, 'variant': 1}),
    (3, 0, 2, 7, 2, 'outflow', (3, 2, 1), 0.6, 36, {'tile': 1, 'zchunk': 0, 'grid': 0, 'xcd': 0, 'variant': 1}),
    (3, 0, 3, 5, 3, 'outflow', (3, 1, 2), 0.3, 318, {'tile': 1, 'zchunk': 5, 'grid': 64, 'xcd': 1, 'variant': 0}),
    (3, 1, 2, 9, 3, 'periodic', (2, 1, 2), 0.3, 848, {'tile': 2, 'zchunk': 0, 'grid': 7, 'xcd': 2, 'variant': 0}),
    (2, 0, 3, 4, 3, 'outflow', (3, 2, 1), 0.6, 860, {'tile': 0, 'zchunk': 3, 'grid': 0, 'xcd': 0, 'variant': 1}),
    (3, 1, 3, 10, 3, 'periodic', (3, 2, 2), 0.6, 582, {'tile': 1, 'zchunk': 5, 'grid': 0, 'xcd': 0, 'variant': 1}),
    (2, 0, 2, 7, 3, 'periodic', (3, 2, 1), 0.3, 194, {'tile': 2, 'zchunk': 0, 'grid': 64, 'xcd': 2, 'variant': 0}),
    (3, 0, 2, 9, 2, 'outflow', (2, 2, 2), 0.3, 307, {'tile': 1, 'zchunk': 0, 'grid': 0, 'xcd': 2, 'variant': 0}),
    (2, 0, 3, 15, 2, 'outflow', (3, 2, 1), 0.3, 77, {'tile': 1, 'zchunk': 5, 'grid': 0, 'xcd': 1, 'variant': 1}),
    (3, 0, 3, 3, 3, 'periodic', (2, 2, 2), 0.6, 836, {'tile': 1, 'zchunk': 0, 'grid': 0, 'xcd': 0, 'variant': 0}),
    (2, 0, 3, 16, 3, 'outflow', (1, 3, 1), 0.6, 212, {'tile': 1, 'zchunk': 0, 'grid': 0, 'xcd': 2, 'variant': 1}),
    (2, 0, 3, 7, 3, 'outflow', (2, 2, 1), 0.3, 437, {'tile': 0, 'zchunk': 0, 'grid': 0, 'xcd': 0, 'variant': 0}),
    (2, 0, 3, 4, 2, 'periodic', (2, 1, 1), 0.3, 668, {'tile': 2, 'zchunk': 5, 'grid': 7, 'xcd': 1, 'variant': 0}),
    (3, 0, 3, 11, 2, 'periodic', (3, 3, 2), 0.6, 104, {'tile': 1, 'zchunk': 5, 'grid': 7, 'xcd': 1, 'variant': 0}),
    (2, 0, 3, 9, 3, 'periodic', (3, 2, 1), 0.3, 272, {'tile': 2, 'zchunk': 3, 'grid': 0, 'xcd': 2, 'variant': 1}),
    (3, 1, 3, 8, 3, 'outflow', (2, 1, 1), 0.6, 530, {'tile': 0, 'zchunk': 0, 'grid': 64, 'xcd': 0, 'variant': 0}),
    (3, 1, 3, 4, 4, 'periodic', (1, 2, 2), 0.3, 504, {'tile': 0, 'zchunk': 0, 'grid': 0, 'xcd': 2, 'variant': 0}),
    (3, 0, 3, 5, 3, 'periodic', (3, 3, 2), 0.6, 505, {'tile': 2, 'zchunk': 0, 'grid': 0, 'xcd': 2, 'variant': 1}),
]


@pytest.mark.parametrize("ndim,recon,rk,n,ng,bc,NB,amp,seed,tune", RANDOM_CASES)
def test_random_problems_bit_for_bit(ndim, recon, rk, n, ng, bc, NB, amp, seed, tune):
    p = W.random_blocks(ndim, n, ng, seed, recon=recon, rk=rk, bc=bc, NB=NB, amp=amp)
    Uo, dto = _ora_run(p, 3)
    Ug, dtg = _gpu_run(p, 3, **tune)
    assert np.array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, f"random {ndim}d recon {recon} n {n} ng {ng} {bc} {NB} {tune}", bitwise=True)


@pytest.mark.parametrize("k", range(8))
def test_materialised_mode_random_problems_bit_for_bit(k):
    """The first eight random problems in HYDRO_MODE_MATERIALISED (one guard
    fill launch per stage, then the non-gathering stage kernel)."""
    ndim, recon, rk, n, ng, bc, NB, amp, seed, tune = RANDOM_CASES[k]
    p = W.random_blocks(ndim, n, ng, seed, recon=recon, rk=rk, bc=bc, NB=NB, amp=amp)
    Uo, dto = _ora_run(p, 3)
    Ug, dtg = _gpu_run(p, 3, **dict(tune, mode=3))
    assert np.array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, f"materialised random {k}", bitwise=True)


def test_materialised_mode_full_size_sedov():
    """The Sedov 128^3 workload (the bench's) in HYDRO_MODE_MATERIALISED gives
    the gathering form's states and dts bit for bit over three steps."""
    p = W.config(1)
    ref, dref = _gpu_run(p, 3)
    Ug, dtg = _gpu_run(p, 3, mode=3)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(dtg, dref)
    assert np.array_equal(Ug[:, m], ref[:, m])
