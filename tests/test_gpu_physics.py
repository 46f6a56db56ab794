"""Gravity source and shock detector on the GPU vs the CPU oracle (needs an
MI355X).  The forward step is compared bit for bit (same arithmetic in the
same order on both sides), the step VJP to 1e-12 per field.  Every call
goes through the C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import _hip
from paper_2401_03378_amd import workloads as W
from parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(p, **tune):
    from paper_2401_03378_amd.solver import Solver
    return Solver(p, tuning=tune or None)


def _gpu_run(p, nsteps, dt_from_previous=False, **tune):
    S = _solver(p, **tune)
    U = S.to_device(p.U0)
    dts = S.run(U, nsteps, dt_from_previous=dt_from_previous)
    S.status()
    out = U.cpu().numpy(), dts.cpu().numpy()
    S.close()
    return out


def _ora_run(p, nsteps, telescoping=False):
    U = p.U0.copy()
    step = O.step_telescoping if telescoping else O.step
    dts = [step(p, U) for _ in range(nsteps)]
    return U, np.array(dts)


def _with(p, grav=None, thresh=None):
    q = p.copy()
    q.grav = grav
    q.shock_thresh = thresh
    return q


G3 = (0.6, -1.1, 0.4)

CASES = [
    # (problem, grav, thresh, steps)
    ("rand2d_plm", lambda: W.random_blocks(2, 12, 2, seed=21, NB=(3, 2, 1)), G3, 0.2, 4),
    ("rand2d_weno", lambda: W.random_blocks(2, 10, 3, seed=22, recon=1, rk=3, bc="outflow"), G3, 0.3, 4),
    ("rand3d_weno", lambda: W.random_blocks(3, 10, 3, seed=23, recon=1, rk=3, NB=(2, 2, 2)), G3, 0.2, 3),
    ("rand3d_plm_outflow", lambda: W.random_blocks(3, 9, 2, seed=24, bc="outflow", NB=(2, 1, 2)), G3, 0.1, 3),
    ("rand3d_grav_only", lambda: W.random_blocks(3, 8, 3, seed=25, recon=1, rk=3), G3, None, 3),
    ("rand3d_shock_only", lambda: W.random_blocks(3, 8, 2, seed=26), None, 0.0, 3),
    ("sod_detector", lambda: W.sod2d(N=64, n=16), None, 0.5, 30),
    ("sedov_detector_gravity", lambda: W.sedov3d(N=32, n=16), (0.0, 0.0, -2.0), 0.5, 12),
    ("atmosphere", lambda: W.atmosphere2d(N=64, n=16), (0.0, -1.0, 0.0), None, 20),
    ("free_fall_3d", lambda: W.free_fall(3, n=8, ng=3, recon=1, rk=3), G3, 0.5, 5),
    ("batched_uneven", lambda: W.batched_uneven(nblocks=40, seed=27), G3, 0.3, 3),
    ("uneven_neighbours", lambda: W.rectilinear(3, ((8, 12, 6), (10, 5), (9, 7)), 3, seed=28, recon=1, rk=3,
                                                bc="outflow"), G3, 0.2, 3),
]


@pytest.mark.parametrize("name,make,grav,thresh,nsteps", CASES, ids=[c[0] for c in CASES])
def test_physics_forward_bit_for_bit(name, make, grav, thresh, nsteps):
    """Every tile shape, z-chunking, the persistent grid, the per-block and
    the materialised forms, and a requested prefetching schedule (the plain
    schedule runs) give the oracle's states and dts bit for bit."""
    base = make()
    p = _with(base, grav if grav is not None else getattr(base, "grav", None), thresh)
    Uo, dto = _ora_run(p, nsteps)
    m = W.interior_mask(p.blocks, p.ncell, p.ndim)
    tunes = [dict(tile=t) for t in (0, 1, 2)]
    tunes += [dict(tile=2, zchunk=5, grid=64, variant=1), dict(mode=_hip.MODE_PERBLOCK),
              dict(mode=_hip.MODE_MATERIALISED, tile=1)]
    for tune in tunes:
        Ug, dtg = _gpu_run(p, nsteps, **tune)
        assert np.array_equal(dtg, dto), (name, tune)
        assert_parity(p, Ug, Uo, f"{name} {tune}", bitwise=True)
    # the fused CFL form (final stage records the maxima of its output)
    Ug, dtg = _gpu_run(p, nsteps, dt_from_previous=True)
    assert np.array_equal(dtg, dto)
    assert np.array_equal(Ug[:, m], Uo[:, m])


def test_physics_changes_the_step():
    """The flags are not ignored: gravity and the detector each change the
    GPU result away from the plain step's, as the oracle's."""
    p = W.random_blocks(3, 10, 3, seed=23, recon=1, rk=3)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    plain, _ = _gpu_run(p, 2)
    for q in (_with(p, G3, None), _with(p, None, 0.2)):
        Ug, _ = _gpu_run(q, 2)
        Uo, _ = _ora_run(q, 2)
        assert not np.array_equal(Ug[:, m], plain[:, m])
        assert np.array_equal(Ug[:, m], Uo[:, m])


def test_gravity_in_the_telescoping_mode():
    """Gravity belongs to every stage's intra-stage chain, so the telescoping
    mode takes it too: the oracle's telescoping step bit for bit, on a
    periodic domain (where it equals the per-stage fill) and at outflow faces."""
    for bc in ("periodic", "outflow"):
        p = _with(W.random_blocks(3, 10, 3, seed=28, recon=1, rk=3, bc=bc), G3, None)
        Uo, dto = _ora_run(p, 2, telescoping=True)
        Ug, dtg = _gpu_run(p, 2, mode=_hip.MODE_TELESCOPING)
        assert np.array_equal(dtg, dto)
        assert_parity(p, Ug, Uo, f"telescoping {bc}", bitwise=True)


def test_detector_refused_where_it_is_not_defined():
    from paper_2401_03378_amd.solver import Solver
    p = _with(W.random_blocks(3, 10, 3, seed=29, recon=1, rk=3), None, 0.5)
    S = Solver(p)
    with pytest.raises(_hip.HydroError):
        S.set_tuning(mode=_hip.MODE_TELESCOPING)
    S.close()


def test_sedov_full_size_with_detector_and_gravity():
    """Sedov 128^3 (512 blocks of 16^3) with the detector and gravity, in the
    default and the tuned launch configurations: 3 steps bit for bit."""
    p = _with(W.sedov3d(N=128, n=16), (0.0, 0.0, -1.0), 0.5)
    Uo, dto = _ora_run(p, 3)
    Ug, dtg = _gpu_run(p, 3)
    assert np.array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, "sedov128 physics", bitwise=True)


# ------------------------------------------------------------------ adjoint

VJP_CASES = [
    (lambda: W.random_blocks(2, 12, 2, seed=31, bc="outflow"), G3, 0.2),
    (lambda: W.random_blocks(2, 10, 3, seed=32, recon=1, rk=3), G3, 0.3),
    (lambda: W.random_blocks(3, 8, 3, seed=33, recon=1, rk=3, bc="outflow"), G3, 0.2),
    (lambda: W.random_blocks(3, 9, 2, seed=34), G3, None),
    (lambda: W.random_blocks(3, 9, 2, seed=35, bc="outflow"), None, 0.1),
    (lambda: W.batched_uneven(nblocks=24, seed=36), G3, 0.3),
]


@pytest.mark.parametrize("k", range(len(VJP_CASES)))
def test_physics_step_vjp(k):
    make, grav, thresh = VJP_CASES[k]
    p = _with(make(), grav, thresh)
    dt = O.cfl_dt(p, p.U0)
    rng = np.random.default_rng(40 + k)
    g = np.where(np.isfinite(p.U0), rng.standard_normal(p.U0.shape), 0.0)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p)
    Ug = S.to_device(p.U0)
    got = S.step_vjp(Ug, S.to_device(g), dt).cpu().numpy()
    S.status()
    S.close()
    assert_parity(p, got, ref, "physics step_vjp")
    assert np.all(got[:, ~W.interior_mask(p.blocks, p.ncell, p.ndim)] == 0.0)


def test_turbulence_full_size_with_detector_and_gravity():
    """The 256^3 turbulence workload (4096 blocks of 16^3) with the detector
    and gravity in its tuned launch configuration: one step bit for bit, and
    the step VJP at full size to 1e-12."""
    from paper_2401_03378_amd import autotune
    import json
    import os
    p = _with(W.turb3d(), (0.3, -0.5, 0.2), 0.3)
    Uo, dto = _ora_run(p, 1)
    tune = None
    if os.path.exists(autotune.CACHE):
        tune = json.load(open(autotune.CACHE)).get(autotune.signature(p), {}).get("tuning")
    Ug, dtg = _gpu_run(p, 1, **(tune or {}))
    assert np.array_equal(dtg, dto)
    assert_parity(p, Ug, Uo, "turb256 physics", bitwise=True)
    dt = float(dto[0])
    rng = np.random.default_rng(77)
    g = np.where(np.isfinite(p.U0), rng.standard_normal(p.U0.shape), 0.0)
    ref = O.step_vjp(p, p.U0, dt, g)
    S = _solver(p)
    got = S.step_vjp(S.to_device(p.U0), S.to_device(g), dt).cpu().numpy()
    S.status()
    S.close()
    assert_parity(p, got, ref, "turb256 physics step_vjp")


def test_physics_central_differences():
    """Central differences of two steps with gravity and the shock detector
    on (smooth random data with a threshold that flags a share of the cells),
    with the kink check of the plain-problem test: a direction whose
    perturbation moves the adjoint by more than O(h) crossed a branch (a
    detector flag, a limiter case, an HLLC region) and is left out; every
    other direction must agree to 1e-6."""
    p = _with(W.random_blocks(2, 16, 2, seed=9, amp=0.1, NB=(4, 4, 1)), (0.7, -1.3, 0.0), 0.02)
    S = _solver(p)
    m = np.isfinite(p.U0)
    U0 = S.to_device(p.U0)
    Ug = p.U0.copy()
    O.fill_guards(p, Ug)
    assert sum(int(O.shock_flags(p, Ug, d).sum()) for d in range(2)) > 20
    dt = float(S.cfl_dt(U0).item())
    rng = np.random.default_rng(11)
    w = torch.nan_to_num(S.to_device(np.where(m, rng.standard_normal(p.U0.shape), 0.0)))

    def grad_at(U):
        U1 = U.clone()
        S.step(U1, dt)
        return S.step_vjp(U, S.step_vjp(U1, w, dt), dt)

    g0 = grad_at(U0)
    scale = float(g0.abs().max())
    accepted, rejected = 0, []
    for trial in range(40):
        v = S.to_device(np.where(m, rng.standard_normal(p.U0.shape), 0.0))
        h = 1e-7 * float(torch.nan_to_num(U0).abs().max()) / float(v.abs().max())
        up, um = U0 + h * v, U0 - h * v
        dev = max(float((grad_at(up) - g0).abs().max()), float((grad_at(um) - g0).abs().max())) / scale
        if dev > 1e-5:
            rejected.append(dev)
            continue
        for U in (up, um):
            S.step(U, dt)
            S.step(U, dt)
        fd = float(torch.nansum(w * (up - um))) / (2 * h)
        ad = float(torch.nansum(g0 * v))
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (trial, fd, ad)
        accepted += 1
        if accepted >= 8:
            break
    S.status()
    S.close()
    print(f"central differences with gravity and the detector: {accepted} directions agree; "
          f"{len(rejected)} crossed a branch")
    assert accepted >= 8
