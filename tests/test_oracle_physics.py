"""Pins of the oracle's gravity source and shock detector (no GPU).

The paper names both steps without formulas: grvAccel heads the intra-stage
chain of Algorithm "Intra stage calculations for Spark" and shockDet sits in
Algorithm "Block initializations for Spark", which the non-telescoping RK
listing of Sec. 4.2 runs per stage.  The readings pinned here:

* gravity: a uniform acceleration g whose source enters the update,
  d(m)/dt += rho g and d(E)/dt += m . g, from the stage's own state;
* detector: a cell is flagged along a direction when the flow compresses
  along it (u of the next cell below u of the previous one) and the
  pressure jumps across it by more than shock_thresh times the smaller of
  the two pressures; a flagged cell reconstructs at first order along that
  direction.

Expected values come from closed forms (free fall), conservation laws, the
exact Riemann solution (Toro 2009, ch. 4), the Sedov similarity radius,
symmetry and convergence, never from the code under test.  Copies of the
oracle with a plausible slip planted in either step (built here with gcc)
must fail these pins.
"""
import ctypes as C
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import analytic as A
import oracle as O
from paper_2401_03378_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")


# ------------------------------------------------------- library wrappers

def _fn(L, name, args, res=C.c_int):
    f = getattr(L, name)
    f.restype = res
    f.argtypes = args
    return f


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _step(L, P, U, dt=None):
    f = _fn(L, "ora_step", [C.POINTER(O._Problem), C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int])
    d = np.array([0.0 if dt is None else float(dt)])
    rc = f(P.ptr, _dp(U), _dp(d), 1 if dt is None else 0)
    assert rc == O.ORA_OK, rc
    return float(d[0])


def _flags(L, P, U, d):
    """Detector flags along d of a state (its guards filled first)."""
    fill = _fn(L, "ora_fill_guards", [C.POINTER(O._Problem), C.POINTER(C.c_double)])
    fl = _fn(L, "ora_shock_flags", [C.POINTER(O._Problem), C.POINTER(C.c_double), C.c_int,
                                    C.POINTER(C.c_int)])
    Ug = np.array(U, copy=True)
    assert fill(P.ptr, _dp(Ug)) == O.ORA_OK
    out = np.zeros(P.ncell, dtype=np.int32)
    assert fl(P.ptr, _dp(Ug), int(d), out.ctypes.data_as(C.POINTER(C.c_int))) == O.ORA_OK
    return out


def _global(p, f):
    """A per-cell array of one variable plane as a global (Nz, Ny, Nx) grid."""
    return W.gather_global(np.asarray(f, dtype=np.float64)[None], p.blocks, p.grid, p.ndim)[0]


# ------------------------------------------------------------------ gravity

def _free_fall_check(L, ndim, recon, rk):
    """A uniform gas in free fall: fluxes cancel in every stage, so the step
    is the linear system rho' = 0, m' = rho g, E' = m . g, whose solution is
    a polynomial of degree two in t; SSP-RK2 and RK3 reproduce it exactly
    (the system matrix is nilpotent of order three).  Closed form:
    m(t) = m0 + rho g t, E(t) = E0 + (m0 . g) t + rho |g|^2 t^2 / 2."""
    p = W.free_fall(ndim, n=8, ng=3 if recon else 2, recon=recon, rk=rk)
    P = O.Problem(p)
    m = W.interior_mask(p.blocks, p.ncell, ndim)
    U = p.U0.copy()
    dt, nsteps = 1e-3, 20
    for _ in range(nsteps):
        _step(L, P, U, dt)
    t = nsteps * dt
    g = np.array(p.grav[:ndim])
    rho = p.U0[0, m][0]
    m0 = np.array([p.U0[1 + d, m][0] for d in range(ndim)])
    E0 = p.U0[ndim + 1, m][0]
    assert np.all(U[0, m] == rho)
    for d in range(ndim):
        want = m0[d] + rho * g[d] * t
        assert np.max(np.abs(U[1 + d, m] - want)) <= 1e-13 * abs(want)
    E = E0 + (m0 @ g) * t + 0.5 * rho * (g @ g) * t * t
    assert np.max(np.abs(U[ndim + 1, m] - E)) <= 1e-13 * E


@pytest.mark.parametrize("ndim,recon,rk", [(2, 0, 2), (3, 1, 3), (2, 1, 3), (3, 0, 2)])
def test_free_fall_closed_form(ndim, recon, rk):
    _free_fall_check(O.lib(), ndim, recon, rk)


def test_gravity_momentum_budget_on_a_periodic_flow():
    """On a periodic domain the fluxes only move momentum around, so each
    step changes the total momentum by exactly dt g times the total mass
    (conserved), to rounding."""
    p = W.random_blocks(3, 8, 3, seed=11, recon=W.WENO5, rk=3)
    p.grav = (0.7, -1.5, 0.4)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    U = p.U0.copy()
    M = math.fsum(U[0, m])
    for _ in range(3):
        before = [math.fsum(U[1 + d, m]) for d in range(3)]
        dt = O.step(p, U)
        assert abs(math.fsum(U[0, m]) - M) <= 1e-13 * M
        for d in range(3):
            gain = dt * p.grav[d] * M
            assert abs((math.fsum(U[1 + d, m]) - before[d]) - gain) <= 1e-11 * abs(gain)


def _atmosphere_drift(N, sign=1.0):
    p = W.atmosphere2d(N=N, n=16)
    p.grav = (0.0, sign * p.grav[1], 0.0)
    U = p.U0.copy()
    t = 0.0
    while t < 0.1:
        t += O.step(p, U)
    G = W.gather_global(U, p.blocks, p.grid, 2)[:, 0]
    band = slice(int(0.3 * N), int(0.7 * N))          # away from the outflow faces
    return float(np.max(np.abs(G[2][band] / G[0][band])))


def test_hydrostatic_atmosphere_stays_at_rest_to_second_order():
    """An isothermal atmosphere rho = p = exp(-y) balances an acceleration of
    1 along -y: the velocities the discretisation error sets up away from the
    boundaries stay small and fall at second order under refinement, while
    the opposite sign of g sets the gas moving at about 2 g t."""
    d64, d128 = _atmosphere_drift(64), _atmosphere_drift(128)
    assert d64 < 1e-5
    assert d128 < d64 / 3.5
    assert _atmosphere_drift(64, sign=-1.0) > 0.1


def test_zero_gravity_is_the_plain_step():
    p = W.random_blocks(2, 8, 2, seed=12)
    U, V = p.U0.copy(), p.U0.copy()
    dts = O.run(p, U, 3)
    q = p.copy()
    q.grav = (0.0, 0.0, 0.0)
    O.run(q, V, 3, dts)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    assert np.array_equal(U[:, m], V[:, m])


def test_gravity_in_the_telescoping_step_and_detector_refused_there():
    """Gravity is part of every stage's intra-stage chain, so the telescoping
    step equals the per-stage-fill step bit for bit on a periodic domain; the
    detector belongs to the block initialisation, which the telescoping
    listing runs once per step, and is refused there."""
    p = W.random_blocks(3, 10, 3, seed=13, recon=W.WENO5, rk=3)
    p.grav = (0.5, 0.0, -1.0)
    U, V = p.U0.copy(), p.U0.copy()
    dt = O.step(p, U)
    O.step_telescoping(p, V, dt)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(U[:, m], V[:, m])
    q = p.copy()
    q.shock_thresh = 0.5
    with pytest.raises(O.OracleError):
        O.step_telescoping(q, q.U0.copy())


def test_physics_parameters_are_validated():
    p = W.random_blocks(2, 8, 2, seed=0)
    for kw in ({"grav": (float("nan"), 0.0, 0.0)}, {"grav": (0.0, float("inf"), 0.0)},
               {"shock_thresh": -0.1}, {"shock_thresh": float("nan")}):
        assert O.validate(O.Problem(p, **kw)) == O.ORA_EINVAL
    assert O.validate(O.Problem(p, grav=(1.0, 2.0, 3.0), shock_thresh=0.0)) == O.ORA_OK


# ------------------------------------------------------------ shock detector

def _sod_flag_check(L, N=128, tend=0.15):
    """Sod's tube with the detector: at t the detector flags x-faces within
    three cells of the exact shock position and nowhere else (not in the
    rarefaction fan, not at the contact, whose pressure is continuous), the
    same in every row, and nothing along y."""
    p = W.sod2d(N=N, n=16)
    p.shock_thresh = 0.5
    P = O.Problem(p)
    U = p.U0.copy()
    t = 0.0
    while t < tend:
        t += _step(L, P, U)
    _, _, _, info = A.riemann_sample(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, [0.0])
    xs = 0.5 + info["right_shock"] * t
    F = _global(p, _flags(L, P, U, 0))[0]
    xc = (np.arange(N) + 0.5) / N
    cols = np.flatnonzero(F[0])
    assert len(cols) >= 1
    assert np.all(np.abs(xc[cols] - xs) * N <= 3.0), (xc[cols], xs)
    assert np.min(np.abs(xc[cols] - xs)) * N <= 1.0
    assert all(np.array_equal(F[j], F[0]) for j in range(N))
    assert not np.any(_flags(L, P, U, 1))


def test_detector_flags_the_sod_shock_only():
    _sod_flag_check(O.lib())


def _sedov_flag_check(L, nsteps=40):
    """Sedov 32^3 with the detector: flags sit in a shell at the shock (at
    least one within two cells of the similarity radius along each axis
    direction, none in the expanding interior inside 0.75 R), mirror
    symmetric about the centre along every axis bit for bit (the detector
    compares the two neighbours symmetrically), equally many along x, y, z."""
    gold = json.load(open(os.path.join(HERE, "golden", "sedov_constant.json")))
    p = W.sedov3d(N=32, n=16)
    p.shock_thresh = 0.5
    P = O.Problem(p)
    U = p.U0.copy()
    t = 0.0
    for _ in range(nsteps):
        t += _step(L, P, U)
    R = A.sedov_radius(1.0, t, 1.0, gold["xi0"])
    xc = (np.arange(32) + 0.5) / 32 - 0.5
    r = np.sqrt(xc[:, None, None] ** 2 + xc[None, :, None] ** 2 + xc[None, None, :] ** 2)
    counts = []
    for d in range(3):
        F = _global(p, _flags(L, P, U, d))
        counts.append(int(F.sum()))
        assert not np.any(F[r < 0.75 * R])
        assert np.any(F[np.abs(r - R) <= 2.0 / 32])
        axis = 2 - d                                  # global arrays are (z, y, x)
        assert np.array_equal(F, np.flip(F, axis=axis))
    assert counts[0] == counts[1] == counts[2] > 0


def test_detector_flags_the_sedov_front_symmetrically():
    _sedov_flag_check(O.lib())


def test_detector_faces_are_first_order_along_the_flagged_direction_only():
    """On a random periodic state with many pressure jumps: a cell flagged
    along d has both faces along d equal to its own primitives, bit for bit;
    every other cell's faces along d are those of the plain reconstruction;
    the flags along d and along the other directions differ."""
    p = W.random_blocks(3, 8, 3, seed=14, recon=W.WENO5, rk=3)
    q = p.copy()
    q.shock_thresh = 0.2
    U = p.U0.copy()
    O.fill_guards(p, U)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    Wp = np.full((5, p.ncell), np.nan)
    Wp[:, m] = O.eos(p, U[:, m].T.copy())[0].T
    flags = [O.shock_flags(q, U, d) for d in range(3)]
    for d in range(3):
        qm0, qp0, fb0 = O.faces(p, U, d)
        qm1, qp1, fb1 = O.faces(q, U, d)
        f = flags[d].astype(bool) & m
        assert f.sum() > 50
        for v in range(5):
            assert np.array_equal(qm1[v, f], Wp[v, f]) and np.array_equal(qp1[v, f], Wp[v, f])
        rest = m & ~f
        assert np.array_equal(qm1[:, rest], qm0[:, rest]) and np.array_equal(qp1[:, rest], qp0[:, rest])
        assert np.array_equal(fb1.astype(bool)[m], (fb0.astype(bool) | f)[m])
    assert not np.array_equal(flags[0], flags[1]) and not np.array_equal(flags[1], flags[2])


def test_detector_inert_threshold_is_the_plain_step():
    p = W.random_blocks(3, 8, 3, seed=15, recon=W.WENO5, rk=3)
    U, V = p.U0.copy(), p.U0.copy()
    dts = O.run(p, U, 2)
    q = p.copy()
    q.shock_thresh = 1e300
    O.run(q, V, 2, dts)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(U[:, m], V[:, m])


def test_detector_conserves_and_keeps_free_stream():
    p = W.random_blocks(3, 8, 3, seed=16, recon=W.WENO5, rk=3)
    p.shock_thresh = 0.1
    m = W.interior_mask(p.blocks, p.ncell, 3)
    U = p.U0.copy()
    tot = [math.fsum(U[v, m]) for v in range(5)]
    O.run(p, U, 3)
    for v in range(5):
        scale = math.fsum(np.abs(U[v, m]))
        assert abs(math.fsum(U[v, m]) - tot[v]) <= 1e-13 * scale
    f = W.free_fall(3, n=8, ng=3, recon=W.WENO5, rk=3)
    f.grav = None
    f.shock_thresh = 0.0
    V = f.U0.copy()
    O.run(f, V, 2)
    mf = W.interior_mask(f.blocks, f.ncell, 3)
    assert np.array_equal(V[:, mf], f.U0[:, mf])


def test_sod_with_the_detector_converges():
    errs = []
    for N in (64, 128):
        p = W.sod2d(N=N, n=16)
        p.shock_thresh = 0.5
        U = p.U0.copy()
        t = 0.0
        while t < 0.15:
            t += O.step(p, U)
        G = W.gather_global(U, p.blocks, p.grid, 2)[:, 0]
        xc = (np.arange(N) + 0.5) / N
        rho, _, _, _ = A.riemann_sample(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (xc - 0.5) / t)
        errs.append(float(np.mean(np.abs(G[0][N // 2] - rho))))
    assert errs[1] < errs[0] / 1.4, errs


# ------------------------------------------------------------------ adjoint

@pytest.mark.parametrize("ndim,recon,rk", [(2, 0, 2), (3, 1, 3)])
def test_step_vjp_with_gravity_and_detector_dot_product(ndim, recon, rk):
    """<w, J v> = <J^T w, v> for whole steps with gravity and the detector
    on, J v from the complex-step derivative of the forward code (the
    detector's branches decided on real parts, as the fallback's)."""
    p = W.random_blocks(ndim, 8 if ndim == 2 else 6, 3 if recon else 2, seed=17, recon=recon, rk=rk,
                        bc="outflow")
    p.grav = (0.8, -1.2, 0.3)
    p.shock_thresh = 0.2
    U = p.U0
    dt = O.cfl_dt(p, U)
    Ug = U.copy()
    O.fill_guards(p, Ug)
    assert sum(int(O.shock_flags(p, Ug, d).sum()) for d in range(ndim)) > 10
    rng = np.random.default_rng(18)
    m = np.isfinite(U)
    for _ in range(3):
        V = np.where(m, rng.standard_normal(U.shape), 0.0)
        Wt = np.where(m, rng.standard_normal(U.shape), 0.0)
        _, Jv = O.step_cs(p, U, V, dt)
        g = O.step_vjp(p, U, dt, Wt)
        a, b = np.sum(Wt[m] * Jv[m]), np.sum(g[m] * V[m])
        assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


# ---------------------------------------------------------------- mutations

_SRC = {
    "shock_du": "    REAL du = w[5 + 1 + d] - w[-5 + 1 + d];",
    "shock_jump": "    REAL jump = RABS(pb - pa);",
    "shock_store": "                    flag[d * np + li] = (unsigned char)FN(shock_flag)(P, &W[5 * (t + 2)], d);",
    "grav_energy": "                        REAL mg = Us[1 * nc + ci] * g[0] + Us[2 * nc + ci] * g[1];",
    "grav_rho": "                        REAL rho = Us[ci];",
}

MUTATIONS = {
    # expansion flagged instead of compression
    "detector_expansion": ("shock_du", "    REAL du = w[-5 + 1 + d] - w[5 + 1 + d];"),
    # one-sided pressure jump (next cell against the cell itself)
    "detector_one_sided_jump": ("shock_jump", "    REAL jump = RABS(pb - w[4]);"),
    # one flag per cell shared by every direction
    "detector_one_flag_per_cell": ("shock_store",
                                   "                    flag[li] = (unsigned char)FN(shock_flag)(P, &W[5 * (t + 2)], d);"),
    # energy source from the velocity instead of the momentum
    "gravity_energy_from_velocity": ("grav_energy",
                                     "                        REAL mg = (Us[1 * nc + ci] / Us[ci]) * g[0] + "
                                     "(Us[2 * nc + ci] / Us[ci]) * g[1];"),
    # source from the step's initial state instead of the stage's
    "gravity_from_step_start": ("grav_rho", "                        REAL rho = Un[ci];"),
}


def _check_all(L):
    _free_fall_check(L, 2, 0, 2)
    _free_fall_check(L, 3, 1, 3)
    _sod_flag_check(L, N=64, tend=0.1)
    _sedov_flag_check(L)


def test_pins_pass_on_the_oracle_itself():
    _check_all(O.lib())


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_a_mutated_step(name, tmp_path):
    key, repl = MUTATIONS[name]
    src = open(os.path.join(ORACLE_DIR, "forward_body.inc")).read()
    assert src.count(_SRC[key]) == 1, "the oracle's source changed: update the mutations"
    mutated = src.replace(_SRC[key], repl)
    if name == "gravity_from_step_start":
        # the momentum and energy terms of the source too
        mutated = mutated.replace("REAL mg = Us[1 * nc + ci] * g[0] + Us[2 * nc + ci] * g[1];",
                                  "REAL mg = Un[1 * nc + ci] * g[0] + Un[2 * nc + ci] * g[1];")
        mutated = mutated.replace("if (nd == 3) mg = mg + Us[3 * nc + ci] * g[2];",
                                  "if (nd == 3) mg = mg + Un[3 * nc + ci] * g[2];")
    for f in ("oracle.c", "oracle_cs.c", "oracle_amr.c", "oracle.h"):
        shutil.copy(os.path.join(ORACLE_DIR, f), tmp_path / f)
    (tmp_path / "forward_body.inc").write_text(mutated)
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                    "-std=gnu11", "-o", str(lib), "oracle.c", "oracle_cs.c", "oracle_amr.c", "-lm"],
                   check=True, cwd=tmp_path, capture_output=True)
    with pytest.raises(AssertionError):
        _check_all(C.CDLL(str(lib)))


def test_mesh_with_levels_refuses_gravity_and_detector():
    for attr, val in (("grav", (0.0, 1.0, 0.0)), ("shock_thresh", 0.5)):
        q = W.amr_problem(2, n=8, ng=2, recon=0, rk=2)
        assert O.amr_validate(q) == O.ORA_OK
        setattr(q, attr, val)
        assert O.amr_validate(q) == O.ORA_EINVAL
