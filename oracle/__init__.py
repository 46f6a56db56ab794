"""CPU oracle for the block-structured compressible-Euler step.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  It shares no code with
the GPU path; the two meet only in the seeded inputs.

The oracle follows the method step by step in plain FP64 C (see oracle.h for
the passages of the paper it follows and the textbook formulas it uses); this
module only marshals numpy arrays into it.  Problems are duck-typed: any
object with ndim, recon, rk, gamma, cfl, dx, dy, dz, blocks (structured array
nx, ny, nz, ng, offset), links (structured array nbr[6]) and ncell.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ORA_OK, ORA_EINVAL, ORA_ENONPHYS, ORA_ENOMEM = 0, -1, -3, -4
# Epsilon of the WENO5 nonlinear weights in Jiang & Shu (1996); a problem may
# carry its own (attribute weno_eps).
WENO_EPS = 1e-6
# Optional physics: a uniform gravitational acceleration (attribute grav, a
# 3-vector, or None) and the shock detector (attribute shock_thresh, or None).
ORA_GRAVITY, ORA_SHOCK = 1, 2


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what}: error {code}")
        self.code = code


class _Block(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("ng", C.c_int32), ("offset", C.c_int64)]


class _Link(C.Structure):
    _fields_ = [("nbr", C.c_int32 * 6)]


class _Amr(C.Structure):
    _fields_ = [("level", C.c_int32), ("kind", C.c_int32 * 6), ("nbr", (C.c_int32 * 4) * 6)]


class _Problem(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("recon", C.c_int32), ("rk", C.c_int32),
                ("nblocks", C.c_int32), ("ncell", C.c_int64),
                ("gamma", C.c_double), ("cfl", C.c_double), ("dx", C.c_double),
                ("dy", C.c_double), ("dz", C.c_double),
                ("blocks", C.c_void_p), ("links", C.c_void_p), ("weno_eps", C.c_double),
                ("grav", C.c_double * 3), ("shock_thresh", C.c_double), ("phys", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _build.needs_build():
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        i64 = C.c_int64
        sig = {
            "ora_validate": (C.c_int, [P]),
            "ora_fill_guards": (C.c_int, [P, dp]),
            "ora_cfl_dt": (C.c_int, [P, dp, dp]),
            "ora_rk_stage": (C.c_int, [P, C.c_int, C.c_double, dp, dp, dp]),
            "ora_step": (C.c_int, [P, dp, dp, C.c_int]),
            "ora_step_vjp": (C.c_int, [P, dp, C.c_double, dp, dp]),
            "ora_step_telescoping": (C.c_int, [P, dp, dp, C.c_int]),
            "ora_cs_step": (C.c_int, [P, dp, dp, C.c_double]),
            "ora_eos_n": (C.c_int, [P, i64, dp, dp]),
            "ora_plm_n": (None, [i64, dp, dp, dp, ip]),
            "ora_weno5_n": (None, [i64, dp, C.c_double, dp, dp]),
            "ora_recon_cell_n": (None, [P, i64, dp, dp, dp, ip]),
            "ora_faces": (C.c_int, [P, dp, C.c_int, dp, dp, ip]),
            "ora_shock_flags": (C.c_int, [P, dp, C.c_int, ip]),
            "ora_hllc_n": (C.c_int, [P, i64, C.c_int, dp, dp, dp, ip]),
            "ora_state_flux_n": (None, [P, i64, C.c_int, dp, dp, dp, dp]),
            "ora_eos_vjp_n": (None, [P, i64, dp, dp, dp]),
            "ora_plm_vjp_n": (None, [i64, dp, dp, dp, dp]),
            "ora_weno5_vjp_n": (None, [i64, dp, C.c_double, dp, dp, dp]),
            "ora_hllc_vjp_n": (None, [P, i64, C.c_int, dp, dp, dp, dp, dp]),
            "ora_cs_eos_n": (None, [P, i64, dp, dp, dp, dp]),
            "ora_cs_plm_n": (None, [i64, dp, dp, dp, dp, dp, dp]),
            "ora_cs_weno5_n": (None, [i64, dp, dp, C.c_double, dp, dp, dp, dp]),
            "ora_cs_hllc_n": (None, [P, i64, C.c_int, dp, dp, dp, dp, dp, dp]),
            "ora_amr_validate": (C.c_int, [P, C.c_void_p]),
            "ora_amr_fill_guards": (C.c_int, [P, C.c_void_p, dp]),
            "ora_amr_cfl_dt": (C.c_int, [P, C.c_void_p, dp, dp]),
            "ora_amr_step": (C.c_int, [P, C.c_void_p, dp, dp, C.c_int, C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_int))


class Problem:
    """ctypes view of a problem description (keeps its arrays alive)."""

    def __init__(self, prob, **override):
        get = lambda k: override.get(k, getattr(prob, k))
        self.ndim = int(get("ndim"))
        self.nvar = self.ndim + 2
        self.ncell = int(get("ncell"))
        blocks = np.ascontiguousarray(get("blocks"))
        links = np.ascontiguousarray(get("links"))
        self._blocks = (_Block * max(len(blocks), 1))()
        for i, b in enumerate(blocks):
            self._blocks[i] = _Block(int(b["nx"]), int(b["ny"]), int(b["nz"]),
                                     int(b["ng"]), int(b["offset"]))
        self._links = (_Link * max(len(links), 1))()
        for i, l in enumerate(links):
            for f in range(6):
                self._links[i].nbr[f] = int(l["nbr"][f])
        amr = override.get("amr", getattr(prob, "amr", None))
        self._amr = None
        if amr is not None:
            amr = np.ascontiguousarray(amr)
            self._amr = (_Amr * max(len(amr), 1))()
            for i, a in enumerate(amr):
                self._amr[i].level = int(a["level"])
                for f in range(6):
                    self._amr[i].kind[f] = int(a["kind"][f])
                    for h in range(4):
                        self._amr[i].nbr[f][h] = int(a["nbr"][f][h])
        self.c = _Problem(self.ndim, int(get("recon")), int(get("rk")), len(blocks),
                          self.ncell, float(get("gamma")), float(get("cfl")),
                          float(get("dx")), float(get("dy")), float(get("dz")),
                          C.cast(self._blocks, C.c_void_p), C.cast(self._links, C.c_void_p),
                          float(override.get("weno_eps", getattr(prob, "weno_eps", WENO_EPS))))
        grav = override.get("grav", getattr(prob, "grav", None))
        thresh = override.get("shock_thresh", getattr(prob, "shock_thresh", None))
        if grav is not None:
            g = [float(x) for x in grav] + [0.0] * (3 - len(grav))
            for d in range(3):
                self.c.grav[d] = g[d]
            self.c.phys |= ORA_GRAVITY
        if thresh is not None:
            self.c.shock_thresh = float(thresh)
            self.c.phys |= ORA_SHOCK

    @property
    def ptr(self):
        return C.byref(self.c)


def _as_problem(prob):
    return prob if isinstance(prob, Problem) else Problem(prob)


def _check(rc, what):
    if rc != ORA_OK:
        raise OracleError(rc, what)


def validate(prob) -> int:
    return lib().ora_validate(_as_problem(prob).ptr)


def fill_guards(prob, U):
    P = _as_problem(prob)
    _check(lib().ora_fill_guards(P.ptr, _dp(U)), "fill_guards")


def cfl_dt(prob, U) -> float:
    P = _as_problem(prob)
    dt = np.zeros(1)
    _check(lib().ora_cfl_dt(P.ptr, _dp(U), _dp(dt)), "cfl_dt")
    return float(dt[0])


def rk_stage(prob, stage, dt, Un, Us, Uout):
    P = _as_problem(prob)
    _check(lib().ora_rk_stage(P.ptr, int(stage), float(dt), _dp(Un), _dp(Us), _dp(Uout)), "rk_stage")


def step(prob, U, dt=None) -> float:
    """One step in place; returns the dt used (CFL dt when dt is None)."""
    P = _as_problem(prob)
    d = np.array([0.0 if dt is None else float(dt)])
    _check(lib().ora_step(P.ptr, _dp(U), _dp(d), 1 if dt is None else 0), "step")
    return float(d[0])


def step_telescoping(prob, U, dt=None) -> float:
    """One telescoping step in place (one thick guard fill per step, stages
    updated on the shrinking extended region); returns the dt used."""
    P = _as_problem(prob)
    d = np.array([0.0 if dt is None else float(dt)])
    _check(lib().ora_step_telescoping(P.ptr, _dp(U), _dp(d), 1 if dt is None else 0), "step_telescoping")
    return float(d[0])


# ------------------------------------------------------------------- AMR

AMR_ALL_LEVELS, AMR_LEVEL_BY_LEVEL, AMR_NO_CORRECTION = 0, 1, 2


def _amr_args(prob):
    P = _as_problem(prob)
    if P._amr is None:
        raise ValueError("problem has no AMR table")
    return P, C.cast(P._amr, C.c_void_p)


def amr_validate(prob) -> int:
    P, A = _amr_args(prob)
    return lib().ora_amr_validate(P.ptr, A)


def amr_fill_guards(prob, U):
    P, A = _amr_args(prob)
    _check(lib().ora_amr_fill_guards(P.ptr, A, _dp(U)), "amr_fill_guards")


def amr_cfl_dt(prob, U) -> float:
    P, A = _amr_args(prob)
    dt = np.zeros(1)
    _check(lib().ora_amr_cfl_dt(P.ptr, A, _dp(U), _dp(dt)), "amr_cfl_dt")
    return float(dt[0])


def amr_step(prob, U, dt=None, order=AMR_ALL_LEVELS) -> float:
    """One step on a mesh with refinement levels, in place; order: flux
    correction for all levels at once, level by level, or (a check only)
    none.  Returns the dt used."""
    P, A = _amr_args(prob)
    d = np.array([0.0 if dt is None else float(dt)])
    _check(lib().ora_amr_step(P.ptr, A, _dp(U), _dp(d), 1 if dt is None else 0, int(order)), "amr_step")
    return float(d[0])


def amr_run(prob, U, nsteps, order=AMR_ALL_LEVELS, dts=None):
    P = _as_problem(prob)
    return [amr_step(P, U, None if dts is None else dts[n], order) for n in range(nsteps)]


def run(prob, U, nsteps, dts=None):
    """nsteps steps in place; returns the list of dts (given or computed)."""
    P = _as_problem(prob)
    out = []
    for n in range(nsteps):
        out.append(step(P, U, None if dts is None else dts[n]))
    return out


def step_vjp(prob, Un, dt, gUnext):
    """Cotangent of U^n for one step at fixed dt (padding of the result = 0)."""
    P = _as_problem(prob)
    g = np.zeros_like(Un)
    _check(lib().ora_step_vjp(P.ptr, _dp(Un), float(dt), _dp(np.ascontiguousarray(gUnext)), _dp(g)),
           "step_vjp")
    return g


def step_cs(prob, U, V, dt, h=1e-30):
    """Complex-step directional derivative of one step at fixed dt.

    Returns (U^{n+1}, J V) with J = dU^{n+1}/dU^n."""
    P = _as_problem(prob)
    re = U.copy()
    im = np.where(np.isnan(U), 0.0, V * h)
    _check(lib().ora_cs_step(P.ptr, _dp(re), _dp(im), float(dt)), "cs_step")
    return re, im / h


# ---------------------------------------------------------------- pieces

def eos(prob, U):
    """U: (n, nvar) -> W: (n, 5) = (rho, ux, uy, uz, p); returns (W, nbad)."""
    P = _as_problem(prob)
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.zeros((U.shape[0], 5))
    bad = lib().ora_eos_n(P.ptr, U.shape[0], _dp(U), _dp(W))
    return W, bad


def plm(q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0]
    qm, qp, code = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int32)
    lib().ora_plm_n(n, _dp(q), _dp(qm), _dp(qp), _ip(code))
    return qm, qp, code


def weno5(q, eps=None):
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0]
    qm, qp = np.zeros(n), np.zeros(n)
    lib().ora_weno5_n(n, _dp(q), WENO_EPS if eps is None else float(eps), _dp(qm), _dp(qp))
    return qm, qp


def recon_cell(prob, w):
    """Reconstruction of cells along a line with the positivity fallback:
    w (n, 2R+1, 5) stencil primitives per cell (R = 1 PLM-MC, 2 WENO5) ->
    (qm, qp) (n, 5) left/right face values and fb (n,) fallback flags."""
    P = _as_problem(prob)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = w.shape[0]
    qm, qp, fb = np.zeros((n, 5)), np.zeros((n, 5)), np.zeros(n, dtype=np.int32)
    lib().ora_recon_cell_n(P.ptr, n, _dp(w), _dp(qm), _dp(qp), _ip(fb))
    return qm, qp, fb


def faces(prob, U, direction):
    """Face values along a direction of every interior cell of a guard-filled
    state U: (qm, qp) (5, ncell) primitives (NaN outside the interior) and
    fb (ncell,) where the positivity fallback fired."""
    P = _as_problem(prob)
    U = np.ascontiguousarray(U, dtype=np.float64)
    qm = np.full((5, P.ncell), np.nan)
    qp = np.full((5, P.ncell), np.nan)
    fb = np.zeros(P.ncell, dtype=np.int32)
    _check(lib().ora_faces(P.ptr, _dp(U), int(direction), _dp(qm), _dp(qp), _ip(fb)), "faces")
    return qm, qp, fb


def shock_flags(prob, U, direction, thresh=None):
    """The shock detector's flags along a direction (the block initialisation
    of a stage) for every interior cell of a guard-filled state U: (ncell,)
    int32, 1 where flagged (0 elsewhere, padding included).  thresh
    overrides the problem's shock_thresh."""
    over = {} if thresh is None else {"shock_thresh": thresh}
    P = prob if (isinstance(prob, Problem) and not over) else Problem(prob, **over)
    U = np.ascontiguousarray(U, dtype=np.float64)
    flag = np.zeros(P.ncell, dtype=np.int32)
    _check(lib().ora_shock_flags(P.ptr, _dp(U), int(direction), _ip(flag)), "shock_flags")
    return flag


def hllc(prob, WL, WR, direction):
    P = _as_problem(prob)
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    n = WL.shape[0]
    F = np.zeros((n, P.nvar))
    tape = np.zeros(n, dtype=np.int32)
    bad = lib().ora_hllc_n(P.ptr, n, int(direction), _dp(WL), _dp(WR), _dp(F), _ip(tape))
    return F, tape, bad


def state_flux(prob, W, direction):
    P = _as_problem(prob)
    W = np.ascontiguousarray(W, dtype=np.float64)
    n = W.shape[0]
    U, F, c = np.zeros((n, P.nvar)), np.zeros((n, P.nvar)), np.zeros(n)
    lib().ora_state_flux_n(P.ptr, n, int(direction), _dp(W), _dp(U), _dp(F), _dp(c))
    return U, F, c


def eos_vjp(prob, U, gW):
    P = _as_problem(prob)
    U = np.ascontiguousarray(U, dtype=np.float64)
    gW = np.ascontiguousarray(gW, dtype=np.float64)
    gU = np.zeros_like(U)
    lib().ora_eos_vjp_n(P.ptr, U.shape[0], _dp(U), _dp(gW), _dp(gU))
    return gU


def plm_vjp(q, gqm, gqp):
    q = np.ascontiguousarray(q, dtype=np.float64)
    gq = np.zeros_like(q)
    lib().ora_plm_vjp_n(q.shape[0], _dp(q), _dp(np.ascontiguousarray(gqm, dtype=np.float64)),
                        _dp(np.ascontiguousarray(gqp, dtype=np.float64)), _dp(gq))
    return gq


def weno5_vjp(q, gqm, gqp, eps=None):
    q = np.ascontiguousarray(q, dtype=np.float64)
    gq = np.zeros_like(q)
    lib().ora_weno5_vjp_n(q.shape[0], _dp(q), WENO_EPS if eps is None else float(eps),
                          _dp(np.ascontiguousarray(gqm, dtype=np.float64)),
                          _dp(np.ascontiguousarray(gqp, dtype=np.float64)), _dp(gq))
    return gq


def hllc_vjp(prob, WL, WR, direction, gF):
    P = _as_problem(prob)
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    gF = np.ascontiguousarray(gF, dtype=np.float64)
    gL, gR = np.zeros_like(WL), np.zeros_like(WR)
    lib().ora_hllc_vjp_n(P.ptr, WL.shape[0], int(direction), _dp(WL), _dp(WR), _dp(gF), _dp(gL), _dp(gR))
    return gL, gR



def eos_cs(prob, U, V, h=1e-30):
    P = _as_problem(prob)
    ur = np.ascontiguousarray(U, dtype=np.float64)
    ui = np.ascontiguousarray(V * h, dtype=np.float64)
    wr, wi = np.zeros((U.shape[0], 5)), np.zeros((U.shape[0], 5))
    lib().ora_cs_eos_n(P.ptr, U.shape[0], _dp(ur), _dp(ui), _dp(wr), _dp(wi))
    return wr, wi / h


def plm_cs(q, v, h=1e-30):
    qr = np.ascontiguousarray(q, dtype=np.float64)
    qi = np.ascontiguousarray(v * h, dtype=np.float64)
    n = q.shape[0]
    mr, mi, pr, pi = (np.zeros(n) for _ in range(4))
    lib().ora_cs_plm_n(n, _dp(qr), _dp(qi), _dp(mr), _dp(mi), _dp(pr), _dp(pi))
    return (mr, mi / h), (pr, pi / h)


def weno5_cs(q, v, h=1e-30, eps=None):
    qr = np.ascontiguousarray(q, dtype=np.float64)
    qi = np.ascontiguousarray(v * h, dtype=np.float64)
    n = q.shape[0]
    mr, mi, pr, pi = (np.zeros(n) for _ in range(4))
    lib().ora_cs_weno5_n(n, _dp(qr), _dp(qi), WENO_EPS if eps is None else float(eps),
                         _dp(mr), _dp(mi), _dp(pr), _dp(pi))
    return (mr, mi / h), (pr, pi / h)


def hllc_cs(prob, WL, WR, direction, VL, VR, h=1e-30):
    P = _as_problem(prob)
    n = WL.shape[0]
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (WL, VL * h, WR, VR * h)]
    fr, fi = np.zeros((n, P.nvar)), np.zeros((n, P.nvar))
    lib().ora_cs_hllc_n(P.ptr, n, int(direction), *[_dp(a) for a in args], _dp(fr), _dp(fi))
    return fr, fi / h
