"""Python front end of the GPU step: device memory and streams from PyTorch,
every computation in libhydro's HIP kernels (through the C ABI)."""
from __future__ import annotations

import ctypes as C
import weakref

import numpy as np
import torch

from . import _hip
from ._hip import HydroError, Tuning


def _ptr(t):
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class CflRecord:
    """Whether a step of U may take its CFL dt from the maxima the previous
    step recorded (HYDRO_DT_FROM_PREVIOUS).  Only when U is the very tensor
    the previous such step wrote: still alive (so its memory cannot have been
    freed and handed to another tensor at the same address) and not written
    through torch since (its version counter is unchanged; the library's own
    writes do not count).  Otherwise the step computes the CFL dt from U and
    records the maxima of the state it writes (HYDRO_DT_RECORD)."""

    def __init__(self):
        self._ref = None
        self._ver = None

    def mode(self, U):
        last = self._ref() if self._ref is not None else None
        if last is U and U._version == self._ver:
            return _hip.HYDRO_DT_FROM_PREVIOUS
        return _hip.HYDRO_DT_RECORD

    def wrote(self, U):
        self._ref = weakref.ref(U)
        self._ver = U._version

    def forget(self):
        self._ref = None
        self._ver = None


class Solver:
    """A problem bound to one GPU and one stream.

    prob: a workload description (ndim, recon, rk, gamma, cfl, dx, dy, dz,
    blocks, links, ncell).  State tensors are float64 (nvar, ncell) on the
    solver's device."""

    def __init__(self, prob, device="cuda", stream=None, tuning=None, level_by_level=False):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the hydro step runs only in its HIP kernels")
        self.prob = prob
        self.device = torch.device(device)
        self.nvar = int(prob.ndim) + 2
        self.ncell = int(prob.ncell)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._L = _hip.lib()
        P, B, L, nb = _hip.tables(prob)
        A = _hip.amr_table(prob)
        ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            if A is None:
                rc = self._L.hydro_create(C.byref(P), B, L, nb, self.ncell,
                                          C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
            else:
                if level_by_level:
                    P.flags |= _hip.FLAG_LEVEL_BY_LEVEL
                rc = self._L.hydro_create_amr(C.byref(P), B, L, A, nb, self.ncell,
                                              C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc != _hip.HYDRO_OK:
            raise HydroError(rc, self._L.hydro_last_error(None).decode())
        self.ctx = ctx
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._cfl = CflRecord()
        if tuning:
            self.set_tuning(**tuning)

    # ------------------------------------------------------------ plumbing
    def _check(self, rc):
        if rc != _hip.HYDRO_OK:
            raise HydroError(rc, self._L.hydro_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self._L.hydro_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def to_device(self, U):
        return torch.as_tensor(np.ascontiguousarray(U), dtype=torch.float64).to(self.device)

    def tuning(self):
        t = Tuning()
        self._check(self._L.hydro_get_tuning(self.ctx, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = Tuning(**cur)
        self._cfl.forget()
        self._check(self._L.hydro_set_tuning(self.ctx, C.byref(t)))

    # ------------------------------------------------------------ the method
    def fill_guards(self, U):
        self._check(self._L.hydro_fill_guards(self.ctx, _ptr(U)))

    def cfl_dt(self, U, out=None):
        out = self.dt if out is None else out
        self._check(self._L.hydro_cfl_dt(self.ctx, _ptr(U), _ptr(out)))
        return out

    def rk_stage(self, stage, Un, Us, Uout, dt=None):
        dt = self.dt if dt is None else dt
        self._cfl.forget()
        self._check(self._L.hydro_rk_stage(self.ctx, int(stage), _ptr(dt), _ptr(Un), _ptr(Us), _ptr(Uout)))

    def step(self, U, dt=None, dt_from_previous=False):
        """One step in place.  dt None: CFL dt (left in self.dt); a float or a
        device tensor: that dt.  dt_from_previous (with dt None): the same dt,
        taken from the maxima the previous such step recorded when U is the
        tensor it wrote and nothing has written it since (CflRecord); else
        computed from U and recorded for the next step."""
        if dt is None:
            mode = self._cfl.mode(U) if dt_from_previous else 1
            self._cfl.forget()
            self._check(self._L.hydro_step(self.ctx, _ptr(U), _ptr(self.dt), mode))
            if dt_from_previous:
                self._cfl.wrote(U)
            return self.dt
        self._cfl.forget()
        if not torch.is_tensor(dt):
            self.dt.fill_(float(dt))
            dt = self.dt
        self._check(self._L.hydro_step(self.ctx, _ptr(U), _ptr(dt), 0))
        return dt

    def run(self, U, nsteps, record_dt=True, dt_from_previous=False):
        """nsteps CFL steps in place; returns the dts (device tensor)."""
        dts = torch.empty(nsteps, dtype=torch.float64, device=self.device)
        for n in range(nsteps):
            self.step(U, dt_from_previous=dt_from_previous)
            if record_dt:
                dts[n:n + 1].copy_(self.dt)
        return dts

    def _dt_tensor(self, dt):
        if torch.is_tensor(dt):
            return dt
        return torch.full((1,), float(dt), dtype=torch.float64, device=self.device)

    def step_keep(self, Un, dt, out=None):
        """One step at dt out of place, stage by stage (hydro_rk_stage):
        returns (U^{n+1}, [U_2 .. U_S]), the stage inputs as step_vjp takes
        them.  Un is not changed (in the per-block and materialised modes,
        whose stages write the guard cells of their input, the first stage
        reads a copy of it).  U^{n+1} is written into the interior of out if
        given (its guard cells are left as they are), else into a new tensor
        whose guard cells are unspecified, as are the stage inputs'."""
        if out is not None and out.data_ptr() == Un.data_ptr():
            raise ValueError("out must not alias Un (step_keep leaves Un as it is)")
        d = self._dt_tensor(dt)
        S = int(self.prob.rk)
        stages = []
        Us = Un
        if self.tuning()["mode"] in (_hip.MODE_PERBLOCK, _hip.MODE_MATERIALISED):
            Us = Un.clone()
        for s in range(1, S):
            buf = torch.empty_like(Un)
            self.rk_stage(s, Un, Us, buf, d)
            stages.append(buf)
            Us = buf
        Unext = torch.empty_like(Un) if out is None else out
        self.rk_stage(S, Un, Us, Unext, d)
        return Unext, stages

    def step_vjp(self, Un, gUnext, dt, gUn=None, stages=None):
        """gUn = (dU^{n+1}/dU^n)^T gUnext at fixed dt.  stages: the stage
        inputs [U_2 .. U_S] of this step (from step_keep), used in place of
        recomputing them."""
        d = self._dt_tensor(dt)
        gUn = torch.empty_like(Un) if gUn is None else gUn
        if stages is None:
            self._check(self._L.hydro_step_vjp(self.ctx, _ptr(Un), _ptr(d), _ptr(gUnext), _ptr(gUn)))
            return gUn
        S = int(self.prob.rk)
        if len(stages) != S - 1:
            raise ValueError(f"{S - 1} stage inputs expected, got {len(stages)}")
        arr = (C.c_void_p * (S - 1))(*[_ptr(t) for t in stages])
        self._check(self._L.hydro_step_vjp_stages(self.ctx, _ptr(Un), arr, _ptr(d), _ptr(gUnext), _ptr(gUn)))
        return gUn

    def status(self):
        n = C.c_int64(0)
        rc = self._L.hydro_status(self.ctx, C.byref(n))
        if rc != _hip.HYDRO_OK:
            raise HydroError(rc, self._L.hydro_last_error(self.ctx).decode())
        return 0
