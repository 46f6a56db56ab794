"""Differentiation of the hydro step: a torch.autograd.Function per step and
a checkpointed multi-step rollout.

The gradient is taken with every dt held fixed (the dt sequence of the
forward pass is recorded and replayed) and with the branches of the forward
pass (limiter slopes, positivity fallback, Riemann-solver region); the
per-step transpose is the library's hydro_step_vjp.

Checkpointing: the forward rollout stores the state every k steps; the
backward pass walks the segments in reverse, recomputes a segment's step
inputs from its checkpoint, then applies the step VJPs in reverse.  Memory is
(N/k + k) states instead of N, plus the stage inputs of the recomputed steps
(S-1 states each), which their VJPs then need not recompute.  The rollout
logic is written against a small stepper interface (step / step_vjp / copy,
optionally step_keep) so that it can be exercised with any implementation of
a step.
"""
from __future__ import annotations

import torch

from . import _hip


class Tape:
    """What a checkpointed forward rollout keeps: states every k steps and
    every dt."""

    def __init__(self, k):
        self.k = k
        self.checkpoints = {}   # step index -> state before that step
        self.dts = []
        self.tail = {}          # step index -> (state before it, kept data), last segment
        self.recomputed_steps = 0


def rollout(stepper, U0, nsteps, k, dts=None, keep_last=False):
    """Advance a copy of U0 by nsteps; returns (U_N, tape).  dts: optional
    fixed time steps; otherwise each step takes its CFL dt (recorded).

    keep_last (for a stepper with step_keep): the steps of the last segment
    run out of place and the tape keeps their inputs and kept data, which the
    backward pass would otherwise recompute first and then hold at once
    anyway; it uses them and releases them.  Without a backward pass this
    holds k states and their kept data for nothing."""
    if k < 1:
        raise ValueError("checkpoint interval must be >= 1")
    tape = Tape(k)
    keep = getattr(stepper, "step_keep", None) if keep_last else None
    last = ((nsteps - 1) // k) * k
    U = stepper.copy(U0)
    for n in range(nsteps):
        dtn = None if dts is None else dts[n]
        if keep is not None and n >= last:
            # out of place from here on: U itself is the checkpoint
            if n == last:
                tape.checkpoints[n] = U
            # the returned state takes its guard cells from U0, as in place:
            # the segment's checkpoint holds them (it was stepped in place;
            # the states step_keep returns in between have unspecified guards)
            out = stepper.copy(tape.checkpoints[last]) if n == nsteps - 1 else None
            Unext, aux, dt = keep(U, dtn, out)
            tape.tail[n] = (U, aux)
            U = Unext
        else:
            if n % k == 0:
                tape.checkpoints[n] = stepper.copy(U)
            dt = stepper.step(U, dtn)
        tape.dts.append(float(dt))
    return U, tape


def rollout_vjp(stepper, tape, gUN):
    """Cotangent of U0 given the cotangent of U_N, by segments in reverse.

    A stepper with step_keep(Un, dt, out=None) -> (U^{n+1}, kept, dt)
    (U^{n+1} in out if given, else in a new state) recomputes a
    segment's steps out of place and keeps what step_vjp(Un, g, dt, kept)
    would otherwise recompute (the stage inputs); the last step of a segment
    is not recomputed forward, so its VJP recomputes its own (except in a
    last segment kept by the forward pass).  A kept last segment is used once:
    the tape then falls back to recomputing it."""
    nsteps = len(tape.dts)
    keep = getattr(stepper, "step_keep", None)
    g = gUN
    starts = sorted(tape.checkpoints)
    for s0 in reversed(starts):
        s1 = min(s0 + tape.k, nsteps)
        if s0 in tape.tail:
            # the last segment as the forward pass kept it
            states = [tape.tail[n][0] for n in range(s0, s1)]
            kept = [tape.tail[n][1] for n in range(s0, s1)]
            tape.tail = {}
        else:
            # recompute the inputs of steps s0 .. s1-1; step_keep leaves its
            # input as it is, so the checkpoint itself serves
            ck = tape.checkpoints[s0]
            states = [ck if keep is not None else stepper.copy(ck)]
            kept = []
            for n in range(s0, s1 - 1):
                if keep is None:
                    U = stepper.copy(states[-1])
                    stepper.step(U, tape.dts[n])
                    kept.append(None)
                else:
                    U, aux, _ = keep(states[-1], tape.dts[n])
                    kept.append(aux)
                tape.recomputed_steps += 1
                states.append(U)
            kept.append(None)
        for n in range(s1 - 1, s0 - 1, -1):
            i = n - s0
            if kept[i] is None:
                g = stepper.step_vjp(states[i], g, tape.dts[n])
            else:
                g = stepper.step_vjp(states[i], g, tape.dts[n], kept[i])
            states[i] = kept[i] = None
    return g


class TorchStepper:
    """Stepper over a Solver (GPU tensors)."""

    def __init__(self, solver):
        self.S = solver

    def copy(self, U):
        return U.clone()

    def step(self, U, dt=None):
        # a rollout steps one state in place: its CFL dt can come from the
        # maxima the previous step recorded (the same dt, bit for bit); the
        # solver allows that only for the tensor that step wrote, so the first
        # step of a rollout (a fresh copy of U0) computes its dt from U
        d = self.S.step(U, dt, dt_from_previous=dt is None)
        return float(d.item()) if torch.is_tensor(d) else float(d)

    def step_keep(self, Un, dt=None, out=None):
        if dt is None:
            dt = float(self.S.cfl_dt(Un).item())
        Unext, stages = self.S.step_keep(Un, dt, out)
        return Unext, stages, dt

    def step_vjp(self, Un, g, dt, stages=None):
        return self.S.step_vjp(Un, g.contiguous(), dt, stages=stages)


class HydroStep(torch.autograd.Function):
    """U_{n+1} = step(U_n) at a given dt, run stage by stage so that the
    stage inputs are saved (S-1 states besides U_n); backward =
    hydro_step_vjp_stages on them.  The output's guard cells are U_n's."""

    @staticmethod
    def forward(ctx, U, dt, solver):
        Un = U.detach()
        if solver.tuning()["mode"] == _hip.MODE_TELESCOPING:
            # no single stages in this mode (and no VJP: backward raises)
            out = Un.clone()
            solver.step(out, float(dt))
            stages = []
        else:
            out, stages = solver.step_keep(Un, float(dt), out=Un.clone())
        ctx.save_for_backward(Un, *stages)
        ctx.dt = float(dt)
        ctx.solver = solver
        return out

    @staticmethod
    def backward(ctx, g):
        U, *stages = ctx.saved_tensors
        return ctx.solver.step_vjp(U, g.contiguous(), ctx.dt, stages=list(stages) or None), None, None


class HydroRollout(torch.autograd.Function):
    """U_N after nsteps CFL steps, with a checkpointed backward pass."""

    @staticmethod
    def forward(ctx, U0, solver, nsteps, k):
        st = TorchStepper(solver)
        UN, tape = rollout(st, U0.detach(), nsteps, k, keep_last=True)
        ctx.stepper = st
        ctx.tape = tape
        return UN

    @staticmethod
    def backward(ctx, g):
        return rollout_vjp(ctx.stepper, ctx.tape, g.contiguous()), None, None, None


def hydro_step(U, dt, solver):
    return HydroStep.apply(U, dt, solver)


def hydro_rollout(U0, solver, nsteps, k):
    return HydroRollout.apply(U0, solver, nsteps, k)


def time_rollouts(cases=((3, 50, 10), (1, 20, 5), (4, 10, 5))):
    """Cost of the checkpointed adjoint against the forward rollout, for
    (workload index, steps, checkpoint interval) cases; one JSON line each."""
    import json
    import time

    from . import autotune
    from . import workloads as W
    from .solver import Solver

    out = []
    for ci, nsteps, k in cases:
        p = W.config(ci)
        S = Solver(p)
        autotune.tuned_or_search(S, p, log=lambda *a: None)
        st = TorchStepper(S)
        U0 = S.to_device(p.U0)
        # warm-up rollout of the same shape (graph capture, VJP scratch, allocator)
        UN, tape = rollout(st, U0, nsteps, k, keep_last=True)
        rollout_vjp(st, tape, torch.nan_to_num(UN).clone())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        UN, tape = rollout(st, U0, nsteps, nsteps + 1)   # forward only (one checkpoint)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        UN, tape = rollout(st, U0, nsteps, k, keep_last=True)
        rollout_vjp(st, tape, torch.nan_to_num(UN).clone())
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        dt = tape.dts[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            S.step_vjp(U0, torch.nan_to_num(U0), dt)
        torch.cuda.synchronize()
        tv = (time.perf_counter() - t0) / 3
        S.status()
        r = dict(cfg=ci, name=p.name, nsteps=nsteps, k=k, t_forward_s=tf, t_fwd_plus_ckpt_bwd_s=tb,
                 adjoint_over_forward=tb / tf, t_step_vjp_s=tv, t_step_fwd_s=tf / nsteps)
        print(json.dumps(r), flush=True)
        out.append(r)
        S.close()
    return out


if __name__ == "__main__":
    time_rollouts()
