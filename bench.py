#!/usr/bin/env python3
"""Throughput of the FP64 Euler step on one MI355X.

Workload: 3D Sedov blast, 128^3 cells as 512 blocks of 16^3 with 3 guard
layers, WENO5 + HLLC + SSP-RK3, CFL 0.5, gamma 1.4 (seeded synthetic input,
see paper_2401_03378_amd/workloads.py).  A step is one whole hydro_step:
CFL dt reduction plus three fused stage launches (captured in a hipGraph).

Prints ONE JSON line: zone-updates per second per RK stage, the roofline of
the dominant kernel (the fused stage kernel, timed with HIP events on its
own stream), and the CPU oracle timed on a bounded sample of the same
workload on the host cores.  The timed loop steps one state, each step
taking its CFL dt from the maxima the previous step's final stage recorded
(the same dt bit for bit; --cfl-pass: a separate pass over U).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per zone-stage of the fused stage kernel
# (+ - * / sqrt = 1, fma = 2; compares, min/max, abs, copysign = 0), with one
# EOS per cell, one reconstruction per cell and direction, one Riemann solve
# per face (star-region branch) and the flux-difference/RK update.
FLOPS_PER_ZONE_STAGE = {("3", "WENO5"): 1781, ("3", "PLM"): 476, ("2", "PLM"): 277, ("2", "WENO5"): 973}
# Algorithmic HBM bytes per zone-stage: read U_s, read U^n (stages >= 2),
# write U_{s+1}; interior cells only.
PEAK_FP64 = 78.6e12          # 256 CU x 64 lanes x 2.4 GHz x 2 (fma)
PEAK_HBM = 8.0e12
PEAK_VALU_LANES = 256 * 64 * 2.4e9   # FP64 lane-instructions per second (16-lane SIMDs, 4 per CU)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the stage kernel's code (comments and layout ignored), to
    tell whether counter records were taken on the kernel as it is: the
    device helpers, and the stage kernel's body and entry points (from
    set_prio up to the CFL kernels) in the kernel file."""
    h = hashlib.sha256()
    for f in ("hydro_common.h", "hydro_fwd.hip"):
        text = open(os.path.join(ROOT, "paper_2401_03378_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        if f == "hydro_fwd.hip":
            a, b = text.find("void set_prio"), text.find("k_cfl_partial(CflArgs")
            if 0 <= a < b:
                text = text[a:b]
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def cpu_baseline(prob, budget_s):
    """Oracle zone-stage rate on the first steps of the same workload."""
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    U = prob.U0.copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        O.step(prob, U)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= prob.nsteps:
            break
    el = time.perf_counter() - t0
    zs = prob.interior_zones * prob.rk * steps
    return {"value": zs / el, "unit": "zone-updates/s", "cores": min(threads, cores), "kind": "oracle",
            "sample": f"first {steps} step(s) of the same workload ({zs} zone-stages, {el:.1f} s)"}


def extras(S, prob, U0, ms_per_step):
    """Adjoint/forward cost of a checkpointed rollout (the config's 20 steps,
    checkpoint every 5, dt frozen) and the plain per-block-launch form of the
    same step, both on this GPU."""
    import torch
    from paper_2401_03378_amd.adjoint import rollout, rollout_vjp, TorchStepper
    st = TorchStepper(S)
    n, k = prob.nsteps, 5
    UN, tape = rollout(st, U0, n, k, keep_last=True)  # warm-up of the same shape: graph,
    rollout_vjp(st, tape, torch.nan_to_num(UN))       # adjoint scratch, allocator blocks
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    UN, tape = rollout(st, U0, n, n + 1)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    UN, tape = rollout(st, U0, n, k, keep_last=True)
    rollout_vjp(st, tape, torch.nan_to_num(UN))
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    S.status()
    tuned = S.tuning()
    S.set_tuning(mode=1, use_graph=0)
    U = U0.clone()
    S.step(U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        S.step(U)
    torch.cuda.synchronize()
    tpb = (time.perf_counter() - t0) / 2
    S.status()
    S.set_tuning(**tuned)
    return {"adjoint_over_forward": round(tb / tf, 3),
            "adjoint_detail": f"{n}-step rollout, checkpoint every {k}: forward {tf * 1e3:.2f} ms, "
                              f"forward + checkpointed backward {tb * 1e3:.2f} ms",
            "perblock_ms_per_step": round(tpb * 1e3, 3),
            "speedup_vs_perblock": round(tpb * 1e3 / ms_per_step, 2)}


def amr_extra(nsteps=10):
    """A two-level mesh: 8^3 coarse blocks of 16^3 cells with the central
    4^3 refined (448 coarse + 512 fine blocks, 3.9 M zones), WENO5 + HLLC +
    SSP-RK3, the density/pressure blob crossing the coarse-fine faces; zone
    updates per second of hydro_step (coarse-fine guard fill, stage, flux
    correction), with the all-levels and the level-by-level order."""
    import torch
    from paper_2401_03378_amd import autotune
    from paper_2401_03378_amd import workloads as W
    from paper_2401_03378_amd.solver import Solver
    prob = W.amr_problem(3, NBc=(8, 8, 8), n=16, ng=3, recon=W.WENO5, rk=3, flow="blob",
                         refine=[(i, j, k) for i in range(2, 6) for j in range(2, 6) for k in range(2, 6)])
    zones = prob.interior_zones
    res = {"workload": "two-level mesh: 448 coarse + 512 fine blocks of 16^3 (central 4^3 coarse blocks refined), "
                       "WENO5 + HLLC + SSP-RK3, flux correction at coarse-fine faces",
           "zones": zones}
    tuning = None
    for lbl in (False, True):
        S = Solver(prob, level_by_level=lbl)
        if tuning is None:    # the autotuner's choice for this mesh (all-levels order), cached
            tuning = autotune.tuned_or_search(S, prob, log=lambda *a: None)
            res["tuning"] = tuning
        else:
            S.set_tuning(**tuning)
        U0 = S.to_device(prob.U0)
        U = U0.clone()
        for _ in range(3):
            S.step(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            S.step(U)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / nsteps
        S.status()
        key = "level_by_level" if lbl else "all_levels"
        res[key] = {"ms_per_step": round(t * 1e3, 4), "zone_updates_per_s": zones * prob.rk / t}
        S.close()
    return {"amr": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work (0 = skip)")
    ap.add_argument("--kernel-steps", type=int, default=10, help="steps timed per stage launch with events")
    ap.add_argument("--calib-copy", action="store_true", help="also run a plain 512 MiB device copy")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cfl-pass", action="store_true",
                    help="compute every step's dt with a separate pass over U (default: from the maxima "
                         "the previous step's final stage recorded)")
    ap.add_argument("--amr-only", action="store_true",
                    help="only time the two-level AMR workload (prints its JSON object)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint/forward and per-block-launch comparisons")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU (blocks are not sharded across GPUs); --gpus must be 1"}))
        sys.exit(2)
    if args.amr_only:
        print(json.dumps(amr_extra(args.steps)), flush=True)
        return

    import torch
    from paper_2401_03378_amd import workloads as W
    from paper_2401_03378_amd.solver import Solver
    from paper_2401_03378_amd import autotune

    prob = W.config(1)
    zones = prob.interior_zones
    S = Solver(prob)
    tuned = None
    if not args.no_autotune:
        tuned = autotune.tuned_or_search(S, prob, log=log)
    U0 = S.to_device(prob.U0)
    U = U0.clone()
    log(f"workload {prob.name}: {prob.nblocks} blocks, {zones} zones, tuning {S.tuning()}")

    if args.calib_copy:
        a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()

    # a time-stepping loop on one state: each step takes its CFL dt from the
    # maxima the previous step's final stage recorded (bitwise the same dt as
    # a separate pass over U; --cfl-pass times that pass instead)
    fused = not args.cfl_pass
    for _ in range(args.warmup):
        S.step(U, dt_from_previous=fused)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.step(U, dt_from_previous=fused)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    S.status()
    ms_per_step = 1000.0 * T / args.steps
    value = zones * prob.rk * args.steps / T
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.4e} zone-updates/s")

    # dominant kernel: one fused stage launch, HIP events on the solver's stream
    stream = S.stream
    Ua = U0.clone()
    B1 = U0.clone()
    B2 = U0.clone()
    dt = S.cfl_dt(Ua)
    evs = []
    with torch.cuda.stream(stream):
        for rep in range(args.kernel_steps):
            for s, (Us, Uo) in enumerate(((Ua, B1), (B1, B2), (B2, Ua)), start=1):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                S.rk_stage(s, Ua, Us, Uo, dt)
                e1.record(stream)
                evs.append((e0, e1))
    torch.cuda.synchronize()
    S.status()
    durs = [a.elapsed_time(b) * 1e-3 for a, b in evs]
    t_stage = sum(durs) / len(durs)
    flops = FLOPS_PER_ZONE_STAGE[(str(prob.ndim), "WENO5" if prob.recon == W.WENO5 else "PLM")] * zones
    achieved = flops / t_stage / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": round(achieved * 1e12 / PEAK_FP64, 4), "traffic": None,
            "kernel": "k_stage (fused guard-gather+EOS+WENO5+HLLC+update)",
            "avg_launch_s": t_stage, "flops_per_launch": flops}
    # counter-derived figures, valid while the kernel source and the launch
    # configuration are those they were measured with
    def measured(name):
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            return None
        rec = json.load(open(path))
        if rec.get("source_sha") != source_hash() or rec.get("tuning") != S.tuning():
            return None
        return rec
    tr = measured("traffic_stage_sedov128.json")
    if tr:
        roof["traffic"] = tr["bytes_per_launch"]
    ct = measured("counters_stage_sedov128.json")
    if ct:
        # issued VALU lane-instructions (rocprofv3 SQ_INSTS_VALU x 64) over the
        # chip's FP64 instruction rate: how busy the vector units are
        roof["valu_issue_frac"] = round(ct["valu_lane_instr_per_launch"] / t_stage / PEAK_VALU_LANES, 4)
        roof["valu_lane_instr_per_zone_stage"] = round(ct["valu_lane_instr_per_launch"] / zones)
    # bytes the method must move per stage (RK3 average: read U_s, U^n for
    # s >= 2, write U_{s+1}) relative to HBM peak at the whole-step rate
    balg = (3 * 40 + 2 * 40 + 3 * 40) / 3.0
    hbm_frac = value * balg / PEAK_HBM

    out = {
        "metric": "zone-updates/s (FP64, per RK stage)",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sedov3d: 128^3 cells as 512 blocks of 16^3 + 3 guard layers, WENO5 + HLLC "
                               "+ SSP-RK3, CFL 0.5, gamma 1.4, E=1 in r<3.5 cells",
                   "zones": zones, "rk_stages": prob.rk, "tuning": S.tuning(),
                   "dt": ("CFL maxima recorded by the previous step's final stage" if fused
                          else "separate CFL pass over U")},
        "roofline": roof,
        "hbm_effective_frac": round(hbm_frac, 4),
    }
    if not args.no_extras:
        out.update(extras(S, prob, U0, ms_per_step))
        out.update(amr_extra())
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(W.config(1), args.cpu_budget)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
