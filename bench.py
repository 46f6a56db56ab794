#!/usr/bin/env python3
"""Throughput of the FP64 Euler step on one MI355X.

Headline workload: 3D turbulence-like flow, 256^3 cells as 4096 blocks of
16^3 with 3 guard layers, periodic, WENO5 + HLLC + SSP-RK3, CFL 0.5, gamma
1.4, Gaussian velocity field with a k^-4 power spectrum at rms Mach 0.5
(seeded synthetic input, see paper_2401_03378_amd/workloads.py).  A step is
one whole hydro_step: the CFL dt plus three fused stage launches (captured in
a hipGraph).  The timed loop steps one state, each step taking its CFL dt
from the maxima the previous step's final stage recorded (the same dt bit
for bit; --cfl-pass: a separate pass over U).

Prints ONE JSON line: zone-updates per second per RK stage, the roofline of
the dominant kernel (the fused stage kernel, timed with HIP events on its
own stream), the CPU oracle timed on a bounded sample of the same workload
on the host cores, and (unless --no-extras) the other named workloads, the
checkpointed adjoint's cost relative to the forward rollout, the plain
per-block launch form, a plain device copy (attainable bandwidth) and a
two-level AMR mesh.
"""
import argparse
import ctypes
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per zone-stage of the fused stage kernel
# (+ - * / sqrt = 1, fma = 2; compares, min/max, abs, copysign = 0), with one
# EOS per cell, one reconstruction per cell and direction, one Riemann solve
# per face (star-region branch) and the flux-difference/RK update.
FLOPS_PER_ZONE_STAGE = {("3", "WENO5"): 1781, ("3", "PLM"): 476, ("2", "PLM"): 277, ("2", "WENO5"): 973}
PEAK_FP64 = 78.6e12          # 256 CU x 64 lanes x 2.4 GHz x 2 (fma)
PEAK_HBM = 8.0e12
PEAK_VALU_LANES = 256 * 64 * 2.4e9   # FP64 lane-instructions per second (16-lane SIMDs, 4 per CU)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def balg_per_zone_stage(prob):
    """Algorithmic HBM bytes per zone-stage: a stage reads U_s (and U^n for
    s >= 2) and writes U_{s+1}, interior cells only; averaged over the
    stages of a step."""
    arrays = (2 + 3 * (prob.rk - 1)) / prob.rk
    return arrays * prob.nvar * 8


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


def _omp_threads(n):
    """Set the OpenMP thread count of this process (the oracle's runtime)."""
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(ctypes.c_int(n))
        return True
    except OSError:
        return False


def cpu_baseline(prob, budget_s):
    """Oracle zone-stage rate on the first steps of the same workload, on
    all host cores; plus one step of the same recipe at 64^3 on one thread
    (a per-core rate)."""
    import oracle as O
    from paper_2401_03378_amd import workloads as W
    cores = len(os.sched_getaffinity(0))
    threads = min(int(os.environ.get("OMP_NUM_THREADS", cores)), cores)
    _omp_threads(threads)
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
    out = {"value": zs / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"first {steps} step(s) of the same workload ({zs} zone-stages, {el:.1f} s)"}
    if prob.name == "turb3d" and _omp_threads(1):
        small = W.turb3d(N=64)
        U = small.U0.copy()
        t0 = time.perf_counter()
        O.step(small, U)
        el1 = time.perf_counter() - t0
        _omp_threads(threads)
        z1 = small.interior_zones * small.rk
        out["per_core"] = {"value": z1 / el1, "unit": "zone-updates/s", "threads": 1,
                           "sample": f"first step of the same recipe at 64^3 (64 blocks of 16^3, {z1} "
                                     f"zone-stages, {el1:.2f} s)"}
    return out


def timed_steps(S, U, steps, fused):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S.step(U, dt_from_previous=fused)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def stage_kernel_time(S, U0, reps):
    """Average duration of one fused stage launch (HIP events recorded on
    the solver's stream around each launch), over reps steps' worth of
    stages on three buffers."""
    import torch
    stream = S.stream
    Ua, B1, B2 = U0.clone(), U0.clone(), U0.clone()
    dt = S.cfl_dt(Ua)
    evs = []
    chain = ((Ua, B1), (B1, B2), (B2, Ua)) if S.prob.rk == 3 else ((Ua, B1), (B1, Ua))
    with torch.cuda.stream(stream):
        for _ in range(reps):
            for s, (Us, Uo) in enumerate(chain, start=1):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                S.rk_stage(s, Ua, Us, Uo, dt)
                e1.record(stream)
                evs.append((e0, e1))
    torch.cuda.synchronize()
    S.status()
    durs = [a.elapsed_time(b) * 1e-3 for a, b in evs]
    return sum(durs) / len(durs)


def adjoint_cost(S, U0, n, k):
    """Adjoint/forward cost of a checkpointed rollout: n steps, checkpoint
    every k, dt frozen; the forward rollout alone against forward plus the
    checkpointed backward pass."""
    import torch
    from paper_2401_03378_amd.adjoint import rollout, rollout_vjp, TorchStepper
    st = TorchStepper(S)
    UN, tape = rollout(st, U0, n, k, keep_last=True)  # warm-up of the same shape: graph,
    rollout_vjp(st, tape, torch.nan_to_num(UN))       # adjoint scratch, allocator blocks
    del UN, tape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    UN, tape = rollout(st, U0, n, n + 1)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    del UN, tape
    t0 = time.perf_counter()
    UN, tape = rollout(st, U0, n, k, keep_last=True)
    rollout_vjp(st, tape, torch.nan_to_num(UN))
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    del UN, tape
    S.status()
    return {"adjoint_over_forward": round(tb / tf, 3),
            "adjoint_detail": f"{n}-step rollout, checkpoint every {k}: forward {tf * 1e3:.2f} ms, "
                              f"forward + checkpointed backward {tb * 1e3:.2f} ms"}


def perblock_form(S, U0, nsteps):
    """The plain per-block launch form of the same step: per stage and block,
    a guard-fill launch and a stage launch; no graph."""
    import torch
    tuned = S.tuning()
    S.set_tuning(mode=1, use_graph=0)
    U = U0.clone()
    S.step(U)
    t = timed_steps(S, U, nsteps, False) / nsteps
    S.status()
    S.set_tuning(**tuned)
    del U
    torch.cuda.synchronize()
    return t


def copy_bandwidth(nbytes=2 ** 31, reps=5):
    """Attainable HBM bandwidth: a plain device-to-device copy of nbytes
    (read + write counted), best of reps, timed with HIP events."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        best = t if best is None else min(best, t)
    del a, b
    return {"bytes": 2 * nbytes, "seconds": best, "GB_per_s": round(2 * nbytes / best / 1e9, 1),
            "frac_of_peak": round(2 * nbytes / best / PEAK_HBM, 4)}


def other_workloads(log):
    """The other named workloads at their own sizes and step counts: the
    tuned persistent form (the Sod problem also in its plain per-block form,
    its defining launch form)."""
    import torch
    from paper_2401_03378_amd import autotune
    from paper_2401_03378_amd import workloads as W
    from paper_2401_03378_amd.solver import Solver
    out = {}
    for prob in (W.sod2d(), W.sedov3d(), W.batched_uneven(), W.kh2d()):
        S = Solver(prob)
        tuning = autotune.tuned_or_search(S, prob, log=log)
        U0 = S.to_device(prob.U0)
        U = U0.clone()
        for _ in range(3):
            S.step(U, dt_from_previous=True)
        t = timed_steps(S, U, prob.nsteps, True) / prob.nsteps
        S.status()
        zs = prob.interior_zones * prob.rk
        r = {"zones": prob.interior_zones, "steps": prob.nsteps, "ms_per_step": round(t * 1e3, 4),
             "zone_updates_per_s": zs / t, "hbm_effective_frac": round(zs / t * balg_per_zone_stage(prob) / PEAK_HBM, 4),
             "tuning": tuning}
        if prob.name == "sod2d":
            tp = perblock_form(S, U0, prob.nsteps)
            r["perblock_ms_per_step"] = round(tp * 1e3, 4)
            r["perblock_zone_updates_per_s"] = zs / tp
        out[prob.name] = r
        S.close()
        del U, U0
        torch.cuda.synchronize()
        log(f"{prob.name}: {t * 1e3:.4f} ms/step")
    return out


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
        t = timed_steps(S, U, nsteps, False) / nsteps
        S.status()
        key = "level_by_level" if lbl else "all_levels"
        res[key] = {"ms_per_step": round(t * 1e3, 4), "zone_updates_per_s": zones * prob.rk / t}
        S.close()
        torch.cuda.synchronize()
    return {"amr": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed steps before the timed ones (the GPU clocks settle over the first few)")
    ap.add_argument("--repeats", type=int, default=5, help="timed loops of --steps steps (the first is the line's value)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work (0 = skip)")
    ap.add_argument("--kernel-steps", type=int, default=5, help="steps timed per stage launch with events")
    ap.add_argument("--calib-copy", action="store_true", help="also run a plain 512 MiB device copy")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cfl-pass", action="store_true",
                    help="compute every step's dt with a separate pass over U (default: from the maxima "
                         "the previous step's final stage recorded)")
    ap.add_argument("--workload", default="turb3d", choices=("turb3d", "sedov3d", "batched", "kh2d", "sod2d"),
                    help="the workload timed (default: the 256^3 turbulence workload)")
    ap.add_argument("--amr-only", action="store_true",
                    help="only time the two-level AMR workload (prints its JSON object)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, the adjoint/forward, per-block and copy comparisons")
    ap.add_argument("--grav", type=float, nargs=3, default=None, metavar=("GX", "GY", "GZ"),
                    help="add a uniform gravitational acceleration (grvAccel) to the workload")
    ap.add_argument("--shock-thresh", type=float, default=None,
                    help="turn on the shock detector (shockDet) with this relative pressure jump")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the checkpointed adjoint rollout of the workload (prints its JSON object)")
    ap.add_argument("--adjoint-steps", type=int, default=None,
                    help="steps of the adjoint rollout (default: 10 for turb3d, else the workload's)")
    ap.add_argument("--adjoint-every", type=int, default=5, help="checkpoint interval of the adjoint rollout")
    ap.add_argument("--tune", nargs="*", default=[], metavar="KEY=VALUE",
                    help="override fields of the launch configuration after the autotuner (e.g. variant=2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the blocks are not sharded across GPUs, "
                                   "so --gpus must be 1"}), flush=True)
        sys.exit(2)
    if args.amr_only:
        print(json.dumps(amr_extra(args.steps)), flush=True)
        return

    import torch
    from paper_2401_03378_amd import workloads as W
    from paper_2401_03378_amd.solver import Solver
    from paper_2401_03378_amd import autotune

    build = {"turb3d": W.turb3d, "sedov3d": W.sedov3d, "batched": W.batched_uneven, "kh2d": W.kh2d,
             "sod2d": W.sod2d}[args.workload]
    prob = build()
    if args.grav is not None:
        prob.grav = tuple(args.grav)
    if args.shock_thresh is not None:
        prob.shock_thresh = args.shock_thresh
    zones = prob.interior_zones
    S = Solver(prob)
    if not args.no_autotune:
        autotune.tuned_or_search(S, prob, log=log)
    if args.tune:
        S.set_tuning(**{k: int(v) for k, v in (kv.split("=", 1) for kv in args.tune)})
    U0 = S.to_device(prob.U0)
    U = U0.clone()
    log(f"workload {prob.name}: {prob.nblocks} blocks, {zones} zones, tuning {S.tuning()}")

    if args.calib_copy:
        a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    nadj = args.adjoint_steps or (10 if prob.name == "turb3d" else prob.nsteps)
    if args.adjoint_only:
        res = {"workload": prob.name, "zones": zones, "tuning": S.tuning()}
        res.update(adjoint_cost(S, U0, nadj, args.adjoint_every))
        S.close()
        print(json.dumps(res), flush=True)
        return

    fused = not args.cfl_pass
    for _ in range(args.warmup):
        S.step(U, dt_from_previous=fused)
    T = timed_steps(S, U, args.steps, fused)
    S.status()
    ms_per_step = 1000.0 * T / args.steps
    value = zones * prob.rk * args.steps / T
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.4e} zone-updates/s")
    reps = [ms_per_step]
    for _ in range(args.repeats - 1):
        reps.append(1000.0 * timed_steps(S, U, args.steps, fused) / args.steps)
    S.status()
    del U

    t_stage = stage_kernel_time(S, U0, args.kernel_steps)
    recon = "WENO5" if prob.recon == W.WENO5 else "PLM"
    flops = FLOPS_PER_ZONE_STAGE[(str(prob.ndim), recon)] * zones
    achieved = flops / t_stage / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": round(achieved * 1e12 / PEAK_FP64, 4), "traffic": None,
            "kernel": f"k_stage (fused guard-gather+EOS+{recon}+HLLC+update)",
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
    tr = measured(f"traffic_stage_{prob.name}.json")
    if tr:
        roof["traffic"] = tr["bytes_per_launch"]
    ct = measured(f"counters_stage_{prob.name}.json")
    if ct:
        # issued VALU lane-instructions (rocprofv3 SQ_INSTS_VALU x 64) over the
        # chip's FP64 instruction rate: how busy the vector units are
        roof["valu_issue_frac"] = round(ct["valu_lane_instr_per_launch"] / t_stage / PEAK_VALU_LANES, 4)
        roof["valu_lane_instr_per_zone_stage"] = round(ct["valu_lane_instr_per_launch"] / zones)
    balg = balg_per_zone_stage(prob)

    desc = {"turb3d": "turbulence 3D: 256^3 cells as 4096 blocks of 16^3 + 3 guard layers, periodic, WENO5 + "
                      "HLLC + SSP-RK3, CFL 0.5, gamma 1.4, k^-4 Gaussian velocity at rms Mach 0.5",
            "sedov3d": "sedov3d: 128^3 cells as 512 blocks of 16^3 + 3 guard layers, WENO5 + HLLC + SSP-RK3, "
                       "CFL 0.5, gamma 1.4, E=1 in r<3.5 cells",
            "batched_uneven": "batched: 4096 periodic blocks (50% 8^3, 40% 16^3, 10% 32^3) + 2 guard layers, PLM-MC + "
                       "HLLC + SSP-RK2, CFL 0.8, gamma 5/3",
            "kh2d": "kh2d: 256^2 cells as 256 blocks of 16^2 + 2 guard layers, PLM-MC + HLLC + SSP-RK2",
            "sod2d": "sod2d: 64^2 cells as 16 blocks of 16^2 + 2 guard layers, PLM-MC + HLLC + SSP-RK2"}[prob.name]
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
        "config": {"workload": desc + ("" if prob.grav is None else f", gravity {tuple(prob.grav)}")
                   + ("" if prob.shock_thresh is None else f", shock detector {prob.shock_thresh}"),
                   "zones": zones, "rk_stages": prob.rk, "tuning": S.tuning(),
                   "dt": ("CFL maxima recorded by the previous step's final stage" if fused
                          else "separate CFL pass over U")},
        "repeats_ms_per_step": [round(r, 4) for r in reps],
        "median_ms_per_step": round(statistics.median(reps), 4),
        "roofline": roof,
        "hbm_effective_frac": round(value * balg / PEAK_HBM, 4),
        "balg_bytes_per_zone_stage": round(balg, 2),
    }
    if not args.no_extras:
        out.update(adjoint_cost(S, U0, nadj, args.adjoint_every))
        tpb = perblock_form(S, U0, 2)
        out["perblock_ms_per_step"] = round(tpb * 1e3, 3)
        out["speedup_vs_perblock"] = round(tpb * 1e3 / ms_per_step, 2)
        S.close()
        del U0
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["copy_bandwidth"] = copy_bandwidth()
        out["workloads"] = other_workloads(log)
        out.update(amr_extra())
    else:
        S.close()
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
