#!/usr/bin/env python3
"""Benchmark of the 1D heat-equation hot path on one MI355X.

A "step" of this benchmark is one complete run of the synchronous large-rod
workload: N = 2^26 points in FP32, r = 0.25, c1 = cN = 0, u0 = eight sine modes
plus noise, K = 2000 time steps (depth-T temporal blocking, autotuned).
`value` is its throughput in GLUP/s (giga lattice-point updates per second,
(N-2)*K per run) with the input already resident in HBM.

The same invocation also measures, and reports under "variants", the other
forms of the hot path: the T sweep (1..32) and the FP64 rod (N = 2^25); the
small rod (N = 4096, FP64, K = 20000) synchronous and emulated-asynchronous;
the asynchronous large rod (N = 2^24, 1024 subdomains, K = 5000,
d in {1, 4, 16}, hardware and emulated) with its synchronous comparators, and
the gradients through its emulated run at d = 4; the
batched ragged rods (4096 rods, one persistent launch in a HIP graph);
forward + adjoint (256 rods of 2^16 FP32 and one FP64 rod of 2^20, K = 2000);
and the paper's own rod as an ensemble of 300 emulated-async runs with
Dirichlet ends and on the periodic ring (N = 100, K = 5000, norm every step).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64
PEAK_HBM_GBS = 8000.0
FLOPS_PER_LUP = 4         # add, multiply, fused multiply-add (the update c + r((a+b) - 2c))
ADJ_FLOPS_PER_LUP = 6     # a lambda update (4) and its dL/dr term (one FMA, 2)
PROFILES = os.path.join(ROOT, "profiles")


def traffic_record(kernel, plan):
    """HBM bytes per launch of `kernel` under `plan` ("T=.. M=..") from the
    counter summaries under profiles/, or None when there is none or the
    kernel's sources have changed since the counters were taken."""
    import hashlib
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)):
            if not line.startswith("traffic-record: "):
                continue
            rec = json.loads(line[len("traffic-record: "):])
            if rec["kernel"] != kernel or rec["plan"] != plan:
                continue
            h = hashlib.sha256()
            try:
                for f in rec["sources"]:
                    with open(os.path.join(ROOT, f), "rb") as fh:
                        h.update(fh.read())
            except OSError:
                continue
            if h.hexdigest() == rec["source_sha256"]:
                return rec
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", default="", help="comma list of variant groups to run "
                    "(f64,small,async,batched,async_adjoint,adjoint,ensemble,ring); default all")
    ap.add_argument("--plan", default="", help="fix the headline plan as T,M[,tiled|pipelined"
                    "[,S[,W]]] (skips sweep and autotune; default kernel pipelined, S=1, "
                    "W wavefronts per tile of the tiled kernel)")
    ap.add_argument("--kernel", default="",
                    choices=["", "async", "batched", "adjoint", "async_adjoint", "ensemble", "ring"],
                    help="run only one workload of one hot-path kernel, once after one warm-up, "
                    "and print its timing (for profiler runs: async = the 2^24 rod, emulated "
                    "and hardware at d = 4; batched = the 4096 ragged rods; adjoint = forward "
                    "+ backward of 256 x 2^16 FP32; ensemble = the paper's 300 members with "
                    "norms every step, Dirichlet; ring = the 2^26-point FP32 ring on fixed wide ring "
                    "tiles T=256 M=32 S=8 W=4; async_adjoint = gradients through the emulated "
                    "run of the 2^24 rod at d = 4)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain device copy of the rod (2^26 floats) so that "
                    "hardware byte counters can be scaled against a known transfer")
    return ap.parse_args()


class Timer:
    def __init__(self, torch):
        self.torch = torch

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        return self

    def __exit__(self, *exc):
        self.torch.cuda.synchronize()
        self.dt = time.perf_counter() - self.t0


def time_runs(torch, fn, reps, warmup=1):
    for _ in range(warmup):
        fn()
    with Timer(torch) as t:
        for _ in range(reps):
            fn()
    return t.dt / reps


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "heat1d runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        log("bench.py: only --gpus 1 is supported (the hot path is measured on one GPU; "
            "the multi-GPU design is described, not built)")
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    import workloads
    from paper_1510_08982_amd import abi
    from paper_1510_08982_amd.heat import (SyncPlan, AsyncPlan, BatchedPlan, AdjointPlan)

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    variants = {}
    if args.kernel:
        if args.calib_copy:
            src = torch.zeros(1 << 26, dtype=torch.float32, device=dev)
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        one_kernel(args.kernel, torch, dev, workloads, abi, AsyncPlan, BatchedPlan, SyncPlan,
                   AdjointPlan)
        return

    # ------------------------------------------------------------ headline
    N, K = 1 << 26, 2000
    log(f"[bench] generating sine-mode rod N={N}")
    rod = workloads.sine_modes_rod(N, seed=0, K=K)
    x32 = torch.from_numpy(rod.u0.astype(np.float32)).to(dev)
    r = float(np.float32(rod.r))
    lups = (N - 2) * K
    if args.calib_copy:
        y = torch.empty_like(x32)
        y.copy_(x32)
        torch.cuda.synchronize()
        del y

    # T sweep (1..128): for each depth the best points-per-lane, for the plain
    # tiled pass and for the pipelined persistent kernel
    kernels = {"tiled": abi.HEAT1D_SYNC_TILED, "pipelined": abi.HEAT1D_SYNC_PIPELINED}
    sweep = {}
    for T in (() if args.plan else (1, 2, 4, 8, 16, 32, 64, 96, 128, 192, 256)):
        row = {}
        families = list(kernels.items()) + [("tiled_W4", abi.HEAT1D_SYNC_TILED),
                                            ("tiled_W8", abi.HEAT1D_SYNC_TILED)]
        for kname, kcode in families:
            G = int(kname[-1]) if kname.startswith("tiled_W") else 0
            if (G and T < 16) or (not G and T > 128):
                continue
            for S in ((1,) if T < 8 else (1, 4, 8) if G else (1, 4)):
                best = None
                Ms = ((16, 32) if T <= 8 else (16, 32, 48) if T <= 32 else (32, 48, 64))
                for M in ((16, 32) if G == 8 else (16, 32, 48) if G == 4 else Ms):
                    try:
                        plan = SyncPlan(N, torch.float32, sync_kernel=kcode, depth_t=T,
                                        pts_per_lane=M, fuse_steps=S, waves=G)
                    except abi.Heat1dError:
                        continue        # no tile of this width holds a halo of T
                    dt = time_runs(torch, lambda: plan.run(x32, r, 0.0, 0.0, K), 1, 1)
                    plan.close()
                    if best is None or dt < best[0]:
                        best = (dt, M)
                if best is not None:
                    row[kname + ("" if S == 1 else f"_S{S}")] = {
                        "glups": round(lups / best[0] / 1e9, 1), "M": best[1],
                        "ms": round(best[0] * 1e3, 3)}
        sweep[str(T)] = row
        log(f"[bench] T={T}: {row}")
    if sweep:
        variants["sync_f32_T_sweep"] = sweep

    if args.plan:
        parts = args.plan.split(",")
        T_fix, M_fix = int(parts[0]), int(parts[1])
        kcode = kernels[parts[2]] if len(parts) > 2 else abi.HEAT1D_SYNC_PIPELINED
        S_fix = int(parts[3]) if len(parts) > 3 else 1
        W_fix = int(parts[4]) if len(parts) > 4 else 0
        plan = SyncPlan(N, torch.float32, sync_kernel=kcode, depth_t=T_fix, pts_per_lane=M_fix,
                        fuse_steps=S_fix, waves=W_fix)
    else:
        plan = SyncPlan(N, torch.float32)
        tuned_ms = plan.autotune(x32, r, 512)
        log(f"[bench] autotuned: {plan.describe()} ({tuned_ms:.3f} ms for 512 steps)")
    out = torch.empty_like(x32)
    for _ in range(args.warmup):
        plan.run(x32, r, 0.0, 0.0, K, out=out)
    plan.set_timing(True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record()
    for i in range(args.steps):
        plan.run(x32, r, 0.0, 0.0, K, out=out)
        marks[i + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_run_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps))
    kern_ms, launches_total = plan.last_kernel_ms()
    plan.set_timing(False)
    kern_total_ms = kern_ms * launches_total
    value = lups * args.steps / elapsed / 1e9
    ms_per_step = elapsed / args.steps * 1e3
    desc = plan.describe()
    log(f"[bench] headline {value:.1f} GLUP/s, {ms_per_step:.3f} ms per run ({desc})")

    # roofline of the dominant kernel: one launch = one pass of T steps over the
    # rod; achieved = algorithmic flops of all timed launches / their summed
    # event-measured durations (= flops per launch / average launch time)
    lups_per_launch = (N - 2) * K * args.steps / max(launches_total, 1)
    flops_per_launch = FLOPS_PER_LUP * lups_per_launch
    achieved_tflops = flops_per_launch / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    tm = desc.split("T=")[1].split() if "T=" in desc else None
    m_s = desc.split("M=")[1].split()[0] if tm else ""
    s_s = desc.split("S=")[1].split()[0] if tm else ""
    w_s = desc.split("W=")[1].split()[0] if "W=" in desc else "1"
    kernel = pass_kernel(desc, "float")
    rec = traffic_record(kernel, f"T={tm[0]} M={m_s} S={s_s} W={w_s}") if tm else None
    # algorithmic HBM bytes: read + write of the rod once per pass
    passes_per_launch = (-(-K // int(tm[0])) * args.steps / max(launches_total, 1)) if tm else 1.0
    bytes_per_launch = 2 * 4 * N * passes_per_launch
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 2) if achieved_tflops else None,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4) if achieved_tflops else None,
                "traffic": rec["bytes_per_launch"] if rec else None,
                "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                "kernel": kernel,
                "kernel_avg_ms": round(kern_ms, 4), "launches_timed": launches_total,
                "lups_per_launch": round(lups_per_launch), "flops_per_lup": FLOPS_PER_LUP,
                "hbm_bytes_per_launch_algorithmic": round(bytes_per_launch),
                "hbm_gbs_algorithmic": round(bytes_per_launch / (kern_ms * 1e-3) / 1e9, 1)
                if kern_ms > 0 else None}
    del out
    plan.close()
    roofline["hbm_gbs_nominal"] = 8000.0
    roofline["hbm_gbs_copy_measured"] = measured_copy_gbs(torch, dev)

    if not args.quick:
        run_variants(args, torch, dev, workloads, abi, SyncPlan, AsyncPlan, BatchedPlan,
                     AdjointPlan, variants, x32, r, rod)
    del x32

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(rod, args.cpu_seconds)
    del rod

    line = {
        "metric": "GLUP/s + HBM roofline fraction: sync vs async vs batched vs fwd+adjoint",
        "value": round(value, 2),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_median": round(per_run_ms[len(per_run_ms) // 2], 4) if per_run_ms else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sync large rod: N=2^26 FP32, r=0.25, c1=cN=0, u0 = 8 sine modes "
                               "(m=8^j) + U[-0.01,0.01] noise, K=2000, temporal blocking autotuned",
                   "N": N, "K": K, "plan": desc, "device": props.name},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


def one_kernel(name, torch, dev, workloads, abi, AsyncPlan, BatchedPlan, SyncPlan, AdjointPlan):
    """One workload of one kernel, one warm-up then one timed run: the
    command profiler summaries are taken with."""
    res = {"kernel": name}
    if name == "async":
        arod = workloads.async_rod(seed=0)
        xa = torch.from_numpy(arod.u0.astype(np.float32)).to(dev)
        ra = float(np.float32(arod.r))
        with AsyncPlan(arod.N, 1024, torch.float32, max_delay=16) as ap:
            for mode, mname in ((abi.HEAT1D_ASYNC_EMULATED, "emulated"),
                                (abi.HEAT1D_ASYNC_HARDWARE, "hardware")):
                dt = time_runs(torch, lambda: ap.run(xa, ra, arod.c1, arod.cN, arod.K, 4, 11, mode),
                               1)
                res[f"{mname}_d4_ms"] = round(dt * 1e3, 3)
                res[f"{mname}_d4_glups"] = round((arod.N - 2) * arod.K / dt / 1e9, 1)
    elif name == "async_adjoint":
        arod, xa, g, ra = async_adjoint_inputs(torch, dev, workloads)
        K = arod.K
        with AsyncPlan(arod.N, 1024, torch.float32, max_delay=16) as ap:
            dt = time_runs(torch, lambda: ap.adjoint(xa, g, ra, arod.c1, arod.cN, K,
                                                     ASYNC_ADJ_D, 11), 1)
        res.update(ms=round(dt * 1e3, 3), K=K,
                   glups_fwd_adj=round(2 * (arod.N - 2) * K / dt / 1e9, 1))
    elif name == "batched":
        batch = workloads.ragged_batch(seed=0)
        with BatchedPlan(np.diff(batch.offsets), batch.K, torch.float32) as bp:
            bargs = [torch.from_numpy(batch.u0.astype(np.float32)).to(dev),
                     torch.from_numpy(batch.offsets).to(dev),
                     torch.from_numpy(batch.r.astype(np.float32).astype(np.float64)).to(dev),
                     torch.from_numpy(batch.c1.astype(np.float32).astype(np.float64)).to(dev),
                     torch.from_numpy(batch.cN.astype(np.float32).astype(np.float64)).to(dev),
                     torch.from_numpy(batch.K.astype(np.int32)).to(dev)]
            bp.autotune(*bargs)
            dt = time_runs(torch, lambda: bp.run(*bargs), 1)
            res.update(ms=round(dt * 1e3, 3), glups=round(batch.lups / dt / 1e9, 1),
                       plan=bp.describe())
    elif name == "ensemble":
        from paper_1510_08982_amd.heat import EnsemblePlan
        rod = workloads.paper_ensemble(members=300, N=100, K=5000, d=3)
        E, N, K, d = 300, rod.N, rod.K, rod.extra["d"]
        x = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(rod.u0, (E, N)))).to(dev)
        seeds = torch.from_numpy(rod.extra["seeds"].view(np.int64).copy()).to(dev)
        with EnsemblePlan(N, E, 0, torch.float64) as plan:
            dt = time_runs(torch, lambda: plan.run(x, rod.r, rod.c1, rod.cN, K, d, seeds, 1), 1)
        res.update(ms=round(dt * 1e3, 3), glups=round(E * (N - 2) * K / dt / 1e9, 2))
    elif name == "ring":
        N, K = 1 << 26, 2000
        rod = workloads.sine_modes_rod(N, seed=0, K=K)
        x = torch.from_numpy(rod.u0.astype(np.float32)).to(dev)
        r = float(np.float32(rod.r))
        with SyncPlan(N, torch.float32, boundary=abi.HEAT1D_BC_PERIODIC,
                      sync_kernel=abi.HEAT1D_SYNC_TILED, depth_t=256, pts_per_lane=32,
                      fuse_steps=8, waves=4) as rp:
            dt = time_runs(torch, lambda: rp.run(x, r, 0.0, 0.0, K), 1)
            res.update(ms=round(dt * 1e3, 3), glups=round(N * K / dt / 1e9, 1),
                       plan=rp.describe())
    else:
        B, NA, KA = 256, 1 << 16, 2000
        rng = np.random.default_rng(0)
        u0 = torch.from_numpy(rng.uniform(-1, 1, B * NA).astype(np.float32)).to(dev)
        with SyncPlan(NA, torch.float32, nrods=B) as tp:
            target = tp.run(u0, float(np.float32(0.35)), 0.0, 0.0, KA)
        r3 = float(np.float32(0.3))
        with AdjointPlan(NA, KA, torch.float32, nrods=B) as adj:
            dt = time_runs(torch, lambda: adj.backward(adj.forward(u0, r3, 0.0, 0.0) - target,
                                                       r3, 0.0, 0.0), 1)
        res.update(ms=round(dt * 1e3, 3), glups_fwd_adj=round(2 * (NA - 2) * KA * B / dt / 1e9, 1))
    print(json.dumps(res), flush=True)


def pass_kernel(desc, ftype, ring=False):
    """The per-pass kernel a synchronous plan description names
    ("tiled|pipelined N=.. rods=.. T=.. M=.. S=.. W=..")."""
    parts = dict(x.split("=") for x in desc.split()[1:] if "=" in x)
    kind = desc.split()[0]
    if kind not in ("tiled", "pipelined") or "M" not in parts:
        return desc
    m, sf, w = parts["M"], parts.get("S", "1"), parts.get("W", "1")
    if ring:
        if w != "1":
            return f"sync_wide_ring_kernel<{ftype}, {m}, {sf}, {w}>"
        return f"sync_ring_kernel<{ftype}, {m}, {sf}>"
    if kind == "pipelined":
        return f"sync_pipelined_kernel<{ftype}, {m}, {sf}>"
    if w != "1":
        return f"sync_wide_kernel<{ftype}, {m}, {sf}, {w}>"
    return f"sync_tiled_kernel<{ftype}, {m}, {sf}>"


def alu_roofline(kernel, flops_per_launch, kern_ms, peak, flops_per_lup, note="", plan=None):
    """Roofline record of one kernel bound by vector ALU work: achieved =
    algorithmic flops per launch / average launch duration (HIP events on the
    launch stream), against the vector peak of its precision.  `traffic` is
    the counter-measured HBM bytes per launch from profiles/ when a record for
    this kernel and plan matches the current sources."""
    if not kern_ms or kern_ms <= 0:
        return None
    achieved = flops_per_launch / (kern_ms * 1e-3) / 1e12
    rec_t = traffic_record(kernel, plan) if plan else None
    rec = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
           "traffic": rec_t["bytes_per_launch"] if rec_t else None,
           "kernel_avg_ms": round(kern_ms, 4), "flops_per_lup": flops_per_lup}
    if rec_t:
        rec["traffic_algorithmic"] = rec_t["algorithmic_bytes"]
    if note:
        rec["note"] = note
    return rec


ASYNC_ADJ_D = 4


def async_adjoint_inputs(torch, dev, workloads):
    """The asynchronous rod's workload (2^24 FP32 points, 1024 subdomains,
    K = 5000) with a seeded dL/du(K) for the gradients."""
    arod = workloads.async_rod(seed=0)
    xa = torch.from_numpy(arod.u0.astype(np.float32)).to(dev)
    g = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, arod.N).astype(np.float32)).to(dev)
    return arod, xa, g, float(np.float32(arod.r))


def run_async_adjoint(torch, dev, workloads, AsyncPlan, variants):
    """Gradients through the emulated asynchronous run of the asynchronous rod
    (d = 4): lockstep forward keeping checkpoints every ~sqrt(K) steps and the
    subdomain-edge records, stretch replays, and the transpose steps."""
    arod, xa, g, ra = async_adjoint_inputs(torch, dev, workloads)
    N, K = arod.N, arod.K
    reps = 2
    with AsyncPlan(N, 1024, torch.float32, max_delay=16) as ap:
        ap.adjoint(xa, g, ra, arod.c1, arod.cN, K, ASYNC_ADJ_D, 11)
        ap.set_timing(True)
        dt = time_runs(torch, lambda: ap.adjoint(xa, g, ra, arod.c1, arod.cN, K, ASYNC_ADJ_D, 11),
                       reps, 0)
        kms, nl = ap.last_kernel_ms()
        ap.set_timing(False)
        ap._adj_ws = None
    # The subdomains (16384 points) are longer than a register tile, so the
    # transpose runs on tiles of up to 32 steps per launch, lambda in
    # registers, every fourth state read and the three between recomputed:
    # counted as the synchronous adjoint is, 6 flops per backward update (the
    # lambda step and its dL/dr term; the recompute is work but not counted),
    # K updates of N-2 points over the launches of one run.
    per_run = max(nl // reps, 1)
    res = {"glups_fwd_adj": round(2 * (N - 2) * K / dt / 1e9, 1), "ms": round(dt * 1e3, 3),
           "d": ASYNC_ADJ_D, "P": 1024, "transpose_launches_per_run": per_run,
           "roofline": alu_roofline("async_adjoint_tiled_kernel<float, false>",
                                    ADJ_FLOPS_PER_LUP * (N - 2) * K / per_run, kms,
                                    PEAK_FP32_TFLOPS, ADJ_FLOPS_PER_LUP,
                                    note="one launch reads lambda once, every fourth u(k) of its "
                                         "steps and writes lambda once: (steps/4 + 2) * 4 * N "
                                         "bytes, far below the HBM roofline",
                                    plan=f"N=2^24 P=1024 d={ASYNC_ADJ_D} K={K}")}
    variants["async_adjoint_N2^24_P1024_K5000_d4_f32"] = res
    log(f"[bench] async adjoint: {res}")
    del xa, g


def run_variants(args, torch, dev, workloads, abi, SyncPlan, AsyncPlan, BatchedPlan, AdjointPlan,
                 variants, x32, r, rod):
    only = set(x for x in args.only.split(",") if x)

    def want(name):
        return not only or name in only

    if want("f64"):
        run_f64(torch, dev, rod, SyncPlan, variants)
    if want("small"):
        run_small(torch, dev, workloads, abi, SyncPlan, AsyncPlan, variants)
    if want("async"):
        run_async_rod(torch, dev, workloads, abi, SyncPlan, AsyncPlan, variants)
    if want("batched"):
        run_batched(torch, dev, workloads, SyncPlan, BatchedPlan, variants)
    if want("async_adjoint"):
        run_async_adjoint(torch, dev, workloads, AsyncPlan, variants)
    if want("adjoint"):
        run_adjoint(torch, dev, SyncPlan, AdjointPlan, variants)
    if want("ensemble"):
        run_ensemble(torch, dev, workloads, variants)
    if want("ring"):
        run_ring(torch, dev, rod, SyncPlan, abi, variants)
        run_async_ring(torch, dev, workloads, abi, SyncPlan, AsyncPlan, variants)


def run_f64(torch, dev, rod, SyncPlan, variants):
    N64, K = 1 << 25, 2000
    x64 = torch.from_numpy(rod.u0[:N64].copy()).to(dev)
    with SyncPlan(N64, torch.float64) as p64:
        p64.autotune(x64, rod.r, 256)
        p64.run(x64, rod.r, 0.0, 0.0, K)
        p64.set_timing(True)
        dt = time_runs(torch, lambda: p64.run(x64, rod.r, 0.0, 0.0, K), 3, 0)
        kms, nl = p64.last_kernel_ms()
        p64.set_timing(False)
        lups = (N64 - 2) * K
        variants["sync_f64_N2^25"] = {
            "glups": round(lups / dt / 1e9, 1), "ms": round(dt * 1e3, 3), "plan": p64.describe(),
            "roofline": alu_roofline(pass_kernel(p64.describe(), "double"),
                                     FLOPS_PER_LUP * lups * 3 / nl, kms, PEAK_FP64_TFLOPS,
                                     FLOPS_PER_LUP)}
    log(f"[bench] FP64 rod: {variants['sync_f64_N2^25']}")
    del x64


def run_small(torch, dev, workloads, abi, SyncPlan, AsyncPlan, variants):
    small = workloads.small_rod(seed=0)
    xs = torch.from_numpy(small.u0).to(dev)
    lups = (small.N - 2) * small.K
    res = {}
    one_cu = PEAK_FP64_TFLOPS / 256
    for name, opts in (("step_per_launch", dict(sync_kernel=abi.HEAT1D_SYNC_STEP)),
                       ("resident_16w", dict(sync_kernel=abi.HEAT1D_SYNC_RESIDENT, waves=16)),
                       ("resident_8w", dict(sync_kernel=abi.HEAT1D_SYNC_RESIDENT, waves=8)),
                       ("resident_4w", dict(sync_kernel=abi.HEAT1D_SYNC_RESIDENT, waves=4)),
                       ("resident_2w", dict(sync_kernel=abi.HEAT1D_SYNC_RESIDENT, waves=2))):
        with SyncPlan(small.N, torch.float64, **opts) as pl:
            dt = time_runs(torch, lambda: pl.run(xs, small.r, small.c1, small.cN, small.K), 2)
        res[name] = {"glups": round(lups / dt / 1e9, 3), "ms": round(dt * 1e3, 3)}
        if name.startswith("resident"):
            res[name]["frac_of_one_cu_fp64"] = round(FLOPS_PER_LUP * lups / dt / 1e12 / one_cu, 4)
    with AsyncPlan(small.N, 16, torch.float64, max_delay=3) as ap:
        for mode, mname in ((abi.HEAT1D_ASYNC_EMULATED, "emulated"),
                            (abi.HEAT1D_ASYNC_HARDWARE, "hardware")):
            dt = time_runs(torch, lambda: ap.run(xs, small.r, small.c1, small.cN, small.K, 3, 1,
                                                 mode), 2)
            res[f"async_{mname}_P16_d3"] = {"glups": round(lups / dt / 1e9, 3),
                                            "ms": round(dt * 1e3, 3), "plan": ap.describe()}
    res["note"] = ("one rod of 4096 points occupies one CU (resident) or 16 CUs (async): "
                   "frac_of_one_cu_fp64 is against one CU's share of the FP64 vector peak")
    variants["small_rod_N4096_f64_K20000"] = res
    log(f"[bench] small rod: {res}")


STATS_NOTE = ("delay_histogram and polls are counted on an untimed run just before the timed one "
              "(the counting kernel instance is a few percent slower than the timed one)")


def run_async_rod(torch, dev, workloads, abi, SyncPlan, AsyncPlan, variants):
    arod = workloads.async_rod(seed=0)
    xa = torch.from_numpy(arod.u0.astype(np.float32)).to(dev)
    ra = float(np.float32(arod.r))
    lups = (arod.N - 2) * arod.K
    res = {}
    with SyncPlan(arod.N, torch.float32) as sp:
        sp.autotune(xa, ra, 256)
        dt = time_runs(torch, lambda: sp.run(xa, ra, arod.c1, arod.cN, arod.K), 2)
        sync_ref = sp.run(xa, ra, arod.c1, arod.cN, arod.K).clone()
        res["sync_tiled"] = {"glups": round(lups / dt / 1e9, 1), "ms": round(dt * 1e3, 3),
                             "plan": sp.describe()}
    with SyncPlan(arod.N, torch.float32, sync_kernel=abi.HEAT1D_SYNC_STEP) as st:
        dt = time_runs(torch, lambda: st.run(xa, ra, arod.c1, arod.cN, arod.K), 1)
    res["sync_step_per_launch"] = {"glups": round(lups / dt / 1e9, 1), "ms": round(dt * 1e3, 3)}
    scale = float(sync_ref.abs().max())
    with AsyncPlan(arod.N, 1024, torch.float32, max_delay=16) as ap:
        for mode, mname in ((abi.HEAT1D_ASYNC_HARDWARE, "hardware"),
                            (abi.HEAT1D_ASYNC_EMULATED, "emulated")):
            for d in ((0, 1, 4, 16) if mode == abi.HEAT1D_ASYNC_HARDWARE else (1, 4, 16)):
                # an untimed run with statistics (the kernel instance that counts
                # delays and polls), then the timed run without them
                stats = torch.zeros(d + 3, dtype=torch.int64, device=dev)
                ap.run(xa, ra, arod.c1, arod.cN, arod.K, d, 11, mode, stats=stats)
                ap.set_timing(True)
                with Timer(torch) as t:
                    outa = ap.run(xa, ra, arod.c1, arod.cN, arod.K, d, 11, mode)
                kms, _ = ap.last_kernel_ms()
                ap.set_timing(False)
                status = ap.status()
                hist = stats.cpu().tolist()
                key = f"async_{mname}_d{d}" if d > 0 else "sync_resident_flags_d0"
                res[key] = {"glups": round(lups / t.dt / 1e9, 1), "ms": round(t.dt * 1e3, 3),
                            "kernel_ms": round(kms, 3), "status": status,
                            "deviation_from_sync": float((outa - sync_ref).abs().max()) / scale,
                            "delay_histogram": hist[:d + 1], "polls": hist[d + 1],
                            "roofline": alu_roofline(
                                f"async_kernel<float, 64, {mode}, false, false>",
                                FLOPS_PER_LUP * lups, kms, PEAK_FP32_TFLOPS, FLOPS_PER_LUP,
                                plan=f"N=2^24 P=1024 d={d} {mname}")}
                log(f"[bench] {key}: {res[key]['glups']} GLUP/s "
                    f"dev={res[key]['deviation_from_sync']:.2e}")
        res["plan"] = ap.describe()
    res["note"] = STATS_NOTE
    # speed-ups at equal accuracy: the emulated runs pass the oracle at the same
    # tolerance as the synchronous ones; hardware runs are reported with their
    # deviation from the synchronous result instead
    base_flags = res["sync_resident_flags_d0"]["ms"]
    base_blocked = res["sync_tiled"]["ms"]
    base_step = res["sync_step_per_launch"]["ms"]
    res["speedups"] = {k: {"vs_sync_persistent_flags_d0": round(base_flags / v["ms"], 2),
                           "vs_sync_temporally_blocked": round(base_blocked / v["ms"], 2),
                           "vs_sync_one_launch_per_step": round(base_step / v["ms"], 2)}
                       for k, v in res.items() if k.startswith("async_")}
    variants["async_rod_N2^24_P1024_K5000_f32"] = res
    del xa, sync_ref


def run_batched(torch, dev, workloads, SyncPlan, BatchedPlan, variants):
    batch = workloads.ragged_batch(seed=0)
    n = np.diff(batch.offsets)
    bp = BatchedPlan(n, batch.K, torch.float32)
    bargs = [torch.from_numpy(batch.u0.astype(np.float32)).to(dev),
             torch.from_numpy(batch.offsets).to(dev),
             torch.from_numpy(batch.r.astype(np.float32).astype(np.float64)).to(dev),
             torch.from_numpy(batch.c1.astype(np.float32).astype(np.float64)).to(dev),
             torch.from_numpy(batch.cN.astype(np.float32).astype(np.float64)).to(dev),
             torch.from_numpy(batch.K.astype(np.int32)).to(dev)]
    bout = torch.empty_like(bargs[0])

    def graph_time():
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            bp.run(*bargs, out=bout)
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                bp.run(*bargs, out=bout)
        torch.cuda.current_stream().wait_stream(s)
        return time_runs(torch, g.replay, 3), g

    # the plan's rule-based work order, then the autotuned one
    dt_rule, g = graph_time()
    plan_rule = bp.describe()
    del g
    tune_ms = bp.autotune(*bargs)
    dt_eager = time_runs(torch, lambda: bp.run(*bargs, out=bout), 3)
    bp.set_timing(True)
    bp.run(*bargs, out=bout)
    kms, _ = bp.last_kernel_ms()
    bp.set_timing(False)
    dt_graph, g = graph_time()
    blups = batch.lups
    # per-rod synchronous baseline on a sample of rods, scaled by work
    rng = np.random.default_rng(1)
    pick = rng.choice(batch.nrods, 128, replace=False)
    t_sample, w_sample = 0.0, 0
    for b in pick:
        s0, e0 = int(batch.offsets[b]), int(batch.offsets[b + 1])
        with SyncPlan(e0 - s0, torch.float32) as pl:
            xb = bargs[0][s0:e0].contiguous()
            t_sample += time_runs(torch, lambda: pl.run(xb, float(batch.r[b]), float(batch.c1[b]),
                                                        float(batch.cN[b]), int(batch.K[b])), 1)
        w_sample += (e0 - s0 - 2) * int(batch.K[b])
    est_per_rod_total = t_sample / w_sample * blups
    variants["batched_4096_rods_f32"] = {
        "glups_graph": round(blups / dt_graph / 1e9, 1), "glups_eager": round(blups / dt_eager / 1e9, 1),
        "ms_graph": round(dt_graph * 1e3, 3), "lups": blups, "plan": bp.describe(),
        "untuned": {"glups_graph": round(blups / dt_rule / 1e9, 1),
                    "ms_graph": round(dt_rule * 1e3, 3), "plan": plan_rule},
        "autotune_best_ms": round(tune_ms, 3),
        "per_rod_sync_estimate_ms": round(est_per_rod_total * 1e3, 1),
        "speedup_vs_per_rod_sync": round(est_per_rod_total / dt_graph, 2),
        "roofline": alu_roofline("batched_kernel<float>", FLOPS_PER_LUP * blups, kms,
                                 PEAK_FP32_TFLOPS, FLOPS_PER_LUP, plan="4096 rods")}
    log(f"[bench] batched: {variants['batched_4096_rods_f32']}")
    del bargs, bout, g
    bp.close()


def run_adjoint(torch, dev, SyncPlan, AdjointPlan, variants):
    B, NA, KA = 256, 1 << 16, 2000
    rng = np.random.default_rng(0)
    u0 = torch.from_numpy(rng.uniform(-1, 1, B * NA).astype(np.float32)).to(dev)
    with SyncPlan(NA, torch.float32, nrods=B) as tp:
        target = tp.run(u0, float(np.float32(0.35)), 0.0, 0.0, KA)
    adj = AdjointPlan(NA, KA, torch.float32, nrods=B)
    r3 = float(np.float32(0.3))

    def fwd_bwd():
        uK = adj.forward(u0, r3, 0.0, 0.0)
        return adj.backward(uK - target, r3, 0.0, 0.0)
    dt = time_runs(torch, fwd_bwd, 2)
    dt_f = time_runs(torch, lambda: adj.forward(u0, r3, 0.0, 0.0), 2)
    gK = adj.forward(u0, r3, 0.0, 0.0) - target
    adj.set_timing(True)
    adj.backward(gK, r3, 0.0, 0.0)
    st_ms, st_n = adj.last_kernel_ms()            # stretch_kernel launches of one backward
    adj.set_timing(False)
    dt_e = time_runs(torch, lambda: adj.ends(gK, r3), 3)
    alups = 2 * (NA - 2) * KA * B
    bwd_lups_per_launch = (NA - 2) * B * KA / max(st_n, 1)
    res = {"glups_fwd_adj": round(alups / dt / 1e9, 1), "ms": round(dt * 1e3, 3),
           "forward_ms": round(dt_f * 1e3, 3), "end_gradients_ms": round(dt_e * 1e3, 3),
           "ckpt_workspace_gb":
           round(adj.workspace(dev).numel() / 1e9, 2),
           "run_frac_of_fp32_peak": round(FLOPS_PER_LUP * alups / dt / 1e12 / PEAK_FP32_TFLOPS, 4),
           "roofline": alu_roofline(
               "stretch_kernel<float, 8, 24, true, true>", ADJ_FLOPS_PER_LUP * bwd_lups_per_launch,
               st_ms, PEAK_FP32_TFLOPS, ADJ_FLOPS_PER_LUP,
               "24 backward steps of all rods per launch; the forward recompute of the "
               "sub-stretch inside the kernel is not counted", plan="256 rods x 2^16, 24 steps")}
    adj.close()
    del u0, target, gK
    N1 = 1 << 20
    u1 = torch.from_numpy(rng.uniform(-1, 1, N1)).to(dev)
    with SyncPlan(N1, torch.float64) as tp:
        t1 = tp.run(u1, 0.35, 0.0, 0.0, KA)
    with AdjointPlan(N1, KA, torch.float64) as adj1:
        dt = time_runs(torch, lambda: adj1.backward(adj1.forward(u1, 0.3, 0.0, 0.0) - t1, 0.3,
                                                    0.0, 0.0), 2)
    res["f64_rod_2^20_glups_fwd_adj"] = round(2 * (N1 - 2) * KA / dt / 1e9, 1)
    variants["fwd_adjoint_256x2^16_f32_K2000"] = res
    log(f"[bench] fwd+adjoint: {res}")


def run_ring(torch, dev, rod, SyncPlan, abi, variants):
    """The synchronous periodic ring (Section 5.3) at the headline's size and
    input: N = 2^26 FP32 points on a ring, r = 0.25, K = 2000, ring tiles
    autotuned."""
    N, K = 1 << 26, 2000
    x = torch.from_numpy(rod.u0.astype(np.float32)).to(dev)
    r = float(np.float32(rod.r))
    with SyncPlan(N, torch.float32, boundary=abi.HEAT1D_BC_PERIODIC) as rp:
        rp.autotune(x, r, 256)
        rp.run(x, r, 0.0, 0.0, K)
        rp.set_timing(True)
        dt = time_runs(torch, lambda: rp.run(x, r, 0.0, 0.0, K), 3, 0)
        kms, nl = rp.last_kernel_ms()
        rp.set_timing(False)
        lups = N * K
        desc = rp.describe()
        variants["sync_ring_f32_N2^26_K2000"] = {
            "glups": round(lups / dt / 1e9, 1), "ms": round(dt * 1e3, 3), "plan": desc,
            "roofline": alu_roofline(pass_kernel(desc, "float", ring=True),
                                     FLOPS_PER_LUP * lups * 3 / max(nl, 1), kms,
                                     PEAK_FP32_TFLOPS, FLOPS_PER_LUP,
                                     plan=" ".join(x for x in desc.split()
                                                   if x[:2] in ("T=", "M=", "S=")
                                                   or (x[:2] == "W=" and x != "W=1")))}
    log(f"[bench] ring: {variants['sync_ring_f32_N2^26_K2000']}")
    del x


def run_async_ring(torch, dev, workloads, abi, SyncPlan, AsyncPlan, variants):
    """The asynchronous rod of Eq.4 closed into a ring (Section 5.3): the
    async rod's input (N = 2^24 FP32, r = 0.45), P = 1024 subdomains with
    subdomains 0 and 1023 neighbours, K = 5000, d = 4, both read policies,
    against the synchronous ring of the same input."""
    arod = workloads.async_rod(seed=0)
    N, K, P, d = arod.N, arod.K, 1024, 4
    x = torch.from_numpy(arod.u0.astype(np.float32)).to(dev)
    r = float(np.float32(arod.r))
    lups = N * K
    res = {}
    with SyncPlan(N, torch.float32, boundary=abi.HEAT1D_BC_PERIODIC) as sp:
        sp.autotune(x, r, 256)
        dt = time_runs(torch, lambda: sp.run(x, r, 0.0, 0.0, K), 2)
        ref = sp.run(x, r, 0.0, 0.0, K).clone()
        res["sync_ring"] = {"glups": round(lups / dt / 1e9, 1), "ms": round(dt * 1e3, 3),
                            "plan": sp.describe()}
    scale = float(ref.abs().max())
    with AsyncPlan(N, P, torch.float32, max_delay=d, periodic=True) as ap:
        for mode, mname in ((abi.HEAT1D_ASYNC_HARDWARE, "hardware"),
                            (abi.HEAT1D_ASYNC_EMULATED, "emulated")):
            stats = torch.zeros(d + 3, dtype=torch.int64, device=dev)
            ap.run(x, r, 0.0, 0.0, K, d, 11, mode, stats=stats)
            ap.set_timing(True)
            with Timer(torch) as t:
                out = ap.run(x, r, 0.0, 0.0, K, d, 11, mode)
            kms, _ = ap.last_kernel_ms()
            ap.set_timing(False)
            hist = stats.cpu().tolist()
            res[f"async_{mname}_d{d}"] = {
                "glups": round(lups / t.dt / 1e9, 1), "ms": round(t.dt * 1e3, 3),
                "kernel_ms": round(kms, 3), "status": ap.status(),
                "deviation_from_sync_ring": float((out - ref).abs().max()) / scale,
                "delay_histogram": hist[:d + 1], "polls": hist[d + 1],
                "roofline": alu_roofline(f"async_kernel<float, 64, {mode}, false, false>",
                                         FLOPS_PER_LUP * lups, kms, PEAK_FP32_TFLOPS,
                                         FLOPS_PER_LUP)}
        res["plan"] = ap.describe()
    res["note"] = STATS_NOTE
    variants["async_ring_N2^24_P1024_K5000_f32"] = res
    log(f"[bench] async ring: " + ", ".join(f"{k} {v['glups']}" for k, v in res.items()
                                            if isinstance(v, dict)))
    del x, ref


def run_ensemble(torch, dev, workloads, variants):
    """The paper's own experiment as an ensemble (Section 5, Figs. 3 and 6):
    300 emulated-async runs of the N = 100 rod, one grid point per subdomain,
    delays 0..3, K = 5000, the 2-norm after every step; Dirichlet ends and the
    periodic ring; and the gradients through every member's run.  FP64."""
    from paper_1510_08982_amd.heat import EnsemblePlan
    rod = workloads.paper_ensemble(members=300, N=100, K=5000, d=3)
    E, N, K, d = 300, rod.N, rod.K, rod.extra["d"]
    x = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(rod.u0, (E, N)))).to(dev)
    seeds = torch.from_numpy(rod.extra["seeds"].view(np.int64).copy()).to(dev)
    res = {"members": E, "N": N, "P": N, "d": d, "K": K}
    for name, periodic in (("dirichlet", False), ("periodic", True)):
        plan = EnsemblePlan(N, E, 0, torch.float64, periodic=periodic)
        out = {}

        def run(with_norms):
            out["r"] = plan.run(x, rod.r, rod.c1, rod.cN, K, d, seeds, 1, with_norms=with_norms)
        lups = E * ((N if periodic else N - 2) * K)
        dt = time_runs(torch, lambda: run(True), 3)
        norms = out["r"][1].cpu().numpy()
        dt0 = time_runs(torch, lambda: run(False), 3)
        plan.set_timing(True)
        run(True)
        kms, _ = plan.last_kernel_ms()
        plan.set_timing(False)
        plan.close()
        fin = norms[:, -1]
        res[name] = {"ms_with_norms": round(dt * 1e3, 3), "glups_with_norms": round(lups / dt / 1e9, 2),
                     "ms_without_norms": round(dt0 * 1e3, 3),
                     "glups_without_norms": round(lups / dt0 / 1e9, 2),
                     "final_norm_mean": round(float(fin.mean()), 6),
                     "final_norm_min": round(float(fin.min()), 6),
                     "final_norm_max": round(float(fin.max()), 6),
                     "initial_norm": round(float(norms[0, 0]), 6),
                     "roofline": alu_roofline(
                         f"ensemble_kernel<double, 1, {'true' if periodic else 'false'}>",
                         FLOPS_PER_LUP * lups, kms, PEAK_FP64_TFLOPS,
                         FLOPS_PER_LUP, "the run with a norm after every step; latency-bound: "
                         "one workgroup barrier per step and member, 98-100 points per member",
                         plan=f"300x100 K=5000 d=3 norms every step {name}")}
    # gradients through every member's run (Dirichlet ends)
    plan = EnsemblePlan(N, E, 0, torch.float64)
    gK = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, (E, N))).to(dev)
    plan.set_timing(True)
    dt = time_runs(torch, lambda: plan.adjoint(x, gK, rod.r, rod.c1, rod.cN, K, d, seeds), 2)
    bwd_ms, _ = plan.last_kernel_ms()
    plan.close()
    res["adjoint"] = {"ms": round(dt * 1e3, 3),
                      "glups_fwd_adj": round(2 * E * (N - 2) * K / dt / 1e9, 2),
                      "backward_kernel_ms": round(bwd_ms, 3),
                      "trajectory_workspace_mb": round((K + 1) * N * E * 8 / 1e6, 1)}
    variants["async_ensemble_paper_300x100_K5000_f64"] = res
    log(f"[bench] ensemble: {res}")


def measured_copy_gbs(torch, dev, nbytes=1 << 30, reps=5):
    """HBM bandwidth of a plain device-to-device copy of `nbytes` (read + write
    counted), timed with events on the current stream after one warm copy."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def cpu_one_thread(seconds=3.0):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1):
    a 2^24-point FP64 rod advanced 4 steps per call for about `seconds`."""
    code = (
        "import sys, time\n"
        "import numpy as np\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.abspath(__file__))!r})\n"
        "import oracle\n"
        "n = 1 << 24\n"
        "u = np.random.default_rng(0).uniform(-1.0, 1.0, n)\n"
        "oracle.sync(u[:4096], 0.25, 0.0, 0.0, 2)\n"
        "k, t0 = 0, time.perf_counter()\n"
        f"while time.perf_counter() - t0 < {seconds}:\n"
        "    u = oracle.sync(u, 0.25, 0.0, 0.0, 4)\n"
        "    k += 4\n"
        "dt = time.perf_counter() - t0\n"
        "print((n - 2) * k / dt / 1e9, oracle.num_threads(), k, dt)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                             timeout=120)
        v, thr, k, dt = res.stdout.split()
    except (subprocess.SubprocessError, ValueError):
        return None
    return {"value": round(float(v), 4), "unit": "GLUP/s", "cores": int(thr),
            "sample": f"a 2^24-point FP64 rod (U[-1,1], r=0.25), {k} steps in {float(dt):.1f} s"}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rod, seconds):
    """The oracle, as it stands, on a bounded sample of the headline workload:
    the whole rod (FP32-rounded input, FP64 arithmetic) advanced by calls of
    doubling length (each call pays the oracle's own set-up, so one short call
    says little about a long one), each sized to the time left at the previous
    call's rate, until about `seconds` of host time or all K steps are spent.
    The rate is all steps over all the time."""
    import oracle
    u = rod.u0.astype(np.float32).astype(np.float64)
    r = float(np.float32(rod.r))
    n = u.shape[0]
    oracle.sync(u[: 1 << 16], r, 0.0, 0.0, 4)      # thread pool and code warm
    done, calls, k, dt = 0, [], 20, 0.0
    while done < rod.K and k > 0:
        k = min(k, rod.K - done)
        t0 = time.perf_counter()
        u = oracle.sync(u, r, 0.0, 0.0, k)
        t = time.perf_counter() - t0
        done += k
        dt += t
        calls.append(k)
        k = int(min(2 * k, (seconds - dt) * k / max(t, 1e-6)))
    glups = (n - 2) * done / dt / 1e9
    log(f"[bench] cpu oracle: {glups:.3f} GLUP/s on {oracle.num_threads()} threads "
        f"({n} points x {done} steps in {dt:.1f} s, calls {calls})")
    one = cpu_one_thread()
    if one:
        log(f"[bench] cpu oracle on one thread: {one['value']:.3f} GLUP/s ({one['sample']})")
    return {"value": round(glups, 4), "unit": "GLUP/s", "cores": oracle.num_threads(),
            "one_thread": one,
            "kind": "oracle", "host_cpu": host_cpu_model(), "nproc": os.cpu_count(), "sample": f"the full N=2^26 rod of the headline workload "
                                        f"(FP32-rounded input, FP64 arithmetic), {done} of its "
                                        f"{rod.K} steps in {len(calls)} calls of doubling length, "
                                        f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
