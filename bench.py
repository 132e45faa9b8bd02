#!/usr/bin/env python3
"""Benchmark of one PDR sweep on one MI355X.

A step is one pass of the hot path over the whole instance: the excess ->
height reduction, the objective and stop test, and the arc update of every
(arc, commodity) pair. The workload is the 100 x 100 bidirectional grid
(n 10,000, m 39,600) with K = 10,000 commodities, demands scaled to load
factor 0.95 (synthetic, seeded; shaped like the paper's grid benchmark family).

Prints ONE JSON line. `value` is edge x commodity updates per second of PDR-ESO
in FP64 with all data resident in HBM. `roofline` prices the arc-update kernel
(the dominant kernel) against the MI355X HBM peak; `cpu_baseline` times the
FP64 CPU oracle on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PDR edge×commodity updates/s + time-to-residual 1e-8, FP32+polish vs FP64"
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")
CSRC = os.path.join(ROOT, "paper_2108_07549_amd", "csrc")


def kernel_sources():
    """The device code: the shared header and every kernel translation unit."""
    names = sorted(n for n in os.listdir(CSRC) if n.startswith("pdr_k_") and n.endswith(".hip"))
    return [os.path.join(CSRC, n) for n in ["pdr_device.h", *names]]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in kernel_sources():
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """Per-launch HBM bytes from the committed rocprofv3 counter summary, if it
    was taken from the current kernel source; else None."""
    try:
        with open(COUNTERS) as fh:
            tab = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = tab.get(key)
    if not entry or entry.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return entry.get("bytes_per_launch")


def time_variant(pdr, inst, method, precision, steps, warmup, **opts):
    """Warm up, then time exactly `steps` sweeps; returns timing and per-kernel ms."""
    ctx = pdr.Context.from_instance(inst, method=method, precision=precision, **opts)
    try:
        ctx.sweep(warmup)
        pdr.device_synchronize()
        t0 = time.perf_counter()
        kms = ctx.profile_sweeps(steps)
        pdr.device_synchronize()
        t1 = time.perf_counter()
        res = ctx.residual()
        tiling = ctx.tiling()
    finally:
        ctx.destroy()
    sec = t1 - t0
    return dict(seconds=sec, ms_per_step=1e3 * sec / steps,
                updates_per_s=inst.m * inst.K * steps / sec,
                kernel_ms_avg=dict(height_objective=kms[0] / steps, arc=kms[1] / steps),
                z_after=res["z"], tiling=dict(lanes_per_arc=tiling[0], vec_per_lane=tiling[1],
                                              Kp=tiling[2]))


def time_to_residual(pdr, inst, method, precision, budget_s, rungs, chunk=2048, window=256):
    """Run from f = 0 for about budget_s seconds (FP32-bulk runs hand over to the
    FP64 polish by pdr_solve's rule, judged on the windows inside each chunk);
    return the wall time and sweep count at which z first fell to each rung,
    and the final state."""
    out = {str(r): None for r in rungs}
    with pdr.Context.from_instance(inst, method=method, precision=precision) as ctx:
        pdr.device_synchronize()
        t0 = time.perf_counter()
        n32 = n64 = 0
        evals = 0
        while True:
            a, b = ctx.solve(min(rungs), chunk, window)
            n32 += a
            n64 += b
            now = time.perf_counter() - t0
            res = ctx.residual()
            new = res["evaluations"]
            zl = ctx.z_log(evals, new - evals)
            for r in rungs:
                if out[str(r)] is None:
                    hit = [q for q, z in enumerate(zl) if z <= r]
                    if hit:
                        # the pass that reached the rung, timed pro rata inside the chunk
                        out[str(r)] = dict(sweeps=evals + hit[0],
                                           seconds=now * (evals + hit[0] + 1) / max(new, 1))
            evals = new
            if res["stopped"] or now > budget_s or a + b == 0:
                break
    return dict(rungs=out, seconds=now, sweeps_fp32=n32, sweeps_fp64=n64, z_final=res["z"],
                precision_final="fp64" if n64 or precision == pdr.FP64 else "fp32")


LADDER = (1e4, 1e3, 1e2, 1e1, 1.0, 1e-1, 1e-2, 1e-4, 1e-6, 1e-8)


def time_to_target(pdr, inst, method, precision, target, cap, window=512, chunk=1_000_000,
                   tag="", seconds=0.0):
    """From f = 0, pdr_solve to z <= target (FP32-bulk runs widen to FP64 and
    polish by its rule; the rule's windows carry over from one solve call to
    the next); the wall time, the passes in each precision, and the first pass
    and (pro rata inside its call) the time at which z fell to each rung of a
    ladder. Runs longer than `chunk` passes are split into pdr_solve calls of
    `chunk` passes, with a progress line after each. seconds > 0 ends the run
    after the call that passes that wall time; the result then says how far it
    got and extrapolates the passes to the target from the descent rate of the
    last tenth of the run (labelled as an extrapolation)."""
    ladder = {str(t): None for t in LADDER if t >= target}
    ladder[str(target)] = None
    out = {}
    with pdr.Context.from_instance(inst, method=method, precision=precision) as ctx:
        pdr.device_synchronize()
        t0 = time.perf_counter()
        n32 = n64 = 0
        ev0 = 0
        handover = None
        floor = None
        while True:
            prev_sec = time.perf_counter() - t0
            a, b = ctx.solve(target, min(chunk, cap - n32 - n64), window)
            pdr.device_synchronize()
            if precision == pdr.FP32_BULK and b > 0 and handover is None:
                handover = n32 + a
            n32, n64 = n32 + a, n64 + b
            sec = time.perf_counter() - t0
            res = ctx.residual()
            if res["z_fp32_floor"] > 0:
                floor = res["z_fp32_floor"]
            ev = res["evaluations"]
            # the z log keeps the last 2^20 evaluations (chunk <= 2^20 covers them all)
            first = max(ev0, ev - (1 << 20))
            zl = ctx.z_log(first, ev - first)
            for thr in ladder:
                if ladder[thr] is None:
                    hit = np.nonzero(zl <= float(thr))[0]
                    if hit.size:
                        q = int(first + hit[0])
                        frac = (q - ev0 + 1) / max(ev - ev0, 1)
                        ladder[thr] = dict(sweeps=q, seconds=prev_sec + frac * (sec - prev_sec))
            ev0 = ev
            done = (res["z"] <= target or n32 + n64 >= cap or a + b == 0
                    or (seconds > 0 and sec >= seconds))
            print(f"[bench] ttr {tag}: {n32} + {n64} passes, z {res['z']:.4e}, {sec:.0f} s",
                  file=sys.stderr, flush=True)
            if done:
                break
        out = dict(seconds=sec, sweeps_fp32=n32, sweeps_fp64=n64, z_final=res["z"],
                   reached=bool(res["z"] <= target), verdict=res["verdict"], rungs=ladder,
                   solve_calls_of=chunk, handover_at_pass=handover, z_fp32_floor=floor)
        if not out["reached"] and ev >= 2:
            tail = max(10, (n32 + n64) // 10)
            first = max(0, ev - min(tail, 1 << 20))
            zl = ctx.z_log(first, ev - first)
            if zl[-1] > 0 and zl[0] > zl[-1]:
                rate = np.log(zl[0] / zl[-1]) / (len(zl) - 1)
                more = float(np.log(zl[-1] / target) / rate)
                # further passes cost what the last call's passes cost (an FP32
                # run that has handed over continues in FP64)
                per_pass = (sec - prev_sec) / max(a + b, 1)
                out["extrapolation"] = dict(
                    kind="extrapolated from the descent rate of the last "
                         f"{len(zl) - 1} passes; not measured",
                    rate_per_pass=float(rate), further_passes=more,
                    total_passes=float(n32 + n64 + more),
                    total_seconds=float(sec + more * per_pass))
    return out


def time_batch(pdr, B, seed, method, precision, steps, warmup, tune_reps):
    """Batched sweeps of the uneven B-instance recipe: wall-clock updates/s of
    plain sweeps before and after the tiling autotuner, and the per-launch
    split from HIP events. With steps and warmup multiples of the batch's
    graph length (32 passes) the timed passes are graph replays, the warm-up
    capturing the graphs."""
    from gen.batch import recipe_batch
    t0 = time.perf_counter()
    insts = recipe_batch(B, seed)
    gen_s = time.perf_counter() - t0
    print(f"[bench] batch: {B} instances generated ({gen_s:.1f} s)", file=sys.stderr, flush=True)
    w = 8 if precision == pdr.FP64 else 4
    upd = sum(i.m * i.K for i in insts)
    sweep_bytes = sum(w * (3 * i.m * i.K + 2 * i.n * i.K) for i in insts)
    cert = {}
    for i in insts:
        cert[i.meta.get("certified", "unknown")] = cert.get(i.meta.get("certified", "unknown"), 0) + 1

    def timed(b):
        b.sweep(warmup)
        pdr.device_synchronize()
        t = time.perf_counter()
        b.sweep(steps)
        pdr.device_synchronize()
        sec = time.perf_counter() - t
        kms = b.profile_sweeps(steps)
        return dict(ms_per_step=1e3 * sec / steps, updates_per_s=upd * steps / sec,
                    frac=sweep_bytes / (sec / steps) / 1e9 / HBM_PEAK_GBS,
                    kernel_ms_avg=dict(height_objective=kms[0] / steps, arc=kms[1] / steps))

    t0 = time.perf_counter()
    with pdr.Batch(insts, method=method, precision=precision) as b:
        init_s = time.perf_counter() - t0
        auto = timed(b)
        auto["buckets"] = b.buckets()
        print(f"[bench] batch: automatic tilings {auto['ms_per_step']:.3f} ms/sweep; tuning",
              file=sys.stderr, flush=True)
        tuned = b.tune(tune_reps)
        after = timed(b)
        after["buckets"] = tuned
        after["height_blocks"] = b.height_blocks
    return dict(workload=f"batch{B}_knn (seed {seed})", instances=B,
                updates_per_sweep=upd, algorithmic_bytes_per_sweep=sweep_bytes,
                certified=cert, generate_s=gen_s, init_s=init_s, auto=auto, tuned=after)


def batch_verdicts(pdr, insts, method, seconds, members=96, chunk=5000):
    """The `members` members of least work (m K) of the batch swept together in
    FP64 for about `seconds` of wall time; every member's verdict (Farkas gap >
    tau: infeasible; z <= 1e-8: feasible) against its certified label
    (gen.batch: column-generation brackets)."""
    order = sorted(range(len(insts)), key=lambda q: insts[q].m * insts[q].K)[:members]
    insts = [insts[q] for q in sorted(order)]
    with pdr.Batch(insts, method=method, precision=pdr.FP64) as b:
        t0 = time.perf_counter()
        passes = 0
        timeline = []  # (passes, seconds, members decided) about once a minute
        next_mark = 60.0
        while True:
            b.sweep(chunk)
            pdr.device_synchronize()
            passes += chunk
            el = time.perf_counter() - t0
            print(f"[bench] batch verdicts: {passes} passes, {el:.0f} s", file=sys.stderr,
                  flush=True)
            if el >= next_mark or el >= seconds:
                dec = sum(b.member(q).residual()["verdict"] != "undecided"
                          for q in range(len(insts)))
                timeline.append(dict(passes=passes, seconds=el, decided=int(dec)))
                next_mark += 60.0
            if el >= seconds:
                break
        sec = time.perf_counter() - t0
        out = dict(members=len(insts), passes=passes, seconds=sec, decided=0, agree=0,
                   disagree=0, undecided=0, by_label={}, timeline=timeline)
        for q, inst in enumerate(insts):
            v = b.member(q).residual()["verdict"]
            lab = inst.meta.get("certified", "uncertified")
            row = out["by_label"].setdefault(lab, dict(members=0, feasible=0, infeasible=0,
                                                       undecided=0))
            row["members"] += 1
            row[v] += 1
            if v == "undecided":
                out["undecided"] += 1
            else:
                out["decided"] += 1
                out["agree" if v == lab else "disagree"] += 1
    return out


def time_long_rows(pdr, steps, warmup):
    """Sweeps of the 2,500-vertex k-NN instance with K = 81,430 (rows streamed
    by the arc kernels), per method and precision, against the HBM roofline of
    the two-phase sweep's algorithmic bytes."""
    from gen.instance import load_instance
    inst = load_instance("knn2500_k81430")
    n, m, K = inst.n, inst.m, inst.K
    out = dict(workload="knn2500_k81430", n=n, m=m, K=K, lf_bracket=inst.meta.get("lf_bracket"))
    for name, meth, prec in (("eso_fp64", pdr.ESO, pdr.FP64), ("eso_fp32", pdr.ESO, pdr.FP32_BULK),
                             ("agd_fp64", pdr.AGD, pdr.FP64), ("gdm_fp64", pdr.GDM, pdr.FP64)):
        r = time_variant(pdr, inst, meth, prec, steps, warmup)
        w = 8 if prec == pdr.FP64 else 4
        sweep_bytes = w * (3 * m * K + 2 * n * K) + (2 * w * m * K if meth == pdr.GDM else 0)
        arc_bytes = w * (2 * m * K + n * K) + (2 * w * m * K if meth == pdr.GDM else 0)
        arc_ms = r["kernel_ms_avg"]["arc"]
        out[name] = dict(ms_per_step=r["ms_per_step"], updates_per_s=r["updates_per_s"],
                         kernel_ms_avg=r["kernel_ms_avg"], tiling=r["tiling"],
                         sweep_frac=sweep_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         arc_frac=arc_bytes / (arc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        print(f"[bench] long rows {name}: {r['ms_per_step']:.3f} ms/sweep", file=sys.stderr,
              flush=True)
    return out


def time_adjoint(pdr, inst, T, checkpoint, forward_ms):
    """Wall time of pdr_adjoint (T forward passes, the recomputation and the
    reverse sweep) from f = 0, and its cost in forward-sweep equivalents."""
    with pdr.Context.from_instance(inst, method=pdr.ESO) as c:
        c.adjoint(1, 1)  # warm up (kernels loaded, buffers touched)
    with pdr.Context.from_instance(inst, method=pdr.ESO) as c:
        pdr.device_synchronize()
        t0 = time.perf_counter()
        z, gu, gd = c.adjoint(T, checkpoint)
        sec = time.perf_counter() - t0
    return dict(T=T, checkpoint=checkpoint, seconds=sec, ms_per_pass=1e3 * sec / T,
                forward_sweeps_per_pass=(1e3 * sec / T) / forward_ms, z=z,
                max_abs_grad_u=float(np.max(np.abs(gu))), max_abs_grad_d=float(np.max(np.abs(gd))))


def host_identity() -> dict:
    """The host CPU as /proc/cpuinfo names it: model, logical CPUs this process
    may use, and physical cores (distinct (package, core) pairs)."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                elif not key and phys is not None and core is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return dict(cpu_model=model, logical_cpus_usable=usable, logical_cpus=os.cpu_count(),
                physical_cores=len(cores) or None)


def cpu_baseline(inst, sweeps, single_sweeps):
    import oracle
    t0 = time.perf_counter()
    oracle.run(inst, oracle.ESO, sweeps)
    sec = time.perf_counter() - t0
    out = dict(value=inst.m * inst.K * sweeps / sec, unit="updates/s",
               cores=oracle.num_threads(), kind="oracle",
               sample=f"{sweeps} PDR-ESO FP64 sweeps of the full workload from f = 0 "
                      f"({sec:.1f} s)", host=host_identity())
    if single_sweeps > 0:
        nt = oracle.num_threads()
        oracle.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            oracle.run(inst, oracle.ESO, single_sweeps)
            sec1 = time.perf_counter() - t0
        finally:
            oracle.set_num_threads(nt)
        out["single_thread"] = dict(
            value=inst.m * inst.K * single_sweeps / sec1, unit="updates/s", cores=1,
            sample=f"{single_sweeps} sweeps from f = 0 ({sec1:.1f} s)")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="grid100_k10000")
    ap.add_argument("--cpu-sweeps", type=int, default=48,
                    help="oracle sweeps of the CPU baseline (about 13 s on 16 host threads)")
    ap.add_argument("--cpu-single-sweeps", type=int, default=8,
                    help="oracle sweeps of the one-thread CPU figure, about 10 s (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=2 << 30,
                    help="buffer size of the plain-copy HBM reference (0: skip)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched 256-instance workload")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint (reverse-mode gradient) timing")
    ap.add_argument("--no-long-rows", action="store_true",
                    help="skip the K = 81,430 (streamed rows) workload")
    ap.add_argument("--verdict-seconds", type=float, default=60.0,
                    help="wall time of the batch verdict run on the 96 members of least "
                         "work (0: skip)")
    ap.add_argument("--ttr-budget", type=float, default=6.0,
                    help="seconds per variant of the time-to-residual ladder (0: skip)")
    ap.add_argument("--ttr-workload", default="knn2500_k1000",
                    help="run FP64 and FP32 bulk + FP64 polish to z <= 1e-8 on this workload "
                         "(about two minutes for ESO and GDM); 'none' skips it")
    ap.add_argument("--ttr-methods", default="eso,gdm",
                    help="methods of --ttr-workload (eso, agd, gdm, cap)")
    ap.add_argument("--ttr-cap", type=int, default=2_000_000,
                    help="pass limit of each --ttr-workload run")
    ap.add_argument("--ttr-seconds", type=float, default=0.0,
                    help="wall-time limit of each --ttr-workload run (0: none); a run that "
                         "stops short reports the rungs it reached and an extrapolation")
    ap.add_argument("--ttr-chunk", type=int, default=1_000_000,
                    help="passes per pdr_solve call of the --ttr-workload runs")
    ap.add_argument("--ttr-precisions", default="fp64,fp32_polish",
                    help="forms of the --ttr-workload runs (fp64, fp32_polish)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design, not a build).", file=sys.stderr)
        sys.exit(2)

    import paper_2108_07549_amd as pdr
    from gen.instance import load_instance

    inst = load_instance(args.workload)
    print(f"[bench] {args.workload}: n {inst.n} m {inst.m} K {inst.K}; "
          f"{args.warmup} warmup + {args.steps} timed sweeps", file=sys.stderr, flush=True)
    head = time_variant(pdr, inst, pdr.ESO, pdr.FP64, args.steps, args.warmup)
    print(f"[bench] eso fp64: {head['ms_per_step']:.3f} ms/sweep", file=sys.stderr, flush=True)

    copy_gbs = None
    if args.copy_bytes > 0:
        copy_gbs = pdr.measure_copy(args.copy_bytes, 5)
        print(f"[bench] plain copy of {args.copy_bytes} bytes: {copy_gbs:.0f} GB/s",
              file=sys.stderr, flush=True)
    n, m, K = inst.n, inst.m, inst.K
    w = 8
    arc_bytes = w * (2 * m * K + n * K)  # read f, write f, read each h row once
    arc_ms = head["kernel_ms_avg"]["arc"]
    achieved = arc_bytes / (arc_ms * 1e-3) / 1e9
    traffic = measured_traffic(f"k_eso_fp64:{args.workload}")
    sweep_bytes = w * (3 * m * K + 2 * n * K)
    out = {
        "metric": METRIC,
        "value": head["updates_per_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "K": K, "method": "eso",
                   "precision": "fp64",
                   # the demands are scaled to this load factor against an explicit
                   # routing; the certified load factor lies in lf_bracket
                   "load_factor_target": inst.meta.get("load_factor"),
                   "lf_bracket": inst.meta.get("lf_bracket"), "tiling": head["tiling"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_eso<double>", "algorithmic_bytes_per_launch": arc_bytes,
                     "avg_launch_ms": arc_ms},
        "sweep_roofline": {"algorithmic_bytes": sweep_bytes,
                           "achieved_GBs": sweep_bytes / (head["ms_per_step"] * 1e-3) / 1e9,
                           "frac": sweep_bytes / (head["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "kernel_ms_avg": head["kernel_ms_avg"],
        "hbm_copy_GBs": copy_gbs,
    }
    if not args.no_variants:
        var = {}
        for name, meth, prec in (("agd_fp64", pdr.AGD, pdr.FP64), ("gdm_fp64", pdr.GDM, pdr.FP64),
                                 ("eso_fp32", pdr.ESO, pdr.FP32_BULK),
                                 ("agd_fp32", pdr.AGD, pdr.FP32_BULK),
                                 ("gdm_fp32", pdr.GDM, pdr.FP32_BULK),
                                 ("cap_fp64", pdr.CAP, pdr.FP64),
                                 # the LDS-tiled height kernel (pdr_options.height_kernel 2)
                                 ("eso_fp64_tiled_height", pdr.ESO, pdr.FP64),
                                 ("eso_fp32_tiled_height", pdr.ESO, pdr.FP32_BULK)):
            opts = dict(height_kernel=2) if name.endswith("_tiled_height") else {}
            r = time_variant(pdr, inst, meth, prec, args.steps, args.warmup, **opts)
            print(f"[bench] {name}: {r['ms_per_step']:.3f} ms/sweep", file=sys.stderr, flush=True)
            var[name] = dict(updates_per_s=r["updates_per_s"], ms_per_step=r["ms_per_step"],
                             kernel_ms_avg=r["kernel_ms_avg"], tiling=r["tiling"])
        out["variants"] = var
    if args.ttr_budget > 0:
        ttr = {}
        for name, prec in (("fp64", pdr.FP64), ("fp32_polish", pdr.FP32_BULK)):
            r = time_to_residual(pdr, inst, pdr.ESO, prec, args.ttr_budget,
                                 [1e5, 1e4, 1e3, 1e2, 1e1, 1.0, 1e-8])
            print(f"[bench] ttr eso {name}: {r}", file=sys.stderr, flush=True)
            ttr[name] = r
        out["time_to_residual"] = dict(method="eso", budget_s_per_variant=args.ttr_budget,
                                       target=1e-8, **ttr)
    if args.ttr_workload and args.ttr_workload != "none":
        tinst = load_instance(args.ttr_workload)
        full = dict(workload=args.ttr_workload, target=1e-8, cap=args.ttr_cap)
        names = {"eso": pdr.ESO, "agd": pdr.AGD, "gdm": pdr.GDM, "cap": pdr.CAP}
        forms = [(p, {"fp64": pdr.FP64, "fp32_polish": pdr.FP32_BULK}[p])
                 for p in args.ttr_precisions.split(",") if p]
        full.update(seconds_limit=args.ttr_seconds or None, solve_call_passes=args.ttr_chunk)
        for mname in [x for x in args.ttr_methods.split(",") if x]:
            for pname, prec in forms:
                print(f"[bench] ttr {args.ttr_workload} {mname} {pname}: running", file=sys.stderr,
                      flush=True)
                r = time_to_target(pdr, tinst, names[mname], prec, 1e-8, args.ttr_cap,
                                   chunk=args.ttr_chunk, tag=f"{args.ttr_workload} {mname} {pname}",
                                   seconds=args.ttr_seconds)
                print(f"[bench] ttr {args.ttr_workload} {mname} {pname}: {r}", file=sys.stderr,
                      flush=True)
                full[f"{mname}_{pname}"] = r
        out["time_to_residual_full"] = full
    if not args.no_adjoint:
        r = time_adjoint(pdr, inst, 8, 4, head["ms_per_step"])
        print(f"[bench] adjoint T=8: {r['ms_per_pass']:.3f} ms per pass "
              f"({r['forward_sweeps_per_pass']:.2f} forward sweeps)", file=sys.stderr, flush=True)
        out["adjoint"] = r
    if not args.no_batch:
        bat = {}
        for name, prec in (("eso_fp32", pdr.FP32_BULK), ("eso_fp64", pdr.FP64)):
            r = time_batch(pdr, 256, 4, pdr.ESO, prec, 64, 32, 3)
            print(f"[bench] batch {name}: auto {r['auto']['ms_per_step']:.3f} ms/sweep, tuned "
                  f"{r['tuned']['ms_per_step']:.3f} ms/sweep", file=sys.stderr, flush=True)
            bat[name] = r
        if args.verdict_seconds > 0:
            from gen.batch import recipe_batch
            v = batch_verdicts(pdr, recipe_batch(256, 4), pdr.GDM, args.verdict_seconds)
            print(f"[bench] batch verdicts: {v}", file=sys.stderr, flush=True)
            bat["verdicts_gdm_fp64"] = v
        out["batch"] = bat
    if not args.no_long_rows:
        out["long_rows"] = time_long_rows(pdr, min(args.steps, 20), min(args.warmup, 3))
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: {args.cpu_sweeps} oracle sweeps", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_sweeps, args.cpu_single_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
