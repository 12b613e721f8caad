"""Benchmark: converged NLP solves/sec of the batched interior-point solver on one MI355X.

A step is one batched solve of the whole workload (every instance run to convergence through
all method steps: derivatives, KKT assembly + inertia-correcting factorization, step, filter
line search with SOC, restoration, barrier update, slot refill).  `value` is the plain form:
C2, figure-eight tracking NMPC, 4096 instances, N = 30, 8 obstacles, FP64, cold start; the timed
batches are streamed one after another through as many slots as the GPU keeps resident in the
asynchronous-slot kernel (hipipm_resident_slots), in one launch: every slot runs passes back to
back and refills from the device queue until the stream is done.

The same run measures the other half of the metric, the warm/mixed form (object `warm_mixed`):
the learned warm start on 16384 point-to-point instances (N = 10, 3 obstacles).  Outside the
timed region the network is trained on cold FP64 solutions of a separate training split and the
warm barrier parameter is picked on a validation split; a timed step is the network's forward
pass plus the warm-started solve with the FP32 factor and FP64 refinement, beside the cold FP64
solve of the same instances, and both are checked against the oracle on a subsample.  A third
leg times one C2 solve with the per-phase kernels so that the factorization and the solve get
durations and roofline fractions of their own.

Prints one JSON line.  The roofline object is the dominant kernel's algorithmic HBM bytes per
launch (`kernel_roofline`: bytes per stage of a factorization and of a solve, times the stages
and the factorizations and solves the launches ran) over its average launch time from HIP events.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


# HBM traffic of the dominant kernel from the two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE)
# scaled by the same counters on a plain device copy of known size, per slot-iteration the
# launches ran; a run's traffic per launch is that times its iterations per launch.  Valid only
# for the kernel sources they were taken on (hash below), the workload and the slot count named.
MEASURED_TRAFFIC = {"k_run": {"csrc": "4229ab4a956f632a", "workload": "C2", "slots": 1024,
                              "bytes_per_iteration": 1.0454e6}}


# the sources the FP64 asynchronous-slot kernel k_run<false> is built from
K_RUN_SOURCES = ("common.h", "kkt.h", "model.h", "slot.h", "run_fp64.hip")


def csrc_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_26341_amd", "csrc")
    for f in K_RUN_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes of the KKT factor/solve per stage (single quadrotor, n_x = 13, n_u = 4, FP64
# words).  A factorization attempt reads the stage Hessian H (17 x 18 / 2 = 153), the dynamics
# Jacobian G (13 x 17 = 221), the dual regularisation Delta (13) and the stage right-hand side
# (30), and writes L_u (10), K = L_u^-1 Hbar^ux (52), S (13 x 14 / 2 = 91) and the affine terms
# (17): 587 words.  A solve reads the factor record (170), G (221) and the right-hand side (30)
# and writes the step (30): 451 words.  There are N + 1 stages (knots).
FACTOR_WORDS_PER_STAGE = 153 + 221 + 13 + 30 + 10 + 52 + 91 + 17
SOLVE_WORDS_PER_STAGE = 170 + 221 + 30 + 30
# flops per stage of one factorization attempt (Schur update G^T S G, Cholesky of Hbar^uu, the
# control elimination and P = Hbar^xx - Y^T Y), for the FP64 fraction
FACTOR_FLOPS_PER_STAGE = 10.8e3


def kernel_roofline(w, st, kt, word_bytes=8.0):
    """Roofline of the dominant kernel from the live HIP-event timings.

    k_fac is charged its factorization attempts, k_sol its solves and the fused pass kernel
    k_iter, and the asynchronous-slot kernel k_run, both (SOC solves included); the pre-processing,
    line-search (and, in k_run, derivative) work is not charged, so their figures are lower bounds.
    `word_bytes` is 4 when the factor runs in FP32."""
    S = w.N + 1
    fb = word_bytes * FACTOR_WORDS_PER_STAGE * S
    sb = word_bytes * SOLVE_WORDS_PER_STAGE * S
    names = ("eval", "pre", "factor", "solve", "linesearch", "fused", "async")
    tot = {k: kt[k][0] for k in names if k in kt and kt[k][1] > 0}
    out = {}
    for k in tot:
        ms, launches = kt[k]
        avg_ms = ms / launches
        if k == "factor":
            units = st["factorizations"] - st["fused_factorizations"]
            per_launch, flops = fb * units / launches, FACTOR_FLOPS_PER_STAGE * S * units / launches
            desc = f"{units} factorizations x {S} stages x {fb / S:.0f} B"
        elif k == "solve":
            units = st["solves"] - st["fused_solves"]
            per_launch, flops = sb * units / launches, 0.0
            desc = f"{units} solves x {S} stages x {sb / S:.0f} B"
        elif k in ("fused", "async"):
            per_launch = (fb * st["fused_factorizations"] + sb * st["fused_solves"]) / launches
            flops = FACTOR_FLOPS_PER_STAGE * S * st["fused_factorizations"] / launches
            desc = (f"{st['fused_factorizations']} factorizations x {S} stages x {fb / S:.0f} B + "
                    f"{st['fused_solves']} solves x {S} stages x {sb / S:.0f} B")
        else:
            continue
        ach = per_launch / (avg_ms * 1e-3) / 1e9
        out["k_" + {"factor": "fac", "solve": "sol", "fused": "iter", "async": "run"}[k]] = dict(
            bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS, traffic=None,
            avg_ms=avg_ms, launches=launches, bytes_per_launch=per_launch, units=desc,
            fp64_tflops=flops / (avg_ms * 1e-3) / 1e12, fp64_frac=flops / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            share_of_gpu_time=ms / sum(tot.values()))
    dom = max(out, key=lambda k: out[k]["share_of_gpu_time"]) if out else None
    return dom, out


def cpu_info():
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(w, sample: int, threads: int):
    """The oracle on a seeded uniform sample of the workload's instances (slow ones included)."""
    import oracle
    idx = np.sort(np.random.default_rng(20261203).choice(w.n_inst, size=min(sample, w.n_inst), replace=False))
    TH = np.stack([w.theta(int(i)) for i in idx])
    t0 = time.perf_counter()
    o = oracle.solve_quad(w, TH, threads=threads)
    dt = time.perf_counter() - t0
    conv = int((o["status"] == oracle.ST_CONVERGED).sum())
    model, _ = cpu_info()
    return dict(value=conv / dt, unit="solves/s", cores=min(threads, len(idx)), kind="oracle",
                sample=f"{len(idx)} {w.name} instances drawn uniformly (seeded) from {w.n_inst}, dense FP64 "
                       f"oracle, one instance per thread, {dt:.1f} s wall, {conv} converged, "
                       f"{int(o['iters'].sum())} iterations",
                cpu=model, host_threads=threads)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C2", help="workload of the plain FP64 cold-start leg (`value`)")
    ap.add_argument("--slots", type=int, default=0,
                    help="slots of the plain and warm/mixed legs (default: the slots the GPU keeps resident in the "
                         "asynchronous-slot kernel, hipipm_resident_slots)")
    ap.add_argument("--instances", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle instances for the CPU baseline (default: about 10-30 s of host work per workload)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm/mixed (C5) leg")
    ap.add_argument("--no-phase-leg", action="store_true", help="skip the per-phase-kernel leg")
    ap.add_argument("--no-stream", action="store_true",
                    help="one solve per timed step instead of streaming the steps' batches through the slots")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (HBM counter calibration) and exit")
    ap.add_argument("--precision", type=int, default=None,
                    help="KKT factor precision of the plain leg: 0 FP64, 1 FP32 + FP64 refinement (default 0)")
    ap.add_argument("--train", type=int, default=190000, help="warm-start training instances (C5)")
    ap.add_argument("--val", type=int, default=10000, help="warm-start validation instances (C5)")
    ap.add_argument("--epochs", type=int, default=30, help="warm-start training epochs (C5)")
    ap.add_argument("--oracle-check", type=int, default=1024, help="C5 instances re-solved by the oracle")
    ap.add_argument("--async-passes", type=int, default=1 << 20,
                    help="passes each slot runs per launch of the asynchronous-slot kernel, plain and warm/mixed "
                         "legs (0: one launch per pass)")
    ap.add_argument("--fuse-below", type=int, default=None,
                    help="unfinished-instance count below which passes use the fused kernel (default: library's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus above 1 is not supported (instances are "
                                   "independent and would shard across GPUs with no exchange)"}))
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = 1 << 25                      # 2^25 doubles = 256 MiB read + 256 MiB written per copy
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "copies": 4}), flush=True)
        return
    from paper_2606_26341_amd import hipipm, workloads as W

    w = W.get(args.workload)
    n_inst = args.instances or w.n_inst
    TH = torch.tensor(w.thetas(0, n_inst), dtype=torch.float64, device="cuda:0")
    opts = dict(timing=1, precision=args.precision or 0, async_passes=args.async_passes)
    if args.fuse_below is not None:
        opts["fuse_below"] = args.fuse_below
    slots = args.slots or hipipm.resident_slots(w, hipipm.default_options(**opts))
    log(f"[bench] plain leg {w.name}: {n_inst} instances, N={w.N}, n={w.n}, m={w.m}, slots={slots}, "
        f"{'streamed' if not args.no_stream else 'one solve per step'}")
    solver = hipipm.Solver(w, slots, hipipm.default_options(**opts))
    dt, conv, out, st, kt = time_solves(solver, TH, args.steps, args.warmup, stream=not args.no_stream)
    log(f"[bench] timed {args.steps} steps in {dt:.3f} s; stats {st}; kernel ms {kt}")
    # one batch on its own (not streamed), after the timed region: the latency of a single batch,
    # bounded below by its slowest instance
    o1 = solver.alloc_outputs(n_inst)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    solver.solve(TH, out=o1)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t1) * 1e3
    del o1
    # the stream's marginal rate (context, not `value`): a stream of half the timed batches beside
    # the timed one; the difference is the cost of the extra batches without the stream's end,
    # which is the slowest instance's own latency
    marginal = None
    if not args.no_stream and args.steps >= 4:
        half = args.steps // 2
        TSh = TH.repeat(half, 1).contiguous()
        oh = solver.alloc_outputs(TSh.shape[0])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        solver.solve(TSh, out=oh)
        torch.cuda.synchronize()
        half_s = time.perf_counter() - t2
        conv_half = int((oh["status"] == 1).sum().item())
        del oh, TSh
        if dt > half_s:
            marginal = dict(batches=[half, args.steps], seconds=[half_s, dt],
                            solves_per_sec=(conv - conv_half) / (dt - half_s))
    dom, roofs = kernel_roofline(w, st, kt, word_bytes=4.0 if opts["precision"] == 1 else 8.0)
    roof = roofs[dom]
    mt = MEASURED_TRAFFIC.get(dom)
    if mt and mt["csrc"] == csrc_hash() and mt["workload"] == w.name and mt["slots"] == slots:
        roof["traffic"] = mt["bytes_per_iteration"] * st["iterations"] / roof["launches"]
    kkt = out["kkt"].cpu().numpy()
    status = out["status"].cpu().numpy()
    desc = {"C2": "C2: figure-eight tracking NMPC, FP64 cold start"}
    res = {
        "metric": "converged NLP solves/sec on 1 MI355X at KKT tol 1e-8 (plain vs warm/mixed)",
        "value": conv / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if opts["precision"] == 0 else "f32 factor + f64 refinement",
        "data": "synthetic",
        "config": {"workload": desc.get(w.name, w.name), "instances": n_inst, "horizon_N": w.N, "n_obs": w.n_obs,
                   "n": w.n, "m": w.m, "slots": slots,
                   "batches": ("the timed steps streamed through the slots in one solve (iteration-level "
                               "batching across batches)") if not args.no_stream else "one solve per step",
                   "pass_kernel": (f"asynchronous slots: every slot runs up to {args.async_passes} whole passes "
                                   "per launch, refilling from the device queue" if args.async_passes > 0
                                   else "one launch per pass"),
                   "obstacles": "centres on the reference path + N(0, 0.5^2 I), kept 0.1 m from the start and "
                                "0.3 m from the first 0.5 s of the reference"},
        "single_batch_ms": single_ms,
        "stream_marginal": marginal,
        "single_batch_solves_per_sec": float((out["status"] == 1).sum().item()) / (single_ms * 1e-3),
        "iterations_per_sec": st["iterations"] / dt,
        "iterations_per_solve": float(out["iters"].float().mean().item()),
        "converged_fraction": float((status == 1).mean()),
        "status_histogram": {hipipm.STATUS[k]: int((status == k).sum()) for k in sorted(hipipm.STATUS)},
        "max_kkt_converged": float(kkt[status == 1].max()) if (status == 1).any() else None,
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": dom,
        "roofline_detail": {k: roof[k] for k in ("avg_ms", "launches", "bytes_per_launch", "units", "fp64_tflops",
                                                 "fp64_frac", "share_of_gpu_time")},
        "kernel_ms": {k: v[0] for k, v in kt.items()},
        "stats": {k: st[k] for k in ("iterations", "resto_iterations", "resto_entries", "soc_tried", "soc_accepted",
                                     "tiny_steps", "factorizations")},
    }
    if not args.no_phase_leg:
        res["per_phase_leg"] = phase_leg(w, TH, n_inst)
    if not args.no_warm:
        res["warm_mixed"] = warm_mixed_leg(args)
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        _, threads = cpu_info()
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_sample or CPU_SAMPLE.get(w.name, 64), threads)
    print(json.dumps(res), flush=True)


# oracle sample sizes sized to about 10-30 s of host work (dense FP64 factorizations grow with N^3)
CPU_SAMPLE = {"C1": 64, "C2": 64, "C4": 32}


def phase_leg(w, TH, slots):
    """One solve of the plain workload with the per-phase kernels (no fused pass kernel), so that
    the factorization (k_fac) and the solve (k_sol) have launch durations and rooflines of their own."""
    from paper_2606_26341_amd import hipipm
    s = hipipm.Solver(w, slots, hipipm.default_options(timing=1, fuse_below=0))
    dt, conv, out, st, kt = time_solves(s, TH, 1, 1)
    _, roofs = kernel_roofline(w, st, kt)
    log(f"[bench] per-phase leg: {dt * 1e3:.1f} ms, kernel ms {kt}")
    return dict(ms_per_step=dt * 1e3, solves_per_sec=conv / dt, kernel_ms={k: v[0] for k, v in kt.items()},
                rooflines={k: {q: v[q] for q in ("achieved", "frac", "avg_ms", "launches", "bytes_per_launch",
                                                 "fp64_tflops", "share_of_gpu_time")} for k, v in roofs.items()})


def warm_mixed_leg(args):
    """The warm/mixed form on C5: network forward pass + warm-started FP32-factor / FP64-refinement
    solve of 16384 instances, beside the cold FP64 solve of the same instances, with the oracle's
    warm solves from the same network rows on a subsample."""
    import torch
    from paper_2606_26341_amd import hipipm, workloads as W
    w = W.get("C5")
    TH = torch.tensor(w.thetas(0, w.n_inst), dtype=torch.float64, device="cuda:0")
    opts = dict(timing=1, precision=1, async_passes=args.async_passes)
    warm_fn, extra = setup_warm_start(w, TH, opts, args)
    slots = args.slots or hipipm.resident_slots(w, hipipm.default_options(**opts))
    s = hipipm.Solver(w, slots, hipipm.default_options(**opts))
    dt, conv, out, st, kt = time_solves(s, TH, args.steps, args.warmup, warm_fn, stream=not args.no_stream)
    log(f"[bench] warm/mixed: {args.steps} steps in {dt:.3f} s; stats {st}")
    res = dict(workload="C5: point-to-point NMPC, 16384 instances, N = 10, 3 obstacles; learned BF16 warm start "
                        "+ FP32 factor with FP64 refinement",
               slots=slots, solves_per_sec=conv / dt, ms_per_step=dt * 1e3 / args.steps,
               iterations_per_solve=float(out["iters"].float().mean().item()),
               max_iterations=int(out["iters"].max().item()),
               converged_fraction=float((out["status"] == 1).float().mean().item()),
               warm_started=st["warm_started"], warm_rejected=st["warm_rejected"],
               warm_restarts=st["warm_restarts"],
               fallback_rate=(st["warm_rejected"] + st["warm_restarts"]) / max(1, st["instances_done"]),
               fp64_refactorizations=st["fp64_fallbacks"], fp32_retakes=st["fp32_retakes"],
               refine_sweeps_per_solve=st["refine_sweeps"] / max(1, st["solves"] + st["soc_tried"]),
               setup=extra)
    res["variants"] = compare_variants(w, TH, out, args, extra, warm_fn)
    res["oracle_check"] = oracle_check(w, TH, out, warm_fn, extra, args.oracle_check)
    return res


def oracle_check(w, TH, out, warm_fn, extra, count):
    """The oracle's warm solves from the same network rows (same warm options) on the first `count`
    instances against the GPU's warm FP32 + refinement results: status, KKT point, and E_0 of the
    GPU point recomputed by the oracle."""
    import oracle
    rows = warm_fn(TH[:count]).cpu().numpy()
    th = TH[:count].cpu().numpy()
    _, threads = cpu_info()
    o = oracle.solve_quad(w, th, threads=threads, warm=rows,
                          opts=oracle.default_opts(warm_mu0=extra["warm_mu0"], warm_iter_cap=extra["warm_iter_cap"]))
    g = {k: out[k][:count].cpu().numpy() for k in ("status", "obj", "x", "y", "zl", "zu", "iters")}
    same_status = int((g["status"] == o["status"]).sum())
    both = np.flatnonzero((g["status"] == 1) & (o["status"] == 1))
    rel = np.abs(g["obj"][both] - o["obj"][both]) / np.maximum(1.0, np.abs(o["obj"][both]))
    dx = np.abs(g["x"][both] - o["x"][both]).max(axis=1)
    e0 = [oracle.kkt_error(w, th[i], g["x"][i], g["y"][i], g["zl"][i], g["zu"][i]) for i in both]
    return dict(instances=count, same_status=same_status, both_converged=int(both.size),
                same_point=int(((rel <= 1e-6) & (dx <= 1e-5)).sum()),
                max_rel_obj=float(rel.max()) if both.size else None, max_dx=float(dx.max()) if both.size else None,
                max_e0_gpu_point=float(max(e0)) if e0 else None,
                same_iterations=int((g["iters"] == o["iters"]).sum()),
                oracle_warm_rejected=int(o["stats"][:, 9].sum()))


def time_solves(solver, TH, steps, warmup, warm_fn=None, stream=False):
    """`warmup` untimed then `steps` timed batched solves of TH (with the warm points computed inside
    the timed region when `warm_fn` is given); returns (seconds, converged count, outputs of the last
    batch, stats, kernel times).

    stream=True: the `steps` batches go through the solver's slots as one stream of
    steps x len(TH) instances in a single solve (iteration-level batching across batches, Sec. V,
    Fig. 2: a slot freed by an instance of one batch takes the next instance while the slowest
    instances of the previous batch still run); warm-up likewise as one stream of `warmup` batches."""
    import torch
    from paper_2606_26341_amd import hipipm
    n = TH.shape[0]
    if stream:
        TS = TH.repeat(max(steps, warmup), 1).contiguous()
        out = solver.alloc_outputs(TS.shape[0])
        if warmup:
            solver.solve(TS[:warmup * n], warm=warm_fn(TS[:warmup * n]) if warm_fn else None,
                         out={k: v[:warmup * n] for k, v in out.items()})
            torch.cuda.synchronize()
            log(f"[bench] warm-up stream of {warmup} batches done")
        solver.reset_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = TS[:steps * n]
        o = {k: v[:steps * n] for k, v in out.items()}
        solver.solve(T, warm=warm_fn(T) if warm_fn else None, out=o)
        conv = int((o["status"] == hipipm.ST_CONVERGED).sum().item())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        last = {k: v[(steps - 1) * n:steps * n] for k, v in o.items()}
        return dt, conv, last, solver.stats(), solver.kernel_times()
    out = solver.alloc_outputs(n)
    for i in range(warmup):
        solver.solve(TH, warm=warm_fn(TH) if warm_fn else None, out=out)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i} done")
    solver.reset_stats()
    conv = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        solver.solve(TH, warm=warm_fn(TH) if warm_fn else None, out=out)
        conv += int((out["status"] == hipipm.ST_CONVERGED).sum().item())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, conv, out, solver.stats(), solver.kernel_times()


def setup_warm_start(w, TH, opts, args):
    """Outside the timed region: solve the training and validation splits cold (FP64) on the GPU,
    train the network on the converged training solutions, pick the warm barrier parameter and the
    divergence cap on the validation split.  Returns the warm-point function and a summary."""
    from paper_2606_26341_amd import warmstart
    t0 = time.perf_counter()
    log(f"[bench] warm start: generating {args.train} training + {args.val} validation instances")
    th_train = warmstart.split(w, args.train, seed_tag=51)
    th_val = warmstart.split(w, args.val, seed_tag=52)
    t1 = time.perf_counter()
    ws, losses, n_fit = warmstart.train_for(w, args.train, seed_tag=51, epochs=args.epochs, thetas=th_train,
                                            log=lambda m: log("[bench]", m) if m.endswith("0") else None)
    t2 = time.perf_counter()
    mu0, cap, table = warmstart.select_options(ws, w, th_val, precision=opts["precision"])
    t3 = time.perf_counter()
    log(f"[bench] trained on {n_fit} solutions (loss {losses[0]:.3e} -> {losses[-1]:.3e}) in {t2 - t1:.1f} s; "
        f"validation: mu0 table {table}, chosen {mu0}, cap {cap}")
    opts.update(warm_mu0=mu0, warm_iter_cap=cap)
    # the network's forward pass alone (its launches go to torch's current stream, so torch events
    # bracket them)
    import torch
    ws.predict(TH)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ws.predict(TH)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 5
    flop = 2.0 * TH.shape[0] * sum(i * o for i, o in ws.net.layout())
    summary = dict(forward_ms=fwd_ms, forward_tflops=flop / (fwd_ms * 1e-3) / 1e12,train_solutions=n_fit, validation=args.val, epochs=args.epochs, loss_first=losses[0],
                   loss_last=losses[-1], warm_mu0=mu0, warm_iter_cap=cap,
                   mu0_table={str(k): v for k, v in table["mu0"].items()},
                   cap_table_ms_conv_maxiter={str(k): v for k, v in table["cap"].items()},
                   setup_s=dict(generate=t1 - t0, solve_and_train=t2 - t1, validate=t3 - t2))
    return ws.predict, summary


def compare_variants(w, TH, warm_out, args, extra, warm_fn):
    """Cold/warm x FP64/FP32+refinement on the same instances, timed the same way, and the share of
    instances where the warm FP32 solve reaches the cold FP64 solve's KKT point."""
    import torch
    from paper_2606_26341_amd import hipipm
    res = {}
    ref = None
    for name, prec, warm in (("cold_fp64", 0, False), ("cold_fp32ir", 1, False), ("warm_fp64", 0, True)):
        o = dict(timing=0, precision=prec, async_passes=args.async_passes)
        fn = None
        if warm:
            o.update(warm_mu0=extra["warm_mu0"], warm_iter_cap=extra["warm_iter_cap"])
            fn = warm_fn
        slots = args.slots or hipipm.resident_slots(w, hipipm.default_options(**o))
        s = hipipm.Solver(w, slots, hipipm.default_options(**o))
        dt, conv, out, st, _ = time_solves(s, TH, args.steps, 1, fn, stream=not args.no_stream)
        res[name] = dict(solves_per_sec=conv / dt, iterations_per_solve=float(out["iters"].float().mean().item()),
                         max_iterations=int(out["iters"].max().item()),
                         converged_fraction=float((out["status"] == 1).float().mean().item()),
                         fp64_fallbacks=st["fp64_fallbacks"],
                         warm_restarts=st["warm_restarts"])
        if name == "cold_fp64":
            ref = {k: v.clone() for k, v in out.items()}
        log(f"[bench] variant {name}: {res[name]}")
    both = (ref["status"] == 1) & (warm_out["status"] == 1)
    rel = (warm_out["obj"] - ref["obj"]).abs() / ref["obj"].abs().clamp(min=1.0)
    dx = (warm_out["x"] - ref["x"]).abs().amax(dim=1)
    same = both & (rel <= 1e-6) & (dx <= 1e-5)
    res["warm_fp32ir_same_point_as_cold_fp64"] = float(same.sum().item()) / max(1, int(both.sum().item()))
    return res


if __name__ == "__main__":
    main()
