"""Benchmark: converged NLP solves/sec of the batched interior-point solver on one MI355X.

A step is one batched solve of the whole workload (every instance run to convergence through
all method steps: derivatives, KKT assembly + inertia-correcting factorization, step, filter
line search with SOC, restoration, barrier update, slot refill).  Default workload: C2,
figure-eight tracking NMPC, 4096 instances, N = 30, 8 obstacles, FP64, cold start.

`--workload C5` measures the learned warm start: 16384 point-to-point instances (N = 10,
3 obstacles); outside the timed region the network is trained on cold FP64 solutions of a
separate training split and the warm barrier parameter is picked on a validation split; a timed
step is the network's forward pass plus the warm-started solve with the FP32 factor and FP64
refinement.  The cold/warm x FP64/FP32 variants of the same instances are reported beside it.

Prints one JSON line.  The roofline object is the dominant kernel's algorithmic HBM bytes per
launch (formula in `kernel_roofline`) over its average launch time from HIP events.
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


# HBM traffic per launch of the dominant kernel, from the two rocprofv3 --pmc runs (FETCH_SIZE,
# WRITE_SIZE) scaled by the same counters on a plain device copy of known size; valid only for
# the kernel sources they were taken on (hash below) and the default C2 run.
MEASURED_TRAFFIC = {"k_iter": {"csrc": "06d33ab38a25685b", "workload": "C2", "bytes_per_launch": 1.7565e8}}


def csrc_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_26341_amd", "csrc")
    for f in ("common.h", "model.h", "kkt.h", "kernels.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# per-knot factor record produced on the regular path: L_R (4x4), Y (4x13), P (13x13),
# Delta^1/2 (13), 1/diag(L_R) (4), flag
FR_WORDS = 16 + 52 + 169 + 13 + 4 + 1


def sd_words(n_obs: int) -> int:
    """Stage data per knot: Hessian diagonal (17), elastic ratios (2 x 13), condensed inequality
    block (9) and 7 words per inequality row, padded to 8 words."""
    return ((17 + 26 + 9 + 7 * n_obs + 7) // 8) * 8


def kernel_roofline(w, st, kt, slots_launched, rec_bytes=8.0):
    """Roofline of the dominant kernel from the live HIP-event timings (algorithmic FP64 bytes).

    One factorization attempt (per slot) reads the stage inputs (G_k 13x17 and W_k 17x17 per
    interval, the stage data per knot) and writes the factor record per knot.  One solve reads
    the factor record and stage data per knot, G_k per interval and the right-hand side (n + m),
    and writes the step (n + m).  k_fac does factorizations only; the fused pass kernel (the
    last instances of a batch) is charged only the bytes of the factorizations and solves it
    runs, so its figure is a lower bound of its traffic.  `rec_bytes` is the width of the factor
    record entries (4 when the factor runs in FP32; the stage data stay FP64).
    """
    N = w.N
    names = ("eval", "pre", "factor", "solve", "linesearch", "fused")
    tot = {k: kt[k][0] for k in names if k in kt}
    dom = max(tot, key=tot.get)
    ms, launches = kt[dom]
    avg_ms = ms / max(1, launches)
    sdw = sd_words(w.n_obs)
    fact_bytes = 8.0 * (N * (13 * 17 + 17 * 17) + (N + 1) * sdw) + rec_bytes * (N + 1) * FR_WORDS
    solve_bytes = 8.0 * ((N + 1) * sdw + N * 13 * 17 + 2 * (w.n + w.m)) + rec_bytes * (N + 1) * FR_WORDS
    if dom == "factor":
        units = st["factorizations"] - st["fused_factorizations"]
        per_launch = fact_bytes * units / max(1, launches)
        kernel, unit_desc = "k_fac", f"{units} factorizations x {fact_bytes:.0f} B"
    elif dom == "fused":
        per_launch = (fact_bytes * st["fused_factorizations"] + solve_bytes * st["fused_solves"]) / max(1, launches)
        kernel = "k_iter"
        unit_desc = (f"{st['fused_factorizations']} factorizations x {fact_bytes:.0f} B + "
                     f"{st['fused_solves']} solves x {solve_bytes:.0f} B")
    else:
        return dict(kernel="k_" + dom, bound="latency", achieved=None, peak=None, unit=None, frac=None,
                    traffic=None, avg_ms=avg_ms, launches=launches)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return dict(kernel=kernel, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=achieved / HBM_PEAK_GBS, traffic=None, avg_ms=avg_ms, launches=launches,
                bytes_per_launch=per_launch, units=unit_desc)


# oracle sample sizes sized to about 10-30 s of host work (dense FP64 factorizations grow with N^3)
CPU_SAMPLE = {"C1": 64, "C2": 48, "C4": 32, "C5": 16384}


def cpu_baseline(w, sample: int):
    import oracle
    TH = w.thetas(0, sample)
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    o = oracle.solve_quad(w, TH, threads=threads)
    dt = time.perf_counter() - t0
    conv = int((o["status"] == oracle.ST_CONVERGED).sum())
    return dict(value=conv / dt, unit="solves/s", cores=min(threads, sample), kind="oracle",
                sample=f"{sample} {w.name} instances (0..{sample - 1}), dense FP64 oracle, one instance per "
                       f"thread, {dt:.1f} s wall, {conv} converged",
                cpu=platform.processor() or platform.machine())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--slots", type=int, default=0, help="concurrent slots (default: all instances)")
    ap.add_argument("--instances", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle instances for the CPU baseline (default: about 10-30 s of host work per workload)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (HBM counter calibration) and exit")
    ap.add_argument("--precision", type=int, default=None,
                    help="KKT factor precision: 0 FP64, 1 FP32 + FP64 refinement (default: the workload's)")
    ap.add_argument("--train", type=int, default=190000, help="warm-start training instances (C5)")
    ap.add_argument("--val", type=int, default=10000, help="warm-start validation instances (C5)")
    ap.add_argument("--epochs", type=int, default=30, help="warm-start training epochs (C5)")
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
    slots = args.slots or n_inst
    TH = torch.tensor(w.thetas(0, n_inst), dtype=torch.float64, device="cuda:0")
    opts = dict(timing=1)
    opts["precision"] = args.precision if args.precision is not None else (1 if w.precision == "fp32ir" else 0)
    if args.fuse_below is not None:
        opts["fuse_below"] = args.fuse_below
    log(f"[bench] workload {w.name}: {n_inst} instances, N={w.N}, n={w.n}, m={w.m}, slots={slots}")
    extra = {}
    warm_fn = None
    if w.name == "C5":
        warm_fn, extra = setup_warm_start(w, TH, slots, opts, args)
    solver = hipipm.Solver(w, slots, hipipm.default_options(**opts))
    dt, conv, out, st, kt = time_solves(solver, TH, args.steps, args.warmup, warm_fn)
    log(f"[bench] timed {args.steps} steps in {dt:.3f} s; stats {st}; kernel ms {kt}")
    roof = kernel_roofline(w, st, kt, min(slots, n_inst), rec_bytes=4.0 if opts["precision"] == 1 else 8.0)
    mt = MEASURED_TRAFFIC.get(roof["kernel"])
    if mt and mt["csrc"] == csrc_hash() and mt["workload"] == w.name and n_inst == w.n_inst and slots == n_inst:
        roof["traffic"] = mt["bytes_per_launch"]
    kkt = out["kkt"].cpu().numpy()
    status = out["status"].cpu().numpy()
    desc = {"C2": "C2: figure-eight tracking NMPC, FP64 cold start",
            "C5": "C5: point-to-point NMPC, learned BF16 warm start + FP32 factor with FP64 refinement"}
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
                   "n": w.n, "m": w.m, "slots": slots},
        "iterations_per_sec": st["iterations"] / dt,
        "iterations_per_solve": float(out["iters"].float().mean().item()),
        "converged_fraction": float((status == 1).mean()),
        "max_kkt_converged": float(kkt[status == 1].max()) if (status == 1).any() else None,
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": roof["kernel"],
        "roofline_detail": {k: roof[k] for k in ("avg_ms", "launches", "bytes_per_launch", "units") if k in roof},
        "kernel_ms": {k: v[0] for k, v in kt.items()},
    }
    if warm_fn is not None:
        res["warm_start"] = dict(extra, warm_started=st["warm_started"], warm_rejected=st["warm_rejected"],
                                 warm_restarts=st["warm_restarts"],
                                 fallback_rate=(st["warm_rejected"] + st["warm_restarts"]) / max(1, st["instances_done"]))
        res["variants"] = compare_variants(w, TH, slots, out, args, extra, warm_fn)
        res["variants"]["warm_fp32ir"] = dict(solves_per_sec=res["value"],
                                              iterations_per_solve=res["iterations_per_solve"],
                                              max_iterations=int(out["iters"].max().item()),
                                              converged_fraction=res["converged_fraction"],
                                              passes_per_solve=st["passes"] / args.steps,
                                              fp64_fallbacks=st["fp64_fallbacks"], warm_restarts=st["warm_restarts"])
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_sample or CPU_SAMPLE.get(w.name, 64))
    print(json.dumps(res), flush=True)


def time_solves(solver, TH, steps, warmup, warm_fn=None):
    """`warmup` untimed then `steps` timed batched solves of TH (with the warm points computed inside
    the timed region when `warm_fn` is given); returns (seconds, converged count, outputs, stats,
    kernel times)."""
    import torch
    from paper_2606_26341_amd import hipipm
    out = solver.alloc_outputs(TH.shape[0])
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


def setup_warm_start(w, TH, slots, opts, args):
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


def compare_variants(w, TH, slots, warm_out, args, extra, warm_fn):
    """Cold/warm x FP64/FP32+refinement on the same instances, timed the same way, and the share of
    instances where the warm FP32 solve reaches the cold FP64 solve's KKT point."""
    import torch
    from paper_2606_26341_amd import hipipm
    res = {}
    ref = None
    for name, prec, warm in (("cold_fp64", 0, False), ("cold_fp32ir", 1, False), ("warm_fp64", 0, True)):
        o = dict(timing=0, precision=prec)
        fn = None
        if warm:
            o.update(warm_mu0=extra["warm_mu0"], warm_iter_cap=extra["warm_iter_cap"])
            fn = warm_fn
        s = hipipm.Solver(w, slots, hipipm.default_options(**o))
        dt, conv, out, st, _ = time_solves(s, TH, args.steps, 1, fn)
        res[name] = dict(solves_per_sec=conv / dt, iterations_per_solve=float(out["iters"].float().mean().item()),
                         max_iterations=int(out["iters"].max().item()),
                         converged_fraction=float((out["status"] == 1).float().mean().item()),
                         passes_per_solve=st["passes"] / args.steps, fp64_fallbacks=st["fp64_fallbacks"],
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
