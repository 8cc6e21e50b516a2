#!/usr/bin/env python3
"""Benchmark: transitive-closure time-to-fixpoint and effective TOPS at N = 8192.

Workload (one "step"): the int8 repeated-squaring closure R = min1(A + R R)
run to its fixpoint on each of nine Erdos-Renyi graphs with N = 8192
constants, edge probability p in {1/N, 4/N, 0.01} and seeds 0, 1, 2 -- ingest,
every squaring step with its fused threshold and counter, the device-side
convergence test and the emit of the 0/1 model.  Inputs are resident in HBM
before the timed region starts.

value = effective TOPS = sum over graphs of 2 N^3 x (products executed,
including the one that confirms the fixpoint) / wall time of the step.

Also reported, each measured once outside the timed steps: per-graph
time-to-fixpoint, the plain FP32 iteration and the fp64 epsilon solve on the
same inputs (with their threshold errors against the int8 model), the bf16
and fp8 variants, same generation at N = 4096 on random forests, the
dominant kernel's roofline figures (HIP events inside the library, on the
launch stream, around the first product launch of each chunk of steps in
the timed region) and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TC time-to-fixpoint & eff. TOPS at N=8192; batched req/s with p50/p99 latency"
N = 8192
PROBS = (("1/N", 1.0 / N), ("4/N", 4.0 / N), ("0.01", 0.01))
SEEDS = (0, 1, 2)
INT8_PEAK_TOPS = 5000.0     # MI355X dense int8 MFMA, 5.0 POP/s
# int8 step kernel of each tile configuration (dl_tune numbering)
STEP_KERNELS = {0: "k_nt_dma<256,256,64,64,128,OpI8,2>", 1: "k_nt_step<128,128,64,64,64,OpI8,2,1>",
                2: "k_nt_step<64,64,32,32,64,OpI8,2,1>", 3: "k_nt_dma<256,256,64,64,128,OpI8x32,2>",
                4: "k_nt_small<OpI8>"}
FP32_PEAK_TFLOPS = 157.3    # MI355X fp32 matrix


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true", help="skip the once-measured variants")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's size rule instead of running the tile autotuner first "
                         "(profiles then see only the timed workload's launches)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests in the Poisson serving stream (0 skips serving)")
    ap.add_argument("--trace-summary", metavar="DB",
                    help="summarise a rocprofv3 --kernel-trace results database and exit")
    ap.add_argument("--eps-only", action="store_true",
                    help="run only the fp64 epsilon solve on the p = 4/N, seed 0 graph (for kernel traces) and exit")
    ap.add_argument("--small-only", action="store_true",
                    help="run only the plain FP32 closure at N = 512 (ER p = 2/N, seeds 0-2) and print its JSON")
    ap.add_argument("--peaks", action="store_true",
                    help="print the measured matrix-core rates and LDS data-path rates (dl_measure_peak) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run three plain 1 GiB device copies (traffic-counter calibration) and exit")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CAL_FETCH_CSV", "CAL_WRITE_CSV"),
                    help="per-launch HBM traffic of the step kernel from rocprofv3 --pmc CSVs and exit")
    ap.add_argument("--mfma-summary", metavar="CSV",
                    help="matrix-core busy fraction and clock of the step kernel and of the register-only "
                         "int8 MFMA loop from a rocprofv3 --pmc CSV and exit")
    ap.add_argument("--counter-summary", metavar="CSV",
                    help="per-launch averages of every counter in a rocprofv3 --pmc CSV for the step kernel, "
                         "per CU cycle, and exit")
    ap.add_argument("--busy-summary", metavar="CSV",
                    help="per kernel name: launches, duration, clock and matrix-core busy fraction from a "
                         "rocprofv3 --pmc CSV holding SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE, and exit")
    ap.add_argument("--kernel", metavar="SUBSTRING",
                    help="with --counter-summary: summarise the kernels whose name contains SUBSTRING "
                         "(the most launched one) instead of the int8 step kernel")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving workload (--serve-requests of them) and print its JSON")
    ap.add_argument("--phase-gaps", type=float, default=0.0, metavar="SECONDS",
                    help="idle time around each timed serving run, so that a kernel trace splits into "
                         "one segment per run (see --trace-busy)")
    ap.add_argument("--trace-busy", metavar="DB",
                    help="split a rocprofv3 --kernel-trace database at device idle gaps of at least "
                         "--gap-ms and print each segment's span, the time some kernel ran, and its "
                         "largest kernels, then exit")
    ap.add_argument("--gap-ms", type=float, default=100.0)
    ap.add_argument("--programs-only", action="store_true",
                    help="run only the layered program workloads (both methods) and print their JSON")
    args = ap.parse_args()
    if args.programs_only:
        import torch

        import paper_1608_00139_amd as dl

        torch.cuda.set_device(0)
        print(json.dumps(run_programs(dl, dl.Context(0), torch)))
        return 0
    if args.small_only:
        import torch

        import paper_1608_00139_amd as dl

        torch.cuda.set_device(0)
        print(json.dumps(run_small_plain(dl, dl.Context(0), torch)))
        return 0
    if args.serving_only:
        import torch

        import paper_1608_00139_amd as dl

        torch.cuda.set_device(0)
        print(json.dumps(run_serving(dl, torch, args.serve_requests, gaps=args.phase_gaps)))
        return 0
    if args.trace_busy:
        return trace_busy(args.trace_busy, args.gap_ms)
    if args.trace_summary:
        return trace_summary(args.trace_summary)
    if args.pmc_summary:
        return pmc_summary(*args.pmc_summary)
    if args.mfma_summary:
        return mfma_summary(args.mfma_summary)
    if args.counter_summary:
        return counter_summary(args.counter_summary, args.kernel)
    if args.busy_summary:
        return busy_summary(args.busy_summary)
    if args.copy_calibration:
        return copy_calibration()
    if args.peaks:
        return peaks()
    if args.eps_only:
        return eps_only()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path, so --gpus above 1 "
              "is not supported", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import dlgen
    import paper_1608_00139_amd as dl

    torch.cuda.set_device(0)
    ctx = dl.Context(0)
    log(f"generating {len(PROBS) * len(SEEDS)} ER graphs, N={N}")
    graphs = []
    for pname, p in PROBS:
        for seed in SEEDS:
            e = dlgen.er_edges(N, p, seed)
            a = dlgen.to_dense(N, e)
            graphs.append({"p": pname, "seed": seed, "edges": int(len(e)), "host": a, "edge_list": e,
                           "dev": torch.from_numpy(a).cuda(),
                           "sha256": dlgen.edges_sha256(N, e)})
    outs = [torch.empty((N, N), dtype=torch.uint8, device="cuda") for _ in graphs]
    torch.cuda.synchronize()

    devs = [g["dev"] for g in graphs]

    def step():
        # one batched call: two fixpoints in flight, so one's counter
        # read-back overlaps the other's products
        _, its = dl.dl_tc_batch(devs, method=dl.DL_TC_SQUARE, prec=dl.DL_I8, outs=outs, ctx=ctx)
        return its

    # tile configuration of the step kernel chosen by the library's autotuner
    if args.no_tune:
        tile_cfg, tile_ms, tile_cand = 0, 0.0, []
    else:
        tile_cfg, tile_ms, tile_cand = ctx.tune("i8", N, candidates=True)
        log(f"autotuner: cfg {tile_cfg} ({tile_ms:.4f} ms), candidates {tile_cand}")

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ctx.kernel_stats(0, reset=True)
    ctx.set_timing(True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = None
    step_ms = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        iters = step()  # returns after its last fixpoint is read back
        step_ms.append(round((time.perf_counter() - ts) * 1e3, 3))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(False)
    launches, kms = ctx.kernel_stats(0, reset=True)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    products = [it - 1 for it in iters]  # step 1 is the input itself, no product
    ops_per_step = sum(2.0 * N ** 3 * k for k in products)
    value = ops_per_step / (ms_per_step * 1e-3) / 1e12
    avg_kernel_ms = kms / max(launches, 1)
    achieved = 2.0 * N ** 3 / (avg_kernel_ms * 1e-3) / 1e12

    # per-graph time-to-fixpoint (median of a few runs each)
    per_graph = []
    for g, out in zip(graphs, outs):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            _, it = dl.dl_tc(g["dev"], method=dl.DL_TC_SQUARE, prec=dl.DL_I8, out=out, ctx=ctx)
            ts.append(time.perf_counter() - a0)
        t = statistics.median(ts)
        per_graph.append({"p": g["p"], "seed": g["seed"], "edges": g["edges"], "iters": it,
                          "time_to_fixpoint_ms": round(t * 1e3, 3),
                          "eff_tops": round(2.0 * N ** 3 * (it - 1) / t / 1e12, 1),
                          "closure_density": round(float(out.sum().item()) / N ** 2, 6)})

    extras = {}
    if not args.no_extras:
        extras = run_extras(dl, ctx, graphs, outs, np, torch)

    serving = None
    if not args.no_extras and args.serve_requests > 0:
        graphs_dev_release(graphs)
        serving = run_serving(dl, torch, args.serve_requests)

    cpu = None if args.no_cpu else cpu_baseline(graphs, iters, outs, torch)

    # matrix-core rate this device sustains on register operands (a reference
    # beside the datasheet peak; the roofline "peak" stays the datasheet one)
    measured_peak = dl.dl_measure_peak("i8", ctx=ctx) / 1e12

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "TOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "step_ms": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic (seeded ER graphs, dense 0/1 int8 in HBM)",
        "config": {"workload": "TC to fixpoint, int8 repeated squaring, N=8192 ER p in {1/N,4/N,0.01} x seeds {0,1,2}, nine fixpoints per step in one batched call",
                   "n": N, "graphs": len(graphs), "iters": iters, "products_per_step": sum(products)},
        "frac_of_int8_peak": round(value / INT8_PEAK_TOPS, 4),
        "roofline": {"bound": "mfma", "kernel": STEP_KERNELS[tile_cfg],
                     "achieved": round(achieved, 1), "peak": INT8_PEAK_TOPS, "unit": "TOPS",
                     "frac": round(achieved / INT8_PEAK_TOPS, 4), "traffic": measured_traffic(STEP_KERNELS[tile_cfg]),
                     "launches": launches, "avg_kernel_ms": round(avg_kernel_ms, 4),
                     "ops_per_launch": 2.0 * N ** 3,
                     "measured_mfma_peak": round(measured_peak, 1),
                     "frac_of_measured_peak": round(achieved / measured_peak, 4),
                     "autotuner": {"cfg": tile_cfg, "ms": round(tile_ms, 4),
                                   "candidates_ms": [round(x, 4) for x in tile_cand]}},
        "per_graph": per_graph,
        "extras": extras,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


def run_extras(dl, ctx, graphs, outs, np, torch):
    """Variants of the hot path, each timed once on the same resident inputs."""
    res = {}
    every = range(len(graphs))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # tile autotuner: every configuration's time per product launch by size
    # (its own context, so the entries do not steer the runs below)
    tctx = dl.Context(0)
    tune = []
    for prec_name in ("i8", "f32"):
        for n in (512, 1024, 2048, 4096, 8192):
            log(f"autotune {prec_name} n={n}")
            cfg, ms, cand = tctx.tune(prec_name, n, candidates=True)
            tune.append({"prec": prec_name, "n": n, "cfg": cfg, "ms": round(ms, 4),
                         "candidates_ms": [round(x, 4) for x in cand]})
    tctx.close()
    res["autotune"] = tune

    # plain FP32 fixpoint (the "Iteration" baseline) and speed-up of int8 squaring
    plain = []
    for i in every:
        g = graphs[i]
        log(f"fp32 plain p={g['p']} seed={g['seed']}")
        tmp = torch.empty_like(outs[i])
        (_, it), t = timed(lambda: dl.dl_tc(g["dev"], method=dl.DL_TC_PLAIN, prec=dl.DL_F32, out=tmp, ctx=ctx))
        (_, it8), t8 = timed(lambda: dl.dl_tc(g["dev"], method=dl.DL_TC_SQUARE, prec=dl.DL_I8, out=outs[i], ctx=ctx))
        mism = int((tmp != outs[i]).sum().item())
        plain.append({"p": g["p"], "seed": g["seed"], "iters": it, "time_ms": round(t * 1e3, 2),
                      "eff_tflops": round(2.0 * N ** 3 * (it - 1) / t / 1e12, 1),
                      "int8_square_ms": round(t8 * 1e3, 2), "speedup_int8_square": round(t / t8, 1),
                      "model_mismatches_vs_int8": mism})
    res["tc_plain_fp32"] = plain

    # bf16 / fp8 squaring variants
    var = []
    for prec_name, prec in (("fp4", dl.DL_FP4), ("fp8", dl.DL_FP8), ("bf16", dl.DL_BF16)):
        for i in every:
            g = graphs[i]
            log(f"{prec_name} square p={g['p']} seed={g['seed']}")
            tmp = torch.empty_like(outs[i])
            dl.dl_tc(g["dev"], method=dl.DL_TC_SQUARE, prec=prec, out=tmp, ctx=ctx)
            (_, it), t = timed(lambda: dl.dl_tc(g["dev"], method=dl.DL_TC_SQUARE, prec=prec, out=tmp, ctx=ctx))
            var.append({"prec": prec_name, "p": g["p"], "seed": g["seed"], "iters": it, "time_ms": round(t * 1e3, 2),
                        "eff_tops": round(2.0 * N ** 3 * (it - 1) / t / 1e12, 1),
                        "model_mismatches_vs_int8": int((tmp != outs[i]).sum().item())})
    res["tc_square_variants"] = var

    # fp64 epsilon solve, eps = 0.5 / (max row sum + 1); one untimed solve
    # first, so that no row carries the process's one-time costs (code
    # loading, workspace allocation: the first solve takes about 40 ms)
    eps_rows = []
    g0 = graphs[every[0]]
    dl.dl_solve_eps(g0["dev"], 0.5 / (1.0 + float(g0["host"].sum(axis=1).max())), out=torch.empty_like(outs[every[0]]),
                    ctx=ctx)
    for i in every:
        g = graphs[i]
        eps = 0.5 / (1.0 + float(g["host"].sum(axis=1).max()))
        log(f"fp64 eps solve p={g['p']} seed={g['seed']}")
        tmp = torch.empty_like(outs[i])
        ctx.kernel_stats(1, reset=True)
        ctx.set_timing(True)
        (_, _, uflow), t = timed(lambda: dl.dl_solve_eps(g["dev"], eps, out=tmp, ctx=ctx, underflow=True))
        ctx.set_timing(False)
        nl, tms = ctx.kernel_stats(1, reset=True)
        eps_rows.append({"p": g["p"], "seed": g["seed"], "eps": eps, "time_ms": round(t * 1e3, 2),
                         "eff_tflops": round(8.0 / 3.0 * N ** 3 / t / 1e12, 2),
                         "executed_tflops": round(3.0 * N ** 3 / t / 1e12, 2),
                         "threshold_errors_vs_int8_model": int((tmp != outs[i]).sum().item()),
                         "underflow_flag": uflow, "update_launches": nl, "update_ms": round(tms, 2),
                         "update_tflops": round(3.0 * N * N * (N - 128) / (tms * 1e-3) / 1e12, 2)
                         if tms > 0 else None})
    res["eps_solve_fp64"] = eps_rows

    # plain FP32 iteration at N = 512, ER p = 2/N (time-to-fixpoint; latency bound)
    res["tc_plain_fp32_n512"] = run_small_plain(dl, ctx, torch)
    import dlgen

    # power-law digraph, N = 32768 (1 GiB int8 operands), repeated squaring
    n = 32768
    log("chung-lu n=32768")
    e = dlgen.chung_lu_edges(n, 0)
    a = torch.from_numpy(dlgen.to_dense(n, e)).cuda()
    o = torch.empty_like(a)
    cl = []
    for prec_name, prec in (("i8", dl.DL_I8), ("fp4", dl.DL_FP4)):
        dl.dl_tc(a, method=dl.DL_TC_SQUARE, prec=prec, out=o, ctx=ctx)
        (_, it), t = timed(lambda: dl.dl_tc(a, method=dl.DL_TC_SQUARE, prec=prec, out=o, ctx=ctx))
        cl.append({"n": n, "prec": prec_name, "edges": int(len(e)), "mean_out_degree": round(len(e) / n, 3),
                   "iters": it, "time_to_fixpoint_ms": round(t * 1e3, 2),
                   "eff_tops": round(2.0 * n ** 3 * (it - 1) / t / 1e12, 1),
                   "closure_density": round(float(o.sum(dtype=torch.int64).item()) / n ** 2, 6)})
    res["tc_chung_lu_n32768"] = cl
    del a, o
    torch.cuda.empty_cache()

    # same generation, N = 4096 random forests

    sg = []
    n = 4096
    for seed in SEEDS:
        p = torch.from_numpy(dlgen.to_dense(n, dlgen.forest_edges(n, seed))).cuda()
        s = torch.empty_like(p)
        dl.dl_sg(p, prec=dl.DL_I8, out=s, ctx=ctx)
        (_, it), t = timed(lambda: dl.dl_sg(p, prec=dl.DL_I8, out=s, ctx=ctx))
        sg.append({"n": n, "seed": seed, "iters": it, "time_to_fixpoint_ms": round(t * 1e3, 2),
                   "eff_tops": round(2 * 2.0 * n ** 3 * (it - 1) / t / 1e12, 1),
                   "model_size": int(s.sum().item())})
    res["sg_n4096"] = sg

    # same generation, epsilon form (fp64 Smith doubling), N = 4096 forests
    sge = []
    for seed in SEEDS:
        ph = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        p = torch.from_numpy(ph).cuda()
        ref = torch.empty_like(p)
        dl.dl_sg(p, prec=dl.DL_I8, out=ref, ctx=ctx)
        s = torch.empty_like(p)
        d = int(ph.sum(axis=1).max())
        eps = 1.0 / (1 + d * d)
        (_, _, dbl), t = timed(lambda: dl.dl_sg_eps(p, eps, out=s, ctx=ctx))
        sge.append({"n": n, "seed": seed, "eps": eps, "doublings": dbl, "time_ms": round(t * 1e3, 2),
                    "executed_tflops": round(6.0 * n ** 3 * dbl / t / 1e12, 2),
                    "threshold_errors_vs_int8_model": int((s != ref).sum().item())})
    res["sg_eps_fp64_n4096"] = sge
    res["measured_mfma_peaks_tops"] = {k: round(dl.dl_measure_peak(k, ctx=ctx) / 1e12, 1)
                                       for k in ("i8", "fp8", "fp4", "bf16", "f32", "f64", "f64_agpr")}
    res["measured_lds_rates_tb_per_s"] = {k: round(dl.dl_measure_peak(k, ctx=ctx) / 1e12, 1)
                                          for k in ("lds_read", "lds_fill")}
    torch.cuda.empty_cache()
    res["programs"] = run_programs(dl, ctx, torch)
    res["paper_workloads"] = run_paper_workloads(dl, ctx, torch)
    return res


def run_small_plain(dl, ctx, torch, n: int = 512, runs: int = 20):
    """The plain FP32 closure at N = 512 on ER p = 2/N, seeds 0-2: median
    time-to-fixpoint of `runs` dl_tc calls each (the one-launch whole-fixpoint
    kernel at this size), per iteration and effective TFLOP/s, as the caller
    sees it (host clock around the call and a device synchronisation) and on
    the device (events recorded on the stream around the call)."""
    import dlgen

    small = []
    stream = torch.cuda.current_stream()
    for seed in SEEDS:
        a = torch.from_numpy(dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n, seed))).cuda()
        o = torch.empty_like(a)
        dl.dl_tc(a, method=dl.DL_TC_PLAIN, prec=dl.DL_F32, out=o, ctx=ctx)
        ts, dts = [], []
        for _ in range(runs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            _, it = dl.dl_tc(a, method=dl.DL_TC_PLAIN, prec=dl.DL_F32, out=o, ctx=ctx, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            dts.append(e0.elapsed_time(e1) * 1e-3)
        t, dt = statistics.median(ts), statistics.median(dts)
        small.append({"n": n, "seed": seed, "iters": it, "time_to_fixpoint_ms": round(t * 1e3, 3),
                      "us_per_iteration": round(t * 1e6 / it, 2),
                      "eff_tflops": round(2.0 * n ** 3 * (it - 1) / t / 1e12, 2),
                      "device_ms": round(dt * 1e3, 3), "device_us_per_iteration": round(dt * 1e6 / it, 2)})
    return small


def run_paper_workloads(dl, ctx, torch):
    """The paper's own closure workloads (ER with self-loops, Sec. 7.1): N = 1000
    at p = 1e-4 .. 1 and N = 10^4 at p = 1e-3, timed with int8 squaring and
    with the fp64 epsilon solve (eps = 1 / (1 + max row sum), the largest the
    bound allows, as in the paper's runs); the two models are compared.  The
    paper's times (Octave on a CPU) are context, not a target."""
    import numpy as np

    import dlgen

    out = []
    for n, ps in ((1000, (1e-4, 1e-3, 1e-2, 1e-1, 1.0)), (10000, (1e-3,))):
        for p in ps:
            log(f"paper workload n={n} p={p}")
            a = dlgen.to_dense(n, dlgen.er_edges(n, p, 0, self_loops=True))
            ad = torch.from_numpy(a).cuda()
            r8 = torch.empty_like(ad)
            re = torch.empty_like(ad)
            eps = 1.0 / (1.0 + float(a.sum(axis=1).max()))

            def med(fn, k=3):
                ts = []
                for _ in range(k):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    fn()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                return sorted(ts)[k // 2]

            t8 = med(lambda: dl.dl_tc(ad, method=dl.DL_TC_SQUARE, prec=dl.DL_I8, out=r8, ctx=ctx))
            _, it8 = dl.dl_tc(ad, method=dl.DL_TC_SQUARE, prec=dl.DL_I8, out=r8, ctx=ctx)
            te = med(lambda: dl.dl_solve_eps(ad, eps, out=re, ctx=ctx))
            out.append({"n": n, "p": p, "edges": int(a.sum()), "iters_int8_square": it8,
                        "int8_square_ms": round(t8 * 1e3, 3), "eps_solve_fp64_ms": round(te * 1e3, 2),
                        "closure_density": round(float(r8.sum().item()) / n ** 2, 6),
                        "model_mismatches_eps_vs_int8": int((r8 != re).sum().item())})
            del ad, r8, re
    return out


PROGRAMS = {
    # four layers: a right-tail closure, two non-recursive layers with negation,
    # and a left-tail recursion over a complemented relation
    "layers_negation": (
        "tc(X,Y) :- e(X,Y).\ntc(X,Y) :- e(X,Z), tc(Z,Y).\n"
        "nr(X,Y) :- not tc(X,Y).\nr(X,Z) :- e(X,Y), not tc(Y,Z).\n"
        "s(X,Z) :- f(X,Z).\ns(X,Z) :- s(X,Y), not e(Y,Z).",
        8192, {"e": ("er", 4.0), "f": ("er", 1.0)}),
    # mutual recursion (walks of odd / even length)
    "even_odd": (
        "odd(X,Z) :- e(X,Z).\nodd(X,Z) :- e(X,Y), even(Y,Z).\neven(X,Z) :- e(X,Y), odd(Y,Z).",
        8192, {"e": ("er", 1.0)}),
    # transposed class (Sec. 6.2): r2(x,z) <- r1(x,y), r2(z,y)
    "transposed": ("r2(X,Z) :- r1(X,Z).\nr2(X,Z) :- r1(X,Y), r2(Z,Y).", 4096, {"r1": ("er", 1.0)}),
    # same generation as a program (two-sided clause with eq)
    "same_generation": ("sg(X,Y) :- eq(X,Y).\nsg(X,Y) :- p(X,U), sg(U,V), p(Y,V).", 4096, {"p": ("forest", 0)}),
}


def run_programs(dl, ctx, torch):
    """Layered evaluation of whole programs: both methods on the same bound
    relations (seed 0; ER with mean degree c as p = c/N), wall time of
    dl_program_run, product-kernel launches and their time, and the number of
    entries where the two methods' models differ (must be 0)."""
    import dlgen

    out = {}
    for name, (text, n, rels) in PROGRAMS.items():
        bound = {}
        for k, (rname, (gen, arg)) in enumerate(rels.items()):
            if gen == "er":
                m = dlgen.to_dense(n, dlgen.er_edges(n, arg / n, k))
            else:
                m = dlgen.to_dense(n, dlgen.forest_edges(n, arg))
            bound[rname] = torch.from_numpy(m).cuda()
        rows, models = [], []
        for method in (dl.DL_EVAL_ITERATION, dl.DL_EVAL_MATRIX):
            prog = dl.Program(text, ctx=ctx)
            for k, t in bound.items():
                prog.bind(k, t)
            prog.run(method)  # warm-up (allocations, first launches)
            ctx.kernel_stats(0, reset=True)
            ctx.set_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prog.run(method)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            ctx.set_timing(False)
            launches, kms = ctx.kernel_stats(0, reset=True)
            np_ = dl.dl_padded_size(n, 0, dl.DL_I8)
            heads = sorted({h for l in prog.layers() for h in l["heads"]})
            got = {h: prog.fetch(h, n=n)[0] for h in heads}
            models.append(got)
            rows.append({"method": "iteration" if method == dl.DL_EVAL_ITERATION else "matrix",
                         "time_ms": round(t * 1e3, 2), "product_launches": launches,
                         "product_kernel_ms": round(kms, 2),
                         "product_kernel_tops": round(2.0 * np_ ** 3 * launches / (kms * 1e-3) / 1e12, 1)
                         if launches else None,
                         "layers": [{"heads": l["heads"], "form": l["form"],
                                     "method": "iteration" if l["method"] == 0 else "matrix",
                                     "iters": l["iters"]} for l in prog.layers()],
                         "ones": {h: int(v.sum().item()) for h, v in got.items()}})
            prog.close()
        diff = sum(int((models[0][h] != models[1][h]).sum().item()) for h in models[0])
        out[name] = {"n": n, "runs": rows, "entries_differing_between_methods": diff}
        log(f"program {name}: " + ", ".join(f"{r['method']} {r['time_ms']} ms" for r in rows) + f", diff {diff}")
        del bound, models
        torch.cuda.empty_cache()
    return out


def graphs_dev_release(graphs):
    """Drop the device copies of the N = 8192 inputs (host copies stay)."""
    for g in graphs:
        g["dev"] = None
    import torch

    torch.cuda.empty_cache()
    return []


def run_serving(dl, torch, count: int, seed: int = 0, gaps: float = 0.0):
    """Serving stream: 70% closure / 30% same generation, n log-uniform in
    [64, 2048], ER p = 3/n or random forests.  A closed-loop burst of
    min(count, 2000) requests (all arriving at t = 0) measures the saturated
    throughput; then `count` requests arrive as a Poisson process at 0.8x that
    rate and are served with continuous batching (and, for the latency curve,
    up to 3000 more at 0.5x and at 0.95x).  Latency = completion -
    arrival.  Relations are generated as edge lists before the run, kept on
    the device, and built into the request's buffers by the library's
    edge-list admission (dl_batch_submit_edges).  gaps > 0 leaves the device
    idle for that many seconds around each timed run (for kernel traces)."""
    import time

    import numpy as np

    import dlgen
    from paper_1608_00139_amd.serve import run_stream

    pool = 8 << 30

    def prepare(reqs):
        # every request's edge list, resident on the device before the run
        flat, offs = [], [0]
        for r in reqs:
            e = dlgen.request_edges(r).astype(np.int32)
            flat.append(e)
            offs.append(offs[-1] + len(e))
        edges = torch.from_numpy(np.concatenate(flat) if flat else np.zeros((0, 2), np.int32)).cuda()
        offs = np.array(offs)

        def make_input(r):
            return edges[offs[r.rid]:offs[r.rid + 1]]
        return make_input

    # grouped-step tile sizes from the library's autotuner (one batch, kept
    # for the runs below)
    tb = dl.Batch(1 << 20, 4)
    tiles = tb.tune()
    tb.close()
    log("serving tiles: " + ", ".join(f"{e['n']}:{e['tile']}" for e in tiles))

    burst_n = min(count, 2000)
    burst = dlgen.serving_stream(burst_n, seed, rate=0.0)
    log(f"serving: closed-loop burst of {burst_n}")
    mk = prepare(burst)
    warm = dlgen.serving_stream(64, seed + 1, rate=0.0)
    run_stream(warm, prepare(warm), pool_bytes=pool, max_active=512, lookahead=1, tiles=tiles)

    def timed_run(reqs, make):
        if gaps > 0:
            torch.cuda.synchronize()
            time.sleep(gaps)
        r = run_stream(reqs, make, pool_bytes=pool, max_active=512, lookahead=1, tiles=tiles)
        if gaps > 0:
            torch.cuda.synchronize()
            time.sleep(gaps)
        return r

    sb, _ = timed_run(burst, mk)
    sat = sb.summary()
    rate = 0.8 * sat["req_per_s"]
    stream = dlgen.serving_stream(count, seed, rate=rate)
    log(f"serving: Poisson stream of {count} at {rate:.0f} req/s")
    mk = prepare(stream)
    st, _ = timed_run(stream, mk)
    ops = 0.0
    for c in st.completions:
        per_step = 2.0 if c.kind == 1 else 1.0
        ops += per_step * 2.0 * ((c.n + 63) // 64 * 64) ** 3 * (c.iters - 1)
    out = st.summary()
    # latency at lighter and heavier load: shorter streams at 0.5x and 0.95x
    # the saturated rate (the 0.8x stream above is the headline)
    sweep = []
    for k, frac in enumerate((0.5, 0.8, 0.95)):
        if frac == 0.8:
            s_ = out
        else:
            sw = dlgen.serving_stream(min(count, 3000), seed + 2 + k, rate=frac * sat["req_per_s"])
            log(f"serving: Poisson stream of {len(sw)} at {frac}x saturation")
            sx, _ = timed_run(sw, prepare(sw))
            s_ = sx.summary()
        sweep.append({"offered_frac": frac, "offered_rate": round(frac * sat["req_per_s"], 1),
                      "requests": s_["requests"], "req_per_s": s_["req_per_s"],
                      "p50_ms": s_["p50_ms"], "p99_ms": s_["p99_ms"]})
    out.update({"offered_rate": round(rate, 1), "saturation": sat, "load_sweep": sweep,
                "tiles": [{"n": e["n"], "tile": e["tile"], "us_per_product_64_128_256": [round(x * 1e3, 2) for x in e["ms"]]}
                          for e in tiles],
                "eff_tops_padded": round(ops / st.wall / 1e12, 2),
                "workload": f"{count} requests, 70% TC (ER p=3/n) / 30% SG (forest), n log-uniform [64, 2048], "
                            f"Poisson arrivals at 0.8x the closed-loop saturation rate, int8 grouped steps, "
                            f"one round of look-ahead"})
    return out


def cpu_baseline(graphs, iters, outs, torch, runs: int = 5):
    """The CPU oracle (semi-naive closure on bitset rows, C with OpenMP) on
    the host's cores, timed as its fixpoint rounds alone.

    Sample: every one of the nine workload graphs, from its in-memory edge
    list to the in-memory model; successor lists and the first iterate are
    built before the clock starts and the dense copy of the model after it
    stops (oracle.tc_seminaive_edges).  Each graph runs `runs` times with one
    thread and `runs` times with the all-core thread count (OpenMP's default:
    OMP_NUM_THREADS, else every usable core); per graph and thread count the
    median is reported, as time-to-fixpoint.  `value` is the all-core rate in
    TOPS-equivalent: the GPU schedule's dense work on the same graphs
    (2 N^3 per squaring product) divided by the oracle's summed medians --
    the oracle does not perform that work (its rounds cost about
    sum(out-degree) x N / 64 word operations), so it is a like-for-like rate
    of finishing the same fixpoints, not a count of the oracle's operations.
    Each graph's oracle model is compared with the GPU's int8 model.
    """
    import numpy as np

    import oracle

    cores = oracle.default_threads()
    cpu_model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    rows = []
    total = {1: 0.0, cores: 0.0}
    work = 0.0
    t_all = 0.0
    for i, g in enumerate(graphs):
        row = {"p": g["p"], "seed": g["seed"]}
        for th in (1, cores):
            ts = []
            for _ in range(runs):
                _, it, ones, secs, used = oracle.tc_seminaive_edges(N, g["edge_list"], threads=th,
                                                                    want_model=False)
                ts.append(secs)
                t_all += secs
            med = statistics.median(ts)
            total[th] += med
            row[f"time_to_fixpoint_ms_{'1thread' if th == 1 else 'allcores'}"] = round(med * 1e3, 3)
        model, it, ones, _, _ = oracle.tc_seminaive_edges(N, g["edge_list"], threads=cores)
        row.update({"iters_plain_rounds": it, "model_ones": ones,
                    "model_mismatches_vs_gpu": int(np.count_nonzero(model != outs[i].cpu().numpy()))})
        rows.append(row)
        work += 2.0 * N ** 3 * (iters[i] - 1)
        log(f"cpu oracle p={g['p']} seed={g['seed']}: {row}")
    by_p = {}
    for pname, _ in PROBS:
        sel = [r for r in rows if r["p"] == pname]
        by_p[pname] = {"median_ms_1thread": round(statistics.median(r["time_to_fixpoint_ms_1thread"] for r in sel), 3),
                       "median_ms_allcores": round(statistics.median(r["time_to_fixpoint_ms_allcores"] for r in sel), 3)}
    return {"value": round(work / total[cores] / 1e12, 3),
            "unit": "TOPS-equivalent (the GPU schedule's 2N^3 per product over the oracle's time)",
            "cores": cores, "kind": "oracle",
            "sample": f"all nine N={N} ER graphs, semi-naive rounds timed alone (edge list in memory to model "
                      f"in memory), median of {runs} runs per graph at 1 thread and at {cores} threads",
            "cpu_model": cpu_model, "threads": [1, cores], "runs_per_graph": runs,
            "value_1thread": round(work / total[1] / 1e12, 3),
            "sum_median_ms_1thread": round(total[1] * 1e3, 2), "sum_median_ms_allcores": round(total[cores] * 1e3, 2),
            "by_p": by_p, "per_graph": rows, "seconds_timed": round(t_all, 2)}


KERNEL_SRC = os.path.join(ROOT, "paper_1608_00139_amd", "csrc", "bool_kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_nt_dma_i8_n8192_traffic.txt")


def source_hash() -> str:
    import hashlib

    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of the step kernel from the committed counter
    summary, or None if it covers another kernel or the kernel source
    changed since it was taken."""
    try:
        fields = dict(line.split(":", 1) for line in open(TRAFFIC_PROFILE) if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    if fields.get("kernel_source_sha256", "").strip() != source_hash():
        return None
    if fields.get("kernel", "").strip() != kernel:
        return None
    return float(fields["traffic_bytes_per_launch"])


def eps_only(reps: int = 3) -> int:
    """fp64 epsilon solve on one N = 8192 graph (ER p = 4/N, seed 0), timed."""
    import torch

    import dlgen
    import paper_1608_00139_amd as dl

    a = dlgen.to_dense(N, dlgen.er_edges(N, 4.0 / N, 0))
    ad = torch.from_numpy(a).cuda()
    eps = 0.5 / (1.0 + float(a.sum(axis=1).max()))
    out = torch.empty_like(ad)
    for r in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dl.dl_solve_eps(ad, eps, out=out)
        torch.cuda.synchronize()
        print(f"eps solve {r}: {(time.perf_counter() - t0) * 1e3:.2f} ms", flush=True)
    return 0


def peaks(reps: int = 3) -> int:
    """dl_measure_peak for every kind, `reps` times each: matrix-core rates in
    TOPS / TFLOP/s, LDS read and global-to-LDS fill rates in TB/s and in
    bytes per clock per CU at 2.4 GHz (256 CUs)."""
    import torch

    import paper_1608_00139_amd as dl

    torch.cuda.set_device(0)
    ctx = dl.Context(0)
    for kind in ("i8", "fp8", "fp4", "bf16", "f32", "f64", "f64_agpr", "lds_read", "lds_fill"):
        vals = [dl.dl_measure_peak(kind, ctx=ctx) for _ in range(reps)]
        if kind.startswith("lds"):
            print(f"{kind}: " + ", ".join(f"{v / 1e12:.1f} TB/s ({v / 256 / 2.4e9:.0f} B/clk/CU)" for v in vals),
                  flush=True)
        else:
            print(f"{kind}: " + ", ".join(f"{v / 1e12:.1f} T/s" for v in vals), flush=True)
    ctx.close()
    return 0


def copy_calibration() -> int:
    """Three plain device copies of 1 GiB: read 1 GiB and write 1 GiB each."""
    import torch

    a = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy calibration: 3 x (1 GiB read + 1 GiB write)")
    return 0


def pmc_summary(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv) -> int:
    """Per-launch HBM traffic of the int8 step kernel (k_nt_dma ... OpI8).

    FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch; each is scaled
    by the ratio of the true bytes of a plain 1 GiB copy to what the same
    counter reads for that copy.  Launches that returned early (fixpoint
    already reached) are excluded by a cut at 10% of the largest value.
    """
    import csv

    def per_kernel(path, pred):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if pred(r["Kernel_Name"])]
        cut = 0.1 * max(vals)
        return [v for v in vals if v >= cut]

    # the step kernel with the most launches (a run after the autotuner also
    # holds a few launches of the other configurations)
    counts = {}
    for r in csv.DictReader(open(fetch_csv)):
        k = r["Kernel_Name"]
        if "k_nt_dma" in k and ("OpI8," in k or "OpI8x32," in k):
            counts[k] = counts.get(k, 0) + 1
    top = max(counts, key=counts.get)
    is_step = lambda k: k == top
    is_copy = lambda k: "copy" in k.lower() or "elementwise" in k
    kernel = STEP_KERNELS[3] if "OpI8x32" in top else STEP_KERNELS[0]
    f = per_kernel(fetch_csv, is_step)
    w = per_kernel(write_csv, is_step)
    cf = per_kernel(cal_fetch_csv, is_copy)
    cw = per_kernel(cal_write_csv, is_copy)
    gib_kib = float(1 << 20)
    ffac = gib_kib / (sum(cf) / len(cf))
    wfac = gib_kib / (sum(cw) / len(cw))
    fetch = sum(f) / len(f) * ffac * 1024
    write = sum(w) / len(w) * wfac * 1024
    algo = 2 * N * N + 2 * N * N  # X and Y read, out and out^T written (no addend read)
    print("# HBM traffic per launch of the int8 step kernel at N=8192 (rocprofv3 --pmc)")
    print(f"kernel: {kernel}")
    print(f"kernel_source_sha256: {source_hash()}")
    print(f"launches_counted: fetch={len(f)} write={len(w)}")
    print(f"calibration_fetch_factor: {ffac:.4f}")
    print(f"calibration_write_factor: {wfac:.4f}")
    print(f"fetch_bytes_per_launch: {fetch:.0f}")
    print(f"write_bytes_per_launch: {write:.0f}")
    print(f"traffic_bytes_per_launch: {fetch + write:.0f}")
    print(f"algorithmic_bytes_per_launch: {algo}  (X, Y read; out, out^T written; int8)")
    print(f"traffic_over_algorithmic: {(fetch + write) / algo:.3f}")
    return 0


def mfma_summary(csv_path: str) -> int:
    """Matrix-core activity per launch from SQ_INSTS_VALU_MFMA_MOPS_I8,
    SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE.

    MOPS_I8 counts int8 MFMA operations in units of 512, so a full step
    launch must read 2 Np^3 / 512.  GRBM_GUI_ACTIVE is summed over the XCDs
    and the busy cycles over every SIMD: busy fraction = busy / (GUI_ACTIVE /
    XCDs * SIMDs), clock = GUI_ACTIVE / XCDs / duration.  Step launches that
    returned early are excluded by a cut at 10% of the largest MOPS value.
    The device's XCD and SIMD counts come from k_agent_info.csv beside the
    counter file (8 and 1024 if it is absent).
    """
    import csv
    import os

    xcds, simds = 8, 1024
    info = os.path.join(os.path.dirname(csv_path), "k_agent_info.csv")
    if os.path.exists(info):
        for r in csv.DictReader(open(info)):
            if r.get("Agent_Type") == "GPU":
                xcds, simds = int(r["Num_Xcc"]), int(r["Simd_Count"])
    disp = {}
    for r in csv.DictReader(open(csv_path)):
        d = disp.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"],
                                               "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    counts = {}
    for d in disp.values():
        if "k_nt_dma" in d["name"] and ("OpI8," in d["name"] or "OpI8x32," in d["name"]):
            counts[d["name"]] = counts.get(d["name"], 0) + 1
    top = max(counts, key=counts.get)  # the timed workload's step kernel
    groups = {"step": lambda k: k == top,
              "peak": lambda k: "k_mfma_peak<0>" in k}
    print("# int8 matrix-core activity (rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_I8 SQ_VALU_MFMA_BUSY_CYCLES "
          "SQ_BUSY_CYCLES GRBM_GUI_ACTIVE)")
    print(f"# device: {xcds} XCDs, {simds} SIMDs")
    for label, pred in groups.items():
        ds = [d for d in disp.values() if pred(d["name"])]
        if not ds:
            continue
        top = max(d["SQ_INSTS_VALU_MFMA_MOPS_I8"] for d in ds)
        ds = [d for d in ds if d["SQ_INSTS_VALU_MFMA_MOPS_I8"] >= 0.1 * top]
        k = len(ds)
        ops = sum(d["SQ_INSTS_VALU_MFMA_MOPS_I8"] for d in ds) / k * 512
        us = sum(d["ns"] for d in ds) / k / 1e3
        ghz = sum(d["GRBM_GUI_ACTIVE"] / xcds / d["ns"] for d in ds) / k
        busy = sum(d["SQ_VALU_MFMA_BUSY_CYCLES"] / (d["GRBM_GUI_ACTIVE"] / xcds * simds) for d in ds) / k
        name = ds[0]["name"].split("(")[0].replace("void ", "")
        print(f"{label}: {name}")
        print(f"  launches: {k}")
        print(f"  int8_ops_per_launch: {ops:.4e}" + (f"  (2 Np^3 = {2.0 * N ** 3:.4e})" if label == "step" else ""))
        print(f"  duration_us: {us:.1f}")
        print(f"  clock_ghz: {ghz:.3f}")
        print(f"  mfma_busy_fraction: {busy:.3f}")
        print(f"  int8_tops: {ops / (us * 1e-6) / 1e12:.0f}")
    return 0


def counter_summary(csv_path: str, kernel: str | None = None) -> int:
    """Averages over the step kernel's full launches (duration above 10% of
    the longest) of each counter in a rocprofv3 --pmc CSV, also divided by
    the kernel's CU cycles (GRBM_GUI_ACTIVE / XCDs x CUs; the CSV must hold
    GRBM_GUI_ACTIVE).  SQ_WAVE_CYCLES counts in units of four cycles on this
    device (sixteen resident waves read four per CU cycle)."""
    import csv
    import os

    xcds, cus = 8, 256
    info = os.path.join(os.path.dirname(csv_path), "k_agent_info.csv")
    if os.path.exists(info):
        for r in csv.DictReader(open(info)):
            if r.get("Agent_Type") == "GPU":
                xcds, cus = int(r["Num_Xcc"]), int(r["Cu_Count"])
    disp = {}
    for r in csv.DictReader(open(csv_path)):
        d = disp.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"],
                                               "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    counts = {}
    for d in disp.values():
        if (kernel is not None and kernel in d["name"]) or (
                kernel is None and "k_nt_dma" in d["name"] and ("OpI8," in d["name"] or "OpI8x32," in d["name"])):
            counts[d["name"]] = counts.get(d["name"], 0) + 1
    top = max(counts, key=counts.get)  # the timed workload's step kernel, or the named one
    ds = [d for d in disp.values() if d["name"] == top]
    top = max(d["ns"] for d in ds)
    ds = [d for d in ds if d["ns"] >= 0.1 * top]
    keys = sorted(k for k in ds[0] if k not in ("name", "ns"))
    avg = {k: sum(d[k] for d in ds) / len(ds) for k in keys}
    cyc = avg["GRBM_GUI_ACTIVE"] / xcds
    ns = sum(d["ns"] for d in ds) / len(ds)
    print(f"kernel: {ds[0]['name'].split('(')[0].replace('void ', '')}")
    print(f"launches: {len(ds)}  duration_us: {ns / 1e3:.1f}  cycles: {cyc:.0f}  clock_ghz: {cyc / ns:.3f}")
    print(f"# {'counter':<34} {'per_launch':>16} {'per_CU_cycle':>13}")
    for k in keys:
        print(f"  {k:<34} {avg[k]:16.0f} {avg[k] / (cyc * cus):13.4f}")
    return 0


def busy_summary(csv_path: str) -> int:
    """Per kernel name of a rocprofv3 --pmc CSV: launches, average duration,
    clock (GRBM_GUI_ACTIVE / XCDs per ns) and the fraction of SIMD cycles the
    matrix cores were busy (SQ_VALU_MFMA_BUSY_CYCLES / (cycles x SIMDs))."""
    import csv
    import os

    xcds, simds = 8, 1024
    info = os.path.join(os.path.dirname(csv_path), "k_agent_info.csv")
    if os.path.exists(info):
        for r in csv.DictReader(open(info)):
            if r.get("Agent_Type") == "GPU":
                xcds, simds = int(r["Num_Xcc"]), int(r["Simd_Count"])
    disp = {}
    for r in csv.DictReader(open(csv_path)):
        d = disp.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"],
                                               "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    by = {}
    for d in disp.values():
        by.setdefault(d["name"], []).append(d)
    print(f"# {'launches':>8} {'avg_us':>10} {'clock_ghz':>9} {'mfma_busy':>9}  kernel")
    for name, ds in by.items():
        ns = sum(d["ns"] for d in ds) / len(ds)
        cyc = sum(d["GRBM_GUI_ACTIVE"] for d in ds) / len(ds) / xcds
        busy = sum(d["SQ_VALU_MFMA_BUSY_CYCLES"] for d in ds) / len(ds) / (cyc * simds)
        print(f"  {len(ds):8d} {ns / 1e3:10.1f} {cyc / ns:9.3f} {busy:9.3f}  {name.split('(')[0].replace('void ', '')}")
    return 0


def trace_busy(db_path: str, gap_ms: float) -> int:
    """Device occupancy of a rocprofv3 kernel trace, per segment: the trace is
    cut wherever no kernel runs for gap_ms or more; for each segment, its span
    (first start to last end), the time at least one kernel was running (the
    union of the kernel intervals) and the kernels with the most time."""
    import sqlite3

    con = sqlite3.connect(db_path)
    rows = sorted(con.execute("select start, end, name from kernels").fetchall())
    if not rows:
        print("no kernels in the trace")
        return 1
    segs, cur, cur_end = [], [], None
    for r in rows:
        if cur and r[0] - cur_end >= gap_ms * 1e6:
            segs.append(cur)
            cur = []
        cur.append(r)
        cur_end = r[1] if not cur_end or len(cur) == 1 else max(cur_end, r[1])
    segs.append(cur)
    print(f"# segments of {db_path} split at device idle gaps >= {gap_ms:g} ms")
    print(f"# {'seg':>3} {'kernels':>8} {'span_ms':>9} {'busy_ms':>9} {'busy':>6}  largest kernels (ms)")
    for i, sg in enumerate(segs):
        t0, t1 = sg[0][0], max(e for _, e, _ in sg)
        busy, reach = 0, t0
        for s, e, _ in sg:
            if e > reach:
                busy += e - max(s, reach)
                reach = e
        per = {}
        for s, e, n in sg:
            k = n.split("(")[0].replace("void ", "")
            per[k] = per.get(k, 0) + (e - s)
        top = sorted(per.items(), key=lambda x: -x[1])[:4]
        print(f"  {i:3d} {len(sg):8d} {(t1 - t0) / 1e6:9.2f} {busy / 1e6:9.2f} {busy / (t1 - t0):6.3f}  "
              + ", ".join(f"{k} {v / 1e6:.2f}" for k, v in top))
    return 0


def trace_summary(db_path: str) -> int:
    """Per-kernel statistics from a rocprofv3 kernel-trace database.

    Besides rocprofv3's own per-kernel average, the step kernels are also
    averaged over the launches that did work: a step launched after the
    fixpoint was reached returns at once (a few microseconds), and those
    launches are separated by a duration cut at 10% of the kernel's longest
    launch.
    """
    import sqlite3

    con = sqlite3.connect(db_path)
    rows = con.execute("select name, duration from kernels").fetchall()
    by = {}
    for name, dur in rows:
        by.setdefault(name, []).append(float(dur))
    total = sum(sum(v) for v in by.values())
    print(f"# kernel trace summary of {db_path}")
    print(f"# {'calls':>7} {'total_ms':>10} {'avg_us':>10} {'pct':>6} {'work_calls':>10} {'work_avg_us':>11}  kernel")
    for name, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        cut = 0.1 * max(v)
        work = [d for d in v if d >= cut]
        print(f"  {len(v):7d} {sum(v) / 1e6:10.3f} {sum(v) / len(v) / 1e3:10.3f} {100 * sum(v) / total:6.2f} "
              f"{len(work):10d} {sum(work) / len(work) / 1e3:11.3f}  {name[:110]}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
