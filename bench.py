#!/usr/bin/env python3
"""Benchmark of the MLMC sample-solve path on one MI355X.

Workload: the four-level FP64 waviness strip (20 x 5 mm orthotropic strip,
Q1 meshes 64x16, 128x32, 256x64, 512x128; Matern-3/2 KL field with 20 modes
plus a sech^2 wrinkle; Jacobi-PCG to rtol 1e-10).  One step is one MLMC
batch round: on every level a batch of coupled samples (Y_0 = Q_0 on level 0,
fine/coarse pairs with shared parameters above) goes through KL synthesis,
lifting, PCG, the QoI and the FP64 level sums.  The per-level batches are a
fixed mix, 2048 / 512 / 128 / 64, that gives every level a batch large
enough to fill the GPU (more samples on the cheaper coarse levels, as MLMC
allocates them); the allocation the MLMC formula itself chooses is what the
time-to-epsilon leg runs.  Parameter rows are generated and copied to the GPU
before the timed region.

Printed: one JSON line with the whole-job rate (coupled samples/s), per-level
rates, the roofline of the dominant kernel (the PCG vector pass) and of the
operator pass (both timed with HIP events on the solve stream), the CPU
oracle timed on the host cores, and two further legs of the metric: the
wall time of adaptive MLMC (Algorithm 1) to a relative RMSE in FP64 and in
mixed precision on the five-level strip, and the serving loop's p50/p99
latency over a mixed strip/panel request stream at 1e2, 1e3 and 1e4
requests/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import mlmc_inputs as mi  # noqa: E402

WORKLOAD = "strip_c2"
DEFAULT_MIX = [2048, 512, 128, 64]
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mix", type=str, default=",".join(map(str, DEFAULT_MIX)))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=str, default="16,8,4,2",
                    help="oracle samples per level for the CPU baseline")
    ap.add_argument("--levels", type=str, default="",
                    help="run only these levels (comma list; profiling runs, the line is then not the benchmark)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="mixed: FP32 operator on FP32 angles inside FP64 refinement")
    ap.add_argument("--mixed", type=str, default="",
                    help="overrides of the mixed-precision settings, e.g. update_factor=0.1,theta_storage=bf16")
    ap.add_argument("--plate", type=str, default="",
                    help="also time the buckling solver: samples per plate level, e.g. 1024,256,32,4")
    ap.add_argument("--plate-config", type=str, default="plate_c4",
                    help="panel workload of the plate leg: plate_c4 (500 mm panel) or plate_t2 (the 636 x 212 mm "
                         "Test Problem II panel)")
    ap.add_argument("--serve", type=str, default="100,1000,10000",
                    help="also run the serving loop over the mixed request stream at these arrival rates "
                         "(requests/s, comma list; empty: no serving leg)")
    ap.add_argument("--serve-duration", type=float, default=3.0,
                    help="seconds of arrivals per rate (0: the serving configuration's)")
    ap.add_argument("--time-to-eps", type=str, default="1e-3,1e-4",
                    help="also run adaptive MLMC (Algorithm 1) to these relative RMSEs, FP64 and mixed precision "
                         "(comma list; empty: no time-to-epsilon leg)")
    ap.add_argument("--tte-config", type=str, default="strip_c3",
                    help="strip workload of the time-to-epsilon runs")
    ap.add_argument("--no-legs", action="store_true",
                    help="only the batch-round benchmark: no time-to-epsilon and no serving leg (profiling runs)")
    ap.add_argument("--plate-mlmc", type=float, default=0.0,
                    help="also run MLMC with selective refinement (Algorithms 1 and 2) on the panel workload of "
                         "--plate-config to this relative tolerance, FP64 and mixed precision")
    ap.add_argument("--plate-mlmc-precisions", type=str, default="fp64,mixed",
                    help="precisions of the --plate-mlmc leg (comma list of fp64, mixed)")
    ap.add_argument("--cosserat", type=str, default="",
                    help="also time the Cosserat Test I workload: coupled samples per level, e.g. "
                         "2048,1024,512,128,32,8")
    ap.add_argument("--cosserat-single", action="store_true",
                    help="Cosserat leg: single solves on every level instead of coupled pairs (profiling)")
    ap.add_argument("--cosserat-eps", type=float, default=0.0,
                    help="also run adaptive MLMC (Algorithm 1) on the Cosserat workload to this relative RMSE")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=JSON",
                    help="override a key of the strip workload definition (tuning runs; the line is then "
                         "not the default benchmark), e.g. --set angle_storage='\"cs\"'")
    ap.add_argument("--calls", choices=["auto", "level", "round"], default="auto",
                    help="solve calls per step: one per level (per-level times inside the timed region), one "
                         "for the whole batch round, or auto (measured: per level for FP64, one call for "
                         "mixed precision)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


# ------------------------------------------------------------------ CPU oracle
_ORACLE_MODELS = None


def _oracle_job(job):
    level, row_idx = job
    models, rows = _ORACLE_MODELS
    row = rows[level][row_idx]
    t0 = time.perf_counter()
    models[level].solve(row)
    if level > 0:
        models[level - 1].solve(row)
    return level, time.perf_counter() - t0


def cpu_baseline(cfg, mix, counts):
    """The oracle (FP64 numpy/scipy, single-threaded BLAS per worker) on a bounded
    sample of the same workload, one worker process per host core."""
    global _ORACLE_MODELS
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle.kl import KL
    from oracle.strip import StripModel
    kl = KL(cfg)
    nl = len(mix)
    models = [StripModel(cfg, l, kl) for l in range(nl)]
    for m in models:          # per-level mode tables (set-up, not timed, as on the GPU)
        m.modes()
    rows = [mi.strip_xi(cfg, l, 10 ** 6, counts[l]) for l in range(nl)]
    _ORACLE_MODELS = (models, rows)
    # one worker per host core of this GPU's share of the host: the boxes
    # this runs on give one GPU 16 cores, whatever the affinity mask shows
    visible = len(os.sched_getaffinity(0))
    cores = min(visible, int(os.environ.get("MLMC_HOST_CORES", "16")))
    jobs = [(l, k) for l in reversed(range(nl)) for k in range(counts[l])]
    res = []
    # one BLAS thread per worker process (the forked workers inherit the limit)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(cores) as pool:
            for r in pool.imap_unordered(_oracle_job, jobs, chunksize=1):
                res.append(r)
                if len(res) % 4 == 0 or len(res) == len(jobs):
                    print(f"cpu baseline: {len(res)}/{len(jobs)} oracle samples done", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
    per_level = [np.mean([t for l, t in res if l == lv]) for lv in range(nl)]
    # throughput on the benchmark's mix: cores workers sharing the per-sample costs
    step_cpu_s = sum(n * t for n, t in zip(mix, per_level))
    value = sum(mix) / (step_cpu_s / cores)
    sample = (f"{'+'.join(str(c) for c in counts)} coupled samples on levels 0..{nl - 1} "
              f"({wall:.1f} s wall on {cores} worker processes); per-sample oracle seconds "
              + ", ".join(f"L{l}={t:.3f}" for l, t in enumerate(per_level)))
    return {"value": value, "unit": "coupled samples/s", "cores": cores, "host_cpus_visible": visible,
            "kind": "oracle", "sample": sample, "per_level_s_per_sample": per_level}


# ------------------------------------------------------------------ GPU
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "{kernel}_strip4lvl_fp64_hbm_traffic.md")
CSRC = os.path.join(ROOT, "paper_1907_10271_amd", "csrc")
# sources that define the operator pass, its launches and the strip solve around it
STRIP_SOURCES = ("api.hip", "common.hpp", "strip_device.hpp", "strip_kernels.hip", "strip_kernels.hpp",
                 "strip_small.hip", "strip_small.hpp")


def profiled_traffic(kernel):
    """HBM bytes per launch of ``kernel`` (k_pass1 or k_pass2) from the
    committed hardware-counter summary of this benchmark, or None when the
    library sources changed since."""
    import hashlib
    path = TRAFFIC_PROFILE.format(kernel=kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if " = " in line:
            k, v = line.split(" = ", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in STRIP_SOURCES:                     # any change to the strip solver invalidates the counters
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    if vals.get("kernel_sources_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def plate_leg(pk, torch, counts, prec, name="plate_c4"):
    """Buckling loads per level of a panel workload (one timed batch per level)."""
    pcfg = mi.load_config(name)
    pctx = pk.Context(mi.config_text(name))
    res = []
    for l, n in enumerate(counts):
        if n <= 0:
            continue
        off = torch.from_numpy(mi.plate_offsets(pcfg, l, 0, n)).to("cuda")
        reqs = [(k, l, False) for k in range(n)]
        pctx.reserve(l, n, prec)                              # the level's workspace, outside the timing
        pctx.buckle_batch(reqs[:1], off, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lf, _, info = pctx.buckle_batch(reqs, off, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res.append({"level": l, "mesh": f"{pcfg['nx0'] << l}x{pcfg['ny0'] << l}", "samples": n,
                    "ms": round(dt * 1e3, 3), "samples_per_s": round(n / dt, 1),
                    "lobpcg_iters_mean": round(float(info["iters_f"].mean()), 1),
                    "all_converged": bool(np.all(info["status_f"] == 0))})
    return res


def serve_leg(pk, rates, duration, prec):
    """Serving loop over the mixed strip/panel request stream at each arrival rate."""
    from paper_1907_10271_amd.serve import serve_sweep
    scfg = mi.load_config("serve_c5")
    stats = serve_sweep(scfg, prec, rates, duration or None,
                        log=lambda m: print("serve: " + m, file=sys.stderr, flush=True))
    return {"workload": "Poisson requests, 70% strip (5 levels 64x16..1024x256) / 30% panel (4 levels 16^2..128^2), "
                        "level mix strip " + str(scfg["strip_level_weights"]) + " panel " +
                        str(scfg["plate_level_weights"]),
            "workers": scfg["workers"], "max_batch": scfg["max_batch"], "mem_budget_gib": scfg["mem_budget_gib"],
            "rates": [{"offered_per_s": r, "requests": s.requests, "served_per_s": round(s.throughput, 1),
                       "p50_ms": round(s.p50_ms, 2), "p99_ms": round(s.p99_ms, 2),
                       "mean_batch": round(s.mean_batch, 2), "failed": s.failed,
                       "per_class": s.per_class} for r, s in zip(rates, stats)]}


def plate_mlmc_leg(pk, torch, name, tau, precisions=("fp64", "mixed")):
    """MLMC with selective refinement for the failure probability of a panel
    workload to a relative tolerance, FP64 and mixed precision."""
    from paper_1907_10271_amd.driver import run_plate_mlmc_sr
    cfg = mi.load_config(name)
    out = {"workload": name, "tau_rel": tau, "lambda_star": cfg["lambda_crit"]}
    for label, prec in (("fp64", pk.FP64), ("mixed", pk.MIXED)):
        if label not in precisions:
            continue
        ctx = pk.Context(mi.config_text(name))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = run_plate_mlmc_sr(ctx, cfg, tau_rel=tau, precision=prec,
                                log=lambda m: print(f"plate mlmc {label}: {m}", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        d = res.as_dict()
        out[label] = {"seconds": round(time.perf_counter() - t0, 2), "estimate": d["estimate"],
                      "rmse": math.sqrt(d["sampling_err2"] + d["bias_estimate"] ** 2), "e_abs": d["e_abs"],
                      "L": d["L"], "converged": d["converged"], "bias_estimate": d["bias_estimate"],
                      "sampling_err2": d["sampling_err2"], "N": [lv["N"] for lv in d["levels"]],
                      "solves_per_level": res.history[-1]["solves_per_level"]}
        ctx.close()
    return out


def cosserat_leg(pk, torch, counts, eps_rel, coupled=True):
    """The Cosserat Test I workload: one timed batch of coupled samples per level
    (synthesis, PCG, QoI, both solves of a pair), and optionally Algorithm 1 to
    a relative RMSE.  The bandwidth figure divides the algorithmic bytes of all
    PCG iterations (117 B per unknown and iteration: 7 FP64 vectors and the
    angle pairs of the operator pass, 7 of the vector pass) by the batch's wall
    time, set-up and QoI included."""
    name = "cosserat_t1"
    cfg = mi.load_config(name)
    ctx = pk.Context(mi.config_text(name))
    out = {"workload": name, "per_level": []}
    for l, n in enumerate(counts):
        if n <= 0:
            continue
        xi = torch.from_numpy(mi.strip_xi(cfg, l, 0, n)).to("cuda")
        pair = coupled and l > 0
        reqs = [(k, l, pair) for k in range(n)]
        ctx.reserve(l, n)
        if pair:
            ctx.reserve(l - 1, n)
        ctx.solve_batch(reqs[:1], xi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qf, qc, info = ctx.solve_batch(reqs, xi)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nd = [ctx.level_info(k)["n_dofs"] for k in range(cfg["n_levels"])]
        work = float(info["iters_f"].sum()) * nd[l] + (float(info["iters_c"].sum()) * nd[l - 1] if pair else 0.0)
        out["per_level"].append({"level": l, "mesh": f"{cfg['nx0'] << l}x{cfg['ny0'] << l}", "samples": n,
                                 "coupled": pair, "ms": round(dt * 1e3, 3), "samples_per_s": round(n / dt, 1),
                                 "pcg_iters_mean": round(float(info["iters_f"].mean()), 1),
                                 "whole_solve_GBs": round(117.0 * work / dt / 1e9, 1),
                                 "all_converged": bool(np.all(info["status_f"] == 0))})
    if eps_rel > 0:
        from paper_1907_10271_amd.driver import run_strip_mlmc
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = run_strip_mlmc(ctx, cfg, precision=pk.FP64, eps_rel=eps_rel,
                             log=lambda m: print(f"cosserat mlmc: {m}", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        d = res.as_dict()
        out["mlmc"] = {"eps_rel": eps_rel, "seconds": round(time.perf_counter() - t0, 2), "estimate": d["estimate"],
                       "L": d["L"], "converged": d["converged"], "e_abs": d["e_abs"],
                       "bias_estimate": d["bias_estimate"], "sampling_err2": d["sampling_err2"],
                       "alpha": d.get("alpha"), "levels": d["levels"]}
    ctx.close()
    return out


def tte_leg(pk, torch, name, eps_rel):
    """Wall time of adaptive MLMC (Algorithm 1) to a relative RMSE, FP64 and mixed precision."""
    from paper_1907_10271_amd.driver import run_strip_mlmc
    cfg = mi.load_config(name)
    out = {"workload": name, "eps_rel": eps_rel}
    for label, prec in (("fp64", pk.FP64), ("mixed", pk.MIXED)):
        ctx = pk.Context(mi.config_text(name))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = run_strip_mlmc(ctx, cfg, precision=prec, eps_rel=eps_rel,
                             log=lambda m: print(f"tte {label}: {m}", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        d = res.as_dict()
        out[label] = {"seconds": round(dt, 2), "estimate": d["estimate"], "L": d["L"], "converged": d["converged"],
                      "e_abs": d["e_abs"], "bias_estimate": d["bias_estimate"],
                      "sampling_err2": d["sampling_err2"], "levels": d["levels"]}
        ctx.close()
    out["speedup_mixed"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: --gpus {args.gpus} is not supported (the path is "
              f"data-parallel over samples; the multi-GPU design shards sample ranges and all-reduces "
              f"the per-level sums, but it is not built)", file=sys.stderr)
        sys.exit(2)
    cfg = mi.load_config(WORKLOAD)
    mix = [int(v) for v in args.mix.split(",")]
    assert len(mix) == cfg["n_levels"]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, mix, [int(v) for v in args.cpu_samples.split(",")])

    import torch
    import paper_1907_10271_amd as pk
    dev = torch.device("cuda:0")
    ccfg = dict(cfg)
    if args.mixed:
        mx = dict(ccfg.get("mixed", {}))
        for kv in args.mixed.split(","):
            k, v = kv.split("=")
            mx[k] = v if k == "theta_storage" else float(v)
        ccfg["mixed"] = mx
    for kv in args.set:
        k, v = kv.split("=", 1)
        ccfg[k] = json.loads(v)
    ctx = pk.Context(ccfg)
    nsteps = args.warmup + args.steps
    xi = []
    for l, n in enumerate(mix):
        rows = mi.strip_xi(cfg, l, 0, n * nsteps)
        xi.append(torch.from_numpy(rows).to(dev))
    torch.cuda.synchronize()
    reqs = [[(k, l, l > 0) for k in range(n)] for l, n in enumerate(mix)]
    prec = pk.MIXED if args.precision == "mixed" else pk.FP64
    levels = [int(v) for v in args.levels.split(",")] if args.levels else list(range(len(mix)))
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()

    def step_levels(s, events=None):
        """The batch round as one solve call per level."""
        accs = []
        for l, n in enumerate(mix):
            if l not in levels:
                accs.append(None)
                continue
            x = xi[l][s * n:(s + 1) * n]
            if events is not None:
                events[l][0].record(stream)
            qf, qc, info = ctx.solve_batch(reqs[l], x, precision=prec)
            acc = ctx.level_stats(l, qf, qc if l > 0 else None)
            if events is not None:
                events[l][1].record(stream)
            accs.append((acc, info))
        return accs

    # the batch round as one call: every level's requests together (the
    # library runs the whole-solve levels beside the lock-step ones and puts
    # the lock-step levels in shared launches); parameter rows of all levels
    # are gathered per step before the timed region
    offs, o = {}, 0
    for l, n in enumerate(mix):
        if l in levels:
            offs[l] = o
            o += n
    all_reqs = [(offs[l] + k, l, l > 0) for l, n in enumerate(mix) if l in levels for k in range(n)]
    xi_round = [torch.cat([xi[l][s * n:(s + 1) * n] for l, n in enumerate(mix) if l in levels]).contiguous()
                for s in range(nsteps)]
    torch.cuda.synchronize()

    def step_round(s, events=None):
        qf, qc, info = ctx.solve_batch(all_reqs, xi_round[s], precision=prec)
        accs = []
        for l, n in enumerate(mix):
            if l not in levels:
                accs.append(None)
                continue
            a, b = offs[l], offs[l] + n
            acc = ctx.level_stats(l, qf[a:b], qc[a:b] if l > 0 else None)
            accs.append((acc, info[a:b]))
        return accs

    # measured on this benchmark: FP64 631 ms per step with one call per level
    # against 648 ms with one call (sharing the operator-pass launches gives
    # level 2 the streaming accesses of the large launch, and the whole-solve
    # levels beside them gain nothing); mixed precision 546 against 517 ms
    per_level_calls = args.calls == "level" or (args.calls == "auto" and prec == pk.FP64)
    step = step_levels if per_level_calls else step_round
    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    ctx.profile(True)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in mix]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for s in range(args.steps):
        results.append(step(args.warmup + s, ev[s]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    k1, k2 = (0, 1) if prec == pk.FP64 else (2, 3)
    p1, p2 = ctx.profile_read(k1), ctx.profile_read(k2)
    dofs1, dofs2 = ctx.profile_read(k1 + 4)["bytes"], ctx.profile_read(k2 + 4)["bytes"]
    ctx.profile(False)
    if not per_level_calls:
        # per-level times (outside the timed region): each level alone, on the
        # parameter rows of the last timed step
        step_levels(args.warmup + args.steps - 1, ev[-1])
        torch.cuda.synchronize()
    per_level = []
    for l, n in enumerate(mix):
        if l not in levels:
            continue
        if per_level_calls:
            ms = np.mean([ev[s][l][0].elapsed_time(ev[s][l][1]) for s in range(args.steps)])
        else:
            ms = ev[-1][l][0].elapsed_time(ev[-1][l][1])
        its_f = np.concatenate([r[l][1]["iters_f"] for r in results])
        ok = all(np.all(r[l][1]["status_f"] == 0) for r in results)
        per_level.append({"level": l, "mesh": f"{cfg['nx0'] << l}x{cfg['ny0'] << l}", "samples": n,
                          "coupled": l > 0, ("ms" if per_level_calls else "ms_alone"): round(float(ms), 3),
                          "samples_per_s": round(n / (ms / 1e3), 1),
                          "pcg_iters_mean": round(float(its_f.mean()), 1), "all_converged": bool(ok)})
    default_run = (mix == DEFAULT_MIX and prec == pk.FP64 and not args.mixed and not args.set
                   and len(levels) == len(mix))
    # Roofline of the two PCG passes, each priced at the algorithmic bytes per
    # unknown of the plain two-pass FP64 iteration (vector pass: read x, r,
    # A p, p, diag(A), write x, r = 7 vectors; operator: read x, write y, and
    # the angles, 4 Gauss points x 8 B per 2 unknowns) times the unknowns of
    # the samples active in the timed launches, over the event-timed launch
    # duration; beside it the kernel's own byte model (which keeps z = r /
    # diag(A), fuses the p-update into the operator pass and moves x every
    # second iteration).  Mixed precision halves the vector bytes and stores
    # FP32 angles.
    w = 8.0 if prec == pk.FP64 else 4.0
    per_unknown = {"k_pass2": 7 * w, "k_pass1": 2 * w + 2 * w}

    def copy_ceiling():
        """Device-to-device copy of 1 GiB through the runtime's copy kernel,
        best of five, timed with HIP events: bytes read plus bytes written over
        the copy's duration, a reference rate for a plain streaming kernel on
        this GPU (not a bound: a tuned stream can exceed it)."""
        n = 1 << 27
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        best = float("inf")
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        del src, dst
        return 2 * 8 * n / (best / 1e3) / 1e9

    # (not in the counter runs, whose calibration counts one 1 GiB copy)
    copy_gbs = None if args.copy_calibration else copy_ceiling()

    def roof(kernel, p, dofs, what):
        if not p["launches"] or p["ms"] <= 0:
            return None
        sec = p["ms"] / 1e3
        alg = per_unknown[kernel] * dofs
        achieved = alg / sec / 1e9
        traffic = profiled_traffic(kernel) if default_run else None
        return {"bound": "hbm", "kernel": f"{kernel}<{'double' if prec == pk.FP64 else 'float'}> ({what})",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "alg_bytes_per_unknown": per_unknown[kernel],
                "unknowns_per_launch": round(dofs / p["launches"], 1),
                "alg_bytes_per_launch": round(alg / p["launches"], 1),
                "avg_launch_us": round(p["ms"] * 1e3 / p["launches"], 3), "timed_launches": p["launches"],
                "timing": "HIP events on the solve stream around the passes of iteration 16 (even blocks) or 17 "
                          "(odd blocks) of every block of 32",
                "kernel_model_bytes_per_launch": round(p["bytes"] / p["launches"], 1),
                "kernel_model_GBs": round(p["bytes"] / sec / 1e9, 1),
                "runtime_copy_GBs": None if copy_gbs is None else round(copy_gbs, 1),
                "vs_runtime_copy": None if copy_gbs is None else round(achieved / copy_gbs, 4)}

    total = sum(n for l, n in enumerate(mix) if l in levels)
    out = {
        "metric": "coupled-sample solves/s (4-level FP64 waviness strip, one MLMC batch round per step)",
        "value": round(total / (ms_per_step / 1e3), 2),
        "unit": "coupled samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == pk.FP64 else "f32 inner, f64 refinement",
        "data": "synthetic (seeded KL parameters and wrinkles)",
        "config": {"workload": "waviness strip 20x5 mm, 4 levels 64x16..512x128, Matern-3/2 20 modes + wrinkle, "
                               "Jacobi-PCG rtol 1e-10, FP64",
                   "batch_per_level": mix, "parallelism": "single GPU, data-parallel over samples",
                   "solve_calls_per_step": "one per level" if per_level_calls else "one for all levels"},
        "per_level": per_level,
        # the vector pass takes the larger share of the GPU time (kernel trace)
        "roofline": roof("k_pass2", p2, dofs2, "PCG vector pass, the dominant kernel"),
        "roofline_operator": roof("k_pass1", p1, dofs1, "PCG operator pass"),
        "cpu_baseline": None if cpu is None else {k: v for k, v in cpu.items() if k != "per_level_s_per_sample"},
    }
    if args.plate:
        out["plate"] = plate_leg(pk, torch, [int(v) for v in args.plate.split(",")], prec, args.plate_config)
        out["plate_workload"] = args.plate_config
    del ctx
    if args.time_to_eps and not args.no_legs:
        out["time_to_eps"] = [tte_leg(pk, torch, args.tte_config, float(e)) for e in args.time_to_eps.split(",")]
    if args.plate_mlmc > 0:
        out["plate_mlmc"] = plate_mlmc_leg(pk, torch, args.plate_config, args.plate_mlmc,
                                           args.plate_mlmc_precisions.split(","))
    if args.cosserat or args.cosserat_eps > 0:
        out["cosserat"] = cosserat_leg(pk, torch, [int(v) for v in args.cosserat.split(",")] if args.cosserat else [],
                                       args.cosserat_eps, coupled=not args.cosserat_single)
    if args.serve and not args.no_legs:
        out["serving"] = serve_leg(pk, [float(v) for v in args.serve.split(",")], args.serve_duration, prec)
    if len(levels) != len(mix):
        out["metric"] = "profiling run on levels " + args.levels + " only (not the benchmark)"
    if cpu is not None:
        out["cpu_baseline"]["value"] = round(cpu["value"], 3)
        out["gpu_over_cpu"] = round(out["value"] / cpu["value"], 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
