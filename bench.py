"""Benchmark: grid-point updates/s of the level-set explicit time step on one
MI355X.

Workload (one "step" of this benchmark = one whole solve): the relative-Dubins
pursuit-evasion tube, ve = vp = 5, |we|,|wp| <= 1, grid 101^3 on
[-6,20]x[-10,10]x[-pi,pi) (psi periodic), V0 = sqrt(x^2+y^2) - 5,
WENO5 + Lax-Friedrichs + TVD-RK3, CFL 0.8, tube to t = 2.8 (820 RK steps,
2460 fused stage launches plus the alpha reduction), FP64.  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line (rank 0).  Also reports the roofline of the dominant
kernel (the fused WENO5 stage kernel, timed with HIP events on the stream it
is launched on) and the FP64 CPU oracle timed on the host's cores.

    python bench.py [--steps K] [--warmup W] [--prec fp64|fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (WENO5+LF+RK3) served vs plain; p50/p99 solve latency"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (KiB per dispatch, scaled by a 512 MiB copy: x2.000 and
# x1.000), keyed by precision, with the hash of the kernel sources they were
# taken on; a changed source reports null until the counters are re-taken.
# An FP32 solve's front band at a long horizon is held to this many times the
# largest band spread of three FP32-storage realizations of the oracle (the
# FP32 kernels perturb each stage by up to 3 ulps, the storage model by half
# an ulp; the amplification of those seeds is linear), or 1e-4.
SPREAD_BAR_FACTOR = 4.0

MEASURED_TRAFFIC = {
    "fp64": {"src_hash": "9ac697e22dbca3da", "fetch_kib": 9827.3, "write_kib": 8049.2,
             "fetch_scale": 2.0, "write_scale": 1.0},
    "fp32": {"src_hash": "9ac697e22dbca3da", "fetch_kib": 4930.6, "write_kib": 4024.6,
             "fetch_scale": 2.0, "write_scale": 1.0},
}


# the sources the per-node stage kernel is compiled from, and its build flags
STAGE_KERNEL_SOURCES = ("hj_internal.h", "hj_stage_impl.h", "hj_launch_impl.h",
                        "hj_stage_f64_exact.hip", "hj_stage_f32.hip")


def source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2507_11542_amd")
    paths = [os.path.join(pkg, "csrc", f) for f in STAGE_KERNEL_SOURCES]
    paths.append(os.path.join(pkg, "build_lib.py"))
    for f in paths:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec: str):
    m = MEASURED_TRAFFIC.get(prec)
    if not m or m["src_hash"] != source_hash():
        return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


# Floating-point operations of the WENO5 formulas (Sec. 3.3), counted on the
# formulas: a window of five first differences w0..w4 (smoothness of the three
# substencils 33, eps = 1e-6 max w^2 + floor 7 with the four maxima, the three
# reciprocal weights (S + eps)^-2 9) and one blend of the third-order
# candidates with them (candidates 15, linear weights 3, weighted sum 5,
# normalisation 3).
WENO_WINDOW_FLOPS = 33 + 7 + 9
WENO_BLEND_FLOPS = 15 + 3 + 5 + 3


def weno5_flops_per_node_stage(ndim: int, executed: bool = False) -> float:
    """Floating-point operations of one RK stage at one node of the WENO5 +
    Lax-Friedrichs + RK3 relative-Dubins step (Sec. 3.3, 4, 5).

    The method's count (executed=False): along each axis a node adds one first
    difference (a subtraction and the 1/dx scaling) and one WENO window, the
    one centred on the interface to its right, which serves the right-biased
    derivative of the node and the left-biased one of its neighbour; two blends
    give p- and p+.  Then p-bar 2/axis, the Lax-Friedrichs term 4/axis, the
    Hamiltonian 17, the sign 1 and the RK combination (13/3, the average of
    the three stages).

    The executed count (executed=True) is what the per-node kernel evaluates:
    every node forms its six first differences per axis and both of its
    windows itself."""
    if executed:
        per_axis = 6 * 2 + 2 * WENO_WINDOW_FLOPS + 2 * WENO_BLEND_FLOPS
    else:
        per_axis = 2 + WENO_WINDOW_FLOPS + 2 * WENO_BLEND_FLOPS
    return ndim * (per_axis + 2 + 4) + 17 + 1 + 13.0 / 3.0


def stage_launch_time(g, v0, out, p, stream, reps: int = 3):
    """Average duration of one stage launch of the solve: HIP events on the
    launch stream around whole hj_solve calls over [t0, tf] and [t0, tf/2]
    (best of `reps` each).  Their difference is K1 - K2 RK steps of three
    back-to-back launches, free of what both calls share (the alpha
    reduction, its read-back, the V0 copy), so launches x this time stays
    within the solve's wall time.  Also returns the per-launch time of the
    whole [t0, tf] solve (those shared parts included)."""
    import torch

    res = {}
    for tf in (p.tf, 0.5 * (p.t0 + p.tf)):
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.solve(v0, out, p.t0, tf, p.mode, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
        res[tf] = (best, g.schedule(p.t0, tf, stream)[2])
    (t1, k1), (t2, k2) = res[p.tf], res[0.5 * (p.t0 + p.tf)]
    return (t1 - t2) / (3 * (k1 - k2)), t1 / (3 * k1)


def bytes_per_node_stage(elem: int, tube: bool) -> float:
    """Algorithmic HBM bytes per node per RK3 stage (average of the three):
    stage 1 reads V and writes A; stage 2 reads A and V and writes B; stage 3
    reads B, V (and V0 for a tube) and writes V."""
    passes = 2 + 3 + (4 if tube else 3)
    return passes * elem / 3.0


def cpu_baseline(p, target_s: float = 15.0):
    import oracle

    threads = oracle.set_threads(0)
    v0 = p.v0()
    alpha, dt, k, _ = oracle.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, p.t0, p.tf)
    t = time.perf_counter()
    oracle.steps(v0, v0, *p.grid_args(), p.dynamics, p.params, p.scheme, p.order, alpha, dt, 1,
                 mode=p.mode)
    one = time.perf_counter() - t
    nsteps = int(max(1, min(k, round(target_s / max(one, 1e-3)))))
    t = time.perf_counter()
    oracle.steps(v0, v0, *p.grid_args(), p.dynamics, p.params, p.scheme, p.order, alpha, dt,
                 nsteps, mode=p.mode)
    el = time.perf_counter() - t
    return {"value": p.points * nsteps / el, "unit": "grid-point updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d of the %d RK3 steps of the same 101^3 tube solve "
                      "(FP64 C oracle, OpenMP over nodes), %.1f s" % (nsteps, k, el)}


def bench_rockets(args):
    """The paper's rockets experiment (Sec. 6.1): 100^3, ENO2 / LF / TVD-RK3,
    the variational-inequality tube over t in [-2.5, 0] through 11 output
    times (590 steps), as one hj_solve_outputs per repetition, FP64 and FP32;
    both precisions' outputs are compared with the stored oracle samples."""
    import numpy as np
    import torch

    from paper_2507_11542_amd import hj, inputs

    p = inputs.rockets()
    times = [float(t) for t in inputs.output_times(p.t0, p.tf)]
    st = torch.cuda.current_stream()
    res = {"workload": "rockets game 100^3 on [-64,64]^2 x [-pi/2,pi/2], a=1, g=32, |u|<=1, "
                       "ENO2+LF+RK3, variational-inequality tube over [-2.5,0], 11 outputs"}
    for prec in ("fp64", "fp32"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        v0 = torch.from_numpy(p.v0()).to("cuda", dtype=dtype)
        outs = torch.empty((len(times),) + tuple(p.n), dtype=dtype, device="cuda")
        g = hj.Grid.from_problem(p, prec)
        g.solve_outputs(v0, outs, p.t0, times, p.mode, st)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(args.rockets_reps):
            t = time.perf_counter()
            g.solve_outputs(v0, outs, p.t0, times, p.mode, st)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        steps = 0
        for a, b in zip([p.t0] + times[:-1], times):
            steps += g.schedule(a, b, st)[2] if b > a else 0
        g.close()
        row = {"solve_s": best, "steps": steps, "updates_per_s": p.points * steps / best,
               "per_output_chunk_s": best / (len(times) - 1)}
        gold = os.path.join(ROOT, "tests", "golden", "rockets_100_vi_samples.txt")
        if os.path.exists(gold):
            data = np.loadtxt(gold)
            host = outs.cpu().numpy()
            err = 0.0
            for o in np.unique(data[:, 0]).astype(int):
                rows = data[data[:, 0] == o]
                vals = host[o].ravel()[rows[:, 1].astype(np.int64)]
                err = max(err, float(np.abs(vals - rows[:, 2]).max()))
            row["error_vs_oracle_fp64"] = err
            row["error_sampled_at"] = "%d stored oracle nodes of the outputs at t=-1.25, 0" \
                % len(data)
        res[prec] = row
    res["paper_table1_context"] = {
        "levelsetpy_gpu_global_s": 11.5153, "levelsetpy_gpu_avg_local_s": 1.1833,
        "levelsetpy_cpu_global_s": 107.84, "toolboxls_matlab_global_s": 138.50,
        "hardware": "Quadro RTX 4000 (CuPy, FP64) / i9-10885H one thread; step counts "
                    "and CFL number not stated, so not the same arithmetic"}
    return res


def bench_dubins4d(args):
    """4-D Dubins car with speed state, 61^4 on [-5,5]^2 x [-pi,pi) x [0,4],
    WENO5+LF+RK3, reachable set to t = 2 (182 steps), FP64 and FP32 side by
    side: one hj_solve per repetition, V0 resident; both results against the
    stored FP64 oracle values at 4096 seeded nodes, and FP32 against FP64."""
    import numpy as np
    import torch

    from paper_2507_11542_amd import hj, inputs

    p = inputs.dubins4d()
    st = torch.cuda.current_stream()
    gold = os.path.join(ROOT, "tests", "golden", "dubins4d_61_set_samples.txt")
    data = np.loadtxt(gold) if os.path.exists(gold) else None
    res = {"workload": "4-D Dubins 61^4 on [-5,5]^2 x [-pi,pi) x [0,4], |w|,|a| <= 1, "
                       "WENO5+LF+RK3, reachable set to t=2"}
    sampled = {}
    for prec in ("fp64", "fp32"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        v0 = torch.from_numpy(p.v0()).to("cuda", dtype=dtype)
        out = torch.empty_like(v0)
        g = hj.Grid.from_problem(p, prec)
        g.solve(v0, out, p.t0, p.tf, p.mode, st)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(args.rockets_reps):
            t = time.perf_counter()
            g.solve(v0, out, p.t0, p.tf, p.mode, st)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        steps = g.schedule(p.t0, p.tf, st)[2]
        g.close()
        row = {"solve_s": best, "steps": steps, "updates_per_s": p.points * steps / best}
        if data is not None:
            idx = torch.from_numpy(data[:, 0].astype(np.int64)).to("cuda")
            vals = out.reshape(-1).index_select(0, idx).double().cpu().numpy()
            sampled[prec] = vals
            row["error_vs_oracle_fp64"] = float(np.abs(vals - data[:, 1]).max())
            row["error_sampled_at"] = "%d stored oracle nodes (whole grid)" % len(data)
        res[prec] = row
        del v0, out
    if len(sampled) == 2:
        res["fp32_vs_fp64_max_abs"] = float(np.abs(sampled["fp32"] - sampled["fp64"]).max())
        # stored nodes in the front band, 6 cells or more from a bounded edge
        ii = np.unravel_index(data[:, 0].astype(np.int64), p.n)
        keep = np.abs(data[:, 1]) < 3 * float(inputs.cell_sizes(*p.grid_args()).max())
        for d, per in enumerate(p.periodic):
            if not per:
                keep &= (ii[d] >= 6) & (ii[d] < p.n[d] - 6)
        res["fp32"]["band_error_vs_oracle_fp64"] = float(
            np.abs(sampled["fp32"] - data[:, 1])[keep].max())
        res["fp32"]["band_nodes_sampled"] = int(keep.sum())
    return res


def bench_batched(args):
    """64 relative-Dubins tubes of uneven size (N ~ U{51,61,81,101}, seeded
    speeds and turn bounds), FP32 with FP64 time: one batched solve (round
    launches replayed from a captured graph, autotuned tile shape) against the
    same instances one at a time through hj_solve."""
    import numpy as np
    import torch

    from paper_2507_11542_amd import autotune, hj, inputs

    prec = "fp32"
    probs = inputs.rel_dubins_batch(args.batch_count, seed=0)
    stream = torch.cuda.current_stream()
    grids = [hj.Grid.from_problem(p, prec) for p in probs]
    v0s = [torch.from_numpy(p.v0()).to("cuda", torch.float32) for p in probs]
    outs = [torch.empty_like(v) for v in v0s]
    steps = [g.schedule(p.t0, p.tf, stream)[2] for g, p in zip(grids, probs)]
    updates = float(sum(p.points * k for p, k in zip(probs, steps)))
    (tile, wg), timings = autotune.tune(probs, grids, v0s, prec, stream=stream)
    b = hj.Batch(tile_nodes=tile, workgroups=wg, use_graph=True)
    t0s = [p.t0 for p in probs]
    tfs = [p.tf for p in probs]
    modes = [p.mode for p in probs]
    b.solve(grids, v0s, outs, t0s, tfs, modes, stream)  # warm-up (capture)
    b.wait(len(probs), stream)
    t = time.perf_counter()
    b.solve(grids, v0s, outs, t0s, tfs, modes, stream)
    tfin, items = b.wait(len(probs), stream)
    batched_s = time.perf_counter() - t
    # plain: the same instances one at a time
    plain_out = [torch.empty_like(v) for v in v0s]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for g, p, v, o in zip(grids, probs, v0s, plain_out):
        g.solve(v, o, p.t0, p.tf, p.mode, stream)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t
    same = all(torch.equal(a, c) for a, c in zip(outs, plain_out))
    accuracy = batch_accuracy(probs, outs) if args.batch_count == 64 else None
    b.close()
    for g in grids:
        g.close()
    return {"workload": "%d relative-Dubins tubes, N~U{51,61,81,101}, ve,vp~U[3,6], "
                        "we,wp~U[0.5,1.5] (rng 0), WENO5+LF+RK3, t=2.8" % len(probs),
            "dtype": "f32 (FP64 t, dt, alpha)", "points": int(sum(p.points for p in probs)),
            "rk_steps_total": int(sum(steps)), "updates": updates,
            "batched_s": batched_s, "batched_updates_per_s": updates / batched_s,
            "plain_s": plain_s, "plain_updates_per_s": updates / plain_s,
            "speedup_vs_plain": plain_s / batched_s, "tile_nodes": tile, "workgroups": wg,
            "autotune_ms_per_step": timings, "batched_equals_plain_bitwise": bool(same),
            "t_final_max_err": float(max(abs(a - p.tf) for a, p in zip(tfin, probs))),
            "fp32_vs_oracle_fp64": accuracy}


def batch_accuracy(probs, outs):
    """Error of the batched FP32 results against the FP64 oracle at its
    stored front-band nodes, every instance, beside the band spread of three
    FP32-storage realizations of the oracle itself (single-precision storage,
    FP64 arithmetic, V0 differing in its last bits)."""
    import numpy as np

    gold = os.path.join(ROOT, "tests", "golden", "rel_dubins_batch_samples.txt")
    if not os.path.exists(gold):
        return None
    spread, rows = {}, []
    with open(gold) as f:
        for line in f:
            w = line.split()
            if line.startswith("# instance") and w[2].isdigit():
                spread[int(w[2])] = [float(x) for x in w[w.index("storage_spread") + 1:]]
            elif w and w[0] == "s":
                rows.append([float(x) for x in w[1:]])
    data = np.array(rows, dtype=np.float64)
    per = {}
    for k in sorted(spread):
        sel = data[data[:, 0] == k]
        got = outs[k].double().cpu().numpy().ravel()[sel[:, 1].astype(np.int64)]
        err = float(np.abs(got - sel[:, 2]).max())
        per[k] = {"band_max_abs": err, "oracle_fp32_storage_spread_max": max(spread[k]),
                  "within_1e-4": err <= 1e-4,
                  "within_spread_bar": err <= max(1e-4, SPREAD_BAR_FACTOR * max(spread[k]))}
    return {"sampled_at": "%d stored front-band nodes of all %d instances (t=2.8)"
                          % (len(data), len(spread)),
            "band_max_abs": max(v["band_max_abs"] for v in per.values()),
            "instances_within_1e-4": sum(v["within_1e-4"] for v in per.values()),
            "instances_within_spread_bar": sum(v["within_spread_bar"] for v in per.values()),
            "per_instance": per}


def bench_served(args):
    """Poisson stream of double-integrator (101^2..401^2), relative-Dubins
    (51^3..121^3) and 4-D Dubins (41^4..61^4) requests, WENO5+LF+RK3, FP32,
    horizons U[0.5,3]: served with continuous batching at several arrival
    rates (relative to the saturated completion rate) against the same
    requests one at a time through hj_solve.  By default both sides return
    FP64 results with the tube minimum retaken in FP64 near the zero level
    set (served: hj_tube_finish per finished request; plain: hj_solve_mixed).
    """
    import numpy as np

    from paper_2507_11542_amd import inputs
    from paper_2507_11542_amd.serve import GpuBackend, Server, run_plain

    n = args.serve_requests
    base = inputs.serving_stream(count=n, rate=1.0, seed=0)
    v0_dtype = np.float64 if args.fp64_finish else np.float32
    v0_cache = ({} if args.device_v0 else
                {k: r.problem.v0().astype(v0_dtype) for k, r in enumerate(base)})

    def at_rate(rate):
        return [inputs.Request(r.arrival / rate, r.problem) for r in base]

    def served(rate):
        print("[bench] served at %.3g req/s" % rate, file=sys.stderr, flush=True)
        be = GpuBackend(prec="fp32", v0_cache=v0_cache, device_v0=args.device_v0,
                        fp64_finish=args.fp64_finish)
        try:
            rep, _ = Server(be, hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                            macro_steps=args.macro_steps,
                            macro_updates=args.macro_updates).run(at_rate(rate))
        finally:
            be.close()
        return rep.as_dict()

    def plain(rate):
        print("[bench] plain at %.3g req/s" % rate, file=sys.stderr, flush=True)
        rep, _ = run_plain(at_rate(rate), prec="fp32", v0_cache=v0_cache,
                           device_v0=args.device_v0, fp64_finish=args.fp64_finish)
        return rep.as_dict()

    def accuracy():
        """The smallest and the largest request of each family served again
        (all at once; a result does not depend on the mix) against the FP64
        oracle's stored values, beside the storage spread: how far the FP64
        method itself moves with single-precision storage."""
        gold = os.path.join(ROOT, "tests", "golden", "serving_stream_samples.txt")
        if not os.path.exists(gold) or n != 256:
            return None
        rows = np.loadtxt(gold)
        spread, sampled_spread = {}, {}
        with open(gold) as f:
            for line in f:
                w = line.split()
                if line.startswith("# request"):
                    for key, into in (("storage_spread", spread), ("sampled_spread", sampled_spread)):
                        vals = []
                        for x in (w[w.index(key) + 1:] if key in w else []):
                            try:
                                vals.append(float(x))
                            except ValueError:
                                break
                        into[int(w[2])] = max(vals) if vals else None
        ids = sorted({int(k) for k in rows[:, 0]})
        reqs = [inputs.Request(0.0, base[k].problem) for k in ids]
        be = GpuBackend(prec="fp32", v0_cache={i: v0_cache[k] for i, k in enumerate(ids)}
                        if v0_cache else None, device_v0=args.device_v0,
                        fp64_finish=args.fp64_finish)
        try:
            _, jobs = Server(be, hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                             macro_steps=args.macro_steps,
                             macro_updates=args.macro_updates).run(reqs, keep_results=True)
        finally:
            be.close()
        out = []
        for k, j in zip(ids, jobs):
            sel = rows[rows[:, 0] == k]
            err = np.abs(j.result.ravel()[sel[:, 1].astype(np.int64)] - sel[:, 3])
            band = sel[:, 2] == 1
            out.append({
                "request": k, "dynamics": j.problem.dynamics, "grid": list(j.problem.n),
                "horizon": j.problem.tf,
                "band_max_abs": float(err[band].max()) if band.any() else None,
                "sampled_max_abs": float(err.max()),
                "oracle_storage_spread": spread.get(k),
                "oracle_sampled_spread": sampled_spread.get(k)})
        return out

    sat = served(1e9)  # everything arrives at once: saturated throughput
    lam_sat = sat["completed"] / sat["makespan_s"]
    runs = {"saturated": sat}
    plains = {"saturated": plain(1e9)}
    for f in args.serve_rates:
        runs["%.2fx" % f] = dict(served(f * lam_sat), rate_req_per_s=f * lam_sat)
        plains["%.2fx" % f] = dict(plain(f * lam_sat), rate_req_per_s=f * lam_sat)
    return {"workload": "%d requests, thirds DI 101^2..401^2 / rel-Dubins 51^3..121^3 / "
                        "4-D Dubins 41^4..61^4, WENO5+LF+RK3, FP32, Poisson (seed 0)" % n,
            "macro_steps": args.macro_steps, "macro_updates": args.macro_updates,
            "v0": ("built on the GPU from each request's shape recipe (hj_init_shapes)"
                   if args.device_v0 else "uploaded from the host per request"),
            "results": ("FP64: FP32 solve, tube minimum retaken in FP64 on |V| <= 3 max dx"
                        if args.fp64_finish else "FP32"),
            "saturated_rate_req_per_s": lam_sat,
            "by_rate": {k: {"served_updates_per_s": runs[k]["updates_per_s"],
                            "plain_updates_per_s": plains[k]["updates_per_s"],
                            "served_vs_plain": runs[k]["updates_per_s"]
                            / plains[k]["updates_per_s"],
                            "served_p50_s": runs[k]["p50_s"], "served_p99_s": runs[k]["p99_s"],
                            "plain_p50_s": plains[k]["p50_s"], "plain_p99_s": plains[k]["p99_s"]}
                        for k in runs},
            "served": runs, "plain": plains,
            "served_vs_oracle_fp64": accuracy(),
            "served_vs_plain_updates_per_s":
                sat["updates_per_s"] / plains["saturated"]["updates_per_s"]}


def profile_batch():
    """One warm-up and one timed flat graph-replayed solve of the 64-instance
    relative-Dubins batch (FP32), HIP events around the timed one: the run a
    kernel trace of the batch rounds is taken on."""
    import torch

    from paper_2507_11542_amd import hj, inputs

    probs = inputs.rel_dubins_batch()
    st = torch.cuda.current_stream()
    grids = [hj.Grid.from_problem(p, "fp32") for p in probs]
    v0s = [torch.from_numpy(p.v0()).to("cuda", torch.float32) for p in probs]
    outs = [torch.empty_like(v) for v in v0s]
    b = hj.Batch(256, 0, True)
    args = (grids, v0s, outs, [p.t0 for p in probs], [p.tf for p in probs],
            [p.mode for p in probs], st)
    b.solve(*args)
    b.wait(len(probs), st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    b.solve(*args)
    e1.record(st)
    b.wait(len(probs), st)
    torch.cuda.synchronize()
    steps = [g.schedule(p.t0, p.tf, st)[2] for g, p in zip(grids, probs)]
    b.close()
    for g in grids:
        g.close()
    return {"timed_batch_ms": e0.elapsed_time(e1), "rounds": 3 * max(steps)}


def stage_sweep():
    """Per-launch stage time against grid size: n^3 grids, n = 32..160, of the
    WENO5 relative-Dubins and the ENO2 rockets stage kernels in both
    precisions, each from the differential of two solves (40 and 20 steps);
    and a least-squares line over the grids of 300k nodes or more."""
    import numpy as np
    import torch

    from paper_2507_11542_amd import hj, inputs

    st = torch.cuda.current_stream()

    def per_launch(p, prec, k1=40, k2=20, reps=3):
        dtp = torch.float64 if prec == "fp64" else torch.float32
        v0 = torch.from_numpy(p.v0()).to("cuda", dtp)
        out = torch.empty_like(v0)
        g = hj.Grid.from_problem(p, prec)
        _, dt, _ = g.schedule(p.t0, p.tf, st)
        res = {}
        for k in (k1, k2):
            tf = p.t0 + (k - 0.5) * dt
            g.solve(v0, out, p.t0, tf, p.mode, st)
            best = float("inf")
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                g.solve(v0, out, p.t0, tf, p.mode, st)
                e1.record(st)
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1))
            res[k] = (best, g.schedule(p.t0, tf, st)[2])
        g.close()
        (ta, ka), (tb, kb) = res[k1], res[k2]
        return (ta - tb) * 1e3 / (3 * (ka - kb))

    rows = []
    for n in (32, 48, 64, 80, 96, 112, 128, 144, 160):
        rd = inputs.rel_dubins_3d(n=n)
        rk = inputs.rockets().with_(n=(n, n, n))
        row = {"n": n, "nodes": n ** 3}
        for prec in ("fp64", "fp32"):
            row["weno5_" + prec + "_us"] = per_launch(rd, prec)
            row["eno2_" + prec + "_us"] = per_launch(rk, prec)
        print(json.dumps(row), file=sys.stderr, flush=True)
        rows.append(row)
    nodes = np.array([r["nodes"] for r in rows], dtype=float)
    fits = {}
    for key in ("weno5_fp64", "weno5_fp32", "eno2_fp64", "eno2_fp32"):
        y = np.array([r[key + "_us"] for r in rows])
        sel = nodes >= 300000
        b, a = np.polyfit(nodes[sel], y[sel], 1)
        fits[key] = {"us_per_launch": float(a), "ps_per_node": float(b * 1e6)}
    return {"rows": rows, "fits": fits}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rockets", action="store_true",
                    help="skip the rockets and 4-D Dubins legs")
    ap.add_argument("--rockets-reps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[0.5, 0.9, 1.2])
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--host-v0", dest="device_v0", action="store_false",
                    help="serving legs upload V0 from the host instead of building it on "
                         "the GPU from the request's shape recipe")
    ap.add_argument("--fp32-results", dest="fp64_finish", action="store_false",
                    help="serving legs return the FP32 solves as they are, without the "
                         "FP64 tube finish")
    ap.add_argument("--macro-steps", type=int, default=64,
                    help="most RK steps per instance in one serving macro-iteration")
    ap.add_argument("--macro-updates", type=float, default=1.5e8,
                    help="node-steps a family's serving macro-iteration aims at")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates "
                         "the HBM byte counters of a profiler run)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="only: one warm-up and one timed 64-instance batched solve "
                         "(the run a trace of the batch rounds is taken on)")
    ap.add_argument("--stage-sweep", action="store_true",
                    help="only: per-launch stage time against grid size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2507_11542_amd import hj, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.profile_batch:
        print(json.dumps(profile_batch()))
        return 0
    if args.stage_sweep:
        print(json.dumps(stage_sweep()))
        return 0
    p = inputs.rel_dubins_3d()
    dtype = torch.float64 if args.prec == "fp64" else torch.float32
    elem = 8 if args.prec == "fp64" else 4
    stream = torch.cuda.current_stream()
    v0 = torch.from_numpy(p.v0()).to("cuda", dtype=dtype)
    out = torch.empty_like(v0)
    g = hj.Grid.from_problem(p, args.prec)
    alpha, dt, nsteps = g.schedule(p.t0, p.tf, stream)
    updates_per_solve = p.points * nsteps

    for _ in range(args.warmup):
        g.solve(v0, out, p.t0, p.tf, p.mode, stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        g.solve(v0, out, p.t0, p.tf, p.mode, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms_per_step = 1e3 * elapsed / args.steps
    value = updates_per_solve * args.steps / elapsed

    # dominant kernel: the fused stage kernel, 3 launches per RK3 step, timed
    # on the stream it is launched on by the differential of two solves
    launch_s, step_launch_s = stage_launch_time(g, v0, torch.empty_like(out), p, stream)
    flops = weno5_flops_per_node_stage(p.ndim) * p.points
    achieved = flops / launch_s / 1e12
    peak = FP64_PEAK_TFLOPS if args.prec == "fp64" else FP32_PEAK_TFLOPS
    hbm_gbs = bytes_per_node_stage(elem, p.mode == "tube") * p.points / launch_s / 1e9

    # error of the timed result against the FP64 oracle at stored samples
    err = None
    gold = os.path.join(ROOT, "tests", "golden", "rel_dubins_3d_101_tube_samples.txt")
    if os.path.exists(gold):
        data = np.loadtxt(gold)
        idx = data[:, 0].astype(np.int64)
        got = out.double().cpu().numpy().ravel()[idx]
        err = float(np.abs(got - data[:, 1]).max())
    g.close()

    if args.copy_mib:
        src = torch.empty(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32",
        "data": "synthetic (analytic dynamics and signed-distance V0)",
        "config": {"workload": "rel_dubins_3d 101^3 WENO5+LF+RK3 tube t=2.8, plain solve",
                   "grid": list(p.n), "rk_steps": nsteps, "dt": dt, "alpha": alpha,
                   "path": "plain (hj_solve, one solve at a time)"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(args.prec),
                     "traffic_unit": "bytes per launch",
                     "kernel": "stage_kernel<%s,3,WENO5,REL_DUBINS>" % args.prec,
                     "launch_us": launch_s * 1e6,
                     "launch_us_whole_solve": step_launch_s * 1e6,
                     "launches_per_solve": 3 * nsteps,
                     "algorithmic_hbm_GBs": hbm_gbs,
                     "measured_hbm_GBs": (measured_traffic(args.prec) / launch_s / 1e9
                                          if measured_traffic(args.prec) else None),
                     "hbm_peak_GBs": 8000.0,
                     "flops_per_node_stage": weno5_flops_per_node_stage(p.ndim),
                     "flops_per_node_stage_executed":
                         weno5_flops_per_node_stage(p.ndim, executed=True),
                     "flop_count": "the method's: one WENO window per interface per axis"},
        "error_vs_oracle_fp64": err,
    }
    if not args.no_rockets:
        print("[bench] rockets leg", file=sys.stderr, flush=True)
        rec["rockets"] = bench_rockets(args)
    if not args.no_rockets:
        print("[bench] 4-D leg", file=sys.stderr, flush=True)
        rec["dubins4d"] = bench_dubins4d(args)
    if not args.no_batch:
        print("[bench] batched leg", file=sys.stderr, flush=True)
        rec["batched"] = bench_batched(args)
    if not args.no_serve:
        print("[bench] served leg", file=sys.stderr, flush=True)
        rec["served"] = bench_served(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
