"""Solves/s to a 1e-10 relative residual on one MI355X.

Workload: [0,1]^2 minus 3 seeded disks (radius U[0.05, 0.15]), 1024 x 1024
cells, a=1, b=0.5, c=2, Dirichlet outside, Neumann on the holes, 6 seeded
sine modes (seed 0).  A step is one whole solve from u = 0 (V-cycles of
Algorithm 3 with nu = (6, 6) until ||b - A u||_inf <= 1e-10 ||b||_inf) with
the inputs already resident on the device.  `value` is the mixed-precision
rate (FP32 V-cycles inside FP64 defect correction); the plain FP64 rate is
reported beside it, the same solve with the FMG cycle of Algorithm 4 and with
nu = (3, 3) as variants, and the 4096^2 star workload (Robin hole, cross
term) as a second line with its own roofline figure.

Prints one JSON line.  --gpus above 1 is refused: the solver runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# smoothing steps (nu1, nu2) of every solve here; the paper's (3, 3) is reported
# as a variant
NU = (6, 6)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2601_02975_amd", "csrc", "kernels.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic_for(name, precision):
    """HBM bytes per launch of the finest-level smoother launch A of a workload
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_smooth_a_%s.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(precision)


def timed_solves(torch, S, f, g, steps, warmup, tol, record=False):
    u = torch.zeros_like(f)
    iters = []
    for _ in range(warmup):
        u.zero_()
        it, rel, code = S.solve(f, g, u, tol)
        if code != 0:
            raise RuntimeError("solve did not converge (code %d, rel %.2e after %d)" % (code, rel, it))
    torch.cuda.synchronize()
    if record:
        S.kernel_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        it, rel, code = S.solve(f, g, u, tol)
        iters.append(it)
        if code != 0:
            raise RuntimeError("solve did not converge (code %d, rel %.2e after %d)" % (code, rel, it))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, avg_ms = S.kernel_timing(False) if record else (0, 0.0)
    return dt, iters, rel, u, launches, avg_ms


def cpu_baseline(P, gpu_iters, sample_cycles, cycle):
    """The oracle (plain NumPy/SciPy, FP64) on the same workload: time a
    bounded number of its cycles (FMG on the residual equation, or V-cycles)
    and scale to one solve with the iteration count the solve needs (the GPU
    FP64 iteration count: the iterates agree)."""
    from threadpoolctl import threadpool_limits

    from oracle.multigrid import Hierarchy
    from oracle.rhs import rhs
    with threadpool_limits(1):
        t0 = time.perf_counter()
        H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, nu=NU,
                      progress=lambda msg: print("oracle setup: " + msg, file=sys.stderr, flush=True))
        t_setup = time.perf_counter() - t0
        b, _, _ = rhs(H.levels[0], P.solution)
        A = H.levels[0].A
        u = b * 0.0
        t0 = time.perf_counter()
        for _ in range(sample_cycles):
            u = u + H.fmg(0, b - A @ u) if cycle == "FMG" else H.vcycle(0, u, b)
            r = b - A @ u
            _ = float(abs(r).max())
        t_cycle = (time.perf_counter() - t0) / sample_cycles
    per_solve = gpu_iters * t_cycle
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "%d %s-cycles, nu = (6, 6), (with residual norms) of the FP64 oracle on the same 1024^2 workload, "
                      "%.3f s each, scaled by the %d cycles a solve to 1e-10 takes; oracle setup %.1f s "
                      "not included" % (sample_cycles, cycle, t_cycle, gpu_iters, t_setup)}


def serving_leg(torch, mg, W, geoms, n_rhs, qps, slots, tol, label):
    """Serving with resident hierarchies: every geometry is set up in the
    server by one warm-up request; then n_rhs right-hand sides per geometry
    arrive as a Poisson process at qps and are solved in mixed precision in
    `slots` slots.  Reported beside the same solves run one after another on
    resident hierarchies (mixed and FP64)."""
    import numpy as np
    n_geom = len(geoms)
    reqs = [(k, W.with_solution(P, 1000 * k + r, 6)) for k, P in enumerate(geoms) for r in range(n_rhs)]
    rng = np.random.default_rng(12345)
    order = rng.permutation(len(reqs))
    gaps = rng.exponential(1.0 / qps, size=len(reqs))
    seq = {p: [mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=p, max_iters=1000, nu=NU)
               for P in geoms] for p in (mg.FP64, mg.MIXED)}
    inputs = []
    for k, P in reqs:
        f, g = seq[mg.FP64][k].project(P.solution)
        inputs.append((torch.tensor(f, device="cuda"), torch.tensor(g, device="cuda")))
    seq_rate = {}
    for p, name in ((mg.FP64, "fp64"), (mg.MIXED, "mixed")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (k, P), (f, g) in zip(reqs, inputs):
            u = torch.zeros_like(f)
            seq[p][k].solve(f, g, u, tol)
        torch.cuda.synchronize()
        seq_rate[name] = len(reqs) / (time.perf_counter() - t0)
        for S in seq[p]:
            S.close()
    srv = mg.Server(max_active=slots, hbm_budget=64 << 30)
    pids = [srv.add_problem(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
            for P in geoms]
    warm = []
    for k in range(n_geom):                        # setup of every hierarchy (not timed)
        f, g = inputs[k * n_rhs]
        warm.append(srv.submit(pids[k], f, g, torch.zeros_like(f), tol))
    setup_lat = [srv.wait(t)["latency_s"] for t in warm]
    outs = [torch.zeros_like(inputs[i][0]) for i in range(len(reqs))]
    torch.cuda.synchronize()
    tickets = []
    t_start = time.perf_counter()
    for i, gap in zip(order, gaps):
        time.sleep(float(gap))
        f, g = inputs[i]
        tickets.append(srv.submit(pids[reqs[i][0]], f, g, outs[i], tol))
    res = [srv.wait(t) for t in tickets]
    t_all = time.perf_counter() - t_start
    srv.close()
    lat = sorted(r["latency_s"] for r in res)
    pct = lambda q: lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]
    return {"workload": "%s, resident after one warm-up request each; %d right-hand sides per geometry arriving "
                        "as a Poisson process at %g/s; %d slots; V-cycles (nu = (6, 6)) in mixed precision to %g" % (
                            label, n_rhs, qps, slots, tol),
            "requests": len(reqs), "failed": sum(r["status"] != 0 for r in res),
            "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99), "solves_per_s": len(reqs) / t_all,
            "sequential_mixed_solves_per_s": seq_rate["mixed"], "sequential_fp64_solves_per_s": seq_rate["fp64"],
            "setup_latency_s_max": max(setup_lat)}


def roofline(S, n_cells, avg_ms, launches, traffic, kernel="k_smooth_a<float> (finest level: SFV Jacobi tiles + "
                                                                 "PLG segment solves)"):
    """Finest-level FP32 launch A: u, b read and u written on the SFV cells,
    the PLG segment inverses read once, b read and u/y written on the PLG rows
    (words of 4 bytes), plus one byte of class mask per cell."""
    alg_bytes = 4 * S.info["sweep_words"][0] + n_cells
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    return {"bound": "hbm", "kernel": kernel,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "launches_timed": launches, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": alg_bytes}


def star_leg(torch, mg, W, steps, warmup, tol):
    """The 4096^2 star workload (Robin star hole, a=2, b=-1, c=1): V-cycles
    with NU in mixed precision and FP64."""
    P = W.star_config(0, 4096)
    t0 = time.perf_counter()
    S32 = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
    t_setup = time.perf_counter() - t0
    S64 = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.FP64, max_iters=1000, nu=NU)
    fh, gh = S32.project(P.solution)
    f = torch.tensor(fh, device="cuda")
    g = torch.tensor(gh, device="cuda")
    print("star 4096: setup %.1f s, levels %s, PLG cells %s" % (t_setup, S32.info["nx"], S32.info["n_plg"]),
          file=sys.stderr, flush=True)
    dt64, it64, rel64, u64, _, _ = timed_solves(torch, S64, f, g, steps, warmup, tol)
    print("star 4096 fp64: %.4f s/solve, %d iterations" % (dt64 / steps, it64[-1]), file=sys.stderr, flush=True)
    dt32, it32, rel32, u32, nl, avg_ms = timed_solves(torch, S32, f, g, steps, warmup, tol, True)
    print("star 4096 mixed: %.4f s/solve, %d iterations" % (dt32 / steps, it32[-1]), file=sys.stderr, flush=True)
    diff = float((u32 - u64).abs().max() / u64.abs().max())
    n_cells = P.grid.nx * P.grid.ny
    out = {"workload": "star_4096x4096_seed0 (8-point star with arcs, Robin (1, 0.5) on the star, Dirichlet box; "
                       "a=2, b=-1, c=1; 8 sine modes)", "levels": S32.info["nx"], "plg_cells": S32.info["n_plg"],
           "solver": "V-cycles (Algorithm 3), nu = %s" % (NU,),
           "mixed": {"value": steps / dt32, "unit": "solves/s", "iterations": it32[-1], "rel_residual": rel32,
                     "max_rel_diff_vs_fp64": diff},
           "fp64": {"value": steps / dt64, "unit": "solves/s", "iterations": it64[-1], "rel_residual": rel64},
           "speedup_mixed_over_fp64": dt64 / dt32,
           "roofline": roofline(S32, n_cells, avg_ms, nl, load_traffic_for("star4096", "fp32"),
                                "launch A on the finest level: k_smooth_tiles<float> (SFV Jacobi tiles) then "
                                "k_smooth_a<float> (PLG segment solves)")}
    S32.close()
    S64.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cpu-cycles", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-star", action="store_true")
    ap.add_argument("--only-star", action="store_true", help="run only the 4096^2 star leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also move 256 MiB with the runtime's copy kernel and with an elementwise kernel "
                         "(references for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2601_02975_amd as mg
    import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src_t = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        # the same bytes through an ordinary elementwise kernel (plain loads
        # and stores, unlike the runtime's copy kernel)
        for _ in range(3):
            torch.mul(src_t, 2.0, out=dst_t)
        torch.cuda.synchronize()
        print("calibration copy: 3 + 3 x %d bytes read and written" % (src_t.numel() * 8), file=sys.stderr)
        del src_t, dst_t
    if args.only_star:
        print(json.dumps({"star4096": star_leg(torch, mg, W, args.steps, args.warmup, args.tol)}))
        return

    P = W.three_disks_config(0, args.n)
    t0 = time.perf_counter()
    S32 = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
    t_setup = time.perf_counter() - t0
    S64 = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.FP64, max_iters=1000, nu=NU)
    fh, gh = S64.project(P.solution)
    f = torch.tensor(fh, device="cuda")
    g = torch.tensor(gh, device="cuda")
    print("setup %.2f s, levels %s, PLG cells %s, separators %s" % (
        t_setup, S64.info["nx"], S64.info["n_plg"], S64.info["n_sep"]), file=sys.stderr, flush=True)

    dt64, it64, rel64, u64, _, _ = timed_solves(torch, S64, f, g, args.steps, args.warmup, args.tol)
    print("fp64: %.4f s/solve, %d iterations" % (dt64 / args.steps, it64[-1]), file=sys.stderr, flush=True)
    dt32, it32, rel32, u32, nl, avg_ms = timed_solves(torch, S32, f, g, args.steps, args.warmup, args.tol, True)
    print("mixed: %.4f s/solve, %d iterations" % (dt32 / args.steps, it32[-1]), file=sys.stderr, flush=True)
    diff = float((u32 - u64).abs().max() / u64.abs().max())
    n_cells = P.grid.nx * P.grid.ny
    out = {
        "metric": "solves/s to 1e-10 rel. residual (mixed vs FP64 GPU), HBM GB/s; p50/p99 latency",
        "value": args.steps / dt32,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycles in f64 defect correction",
        "data": "synthetic",
        "config": {"workload": "three_disks_1024x1024_seed0 (a=1, b=0.5, c=2; Dirichlet box, Neumann holes; "
                               "6 sine modes)", "tol": args.tol, "cells": n_cells,
                   "solver": "V-cycles (Algorithm 3), nu = %s, omega = 1/2" % (NU,),
                   "levels": S64.info["nx"], "plg_cells": S64.info["n_plg"]},
        "fp64": {"value": args.steps / dt64, "unit": "solves/s", "iterations": it64[-1], "rel_residual": rel64},
        "mixed": {"iterations": it32[-1], "rel_residual": rel32, "max_rel_diff_vs_fp64": diff},
        "speedup_mixed_over_fp64": dt64 / dt32,
        "roofline": roofline(S32, n_cells, avg_ms, nl, load_traffic_for("three_disks1024", "fp32")),
    }
    S32.close()
    S64.close()
    if not args.no_variants:
        # the same solve with the paper's FMG cycle and with nu = (3, 3)
        var = {}
        for cyc, nu, name in ((mg.CYCLE_FMG, NU, "fmg_nu%d%d" % NU), (mg.CYCLE_V, (3, 3), "v_nu33"),
                              (mg.CYCLE_FMG, (3, 3), "fmg_nu33")):
            S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000,
                          nu=nu, cycle=cyc)
            dt, it, rel, _, _, _ = timed_solves(torch, S, f, g, args.steps, args.warmup, args.tol)
            S.close()
            var[name] = {"value": args.steps / dt, "unit": "solves/s", "iterations": it[-1], "rel_residual": rel,
                         "precision": "mixed"}
            print("variant %s: %.4f s/solve, %d iterations" % (name, dt / args.steps, it[-1]), file=sys.stderr,
                  flush=True)
        out["variants"] = var
    if not args.no_star:
        out["star4096"] = star_leg(torch, mg, W, args.steps, args.warmup, args.tol)
    if not args.no_serving:
        out["serving"] = serving_leg(torch, mg, W, [W.three_disks_config(s, 512) for s in range(1, 5)], 8, 400.0, 4,
                                     args.tol, "4 three-disk geometries (seeds 1-4) at 512^2")
        print("serving: p50 %.3f s, p99 %.3f s, %.1f solves/s" % (
            out["serving"]["p50_latency_s"], out["serving"]["p99_latency_s"], out["serving"]["solves_per_s"]),
            file=sys.stderr, flush=True)
        # the request distribution of the serving trace: grids of 128^2 to
        # 2048^2, 1-5 holes with mixed boundary conditions, seeded (a, b, c)
        mix = [W.serving_request(0, k) for k in range(8)]
        out["serving_mix"] = serving_leg(torch, mg, W, mix, 4, 200.0, 4, args.tol,
                                         "the first 8 requests of serving trace 0 as geometries (grids %s; 1-5 "
                                         "holes, mixed boundary conditions, seeded a, b, c)"
                                         % "/".join(str(P.grid.nx) for P in mix))
        print("serving mix: p50 %.3f s, p99 %.3f s, %.1f solves/s" % (
            out["serving_mix"]["p50_latency_s"], out["serving_mix"]["p99_latency_s"],
            out["serving_mix"]["solves_per_s"]), file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(P, it64[-1], args.cpu_cycles, "V")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
