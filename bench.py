"""Solves/s to a 1e-10 relative residual on one MI355X.

Headline workload: [0,1]^2 minus a seeded 8-point star joined to circular
arcs, 4096 x 4096 cells, a=2, b=-1, c=1, Robin (1, 0.5) on the star,
Dirichlet outside, 8 seeded sine modes (seed 0).  A step is one whole solve
from u = 0 (V-cycles of Algorithm 3 with nu = (6, 4) until
||b - A u||_inf <= 1e-10 ||b||_inf) with the inputs already resident on the
device.  `value` is the mixed-precision rate (FP32 V-cycles inside FP64
defect correction); the plain FP64 rate is reported beside it, timed the same
way (replays of the captured outer iteration).  Further lines: the 1024^2
three-disk workload, the FMG cycle and nu = (3, 3) as variants, two serving
traces, and the FP64 oracle on the host cores.

Prints one JSON line.  --gpus above 1 is refused: the solver runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# smoothing steps (nu1, nu2) of every solve here (--nu); the paper's (3, 3)
# is reported as a variant (deep V(3,3)-cycles are not h-independent with the
# piecewise-constant interpolation of eq. (5.9)); (6, 4) is the fastest of
# (5,5) .. (8,8), (6,4), (4,6), (8,4), (8,6) on the 4096^2 star
NU = (6, 4)
# Gauss points per direction for the cell averages <f> over full cells
# (exact to degree 2 GP - 1 per variable; the cut cells use the library's
# own rules): 8 up to 1024^2, 4 above, where the quadrature error of a
# degree-7 rule on cells of h <= 1/2048 is far below the solver tolerance
def gauss_points(n):
    return 8 if n <= 1024 else 4


# Gauss points per direction for the serving requests' inputs: the serving
# figures measure the solver, and a 2 x 2 rule (exact to degree 3) keeps the
# host-side projection of many 2048^2 inputs short
SERVING_GAUSS = 2


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2601_02975_amd", "csrc", "kernels.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic_for(name, kernel):
    """HBM bytes per launch of `kernel` on a workload's finest level from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def timed_solves(torch, S, f, g, steps, warmup, tol):
    """`steps` solves from u = 0 after `warmup` untimed ones; every solve
    replays the captured outer iteration."""
    u = torch.zeros_like(f)
    for _ in range(warmup):
        u.zero_()
        it, rel, code = S.solve(f, g, u, tol)
        if code != 0:
            raise RuntimeError("solve did not converge (code %d, rel %.2e after %d)" % (code, rel, it))
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        it, rel, code = S.solve(f, g, u, tol)
        iters.append(it)
        if code != 0:
            raise RuntimeError("solve did not converge (code %d, rel %.2e after %d)" % (code, rel, it))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, iters, rel, u


def kernel_time(torch, S, f, g, solves, tol):
    """Average duration of the finest level's SFV tile kernel over `solves`
    solves launched eagerly (no graph replay) with a pair of HIP events that
    take the start and end of each of its launches (hipExtLaunchKernel on
    the stream it runs on), and the time per
    solve in that mode."""
    u = torch.zeros_like(f)
    S.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(solves):
        u.zero_()
        S.solve(f, g, u, tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, avg_ms = S.kernel_timing(False)
    return launches, avg_ms, dt / max(solves, 1)


def roofline(S, avg_ms, launches, traffic):
    """The dominant kernel of the mixed solve on the finest level, over its
    average duration: with two-sweep tiles k_smooth_pair<float> (the first
    sweep of a pair on every SFV cell, u and b read and u written, 3 w per
    cell, w = 4 bytes, plus the second sweep's u written on the cells of the
    two-sweep tiles, w per cell), else k_smooth_tiles<float> (3 w per SFV
    cell)."""
    n_sfv, n_pair = S.info["n_sfv"][0], S.info["n_pair_sfv"][0]
    alg_bytes = 12 * n_sfv + 4 * n_pair
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    kernel = ("k_smooth_pair<float> (finest level: two omega-Jacobi sweeps on the SFV cells of the two-sweep "
              "tiles, the first sweep on the other SFV cells)" if n_pair else
              "k_smooth_tiles<float> (finest level: omega-Jacobi on the SFV cells)")
    return {"bound": "hbm", "kernel": kernel,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "launches_timed": launches, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": alg_bytes,
            "sfv_cells": n_sfv, "two_sweep_sfv_cells": n_pair}


def fp64_floor(torch, S, f, g, tols=(1e-11, 1e-12, 1e-13, 1e-14)):
    """Where the GPU's FP64 iteration stagnates: the smallest of `tols` it
    reaches (V-cycles from u = 0; an iteration whose residual grows three
    times in a row stops as diverged, which here means stagnation)."""
    import paper_2601_02975_amd as mg
    out = {"reached": None, "not_reached": None}
    for tol in tols:
        u = torch.zeros_like(f)
        it, rel, code = S.solve(f, g, u, tol)
        if code == 0:
            out["reached"] = {"tol": tol, "cycles": it, "rel_residual": rel}
        else:
            out["not_reached"] = {"tol": tol, "status": mg.STATUS.get(code, code), "cycles": it,
                                  "last_rel_residual": rel}
            break
    return out


# --------------------------------------------------------------------------
# the oracle on the host cores
def _oracle_cycles(H, b, seconds, out):
    import numpy as np
    A = H.levels[0].A
    u = np.zeros_like(b)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        u = H.vcycle(0, u, b)
        _ = float(np.abs(b - A @ u).max())
        n += 1
    out.put((n, time.perf_counter() - t0))


_ORACLE = {}


def _oracle_worker(seconds, q):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        _oracle_cycles(_ORACLE["H"], _ORACLE["b"], seconds, q)


def cpu_baseline(n_sample, gpu_iters, n_cells_headline, seconds):
    """The FP64 oracle (plain NumPy/SciPy, as it stands): V-cycles with NU on
    the three-disk workload at n_sample^2 (the same 25-point operator as the
    headline's, b != 0; the oracle sets it up in about a minute, the star
    at that size takes several) for `seconds` on one core, then one process
    per core (at most 16) for the same time; scaled to the headline's cells
    (the V-cycle is linear in the cells) and the GPU's iteration count."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.multigrid import Hierarchy
    from oracle.rhs import rhs
    P = W.three_disks_config(0, n_sample)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        H = Hierarchy(P.grid, P.curves, P.a, P.b, P.c, P.eps, nu=NU)
        t_setup = time.perf_counter() - t0
        b, _, _ = rhs(H.levels[0], P.solution)
    _ORACLE["H"], _ORACLE["b"] = H, b
    ctx = mp.get_context("fork")
    q = ctx.Queue()
    _oracle_worker(seconds, q)
    n1, t1 = q.get()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = min(cores, 16)            # the host share of one GPU
    procs = [ctx.Process(target=_oracle_worker, args=(seconds, q)) for _ in range(cores)]
    for p in procs:
        p.start()
    res = [q.get() for _ in procs]
    for p in procs:
        p.join()
    cyc_all = sum(n for n, _ in res) / max(t for _, t in res)
    scale = n_cells_headline / float(P.grid.nx * P.grid.ny)
    t_cycle_1 = t1 / n1
    per_solve_1 = gpu_iters * t_cycle_1 * scale
    per_solve_all = gpu_iters * scale / cyc_all
    try:
        lscpu = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        model = next((l.split(":", 1)[1].strip() for l in lscpu.splitlines() if l.startswith("Model name")), "")
    except Exception:
        model = platform.processor()
    return {"value": 1.0 / per_solve_all, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "one_core": {"value": 1.0 / per_solve_1, "unit": "solves/s", "cores": 1},
            "host": {"cpu": model, "cores_available": cores, "nproc": os.cpu_count()},
            "sample": "FP64 oracle V-cycles (nu = %s, residual norm each) on the three-disk workload at %d^2 "
                      "(oracle setup %.1f s, not timed): %d cycles in %.1f s on 1 core (%.3f s each); "
                      "%d processes, one per core, %.1f cycles/s together; scaled by the cells (x%.0f) and the "
                      "%d cycles of the GPU's solve" % (NU, n_sample, t_setup, n1, t1, t_cycle_1, cores,
                                                         cyc_all, scale, gpu_iters)}


# --------------------------------------------------------------------------
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
    seq = {}
    for p in (mg.FP64, mg.MIXED):
        seq[p] = []
        for k, P in enumerate(geoms):
            seq[p].append(mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=p, max_iters=1000, nu=NU))
            print("%s: setup %d/%d (%d^2, precision %d)" % (label[:24], k + 1, n_geom, P.grid.nx, p),
                  file=sys.stderr, flush=True)
    inputs = []
    for k, P in reqs:
        inputs.append(seq[mg.FP64][k].project(P.solution, SERVING_GAUSS))
        print("%s: input %d/%d projected (%d^2)" % (label[:24], len(inputs), len(reqs), P.grid.nx),
              file=sys.stderr, flush=True)
    seq_rate = {}
    for p, name in ((mg.FP64, "fp64"), (mg.MIXED, "mixed")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (k, P), (f, g) in zip(reqs, inputs):
            u = torch.zeros_like(f)
            seq[p][k].solve(f, g, u, tol)
        torch.cuda.synchronize()
        seq_rate[name] = len(reqs) / (time.perf_counter() - t0)
        print("%s: sequential %s %.1f solves/s" % (label[:24], name, seq_rate[name]), file=sys.stderr, flush=True)
        for S in seq[p]:
            S.close()
    srv = mg.Server(max_active=slots, hbm_budget=64 << 30)
    pids = [srv.add_problem(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
            for P in geoms]
    warm = []
    for k in range(n_geom):                        # setup of every hierarchy (not timed)
        f, g = inputs[k * n_rhs]
        warm.append(srv.submit(pids[k], f, g, torch.zeros_like(f), tol))
    setup_lat = []
    for t in warm:
        setup_lat.append(srv.wait(t)["latency_s"])
        print("%s: server warm-up %d/%d done" % (label[:24], len(setup_lat), n_geom), file=sys.stderr, flush=True)
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
    st = srv.stats()
    srv.close()
    lat = sorted(r["latency_s"] for r in res)
    pct = lambda q: lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]
    return {"workload": "%s, resident after one warm-up request each; %d right-hand sides per geometry arriving "
                        "as a Poisson process at %g/s; %d slots; V-cycles (nu = %s) in mixed precision to %g" % (
                            label, n_rhs, qps, slots, NU, tol),
            "requests": len(reqs), "failed": sum(r["status"] != 0 for r in res),
            "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99), "solves_per_s": len(reqs) / t_all,
            "sequential_mixed_solves_per_s": seq_rate["mixed"], "sequential_fp64_solves_per_s": seq_rate["fp64"],
            "setup_latency_s_max": max(setup_lat),
            "server_sweep_gbs": st["sweep_gbs"]}


def _project_all(torch, mg, probs, threads=4):
    """Device inputs (f, g) of every problem, each projected with a handle of
    its own (set up in parallel host threads; the library releases the
    interpreter during setup)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(P):
        S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, max_iters=1000, nu=NU)
        fg = S.project(P.solution, SERVING_GAUSS)
        S.close()
        return fg
    out = []
    with ThreadPoolExecutor(threads) as pool:
        for k, fg in enumerate(pool.map(one, probs)):
            out.append(fg)
            print("projected %d/%d" % (k + 1, len(probs)), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return out


def _run_trace(torch, mg, probs, inputs, pids, srv, rate, seed, tol):
    """Submits request k (problem pids[k], inputs[k]) at Poisson arrival
    times of the given rate (rate = inf: all at once); returns the per-request
    results and the wall time from the first submission to the last result."""
    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(probs)) if math.isfinite(rate) else np.zeros(len(probs))
    outs = [torch.zeros_like(f) for f, _ in inputs]
    torch.cuda.synchronize()
    tickets = []
    t0 = time.perf_counter()
    for k, gap in enumerate(gaps):
        if gap > 0:
            time.sleep(float(gap))
        f, g = inputs[k]
        tickets.append(srv.submit(pids[k], f, g, outs[k], tol))
    res = []
    for t in tickets:
        res.append(srv.wait(t))
        if len(res) % 16 == 0:
            print("trace: %d/%d done" % (len(res), len(tickets)), file=sys.stderr, flush=True)
    return res, time.perf_counter() - t0


def _latency_summary(res, wall):
    lat = sorted(r["latency_s"] for r in res)
    pct = lambda q: lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]
    return {"requests": len(res), "failed": sum(r["status"] != 0 for r in res), "p50_latency_s": pct(0.5),
            "p99_latency_s": pct(0.99), "solves_per_s": len(res) / wall, "wall_s": wall}


def serving_fresh_trace(torch, mg, W, n_req, slots, tol):
    """Requests of the serving trace, each with a geometry of its own (grids
    128^2 to 2048^2, 1-5 holes, mixed boundary conditions, seeded a, b, c),
    so every request pays its setup inside its latency.  First all requests
    at once (saturation), then Poisson arrivals at 25/50/75/100% of that
    rate, each trace on a fresh server."""
    probs = [W.serving_request(0, k) for k in range(n_req)]
    inputs = _project_all(torch, mg, probs)
    out = {"workload": "%d requests of serving trace 0 (grids %s), a fresh geometry each; mixed precision, "
                       "V-cycles nu = %s, to %g; %d slots" % (
                           n_req, "/".join(sorted({str(P.grid.nx) for P in probs}, key=int)), NU, tol, slots)}
    rate_sat = None
    for frac in (None, 0.25, 0.5, 0.75, 1.0):
        srv = mg.Server(max_active=slots, hbm_budget=128 << 30)
        pids = [srv.add_problem(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000,
                                nu=NU) for P in probs]
        rate = float("inf") if frac is None else frac * rate_sat
        res, wall = _run_trace(torch, mg, probs, inputs, pids, srv, rate, 100 + int(100 * (frac or 0)), tol)
        srv.close()
        summ = _latency_summary(res, wall)
        if frac is None:
            rate_sat = summ["solves_per_s"]
            out["saturation"] = summ
        else:
            summ["offered_qps"] = rate
            out["qps_%d%%" % int(100 * frac)] = summ
        print("fresh trace %s: %s" % (frac, summ), file=sys.stderr, flush=True)
    return out


def serving_resident(torch, mg, W, n_geom, n_rhs, slots, tol, budget):
    """n_geom seeded 2048^2 geometries (stars and disks, mixed boundary
    conditions), each receiving n_rhs right-hand sides in a seeded random
    order at Poisson arrivals of 80% of the saturation rate; hierarchies stay
    resident within an HBM budget; against the same solves one after another
    in FP64 on resident hierarchies."""
    import numpy as np
    geoms = [W.serving_geometry(s, 2048) for s in range(n_geom)]
    probs = [W.with_solution(G, 1000 * k + r, 6) for k, G in enumerate(geoms) for r in range(n_rhs)]
    owner = [k for k in range(n_geom) for _ in range(n_rhs)]
    order = np.random.default_rng(77).permutation(len(probs))
    probs = [probs[i] for i in order]
    owner = [owner[i] for i in order]
    inputs = _project_all(torch, mg, probs)
    # sequential FP64 reference on resident hierarchies
    seq = [mg.Solver(G.grid, G.curves, G.a, G.b, G.c, eps=G.eps, precision=mg.FP64, max_iters=1000, nu=NU)
           for G in geoms]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (f, g) in zip(owner, inputs):
        u = torch.zeros_like(f)
        seq[k].solve(f, g, u, tol)
    torch.cuda.synchronize()
    seq_rate = len(probs) / (time.perf_counter() - t0)
    for S in seq:
        S.close()
    print("resident: sequential FP64 %.1f solves/s" % seq_rate, file=sys.stderr, flush=True)
    srv = mg.Server(max_active=slots, hbm_budget=budget)
    gp = [srv.add_problem(G.grid, G.curves, G.a, G.b, G.c, eps=G.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
          for G in geoms]
    pids = [gp[k] for k in owner]
    # warm-up: one request per geometry sets the hierarchies up (not timed)
    first = {}
    for i, k in enumerate(owner):
        first.setdefault(k, i)
    warm = [srv.submit(gp[k], inputs[i][0], inputs[i][1], torch.zeros_like(inputs[i][0]), tol)
            for k, i in sorted(first.items())]
    for t in warm:
        srv.wait(t)
    res, wall = _run_trace(torch, mg, probs, inputs, pids, srv, float("inf"), 5, tol)
    sat = len(res) / wall
    res, wall = _run_trace(torch, mg, probs, inputs, pids, srv, 0.8 * sat, 6, tol)
    st = srv.stats()
    srv.close()
    summ = _latency_summary(res, wall)
    summ.update({"workload": "%d seeded 2048^2 geometries (stars and disks, mixed boundary conditions), %d "
                             "right-hand sides each in a random order, Poisson arrivals at 80%% of the saturation "
                             "rate (%.1f solves/s); hierarchies resident within a %.0f GiB budget; mixed "
                             "precision, V-cycles nu = %s, to %g; %d slots" % (
                                 n_geom, n_rhs, sat, budget / 2 ** 30, NU, tol, slots),
                 "sequential_fp64_solves_per_s": seq_rate, "resident_bytes": st["resident_bytes"],
                 "evictions": st["evictions"], "server_sweep_gbs": st["sweep_gbs"]})
    print("resident: %s" % summ, file=sys.stderr, flush=True)
    return summ


def solve_leg(torch, mg, P, steps, warmup, tol, timing_solves, label):
    """Mixed and FP64 solves of one workload, both replaying graphs; the
    tile kernel's duration from a separate eager pass with HIP events."""
    n = P.grid.nx
    t0 = time.perf_counter()
    S32 = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
    t_setup = time.perf_counter() - t0
    S64 = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.FP64, max_iters=1000, nu=NU)
    f, g = S32.project(P.solution, gauss_points(n))
    print("%s: setup %.1f s, levels %s, PLG cells %s, separators %s" % (
        label, t_setup, S32.info["nx"], S32.info["n_plg"], S32.info["n_sep"]), file=sys.stderr, flush=True)
    dt64, it64, rel64, u64 = timed_solves(torch, S64, f, g, steps, warmup, tol)
    print("%s fp64: %.4f s/solve, %d iterations" % (label, dt64 / steps, it64[-1]), file=sys.stderr, flush=True)
    dt32, it32, rel32, u32 = timed_solves(torch, S32, f, g, steps, warmup, tol)
    print("%s mixed: %.4f s/solve, %d iterations" % (label, dt32 / steps, it32[-1]), file=sys.stderr, flush=True)
    launches, avg_ms, t_timed = kernel_time(torch, S32, f, g, timing_solves, tol)
    print("%s tile kernel: %d launches, %.2f us each" % (label, launches, 1e3 * avg_ms), file=sys.stderr, flush=True)
    diff = float((u32 - u64).abs().max() / u64.abs().max())
    out = {"levels": S32.info["nx"], "plg_cells": S32.info["n_plg"], "separators": S32.info["n_sep"],
           "sfv_cells": S32.info["n_sfv"], "setup_s": t_setup,
           "setup_stage_s": dict(zip(("cut_cells", "classification_lattices_moments", "fits", "plg_solver",
                                      "bottom_inverse", "other"), S32.info["setup_stage_seconds"])),
           "cond_A22": S32.info["cond_A22"],
           "mixed": {"value": steps / dt32, "unit": "solves/s", "ms_per_solve": 1e3 * dt32 / steps,
                     "iterations": it32[-1], "rel_residual": rel32, "max_rel_diff_vs_fp64": diff},
           "fp64": {"value": steps / dt64, "unit": "solves/s", "ms_per_solve": 1e3 * dt64 / steps,
                    "iterations": it64[-1], "rel_residual": rel64},
           "speedup_mixed_over_fp64": dt64 / dt32,
           "ms_per_solve_with_kernel_events": 1e3 * t_timed}
    return out, S32, S64, f, g, dt32, it64, (launches, avg_ms)


def main():
    global NU
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--nu", default="%d,%d" % NU, help="smoothing steps nu1,nu2 of every solve")
    ap.add_argument("--timing-solves", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--cpu-n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 1024^2 three-disk line")
    ap.add_argument("--no-floor", action="store_true", help="skip the FP64 floor measurement")
    ap.add_argument("--only-headline", action="store_true", help="the 4096^2 star line only")
    ap.add_argument("--only-secondary", action="store_true",
                    help="the 1024^2 three-disk line only (for profiling its kernels)")
    ap.add_argument("--serving-traces", action="store_true",
                    help="run only the serving traces with fresh geometries and with resident 2048^2 geometries")
    ap.add_argument("--trace-requests", type=int, default=64)
    ap.add_argument("--resident-geometries", type=int, default=16)
    ap.add_argument("--resident-rhs", type=int, default=8)
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-iters", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-cells", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also move 256 MiB with the runtime's copy kernel and with an elementwise kernel "
                         "(references for HBM byte counters)")
    args = ap.parse_args()
    NU = tuple(int(v) for v in args.nu.split(","))
    if len(NU) != 2 or min(NU) < 0:
        ap.error("--nu takes two non-negative integers nu1,nu2")
    if args.cpu_baseline_worker:
        print(json.dumps(cpu_baseline(args.cpu_n, args.cpu_iters, args.cpu_cells, args.cpu_seconds)))
        return
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
        for _ in range(3):
            torch.mul(src_t, 2.0, out=dst_t)
        torch.cuda.synchronize()
        print("calibration copy: 3 + 3 x %d bytes read and written" % (src_t.numel() * 8), file=sys.stderr)
        del src_t, dst_t

    if args.serving_traces:
        out = {"serving_fresh": serving_fresh_trace(torch, mg, W, args.trace_requests, 4, args.tol),
               "serving_resident": serving_resident(torch, mg, W, args.resident_geometries, args.resident_rhs, 4,
                                                    args.tol, 64 << 30)}
        print(json.dumps(out))
        return
    if args.only_secondary:
        P2 = W.three_disks_config(0, 1024)
        sec, S32b, S64b, f2, g2, _, _, (nl2, ms2) = solve_leg(
            torch, mg, P2, args.steps, args.warmup, args.tol, args.timing_solves, "three disks 1024")
        sec["roofline"] = roofline(S32b, ms2, nl2, load_traffic_for("three_disks1024", "k_smooth_a_fp32"))
        sec["roofline"]["kernel"] = "k_smooth_a<float> (finest level: SFV tiles and PLG groups, one kernel)"
        S32b.close()
        S64b.close()
        print(json.dumps({"three_disks1024": sec}))
        return
    P = W.star_config(0, 4096)
    head, S32, S64, f, g, dt32, it64, (launches, avg_ms) = solve_leg(
        torch, mg, P, args.steps, args.warmup, args.tol, args.timing_solves, "star 4096")
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
        "config": {"workload": "star_4096x4096_seed0: [0,1]^2 minus an 8-point star joined to circular arcs; "
                               "a=2, b=-1, c=1; Robin (1, 0.5) on the star, Dirichlet box; 8 sine modes",
                   "tol": args.tol, "cells": n_cells,
                   "solver": "V-cycles (Algorithm 3), nu = %s, omega = 1/2; graph replay" % (NU,)},
    }
    out.update(head)
    out["roofline"] = roofline(S32, avg_ms, launches, load_traffic_for(
        "star4096", "k_smooth_pair_fp32" if S32.info["n_pair_sfv"][0] else "k_smooth_tiles_fp32"))
    S32.close()
    S64.close()
    if not args.no_floor:
        Sf = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=mg.FP64, max_iters=60, nu=NU)
        out["fp64_floor"] = fp64_floor(torch, Sf, f, g)
        Sf.close()
        print("fp64 floor: %s" % out["fp64_floor"], file=sys.stderr, flush=True)
    if not args.no_variants and not args.only_headline:
        # the same solve with the FMG cycle, fewer sweeps, and the
        # multicolour smoother
        var = {}
        nn = "%d%d" % NU
        for kw, name in ((dict(pair_sweeps=-1), "v_nu%s_single_sweep_tiles" % nn), (dict(nu=(6, 6)), "v_nu66"),
                         (dict(cycle=mg.CYCLE_FMG), "fmg_nu%s" % nn), (dict(nu=(4, 4)), "v_nu44"),
                         (dict(colouring=mg.SMOOTH_MULTICOLOUR), "v_nu%s_multicolour" % nn),
                         (dict(colouring=mg.SMOOTH_MULTICOLOUR, nu=(4, 4)), "v_nu44_multicolour")):
            opts = dict(eps=P.eps, precision=mg.MIXED, max_iters=1000, nu=NU)
            opts.update(kw)
            S = mg.Solver(P.grid, P.curves, P.a, P.b, P.c, **opts)
            try:
                dt, it, rel, _ = timed_solves(torch, S, f, g, args.steps, args.warmup, args.tol)
                var[name] = {"value": args.steps / dt, "unit": "solves/s", "iterations": it[-1],
                             "rel_residual": rel, "precision": "mixed"}
                print("star variant %s: %.4f s/solve, %d iterations" % (name, dt / args.steps, it[-1]),
                      file=sys.stderr, flush=True)
            except (RuntimeError, mg.MGError) as e:
                var[name] = {"error": str(e)}
            S.close()
        out["variants"] = var
    del f, g
    if not args.only_headline:
        if not args.no_secondary:
            P2 = W.three_disks_config(0, 1024)
            sec, S32b, S64b, f2, g2, _, _, (nl2, ms2) = solve_leg(
                torch, mg, P2, args.steps, args.warmup, args.tol, args.timing_solves, "three disks 1024")
            sec["workload"] = ("three_disks_1024x1024_seed0: [0,1]^2 minus 3 seeded disks; a=1, b=0.5, c=2; "
                               "Dirichlet box, Neumann holes; 6 sine modes")
            sec["roofline"] = roofline(S32b, ms2, nl2, load_traffic_for("three_disks1024", "k_smooth_a_fp32"))
            sec["roofline"]["kernel"] = "k_smooth_a<float> (finest level: SFV tiles and PLG groups, one kernel)"
            S32b.close()
            S64b.close()
            if not args.no_variants:
                var = {}
                for cyc, nu, name in ((mg.CYCLE_FMG, NU, "fmg_nu%d%d" % NU), (mg.CYCLE_V, (3, 3), "v_nu33"),
                                      (mg.CYCLE_FMG, (3, 3), "fmg_nu33")):
                    S = mg.Solver(P2.grid, P2.curves, P2.a, P2.b, P2.c, eps=P2.eps, precision=mg.MIXED,
                                  max_iters=1000, nu=nu, cycle=cyc)
                    dt, it, rel, _ = timed_solves(torch, S, f2, g2, args.steps, args.warmup, args.tol)
                    S.close()
                    var[name] = {"value": args.steps / dt, "unit": "solves/s", "iterations": it[-1],
                                 "rel_residual": rel, "precision": "mixed"}
                    print("variant %s: %.4f s/solve, %d iterations" % (name, dt / args.steps, it[-1]),
                          file=sys.stderr, flush=True)
                sec["variants"] = var
            out["three_disks1024"] = sec
            del f2, g2
        if not args.no_serving:
            out["serving"] = serving_leg(torch, mg, W, [W.three_disks_config(s, 512) for s in range(1, 5)], 8,
                                         400.0, 4, args.tol, "4 three-disk geometries (seeds 1-4) at 512^2")
            print("serving: p50 %.3f s, p99 %.3f s, %.1f solves/s" % (
                out["serving"]["p50_latency_s"], out["serving"]["p99_latency_s"], out["serving"]["solves_per_s"]),
                file=sys.stderr, flush=True)
            mix = [W.serving_request(0, k) for k in range(6)]
            out["serving_mix"] = serving_leg(torch, mg, W, mix, 4, 200.0, 4, args.tol,
                                             "the first 6 requests of serving trace 0 as geometries (grids %s; "
                                             "1-5 holes, mixed boundary conditions, seeded a, b, c)"
                                             % "/".join(str(Q.grid.nx) for Q in mix))
            print("serving mix: p50 %.3f s, p99 %.3f s, %.1f solves/s" % (
                out["serving_mix"]["p50_latency_s"], out["serving_mix"]["p99_latency_s"],
                out["serving_mix"]["solves_per_s"]), file=sys.stderr, flush=True)
        if not args.no_cpu:
            # in a fresh interpreter that never touches the GPU (its worker
            # processes are forked from it)
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                                "--cpu-n", str(args.cpu_n), "--cpu-seconds", str(args.cpu_seconds),
                                "--cpu-iters", str(it64[-1]), "--cpu-cells", str(n_cells), "--nu", args.nu],
                               capture_output=True, text=True, timeout=900)
            if r.returncode != 0:
                raise RuntimeError("cpu baseline failed: " + r.stderr[-2000:])
            out["cpu_baseline"] = json.loads(r.stdout.strip().splitlines()[-1])
            print("cpu baseline: %s" % out["cpu_baseline"]["sample"], file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
