"""The solve server (mg_server_*): a request's result is the same alone and
in a mix of concurrent requests, also when the device-memory budget forces
hierarchies out and back in.  Bitwise: each request runs the same kernels on
the same data whatever else runs."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _requests():
    base = [W.unit_disk_config(0, 64), W.three_disks_config(0, 128), W.star_config(0, 128),
            W.serving_request(0, 2)]
    base[3] = W.with_grid(base[3], 128)
    reqs = []
    for k, P in enumerate(base):
        for r in range(2 if k < 2 else 1):
            reqs.append((k, W.with_solution(P, 100 * k + r, 4) if r else P))
    return base, reqs


@pytest.mark.parametrize("budget", [64 << 30, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_server_results_equal_alone(budget, precision):
    torch = _torch()
    import paper_2601_02975_amd as mg
    base, reqs = _requests()
    # inputs from each geometry's own projection
    solvers = [mg.Solver(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=precision) for P in base]
    inputs = []
    for k, P in reqs:
        inputs.append(solvers[k].project(P.solution))
    alone = []
    for (k, P), (f, g) in zip(reqs, inputs):
        u = torch.zeros_like(f)
        it, rel, code = solvers[k].solve(f, g, u, 1e-10)
        assert code == 0, (P.name, code)
        alone.append((u, it, rel))
    for S in solvers:
        S.close()
    srv = mg.Server(max_active=3, hbm_budget=budget)
    pids = [srv.add_problem(P.grid, P.curves, P.a, P.b, P.c, eps=P.eps, precision=precision) for P in base]
    outs, tickets = [], []
    for (k, P), (f, g) in zip(reqs, inputs):
        u = torch.zeros_like(f)
        outs.append(u)
        tickets.append(srv.submit(pids[k], f, g, u, 1e-10))
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    for (u0, it0, rel0), u, r in zip(alone, outs, res):
        assert r["status"] == 0, r
        assert r["iters"] == it0 and r["rel_residual"] == rel0
        assert torch.equal(u, u0)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["p99_latency_s"] >= st["p50_latency_s"] > 0
    assert 0 < st["sweep_gbs"] < 8000       # the smoothing bytes of the solves, below the HBM peak
    if budget == 1:
        assert st["evictions"] > 0 and st["resident_problems"] <= 1
    print(st)


def test_small_request_overtakes_a_large_setup():
    """A slot setting up a large new geometry does not hold the other slots:
    a small request submitted just after it (a new geometry too, so it also
    sets up and captures its graphs) completes first."""
    torch = _torch()
    import paper_2601_02975_amd as mg
    big = W.three_disks_config(3, 1024)
    small = W.unit_disk_config(0, 64)
    Sb = mg.Solver(big.grid, big.curves, big.a, big.b, big.c, eps=big.eps)
    Ss = mg.Solver(small.grid, small.curves, small.a, small.b, small.c, eps=small.eps)
    fb, gb = Sb.project(big.solution)
    fs, gs = Ss.project(small.solution)
    Sb.close()
    Ss.close()
    srv = mg.Server(max_active=2, hbm_budget=64 << 30)
    pb = srv.add_problem(big.grid, big.curves, big.a, big.b, big.c, eps=big.eps, nu=(6, 6), max_iters=1000)
    ps = srv.add_problem(small.grid, small.curves, small.a, small.b, small.c, eps=small.eps)
    tb = srv.submit(pb, fb, gb, torch.zeros_like(fb), 1e-10)
    ts = srv.submit(ps, fs, gs, torch.zeros_like(fs), 1e-10)
    rs = srv.wait(ts)
    done_b = srv.poll(tb)
    rb = srv.wait(tb)
    srv.close()
    print("small request %.3f s, large request (with setup) %.3f s" % (rs["latency_s"], rb["latency_s"]))
    assert rs["status"] == 0 and rb["status"] == 0
    assert done_b is None, "the small request waited for the large setup"
    assert rs["latency_s"] < 0.5 * rb["latency_s"]
