"""GPU tests of the serving form: the continuous-batching server returns, for every request,
exactly (bitwise) what a direct solve of the same request returns, whatever else runs
beside it; admission respects the memory budget."""
import sys

import numpy as np
import pytest

from paper_2401_17806_amd.inputs import lattice_mesh, random_vector

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _disc(n, p):
    from paper_2401_17806_amd import sld
    xy, tri, per = lattice_mesh(n, seed=n + 100 * p)
    mesh = sld.Mesh(xy, tri, per, device=0)
    return sld.Disc(mesh, p)


def _rhs(torch, disc, seed):
    b = random_vector(disc.main_shape, seed)
    return torch.from_numpy(b - b.mean()).to("cuda:0")


def test_server_results_equal_direct_solves(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import sld
    _say("[server] alone vs mix")
    specs = [(12, 2, "fp64"), (16, 3, "fp64"), (8, 4, "mixed"), (10, 1, "mixed"), (14, 3, "fp64")]
    discs = [_disc(n, p) for n, p, _ in specs]
    rhs = [_rhs(torch, d, 50 + k) for k, d in enumerate(discs)]
    alone = []
    for (n, p, prec), d, b in zip(specs, discs, rhs):
        x, rep = d.sld_cg_solve(b, rtol=1e-12 if prec == "fp64" else 1e-11, precision=prec,
                                graph_block=16)
        assert rep["status"] == "SLD_OK"
        alone.append(x)
    torch.cuda.synchronize()
    server = sld.Server(device=0, budget_bytes=8 << 30, workers=4)
    tickets = []
    outs = []
    for rnd in range(2):  # every disc twice: the repeat waits for the first on the same disc
        for (n, p, prec), d, b in zip(specs, discs, rhs):
            out = torch.empty_like(b)
            t = server.sld_server_submit(d, b, out, rtol=1e-12 if prec == "fp64" else 1e-11,
                                         precision=prec, graph_block=16)
            tickets.append(t)
            outs.append(out)
    reps = [server.sld_server_poll(t, wait=True) for t in tickets]
    stats = server.sld_server_stats()
    server.close()
    assert stats["completed"] == len(tickets) and stats["queued"] == 0
    for k, (rep, out) in enumerate(zip(reps, outs)):
        assert rep["status"] == "SLD_OK", rep
        assert torch.equal(out, alone[k % len(specs)]), k


def test_server_budget_admission(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import sld
    _say("[server] budget")
    d1, d2 = _disc(12, 2), _disc(12, 3)
    need = max(d1.footprint(), d2.footprint()) + 12 * 12 * 2 * 10 * 16
    server = sld.Server(device=0, budget_bytes=need, workers=3)
    b1, b2 = _rhs(torch, d1, 7), _rhs(torch, d2, 8)
    o1, o2 = torch.empty_like(b1), torch.empty_like(b2)
    t1 = server.sld_server_submit(d1, b1, o1, rtol=1e-10, graph_block=8)
    t2 = server.sld_server_submit(d2, b2, o2, rtol=1e-10, graph_block=8)
    assert server.sld_server_poll(t1, wait=True)["status"] == "SLD_OK"
    assert server.sld_server_poll(t2, wait=True)["status"] == "SLD_OK"
    big = _disc(40, 4)
    bb = _rhs(torch, big, 9)
    with pytest.raises(sld.SldError) as e:
        server.sld_server_submit(big, bb, torch.empty_like(bb), rtol=1e-10)
    assert e.value.status == 7
    server.close()


def test_serving_loop_poisson_small(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import serve
    _say("[serve] poisson loop")
    reqs = serve.request_mix(12, seed=5, sizes=(8, 12), degrees=(1, 2, 3))
    arr = serve.poisson_arrivals(len(reqs), rate=200.0, seed=6)
    recs, wall = serve.run(reqs, arr, workers=3, keep_solutions=True, kmax=4)
    assert all(r is not None for r in recs)
    summ = serve.summarize(recs, wall)
    _say("   ", summ)
    assert summ["statuses"] == {"SLD_OK": len(reqs)}
    assert all(r["latency"] > 0 for r in recs)
    # each served result equals the same request solved alone, bitwise
    from paper_2401_17806_amd import sld
    side = torch.cuda.Stream(device=0)
    with torch.cuda.stream(side):
        for q, rec in zip(reqs, recs):
            mesh = sld.Mesh(*q["mesh"], device=0)
            disc = sld.Disc(mesh, q["p"])
            b = serve._rhs(disc, q["seed"], 4, torch)
            tol = 1e-10
            x, rep = disc.sld_cg_solve(b, rtol=tol, precision=q["precision"], graph_block=32,
                                       maxit=200000)
            assert rep["iters"] == rec["iters"]
            assert torch.equal(x, rec["solution"]), q["id"]


def _tgv_dual(disc, nu=1e-2):
    x = disc.dual_nodes()
    u = np.sin(x[..., 0]) * np.cos(x[..., 1])
    w = -np.cos(x[..., 0]) * np.sin(x[..., 1])
    return np.ascontiguousarray(np.stack([u, w], axis=1))  # [nd, 2, Npsi]


def test_server_imex_steps_equal_direct_steps(torch_dev):
    """IMEX-step requests (two consecutive steps per state, queued back to back) mixed with
    pressure solves on other discs: every result equals, bitwise, the same work done alone."""
    torch = torch_dev
    from paper_2401_17806_amd import sld
    _say("[server] imex steps in the mix")
    nu = 1e-2
    ispecs = [(8, 2), (12, 3), (10, 1)]
    idiscs = [_disc(n, p) for n, p in ispecs]
    sspecs = [(16, 3), (14, 2)]
    sdiscs = [_disc(n, p) for n, p in sspecs]
    rhs = [_rhs(torch, d, 70 + k) for k, d in enumerate(sdiscs)]
    v0 = [torch.from_numpy(_tgv_dual(d)).to("cuda:0") for d in idiscs]
    dts = [0.5 * 2 * np.pi / n for n, _ in ispecs]
    # alone
    alone_v, alone_p = [], []
    for d, v, dt in zip(idiscs, v0, dts):
        st = sld.State(d)
        vv = v.clone()
        pp = torch.zeros(d.main_shape, dtype=torch.float64, device="cuda:0")
        for _ in range(2):
            rep = st.sld_imex_step(vv, pp, dt, nu, graph_block=16)
            assert rep["status"] == "SLD_OK"
        alone_v.append(vv)
        alone_p.append(pp)
    alone_x = []
    for d, b in zip(sdiscs, rhs):
        x, rep = d.sld_cg_solve(b, graph_block=16)
        assert rep["status"] == "SLD_OK"
        alone_x.append(x)
    torch.cuda.synchronize()
    # in the mix
    server = sld.Server(device=0, budget_bytes=8 << 30, workers=4)
    states = [sld.State(d) for d in idiscs]
    vs = [v.clone() for v in v0]
    ps = [torch.zeros(d.main_shape, dtype=torch.float64, device="cuda:0") for d in idiscs]
    xs = [torch.empty_like(b) for b in rhs]
    tickets = []
    for step in range(2):
        for k in range(len(idiscs)):
            tickets.append(server.sld_server_submit_imex(states[k], vs[k], ps[k], dts[k], nu,
                                                         graph_block=16))
            if step == 0 and k < len(sdiscs):
                tickets.append(server.sld_server_submit(sdiscs[k], rhs[k], xs[k], graph_block=16))
    reps = [server.sld_server_poll(t, wait=True) for t in tickets]
    stats = server.sld_server_stats()
    server.close()
    assert stats["completed"] == len(tickets) and stats["queued"] == 0
    assert all(r["status"] == "SLD_OK" for r in reps), reps
    for k in range(len(idiscs)):
        assert torch.equal(vs[k], alone_v[k]) and torch.equal(ps[k], alone_p[k]), k
    for k in range(len(sdiscs)):
        assert torch.equal(xs[k], alone_x[k]), k


def test_serving_loop_with_imex_requests(torch_dev):
    """The serving loop with half of the requests IMEX steps: every request ends SLD_OK, and each
    served IMEX step's pressure equals the same step run alone, bitwise."""
    torch = torch_dev
    from paper_2401_17806_amd import serve, sld
    _say("[serve] poisson loop with imex steps")
    reqs = serve.request_mix(12, seed=8, sizes=(8, 12), degrees=(1, 2, 3), imex_fraction=0.5)
    assert 0 < sum(q["kind"] == "imex" for q in reqs) < len(reqs)
    arr = serve.poisson_arrivals(len(reqs), rate=200.0, seed=9)
    recs, wall = serve.run(reqs, arr, workers=3, keep_solutions=True, kmax=4)
    summ = serve.summarize(recs, wall)
    _say("   ", summ)
    assert summ["statuses"] == {"SLD_OK": len(reqs)}
    side = torch.cuda.Stream(device=0)
    with torch.cuda.stream(side):
        for q, rec in zip(reqs, recs):
            if q["kind"] != "imex":
                continue
            mesh = sld.Mesh(*q["mesh"], device=0)
            disc = sld.Disc(mesh, q["p"])
            st = sld.State(disc)
            v = serve._tgv_dual(disc, torch)
            p = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
            tol = 1e-10
            rep = st.sld_imex_step(v, p, 0.5 * 2 * np.pi / q["n"], 1e-2, rtol=tol,
                                   precision=q["precision"], graph_block=32, maxit=200000,
                                   warm_start=False)
            assert rep["status"] == "SLD_OK"
            assert torch.equal(p, rec["solution"]), q["id"]
