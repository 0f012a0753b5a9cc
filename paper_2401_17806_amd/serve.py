"""Serving loop for the pressure solve and the IMEX step: a stream of independent requests on
meshes of different sizes and degrees, run through the library's continuous-batching server
(sld_server_*).

Each request is (mesh n, degree p, precision, seed): the pressure stage right-hand side
b = D v* of a seeded Gaussian random Fourier velocity field v* (|k| <= kmax, amplitude ~ |k|^-2)
sampled at the dual nodes, solved to a recomputed FP64 relative residual of 1e-10 in both
precisions (the FP64 rounding floor of K x - b is about 1e-11 on the largest meshes of the
mix, so tighter tolerances cannot be confirmed there).  Every request brings its own jittered
mesh (seed =
request seed).  On arrival it is set up on the device (mesh tables, discretisation, right-hand
side) as soon as the device-memory budget allows, submitted to the server, and freed when its
result is in.  Latency = arrival -> result ready on the host, setup included.

A fraction of the requests (imex_fraction) can be IMEX steps instead: one R = 0
semi-Lagrangian IMEX step of the Taylor-Green vortex (nu = 1e-2, dt = 0.5 h) on the request's
mesh, its velocity interpolated at the dual nodes, the pressure solved to the same tolerance.
"""
from __future__ import annotations

import collections
import sys
import time

import numpy as np

from . import sld
from .inputs import lattice_mesh


def request_mix(nreq: int, seed: int, sizes=(16, 32, 64, 128, 256), degrees=(1, 2, 3, 4),
                mixed_fraction: float = 0.5, imex_fraction: float = 0.0):
    """Seeded heterogeneous request list: n and p uniform, FP64/mixed by a Bernoulli draw, IMEX
    step or pressure solve by a second Bernoulli draw (its own stream, so the solve mix does
    not depend on imex_fraction)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kind_rng = np.random.Generator(np.random.PCG64(seed + 7))
    out = []
    for r in range(nreq):
        out.append({"id": r, "n": int(rng.choice(sizes)), "p": int(rng.choice(degrees)),
                    "precision": "mixed" if rng.random() < mixed_fraction else "fp64",
                    "kind": "imex" if kind_rng.random() < imex_fraction else "solve",
                    "seed": 1000 + r})
    return out


def poisson_arrivals(nreq: int, rate: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=nreq))


def prepare(requests, length: float = 2 * np.pi):
    """Client side of each request: its jittered periodic mesh (seed = the request's seed)."""
    for q in requests:
        if "mesh" not in q:
            q["mesh"] = lattice_mesh(q["n"], length=length, seed=q["seed"])
    return requests


def _rhs(disc, seed, kmax, torch):
    """b = D v* with v* a seeded random Fourier field at the dual nodes: modes k on the half
    plane with 0 < |k| <= kmax, coefficients a_k, b_k ~ N(0, |k|^-4) per component, summed mode
    by mode on the device (elementwise, no temporaries beyond one phase array)."""
    pts = torch.from_numpy(disc.dual_nodes()).to(f"cuda:{disc.mesh.device}")  # [nd, npsi, 2]
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = [(kx, ky) for kx in range(0, kmax + 1) for ky in range(-kmax, kmax + 1)
          if not (kx == 0 and ky <= 0) and kx * kx + ky * ky <= kmax * kmax]
    std = np.array([float(kx * kx + ky * ky) ** -1.0 for kx, ky in ks])
    ca = rng.standard_normal((len(ks), 2)) * std[:, None]
    cb = rng.standard_normal((len(ks), 2)) * std[:, None]
    x, y = pts[..., 0], pts[..., 1]
    v = torch.zeros(pts.shape[0], 2, pts.shape[1], dtype=torch.float64, device=pts.device)
    for m, (kx, ky) in enumerate(ks):
        ph = torch.add(x * float(kx), y, alpha=float(ky))
        c, sn = torch.cos(ph), torch.sin(ph)
        for comp in range(2):
            v[:, comp].add_(c, alpha=float(ca[m, comp])).add_(sn, alpha=float(cb[m, comp]))
    return disc.sld_pressure_rhs(v, 1.0)


def _tgv_dual(disc, torch):
    """Taylor-Green velocity [nd, 2, Npsi] interpolated at the dual nodes (t = 0)."""
    x = disc.dual_nodes()
    u = np.stack([np.sin(x[..., 0]) * np.cos(x[..., 1]),
                  -np.cos(x[..., 0]) * np.sin(x[..., 1])], axis=1)
    return torch.from_numpy(np.ascontiguousarray(u)).to(f"cuda:{disc.mesh.device}")


def run(requests, arrivals, *, workers=4, budget_bytes=32 << 30, rtol=1e-10,
        mixed_rtol=1e-10, kmax=8, graph_block=32, poll_sleep=50e-6, keep_solutions=False,
        progress=0):
    """Submit each request at its arrival time (seconds after start); returns per-request
    records with latency.  arrivals = None means all at t = 0 (closed-loop saturation)."""
    import torch
    # right-hand sides are built on a side stream: library setup and graph capture on the
    # server's workers must not meet work on the legacy null stream
    side = torch.cuda.Stream(device=0)
    with torch.cuda.stream(side):
        return _run(torch, prepare(requests), arrivals, workers, budget_bytes, rtol, mixed_rtol,
                    kmax, graph_block, poll_sleep, keep_solutions, progress)


def _run(torch, requests, arrivals, workers, budget_bytes, rtol, mixed_rtol, kmax,
         graph_block, poll_sleep, keep_solutions, progress):
    server = sld.Server(device=0, budget_bytes=budget_bytes, workers=workers)
    footprint = {}  # (n, p) -> device bytes of one mesh + disc, learnt from the first one built
    resident = 0
    pending = collections.deque(range(len(requests)))
    waiting = collections.deque()  # arrived, not yet set up on the device
    inflight = {}
    records = [None] * len(requests)
    ndone = 0
    arr = np.zeros(len(requests)) if arrivals is None else np.asarray(arrivals)
    t0 = time.perf_counter()
    while pending or waiting or inflight:
        now = time.perf_counter() - t0
        while pending and arr[pending[0]] <= now:
            waiting.append(pending.popleft())
        # set up arrived requests in arrival order while the budget allows (a request is always
        # set up when nothing is resident, so a large one cannot starve)
        while waiting:
            q = requests[waiting[0]]
            key = (q["n"], q["p"])
            if resident and resident + footprint.get(key, 0) > budget_bytes:
                break
            r = waiting.popleft()
            xy, tri, per = q["mesh"]
            mesh = sld.Mesh(xy, tri, per, device=0)
            disc = sld.Disc(mesh, q["p"])
            tol = mixed_rtol if q["precision"] == "mixed" else rtol
            state = None
            if q.get("kind", "solve") == "imex":
                state = sld.State(disc)
                # the state's workspace and the request's velocity and pressure
                fb = disc.footprint() + 8 * (8 * mesh.ne * disc.nphi + 3 * mesh.nd * disc.npsi)
                v = _tgv_dual(disc, torch)
                p = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
                t = server.sld_server_submit_imex(state, v, p, 0.5 * 2 * np.pi / q["n"], 1e-2,
                                                  rtol=tol, precision=q["precision"],
                                                  graph_block=graph_block, maxit=200000,
                                                  warm_start=False)
            else:
                fb = disc.footprint()
                b = _rhs(disc, q["seed"], kmax, torch)
                p = torch.empty_like(b)
                t = server.sld_server_submit(disc, b, p, rtol=tol, precision=q["precision"],
                                             graph_block=graph_block, maxit=200000)
            footprint[key] = max(footprint.get(key, 0), fb)
            resident += fb
            inflight[t] = (r, disc, mesh, p, fb, state)
        for t in list(inflight):
            rep = server.sld_server_poll(t)
            if rep is None:
                continue
            r, disc, mesh, p, fb, state = inflight.pop(t)
            done = time.perf_counter() - t0
            q = requests[r]
            records[r] = {k: v for k, v in q.items() if k != "mesh"}
            records[r].update(arrival=float(arr[r]), done=done, latency=done - float(arr[r]),
                              iters=rep["iters"], outer_iters=rep["outer_iters"],
                              status=rep["status"], rel_res_true=rep["rel_res_true"],
                              dofs=disc.mesh.ne * disc.nphi,
                              solution=p if keep_solutions else None)
            if state is not None:
                state.close()
            disc.close()
            mesh.close()
            resident -= fb
            ndone += 1
            if progress and ndone % progress == 0:
                print(f"[serve] {ndone}/{len(requests)} done at {done:.2f} s", file=sys.stderr,
                      flush=True)
        time.sleep(poll_sleep)
    wall = time.perf_counter() - t0
    server.close()
    return records, wall


def summarize(records, wall):
    """Throughput (solves/s, DOF-updates/s = sum of DOFs x CG iterations over wall time) and
    latency percentiles, overall and per precision."""
    lat = np.array([r["latency"] for r in records])
    dof_updates = sum(r["dofs"] * r["iters"] for r in records)
    out = {"requests": len(records), "wall_s": wall, "solves_per_s": len(records) / wall,
           "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
           "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
           "dof_updates_per_s": dof_updates / wall,
           "max_rel_res_true": float(max(r["rel_res_true"] for r in records)),
           "statuses": dict(collections.Counter(r["status"] for r in records))}
    for pr in ("fp64", "mixed"):
        lp = np.array([r["latency"] for r in records if r["precision"] == pr])
        if len(lp):
            out[f"{pr}_latency_ms_p50"] = float(np.percentile(lp, 50) * 1e3)
            out[f"{pr}_latency_ms_p99"] = float(np.percentile(lp, 99) * 1e3)
    kinds = collections.Counter(r.get("kind", "solve") for r in records)
    if len(kinds) > 1:
        for kd in kinds:
            lk = np.array([r["latency"] for r in records if r.get("kind", "solve") == kd])
            out[f"{kd}_requests"] = int(len(lk))
            out[f"{kd}_latency_ms_p50"] = float(np.percentile(lk, 50) * 1e3)
            out[f"{kd}_latency_ms_p99"] = float(np.percentile(lk, 99) * 1e3)
    return out


def main(argv=None):
    """Two passes over one seeded request mix: closed loop (all requests at t = 0) gives the peak
    rate; then Poisson arrivals at `load` x that rate give the latency distribution."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--sizes", default="16,32,64,128,256")
    ap.add_argument("--degrees", default="1,2,3,4")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--imex-fraction", type=float, default=0.0,
                    help="share of the requests that are IMEX steps instead of pressure solves")
    a = ap.parse_args(argv)
    sizes = tuple(int(x) for x in a.sizes.split(","))
    degrees = tuple(int(x) for x in a.degrees.split(","))
    reqs = request_mix(a.requests, a.seed, sizes=sizes, degrees=degrees,
                       imex_fraction=a.imex_fraction)
    budget = int(a.budget_gib * (1 << 30))
    prepare(reqs)
    # warm pass: load the kernels of every degree and precision once, on the smallest mesh
    kinds = ("solve", "imex") if a.imex_fraction > 0 else ("solve",)
    warm = [{"id": k, "n": min(sizes), "p": p, "precision": pr, "kind": kd, "seed": 900 + k}
            for k, (p, pr, kd) in enumerate((p, pr, kd) for p in degrees
                                            for pr in ("fp64", "mixed") for kd in kinds)]
    run(warm, None, workers=a.workers, budget_bytes=budget)
    recs, wall = run(reqs, None, workers=a.workers, budget_bytes=budget, progress=32)
    closed = summarize(recs, wall)
    print(json.dumps({"pass": "closed_loop", **closed}), flush=True)
    rate = a.load * closed["solves_per_s"]
    arr = poisson_arrivals(len(reqs), rate, a.seed + 1)
    recs, wall = run(reqs, arr, workers=a.workers, budget_bytes=budget, progress=32)
    open_ = summarize(recs, wall)
    print(json.dumps({"pass": "poisson", "rate_per_s": rate, **open_}), flush=True)


if __name__ == "__main__":
    main()
