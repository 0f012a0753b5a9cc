"""GPU parity of the pipelined CG (Ghysels and Vanroose's reformulation of the CG of Section 3.3:
the same iterates in exact arithmetic, the operator applied to a vector the previous iteration
completed) against the FP64 oracle on the same seeded inputs:
  * pressure solves at rtol 1e-12 (residual replacement as for CG) equal the oracle's solution
    to 1e-9, periodic and walled meshes, p = 1..4, one tile up to many tiles with a ragged last
    tile; the iteration count is within 25% of the classic iteration's (its longer recurrences
    carry rounding errors further);
  * repeated solves are bitwise identical; a warm start converges;
  * the 128x128x2, p = 3 pressure matches the oracle's stored sample to 1e-9 of its max norm;
  * requests it cannot serve (mixed precision, meshes beyond one tile per block) are refused."""
import math
import os
import sys

import numpy as np
import pytest

from oracle import solve
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
A_SS = 0.43586652150845967


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


_CACHE = {}


def _setup(n, p, periodic=True, seed=3, oracle=True):
    key = (n, p, periodic, seed, oracle)
    if key not in _CACHE:
        from paper_2401_17806_amd import sld
        xy, tri, per = lattice_mesh(n, seed=seed, periodic=periodic,
                                    length=(2 * np.pi if periodic else 1.0))
        od = OracleDisc(OracleMesh(xy, tri, per), p) if oracle else None
        K = solve.assemble_K(od) if oracle else None
        mesh = sld.Mesh(xy, tri, per, device=0)
        _CACHE[key] = (od, K, mesh, sld.Disc(mesh, p))
    return _CACHE[key]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [(3, 1, True), (3, 2, True), (12, 3, True), (12, 4, True), (45, 3, True), (20, 2, False),
         (24, 3, False)]


@pytest.mark.parametrize("n,p,periodic", CASES)
def test_pcg_matches_oracle_and_classic(torch_dev, n, p, periodic):
    torch = torch_dev
    _say(f"[pcg] n={n} p={p} periodic={periodic}")
    od, K, mesh, disc = _setup(n, p, periodic)
    f = random_fourier_field(23, kmax=4, length=(2 * np.pi if periodic else 1.0))
    b = solve.divergence(od, f(od.dual_node_xy()).transpose(0, 2, 1))
    x_or, _ = solve.cg(K, b, tol=1e-13)
    x_or = solve.gauge(od, x_or)
    bt = torch.from_numpy(b).to("cuda:0")
    pp, rp = disc.sld_cg_solve(bt, rtol=1e-12, maxit=40000, graph_block=16, algorithm="pipelined")
    pc, rc = disc.sld_cg_solve(bt, rtol=1e-12, maxit=40000, graph_block=16, algorithm="classic")
    err = _rel(pp.cpu().numpy(), x_or)
    _say(f"    pipelined: {rp['iters']} iterations, {rp['outer_iters']} replacements, "
         f"{rp['status']}, rel res {rp['rel_res_true']:.2e}, error vs oracle {err:.2e}; "
         f"classic {rc['iters']} iterations")
    assert rp["status"] == "SLD_OK" and rp["converged"] and rp["rel_res_true"] <= 1e-12
    assert err <= 1e-9
    # its longer recurrences carry rounding further than CG's: a few more iterations
    assert rp["iters"] <= 1.25 * rc["iters"] + 2
    p2, _ = disc.sld_cg_solve(bt, rtol=1e-12, maxit=40000, graph_block=16, algorithm="pipelined")
    assert np.array_equal(p2.cpu().numpy(), pp.cpu().numpy())


def test_pcg_warm_start(torch_dev):
    torch = torch_dev
    od, K, mesh, disc = _setup(12, 3, True)
    f = random_fourier_field(29, kmax=4)
    b = solve.divergence(od, f(od.dual_node_xy()).transpose(0, 2, 1))
    x_or, _ = solve.cg(K, b, tol=1e-13)
    x_or = solve.gauge(od, x_or)
    rng = np.random.default_rng(4)
    guess = torch.from_numpy(x_or + 1e-3 * rng.standard_normal(x_or.shape)).to("cuda:0")
    bt = torch.from_numpy(b).to("cuda:0")
    pw, rw = disc.sld_cg_solve(bt, p=guess, rtol=1e-12, warm_start=True, graph_block=16,
                               algorithm="pipelined")
    _say(f"[pcg warm] {rw['iters']} iterations, {rw['status']}")
    assert rw["status"] == "SLD_OK" and _rel(pw.cpu().numpy(), x_or) <= 1e-9


def _read_sample(name):
    idx, val, head = [], [], {}
    for line in open(os.path.join(HERE, "golden", name)):
        if line.startswith("#"):
            parts = line[1:].split()
            for k in range(len(parts) - 1):
                if parts[k] == "maxabs_p":
                    head["maxabs_p"] = float(parts[k + 1])
            continue
        i, v = line.split()
        idx.append(int(i))
        val.append(float(v))
    return np.array(idx), np.array(val), head


def test_pcg_c2_pressure_matches_oracle_sample(torch_dev):
    """128x128x2, p = 3 (the cache-resident workload), the bench right-hand side, rtol 1e-11."""
    torch = torch_dev
    _say("[pcg c2]")
    _, _, mesh, disc = _setup(128, 3, True, seed=2, oracle=False)
    vs = random_fourier_field(102, kmax=8)(disc.dual_nodes()).transpose(0, 2, 1)
    vt = torch.from_numpy(np.ascontiguousarray(vs)).to("cuda:0")
    b = disc.sld_pressure_rhs(vt, 1.0 / (A_SS * 0.5 * (2 * math.pi / 128)))
    pp, rp = disc.sld_cg_solve(b, rtol=1e-11, graph_block=256, maxit=100000, algorithm="pipelined")
    idx, val, head = _read_sample("c2_pressure_sample.txt")
    err = np.abs(pp.cpu().numpy().ravel()[idx] - val).max() / head["maxabs_p"]
    _say(f"    {rp['iters']} iterations, {rp['status']}, rel res {rp['rel_res_true']:.2e}, "
         f"sampled error {err:.2e}")
    assert rp["status"] == "SLD_OK" and rp["rel_res_true"] <= 1e-11 and err <= 1e-9


def test_pcg_refuses_what_it_cannot_serve(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import sld
    _, _, mesh, disc = _setup(12, 2, True, oracle=False)
    b = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sld.SldError):
        disc.sld_cg_solve(b, precision="mixed", algorithm="pipelined")
    # 200x200x2 = 80000 triangles (1250 tiles): more tiles than resident blocks
    _, _, mesh2, disc2 = _setup(200, 1, True, oracle=False)
    b2 = torch.zeros(disc2.main_shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sld.SldError):
        disc2.sld_cg_solve(b2, algorithm="pipelined")
