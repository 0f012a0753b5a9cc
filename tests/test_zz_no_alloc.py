"""sld_cg_solve_static, the CG solve that allocates nothing (its workspace is the library's static
device array), against sld_cg_solve on the same disc and right-hand side: two calls in a row,
the second on a smaller disc, each compared with sld_cg_solve and with the oracle's pressure
(plain CG on the assembled K of eq. pressure_final, Section 3.3); a disc whose workspace does
not fit the array is refused."""
import sys

import numpy as np
import pytest

from oracle import solve
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field

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


def _case(torch, n, p, seed, walls=False):
    from paper_2401_17806_amd import sld
    length = 1.0 if walls else 2 * np.pi
    xy, tri, per = lattice_mesh(n, seed=seed, periodic=not walls, length=length)
    od = OracleDisc(OracleMesh(xy, tri, per), p)
    disc = sld.Disc(sld.Mesh(xy, tri, per, device=0), p)
    vs = random_fourier_field(seed + 100, kmax=4, length=length)(od.dual_node_xy())
    b_h = solve.divergence(od, np.ascontiguousarray(vs.transpose(0, 2, 1)))
    x_or = solve.gauge(od, solve.cg(solve.assemble_K(od), b_h, tol=1e-13)[0])
    return disc, torch.from_numpy(b_h).to("cuda:0"), x_or


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("cases", [[(24, 3, 7, False), (10, 2, 8, False)],
                                   [(20, 4, 9, True), (6, 1, 10, True)]])
def test_static_cg_matches_cg_solve_on_two_calls(torch_dev, cases):
    torch = torch_dev
    for n, p, seed, walls in cases:  # the second call is on a smaller disc
        _say(f"[static cg] n={n} p={p} walls={walls}")
        disc, b, x_or = _case(torch, n, p, seed, walls)
        ref, rr = disc.sld_cg_solve(b, rtol=1e-12, graph_block=8)
        out = torch.full_like(ref, float("nan"))  # every output word must be written
        got, rs = disc.sld_cg_solve_static(b, p=out, rtol=1e-12, graph_block=8)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        _say(f"    cg_solve {rr['status']} {rr['iters']} it; static {rs['status']} {rs['iters']} it; "
             f"static vs cg_solve {_rel(g, r):.2e}, vs oracle {_rel(g, x_or):.2e}")
        assert rs["status"] == rr["status"] == "SLD_OK" and rs["converged"]
        assert rs["iters"] == rr["iters"] and rs["outer_iters"] == rr["outer_iters"]
        assert np.isfinite(g).all()
        assert _rel(g, r) <= 1e-12
        assert _rel(g, x_or) <= 1e-9 and rs["rel_res_true"] <= 1e-12


def test_static_cg_refuses_a_disc_beyond_the_array(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import sld
    xy, tri, per = lattice_mesh(256, seed=1005)
    disc = sld.Disc(sld.Mesh(xy, tri, per, device=0), 4)  # 1.97M DOFs: beyond 9.3e5
    b = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sld.SldError) as ei:
        disc.sld_cg_solve_static(b, rtol=1e-10)
    assert "SLD_E_BUDGET" in str(ei.value) and "static workspace" in str(ei.value)
