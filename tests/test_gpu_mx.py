"""GPU parity of the matrix-core (MFMA) form of the pressure operator (eq. pressure_final with
the reference contractions of Section 3.4.1 as element-batched matrix products) against the
FP64 oracle on the same seeded inputs:
  * FP64 MFMA apply: relative L2 <= 1e-12 (the per-apply bar of every FP64 operator);
  * BF16x3 MFMA apply (FP32 in and out; three-term bfloat16 splits, FP32 accumulation): its
    error against the oracle is stated and bounded at the FP32 level (<= 2e-6 relative L2);
  * CG solves through the MFMA iteration (FP64, and the mixed form whose FP32 inner iterations
    run the BF16x3 operator) converge to the oracle's pressure at 1e-9, the same as the
    vector-unit iteration, and are deterministic;
  * meshes with walls are refused by the MFMA apply.
Meshes span one tile (3x3x2) up to many tiles with halos and a ragged last tile (45x45x2 =
4050 triangles, 63 tiles of 64 and one of 18)."""
import sys

import numpy as np
import pytest

from oracle import solve
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field, random_vector

pytestmark = pytest.mark.gpu

APPLY_TOL = 1e-12
BF3_TOL = 2e-6
SOLVE_TOL = 1e-9


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


def _setup(n, p, periodic=True, seed=3):
    key = (n, p, periodic, seed)
    if key not in _CACHE:
        from paper_2401_17806_amd import sld
        xy, tri, per = lattice_mesh(n, seed=seed, periodic=periodic,
                                    length=(2 * np.pi if periodic else 1.0))
        od = OracleDisc(OracleMesh(xy, tri, per), p)
        K = solve.assemble_K(od)
        mesh = sld.Mesh(xy, tri, per, device=0)
        _CACHE[key] = (od, K, mesh, sld.Disc(mesh, p))
    return _CACHE[key]


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


CASES = [(3, p) for p in (1, 2, 3, 4)] + [(12, p) for p in (1, 2, 3, 4)] + \
        [(45, p) for p in (2, 3, 4)] + [(20, 1)]


@pytest.mark.parametrize("n,p", CASES)
def test_mx_apply_f64_matches_oracle(torch_dev, n, p):
    torch = torch_dev
    _say(f"[mx apply f64] n={n} p={p}")
    od, K, mesh, disc = _setup(n, p)
    x = random_vector((mesh.ne, disc.nphi), seed=700 + n + p)
    want = solve.schur_apply(K, x)
    got = disc.sld_schur_apply_mx(torch.from_numpy(x).to("cuda:0"), "f64").cpu().numpy()
    valu = disc.sld_schur_apply(torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    rel = _rel(got, want)
    _say(f"    rel L2 vs oracle {rel:.2e}, vs vector-unit apply {_rel(got, valu):.2e}")
    assert rel <= APPLY_TOL


@pytest.mark.parametrize("n,p", CASES)
def test_mx_apply_bf16x3_error_vs_oracle(torch_dev, n, p):
    torch = torch_dev
    _say(f"[mx apply bf16x3] n={n} p={p}")
    od, K, mesh, disc = _setup(n, p)
    x = random_vector((mesh.ne, disc.nphi), seed=800 + n + p).astype(np.float32)
    want = solve.schur_apply(K, x.astype(np.float64))
    got = disc.sld_schur_apply_mx(torch.from_numpy(x).to("cuda:0"), "bf16x3").cpu().numpy()
    rel = _rel(got.astype(np.float64), want)
    _say(f"    rel L2 vs FP64 oracle {rel:.2e}")
    assert rel <= BF3_TOL


def test_mx_apply_refuses_walls(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import sld
    od, K, mesh, disc = _setup(6, 2, periodic=False)
    x = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sld.SldError):
        disc.sld_schur_apply_mx(x, "f64")


@pytest.mark.parametrize("n,p", [(3, 2), (12, 3), (20, 4), (45, 3)])
def test_mx_cg_matches_oracle_and_vector_units(torch_dev, n, p):
    torch = torch_dev
    _say(f"[mx cg] n={n} p={p}")
    od, K, mesh, disc = _setup(n, p)
    f = random_fourier_field(17, kmax=4)
    b = solve.divergence(od, f(od.dual_node_xy()).transpose(0, 2, 1))
    x_or, info = solve.cg(K, b, tol=1e-13)
    x_or = solve.gauge(od, x_or)
    bt = torch.from_numpy(b).to("cuda:0")
    res = {}
    for engine in ("mfma", "valu"):
        for prec, rtol in (("fp64", 1e-12), ("mixed", 1e-11)):
            pg, rep = disc.sld_cg_solve(bt, rtol=rtol, maxit=40000, graph_block=16,
                                        precision=prec, engine=engine)
            err = _rel(pg.cpu().numpy(), x_or)
            _say(f"    {engine} {prec}: {rep['iters']} iterations, {rep['status']}, "
                 f"rel res {rep['rel_res_true']:.2e}, error vs oracle {err:.2e}")
            assert rep["status"] == "SLD_OK" and rep["converged"]
            assert err <= SOLVE_TOL
            res[(engine, prec)] = pg.cpu().numpy()
    # deterministic: the same MFMA solve twice, bitwise
    p2, _ = disc.sld_cg_solve(bt, rtol=1e-12, maxit=40000, graph_block=16, engine="mfma")
    assert np.array_equal(p2.cpu().numpy(), res[("mfma", "fp64")])
