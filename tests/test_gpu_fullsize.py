"""GPU parity at the full workload sizes, in the launch configuration bench.py times
(default grid, graph blocks of 64 iterations).  The oracle cannot assemble or solve these
systems quickly, so outputs are checked on samples it computes one by one:
  * the Schur apply on 256 sampled triangles (rows of eq. pressure_final, oracle.schur_rows);
  * the 128x128x2, p = 3 pressure against the oracle's own solve at 512 sampled DOFs
    (tests/golden/c2_pressure_sample.txt, written by make_c2_sample.py from the oracle);
  * the 512x512x2, p = 3 pressure, FP64 and mixed, against the oracle's solve at 1024 sampled
    DOFs (tests/golden/c3_pressure_sample.txt, written by make_c3_sample.py from the oracle),
    and the report of a tolerance below the FP64 rounding floor of the recomputed residual.
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import solve
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field, random_vector

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


def _setup(n, p, seed, walls=False):
    key = (n, p, seed, walls)
    if key not in _CACHE:
        from paper_2401_17806_amd import sld
        xy, tri, per = lattice_mesh(n, seed=seed, periodic=not walls,
                                    length=(1.0 if walls else 2 * np.pi))
        od = OracleDisc(OracleMesh(xy, tri, per), p)
        mesh = sld.Mesh(xy, tri, per, device=0)
        _CACHE[key] = (od, mesh, sld.Disc(mesh, p))
    return _CACHE[key]


def _rhs(torch, od, disc, n, rhs_seed):
    """The bench right-hand side: (1/(a_ss dt)) D v*, v* a seeded Fourier field."""
    coef = A_SS * 0.5 * (2 * math.pi / n)
    vs = random_fourier_field(rhs_seed, kmax=8)(od.dual_node_xy()).transpose(0, 2, 1)
    vt = torch.from_numpy(np.ascontiguousarray(vs)).to("cuda:0")
    return disc.sld_pressure_rhs(vt, 1.0 / coef)


@pytest.mark.parametrize("n,p,seed,walls", [(128, 3, 2, False), (512, 3, 3, False),
                                             (256, 4, 1005, False), (256, 2, 4, True)])
def test_fullsize_schur_apply_sampled_rows(torch_dev, n, p, seed, walls):
    torch = torch_dev
    _say(f"[fullsize apply] n={n} p={p} walls={walls}")
    od, mesh, disc = _setup(n, p, seed, walls)
    x = random_vector((mesh.ne, disc.nphi), seed=500 + n)
    got = disc.sld_schur_apply(torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    ids = np.sort(np.random.default_rng(n).choice(mesh.ne, 256, replace=False))
    if walls:  # make sure wall triangles are among the samples
        ids = np.unique(np.concatenate([ids, np.arange(0, 2 * n, 3)]))
    want = solve.schur_rows(od, x, ids)
    rel = np.linalg.norm(got[ids] - want) / np.linalg.norm(want)
    _say(f"    sampled rel L2 {rel:.2e}")
    assert rel <= 1e-12


def _read_sample(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.fail(f"missing oracle sample {path} (tests/golden/make_*.py writes it)")
    idx, val, head = [], [], {}
    for line in open(path):
        if line.startswith("#"):
            parts = line[1:].split()
            for k in range(0, len(parts) - 1):
                if parts[k] in ("maxabs_p", "norm2_p", "rel_res_true"):
                    head[parts[k]] = float(parts[k + 1])
            continue
        i, v = line.split()
        idx.append(int(i))
        val.append(float(v))
    return np.array(idx), np.array(val), head


def _sample_err(p, sample):
    idx, val, head = sample
    got = p.cpu().numpy().ravel()[idx]
    return np.abs(got - val).max() / head["maxabs_p"]


def test_fullsize_c2_pressure_matches_oracle_sample(torch_dev):
    """128x128x2, p = 3, FP64 to a recomputed residual of 1e-11 (the FP64 rounding floor of
    K x - b is about 3e-12 here), graph blocks of 256: converged, and the pressure at 512 sampled
    DOFs equals the oracle's to 1e-9 of its max norm."""
    torch = torch_dev
    _say("[fullsize c2 solve]")
    od, mesh, disc = _setup(128, 3, 2)
    b = _rhs(torch, od, disc, 128, 102)
    p_gpu, rep = disc.sld_cg_solve(b, rtol=1e-11, graph_block=256, maxit=100000)
    _say("   report", rep)
    err = _sample_err(p_gpu, _read_sample("c2_pressure_sample.txt"))
    _say(f"    sampled max error / max|p| = {err:.2e}")
    assert rep["status"] == "SLD_OK" and rep["converged"] and rep["rel_res_true"] <= 1e-11
    assert err <= 1e-9


def test_fullsize_c3_fp64_and_mixed_match_oracle_sample(torch_dev):
    """512x512x2, p = 3 (the bench workload): FP64 and mixed precision, each to a recomputed
    residual of 1e-10, converge, and each pressure equals the oracle's at 1024 sampled DOFs
    (tests/golden/c3_pressure_sample.txt) to 1e-9 of its max norm; the gauge holds.  The FP32
    process of the mixed form (centred operator inputs, a reliable update at least every 512
    iterations) needs at most 1.2x the FP64 iterations (measured 1.10x; 1.64x without them)."""
    torch = torch_dev
    _say("[fullsize c3 solves]")
    od, mesh, disc = _setup(512, 3, 3)
    b = _rhs(torch, od, disc, 512, 103)
    sample = _read_sample("c3_pressure_sample.txt")
    w = od.main_weights()
    iters = {}
    for prec in ("fp64", "mixed"):
        # graph blocks of 256, as bench.py runs both forms (the FP32 blocks are capped at 128)
        p, rep = disc.sld_cg_solve(b, rtol=1e-10, precision=prec, graph_block=256, maxit=200000)
        err = _sample_err(p, sample)
        _say(f"   {prec} report {rep}; sampled max error / max|p| = {err:.2e}")
        assert rep["status"] == "SLD_OK" and rep["converged"] and rep["rel_res_true"] <= 1e-10
        assert err <= 1e-9
        ph = p.cpu().numpy()
        assert abs((w * ph).sum()) <= 1e-12 * np.abs(ph).max() * w.sum()
        iters[prec] = rep["iters"]
    assert iters["mixed"] <= 1.2 * iters["fp64"]


def test_fullsize_c3_below_the_fp64_floor_is_reported(torch_dev):
    """512x512x2, p = 3, rtol 1e-11: the FP64 rounding error of the recomputed residual K x - b
    itself is about 4e-11 of |b| here, so neither form can confirm 1e-11.  Both stop at that
    floor with SLD_E_NOCONV and converged false, the report names the floor, and the iterate
    still equals the oracle's at the sampled DOFs to 1e-9."""
    torch = torch_dev
    _say("[fullsize c3 floor]")
    od, mesh, disc = _setup(512, 3, 3)
    b = _rhs(torch, od, disc, 512, 103)
    sample = _read_sample("c3_pressure_sample.txt")
    for prec in ("fp64", "mixed"):
        p, rep = disc.sld_cg_solve(b, rtol=1e-11, precision=prec, graph_block=256 if prec == "fp64"
                                   else 64, maxit=200000)
        err = _sample_err(p, sample)
        _say(f"   {prec} report {rep}; sampled max error / max|p| = {err:.2e}")
        assert rep["status"] == "SLD_E_NOCONV" and not rep["converged"]
        assert 1e-11 < rep["rel_res_true"] <= 1e-10
        assert err <= 1e-9


def test_fullsize_cavity_solve_properties(torch_dev):
    """256x256x2 walled unit box, p = 2 (the cavity mesh), FP64 solve to a recomputed residual of
    1e-11 (the FP64 rounding floor of K x - b is about 2e-12 here): converged, the residual on
    sampled rows (wall triangles included) computed by the oracle row by row, zero-mean
    gauge."""
    torch = torch_dev
    _say("[fullsize cavity solve]")
    od, mesh, disc = _setup(256, 2, 4, walls=True)
    coef = A_SS * 0.5 * (1.0 / 256)
    vs = random_fourier_field(104, kmax=8, length=1.0)(od.dual_node_xy()).transpose(0, 2, 1)
    b = disc.sld_pressure_rhs(torch.from_numpy(np.ascontiguousarray(vs)).to("cuda:0"), 1.0 / coef)
    p64, rep = disc.sld_cg_solve(b, rtol=1e-11, graph_block=64, maxit=200000)
    _say("   report", rep)
    assert rep["status"] == "SLD_OK" and rep["converged"] and rep["rel_res_true"] <= 1e-11
    bh = b.cpu().numpy()
    bh = bh - bh.mean()
    ph = p64.cpu().numpy()
    ids = np.unique(np.concatenate([np.arange(0, 512, 2),
                                    np.random.default_rng(9).choice(mesh.ne, 256, replace=False)]))
    res = bh[ids] - solve.schur_rows(od, ph, ids)
    rel = np.linalg.norm(res) / np.linalg.norm(bh[ids])
    _say(f"    sampled true residual {rel:.2e}")
    assert rel <= 1e-9
    w = od.main_weights()
    assert abs((w * ph).sum()) <= 1e-12 * np.abs(ph).max() * w.sum()


def _cavity_setup(torch):
    from oracle import imex as oimex
    from paper_2401_17806_amd import sld
    n, p = 256, 2
    xy, tri, per = lattice_mesh(n, seed=4, periodic=False, length=1.0)
    od = OracleDisc(OracleMesh(xy, tri, per), p)
    disc = sld.Disc(sld.Mesh(xy, tri, per, device=0), p)
    m = od.mesh
    mid = 0.5 * (m.A + m.B)
    side = (~m.interior) & ((np.abs(mid[:, 0]) < 1e-12) | (np.abs(mid[:, 0] - 1.0) < 1e-12))
    t = np.arange(p + 1) / p
    enodes = m.A[:, None, :] + t[None, :, None] * (m.B - m.A)[:, None, :]
    vals = np.ascontiguousarray(0.5 - enodes[..., 0])
    return oimex, od, disc, side, vals


def test_fullsize_cavity_diffusion_residual_on_sampled_rows(torch_dev):
    """256x256x2 walled unit box, p = 2: the temperature diffusion solve (Dirichlet side walls
    with data, adiabatic top and bottom) satisfies (Mbar - c K_W) x = Mbar f + c G_b on sampled
    rows, wall triangles included, computed by the oracle row by row."""
    torch = torch_dev
    _say("[fullsize cavity diffusion]")
    oimex, od, disc, side, vals = _cavity_setup(torch)
    m = od.mesh
    f = random_vector((m.ne, od.nphi), seed=91)
    c = 0.5 / 256 / math.sqrt(1e5 * 0.71)
    x, rep = disc.sld_viscous_solve(torch.from_numpy(f).to("cuda:0"), c,
                                    wall_dirichlet=torch.from_numpy(side.astype(np.uint8)).to("cuda:0"),
                                    wall_values=torch.from_numpy(vals).to("cuda:0"), rtol=1e-12)
    _say("   report", rep)
    xh = x.cpu().numpy()
    ids = np.unique(np.concatenate([np.nonzero(np.isin(np.arange(m.ne), m.left[side]))[0][::7],
                                    np.random.default_rng(3).choice(m.ne, 256, replace=False)]))
    Mb = od.main_mass()[ids]
    gb_all = oimex.dirichlet_rhs(od, side, lambda q: 0.5 - q[..., 0])
    lhs = np.einsum("ekl,el->ek", Mb, xh[ids]) - c * oimex.walls_rows(od, xh, ids, side)
    rhs = np.einsum("ekl,el->ek", Mb, f[ids]) + c * gb_all[ids]
    rel = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
    _say(f"    sampled residual {rel:.2e} over {ids.size} rows")
    assert rep["converged"] and rel <= 1e-10


def test_fullsize_cavity_steps_properties(torch_dev):
    """256x256x2 walled unit box, p = 2, Ra = 1e5, Pr = 0.71, twenty R = 0 steps from rest with
    the mixed-precision pressure solve: divergence-free, zero velocity on the wall cells, the
    temperature within the wall values up to a small overshoot, and the hot side rising."""
    torch = torch_dev
    from paper_2401_17806_amd import sld
    _say("[fullsize cavity steps]")
    oimex, od, disc, side, vals = _cavity_setup(torch)
    m = od.mesh
    nu, kappa = math.sqrt(0.71 / 1e5), 1.0 / math.sqrt(1e5 * 0.71)
    v = torch.zeros(disc.dual_shape, dtype=torch.float64, device="cuda:0")
    T = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
    p = torch.zeros(disc.main_shape, dtype=torch.float64, device="cuda:0")
    st = sld.State(disc)
    mask = torch.from_numpy(side.astype(np.uint8)).to("cuda:0")
    vt = torch.from_numpy(vals).to("cuda:0")
    for k in range(20):
        rep = st.sld_boussinesq_step(v, T, p, 0.5 / 256, nu, kappa, 1.0, temp_dirichlet=mask,
                                     temp_values=vt, rtol=1e-10, precision="mixed",
                                     graph_block=64)
        assert rep["status"] == "SLD_OK"
        dv = float(torch.linalg.norm(disc.sld_divergence(v)))
        assert dv <= 1e-9 * max(float(v.abs().max()), 1e-300) * math.sqrt(m.ne)
        if k % 5 == 4:
            _say(f"    step {k}: |Dv| {dv:.2e} max|v| {float(v.abs().max()):.3e} "
                 f"T [{float(T.min()):.5f}, {float(T.max()):.5f}] p iters {rep['pressure']['iters']} "
                 f"{rep['seconds'] * 1e3:.0f} ms")
    vh = v.cpu().numpy()
    assert np.abs(vh[~m.interior]).max() == 0.0
    assert -0.52 <= float(T.min()) and float(T.max()) <= 0.52
    dn = od.dual_node_xy()
    xs = dn[..., 0]
    inner = m.interior[:, None] & np.isfinite(xs)
    vy = vh[:, 1, :]
    assert vy[inner & (xs < 0.05)].mean() > 0.0 > vy[inner & (xs > 0.95)].mean()
