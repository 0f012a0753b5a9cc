"""GPU parity of sld_sl_advect (Section 3.5) against the oracle's cell-by-cell walk and
Gauss-point projection, element by element, on seeded smooth velocities large enough that
the characteristics cross several cells; periodic and walled boxes, degrees 1..4, several
fields at once; and at the 128x128x2, p = 3 size on sampled triangles."""
import sys

import numpy as np
import pytest

from oracle import advect
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field, random_vector

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _case(n, p, periodic, seed):
    from paper_2401_17806_amd import sld
    length = 2 * np.pi if periodic else 1.0
    xy, tri, per = lattice_mesh(n, seed=seed, periodic=periodic, length=length)
    od = OracleDisc(OracleMesh(xy, tri, per), p)
    mesh = sld.Mesh(xy, tri, per, device=0)
    return od, mesh, sld.Disc(mesh, p), length / n


def _velocity(od, seed, h, cells):
    f = random_fourier_field(seed, kmax=3, length=(2 * np.pi if od.mesh.period is not None else 1.0))
    vb = advect.nodal_velocity(od, f)
    vmax = np.abs(vb).max()
    dt = cells * h / vmax
    return vb, dt


def _to(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n,p,periodic,nc", [(5, 1, True, 1), (5, 2, True, 2), (5, 3, True, 1),
                                             (4, 4, True, 1), (5, 2, False, 1), (6, 3, True, 3),
                                             (5, 3, False, 2)])
def test_sl_advect_parity(torch_dev, n, p, periodic, nc):
    torch = torch_dev
    _say(f"[sl_advect] n={n} p={p} periodic={periodic} nc={nc}")
    od, mesh, disc, h = _case(n, p, periodic, seed=20 + n + p)
    vb, dt = _velocity(od, 30 + p, h, cells=1.7)
    q = random_vector((mesh.ne, nc, disc.nphi), seed=40 + p + nc)
    want = advect.sl_advect(od, vb, q, dt)
    got = disc.sld_sl_advect(_to(torch, vb), _to(torch, q), dt).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    _say(f"    max rel error {err:.2e}")
    assert err <= TOL


def test_sl_advect_rest_and_argument_checks(torch_dev):
    torch = torch_dev
    from paper_2401_17806_amd import sld
    od, mesh, disc, h = _case(4, 3, True, seed=3)
    q = _to(torch, random_vector((mesh.ne, 2, disc.nphi), seed=5))
    zero = torch.zeros(mesh.ne, 2, disc.nphi, dtype=torch.float64, device="cuda:0")
    out = disc.sld_sl_advect(zero, q, 0.3)
    assert float((out - q).abs().max()) <= 1e-12 * float(q.abs().max())
    with pytest.raises(sld.SldError):
        disc.sld_sl_advect(zero, q, 0.3, out=q)
    with pytest.raises(sld.SldError):
        disc.sld_sl_advect(zero, q, float("nan"))


def test_sl_advect_fullsize_sampled(torch_dev):
    """128x128x2, p = 3 (the pressure-stage bench mesh), three fields, CFL about 1: 128
    sampled triangles against the oracle."""
    torch = torch_dev
    _say("[sl_advect fullsize] n=128 p=3")
    od, mesh, disc, h = _case(128, 3, True, seed=2)
    vb, dt = _velocity(od, 77, h, cells=1.0)
    q = random_vector((mesh.ne, 3, disc.nphi), seed=78)
    got = disc.sld_sl_advect(_to(torch, vb), _to(torch, q), dt).cpu().numpy()
    ids = np.sort(np.random.default_rng(6).choice(mesh.ne, 128, replace=False))
    want = advect.sl_advect_rows(od, vb, q, dt, ids)
    err = np.abs(got[ids] - want).max() / np.abs(want).max()
    _say(f"    sampled max rel error {err:.2e}")
    assert err <= TOL
