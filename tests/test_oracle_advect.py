"""Pins of the oracle's semi-Lagrangian advection (Section 3.5) against what the mathematics
fixes: a field at rest is reproduced exactly; on the unjittered lattice a shift by one lattice
vector is an exact permutation of the DOFs; a linear field in a constant velocity is
transported exactly; the walk lands on x_g - dt v (modulo the period) through several cells."""
import numpy as np
import pytest

from oracle import advect
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh, random_vector


def _disc(n, p, periodic=True, jitter=0.1, seed=4):
    xy, tri, per = lattice_mesh(n, seed=seed, periodic=periodic, jitter=jitter,
                                length=(2 * np.pi if periodic else 1.0))
    return OracleDisc(OracleMesh(xy, tri, per), p)


def _const_velocity(d, v):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(v, float)[None, :, None],
                                                (d.mesh.ne, 2, d.nphi)))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_rest_is_identity(p):
    d = _disc(3, p)
    q = random_vector((d.mesh.ne, 2, d.nphi), seed=p)
    out = advect.sl_advect(d, np.zeros((d.mesh.ne, 2, d.nphi)), q, 0.7)
    assert np.abs(out - q).max() <= 1e-12 * np.abs(q).max()


@pytest.mark.parametrize("p", [1, 3])
def test_lattice_shift_is_a_permutation(p):
    n = 4
    d = _disc(n, p, jitter=0.0)
    h = 2 * np.pi / n
    dt = 0.37
    q = random_vector((d.mesh.ne, 1, d.nphi), seed=11)
    out = advect.sl_advect(d, _const_velocity(d, (h / dt, 0.0)), q, dt)
    # square s = a + n b owns triangles 2s, 2s+1; the foot of square (a, b) is in (a-1, b)
    for s in range(n * n):
        a, b = s % n, s // n
        src = ((a - 1) % n) + n * b
        for t in (0, 1):
            assert np.abs(out[2 * s + t] - q[2 * src + t]).max() <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 4])
def test_linear_field_in_constant_velocity_is_exact(p):
    n = 6
    d = _disc(n, p, periodic=False)
    h = 1.0 / n
    dt = 0.1
    v = np.array([0.3 * h / dt, -0.2 * h / dt])
    c = np.array([0.4, -1.3, 2.1])
    xy = d.main_node_xy()
    q = (c[0] + c[1] * xy[..., 0] + c[2] * xy[..., 1])[:, None, :]
    out = advect.sl_advect(d, _const_velocity(d, v), q, dt)
    want = (c[0] + c[1] * (xy[..., 0] - dt * v[0]) + c[2] * (xy[..., 1] - dt * v[1]))[:, None, :]
    P = d.mesh.P
    # triangles whose feet cannot reach a wall
    far = (P[..., 0].min(axis=1) >= h) & (P[..., 1].max(axis=1) <= 1.0 - h)
    assert far.sum() > 10
    assert np.abs(out[far] - want[far]).max() <= 1e-12


def test_walk_lands_on_the_straight_line_foot():
    n, p = 5, 2
    d = _disc(n, p, seed=8)
    h = 2 * np.pi / n
    v = np.array([1.7, -0.9])
    dt = 2.5 * h / np.linalg.norm(v)           # several cell crossings per point
    vb = _const_velocity(d, v)
    pts, _ = advect.sl_rule(p)
    per = d.mesh.period
    crossings = 0
    for i in range(0, d.mesh.ne, 3):
        for g in range(pts.shape[0]):
            xg = d.mesh.P[i, 0] + d.Jmain[i] @ pts[g]
            c, (a, b), steps = advect.walk(d, vb, i, pts[g], dt)
            foot = d.mesh.P[c, 0] + d.Jmain[c] @ np.array([a, b])
            k = (foot - (xg - dt * v)) / per
            assert np.abs(k - np.round(k)).max() <= 1e-9
            crossings += steps - 1
    assert crossings > 50
