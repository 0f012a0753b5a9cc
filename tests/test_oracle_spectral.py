"""Oracle pins from the spectrum of K and from the choice of basis (no GPU).

* Laplace eigenvalues on the periodic box (closed form).  K is the discrete Laplacian of the
  main grid (eq. pressure_final: D Mhat^{-1} Q approximates div grad; Section 3.3), so the
  generalized eigenproblem -K v = lambda Mbar v on the periodic [0, 2 pi]^2 has its smallest
  nonzero eigenvalues near those of -Laplace on that torus: |m|^2 for integer m, i.e. 1 (four
  times: m = (+-1, 0), (0, +-1)) and 2 (four times: m = (+-1, +-1)).  On the unjittered
  split-square lattice the error decays at order at least 2p under refinement (the eigenvalue
  error of a degree-p discretisation), which a wrong sign, scale or dropped term in any block
  of K would break.
* Basis independence (the survey's reading C1).  Moving nodes of the main basis (the interior
  node at p = 3, the hypotenuse's midpoint at p = 2) changes the basis but not the space, so K
  becomes B^T K B and a function-level right-hand side b_k = int phi_k f becomes B^T b: the
  pressure as a function is unchanged.  The oracle's K is assembled from its integral
  definitions in physical space, so this checks that nothing in it relies on the equispaced
  node positions.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import basis, solve
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from paper_2401_17806_amd.inputs import lattice_mesh


def _laplace_eigs(n, p):
    xy, tri, per = lattice_mesh(n, jitter=0.0, seed=1)
    d = OracleDisc(OracleMesh(xy, tri, per), p)
    K = solve.assemble_K(d)
    import scipy.sparse as sp
    M = sp.block_diag(list(d.main_mass()), format="csc")
    lam = spla.eigsh((-K).tocsc(), k=12, M=M, sigma=0.7, which="LM", return_eigenvectors=False)
    return np.sort(lam)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_laplace_eigenvalues_on_periodic_box(p):
    errs = []
    for n in (8, 16):
        lam = _laplace_eigs(n, p)
        one = lam[(lam > 0.5) & (lam < 1.5)]
        two = lam[(lam > 1.5) & (lam < 2.5)]
        # exactly one (numerically) zero eigenvalue, the constants
        assert (np.abs(lam) < 1e-8).sum() == 1, lam
        assert one.size == 4 and two.size == 4, lam
        errs.append(max(np.abs(one - 1.0).max(), np.abs(two - 2.0).max() / 2.0))
    order = math.log2(errs[0] / errs[1])
    assert errs[1] < 10.0 ** (-p - 0.5) and order > 2 * p - 0.5, (errs, order)


def _load_vector(d, f):
    """b_k = int_{T_i} phi_k f dx by the disc's triangle rule (exact up to the rule's order)."""
    m = d.mesh
    u, v = d.tri_pts[:, 0], d.tri_pts[:, 1]
    P = m.P
    x = P[:, None, 0] + u[None, :, None] * (P[:, None, 1] - P[:, None, 0]) + \
        v[None, :, None] * (P[:, None, 2] - P[:, None, 0])
    ph = basis.phi(d.p, u, v)  # [q, k]
    return np.einsum("q,e,qk,eq->ek", d.tri_w, 2.0 * m.area, ph, f(x))


def _pressure_function(n, p, nodes_override):
    """Zero-mean solution of K p = b, b the load of f, evaluated at fixed reference points of
    every triangle; nodes_override replaces the main node set of degree p (or None)."""
    saved = basis.main_nodes
    basis._COEF_CACHE.clear()
    if nodes_override is not None:
        basis.main_nodes = lambda q: nodes_override if q == p else saved(q)
    try:
        xy, tri, per = lattice_mesh(n, seed=5)
        d = OracleDisc(OracleMesh(xy, tri, per), p)
        K = solve.assemble_K(d)
        f = lambda x: np.sin(x[..., 0]) * np.cos(2 * x[..., 1]) + 0.5 * np.cos(3 * x[..., 0])
        b = _load_vector(d, f)
        # the load of f - c with c its discrete mean: sum_k b_k = 0 exactly in every Lagrange
        # basis (a Euclidean projection of b onto 1^perp would depend on the basis)
        w = d.main_weights()
        b = b - w * (b.sum() / w.sum())
        x = solve.gauge(d, solve.dense_bordered_solve(K, b))
        ref = np.array([[0.1, 0.2], [0.6, 0.15], [0.25, 0.5], [1 / 3, 1 / 3], [0.05, 0.9]])
        return np.einsum("sk,ek->es", basis.phi(p, ref[:, 0], ref[:, 1]), x)
    finally:
        basis.main_nodes = saved
        basis._COEF_CACHE.clear()


@pytest.mark.parametrize("p", [2, 3])
def test_pressure_function_is_basis_independent(p):
    nodes = basis.main_nodes(p).copy()
    idx = basis.main_index(p)
    if p == 3:
        nodes[idx[(1, 1)]] = [0.29, 0.37]          # the interior node
    else:
        nodes[idx[(1, 1)]] = [0.43, 0.57]          # along the hypotenuse
    a = _pressure_function(4, p, None)
    b = _pressure_function(4, p, nodes)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()
