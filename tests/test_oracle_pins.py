"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them compares the oracle
with itself: they use closed forms, textbook matrices, the paper's worked
example, exact polynomial reproduction, structural identities, brute-force
dense solves and convergence at the expected order.
"""
import math
import os

import numpy as np
import pytest

from oracle import basis, solve
from oracle.mesh import OracleMesh, MeshError
from oracle.operators import OracleDisc
from oracle.quadrature import gauss_legendre_01, triangle_rule
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field, random_vector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_triangle_rule_exact_on_monomials(n):
    pts, w = triangle_rule(n)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = float((w * pts[:, 0] ** a * pts[:, 1] ** b).sum())
            assert abs(got - exact) <= 1e-15 + 1e-13 * exact


@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_gauss_legendre_exact(n):
    t, w = gauss_legendre_01(n)
    for k in range(2 * n):
        assert abs((w * t ** k).sum() - 1.0 / (k + 1)) < 1e-14


# ---------------------------------------------------------------- basis (Section 3.2)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_main_basis_lagrange_unity(p):
    nd = basis.main_nodes(p)
    V = basis.phi(p, nd[:, 0], nd[:, 1])
    assert np.abs(V - np.eye(basis.n_phi(p))).max() < 1e-12
    rng = np.random.default_rng(0)
    x = rng.random(50)
    y = rng.random(50) * (1 - x)
    assert np.abs(basis.phi(p, x, y).sum(-1) - 1).max() < 1e-12
    assert np.abs(basis.grad_phi(p, x, y).sum(-2)).max() < 1e-10
    assert basis.n_phi(p) == (p + 1) * (p + 2) // 2


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_dual_basis_lagrange_unity_c0(p):
    nd = basis.dual_nodes(p)
    V = basis.psi(p, nd[:, 0], nd[:, 1])
    assert np.abs(V - np.eye(basis.n_psi(p))).max() < 1e-12
    assert basis.n_psi(p) == (p + 1) ** 2
    rng = np.random.default_rng(1)
    x, y = rng.random(100), rng.random(100)
    assert np.abs(basis.psi(p, x, y).sum(-1) - 1).max() < 1e-12
    # C0 across the diagonal xi + eta = 1: limits from both sides agree
    t = rng.random(40)
    eps = 1e-9
    below = basis.psi(p, t - eps, 1 - t - eps)
    above = basis.psi(p, t + eps, 1 - t + eps)
    assert np.abs(below - above).max() < 1e-6


def test_dual_basis_p1_worked_example():
    """The p = 1 example of Section 3.2, written out in tests/golden/dual_basis_p1.txt."""
    rows = _read_rows("dual_basis_p1.txt")
    rng = np.random.default_rng(2)
    x, y = rng.random(200), rng.random(200)
    low = (x + y) <= 1
    ps = basis.psi(1, x, y)
    ph_low = basis.phi(1, x, y)
    ph_up = basis.phi(1, 1 - y, 1 - x)
    for k, branch, m in rows:
        k, m = int(k) - 1, int(m) - 1
        mask = low if branch == "lower" else ~low
        ref = np.zeros(200) if m < 0 else (ph_low if branch == "lower" else ph_up)[:, m]
        assert np.abs(ps[mask, k] - ref[mask]).max() < 1e-14


# ---------------------------------------------------------------- mass matrices (Section 3.4.1)
def _single(tri_xy):
    return OracleMesh(np.asarray(tri_xy, float), np.array([[0, 1, 2]]), None)


def test_p1_mass_matrix_textbook():
    rows = np.array(_read_rows("p1_mass_matrix.txt"), dtype=float) / 24.0
    d = OracleDisc(_single([[0, 0], [1, 0], [0, 1]]), 1)
    assert np.abs(d.main_mass()[0] - rows).max() < 1e-15


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_main_mass_scaling_and_area(p):
    """eq. MassMatrixM: Mbar_i = A_i Mbar_ref with A_i = 2|T_i|; 1^T Mbar_i 1 = |T_i|."""
    ref = OracleDisc(_single([[0, 0], [1, 0], [0, 1]]), p).main_mass()[0]
    tri = [[0.3, -0.2], [2.1, 0.4], [0.9, 1.7]]
    d = OracleDisc(_single(tri), p)
    M = d.main_mass()[0]
    area = d.mesh.area[0]
    assert abs(M.sum() - area) < 1e-13
    assert np.abs(M - 2 * area * ref).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_dual_mass_invariants(p):
    """eq. MassMatrixD: 1^T Mhat_j 1 = |T_lj| + |T_rj| = (|T_l| + |T_r|)/3; SPD; sum |R_j| = |Omega|."""
    xy, tri, per = lattice_mesh(4, seed=3)
    m = OracleMesh(xy, tri, per)
    d = OracleDisc(m, p)
    blk = d.edge_blocks(np.arange(m.nd))
    tot = blk["Mhat"].sum(axis=(1, 2))
    assert np.abs(tot - (m.area[m.left] + m.area[m.right]) / 3).max() < 1e-13
    assert abs(tot.sum() - (2 * math.pi) ** 2) < 1e-11
    ev = np.linalg.eigvalsh(blk["Mhat"])
    assert ev.min() > 0
    # Mhat_j = A_lj M^L + A_rj M^R with fixed reference matrices: normalised blocks agree
    bmin = blk["Mhat"] / tot[:, None, None]
    assert np.isfinite(bmin).all()


# ---------------------------------------------------------------- operators (Section 3.3)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_divergence_is_minus_gradient_transpose(p):
    """D = -Q^T (Section 3.3 after eq. ad5), from two separate integrations."""
    xy, tri, per = lattice_mesh(4, seed=5)
    m = OracleMesh(xy, tri, per)
    blk = OracleDisc(m, p).edge_blocks(np.arange(m.nd))
    scale = np.abs(blk["Ql"]).max()
    assert np.abs(blk["Dl"] + blk["Ql"].transpose(0, 2, 1, 3)).max() < 1e-14 * scale * 10
    assert np.abs(blk["Dr"] + blk["Qr"].transpose(0, 2, 1, 3)).max() < 1e-14 * scale * 10


@pytest.mark.parametrize("n", [3, 4])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_schur_operator_symmetric_nullspace_semidefinite(n, p):
    """eq. pressure_final: K symmetric, K 1 = 0, -K PSD with a one-dimensional kernel."""
    xy, tri, per = lattice_mesh(n, seed=7)
    d = OracleDisc(OracleMesh(xy, tri, per), p)
    K = solve.assemble_K(d).toarray()
    s = np.abs(K).max()
    assert np.abs(K - K.T).max() < 1e-14 * s * 10
    assert np.abs(K.sum(axis=1)).max() < 1e-13 * s * 10
    ev = np.linalg.eigvalsh(-0.5 * (K + K.T))
    assert ev.min() > -1e-12 * ev.max()
    assert (np.abs(ev) < 1e-10 * ev.max()).sum() == 1


def _walls(n, p, seed=11):
    xy, tri, per = lattice_mesh(n, length=1.0, periodic=False, seed=seed)
    return OracleDisc(OracleMesh(xy, tri, per), p)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gradient_reproduces_polynomial_gradients(p):
    """eq. ad4.2: for a continuous polynomial p of degree <= p with grad p in the dual space
    (affine for p = 1, quadratic for p >= 2) the jump term vanishes and the L2 projection is
    exact: ghat_j = grad p at the dual nodes on every interior edge."""
    d = _walls(4, p)
    c = np.array([0.7, -1.3, 0.4, 2.0, -0.6, 0.9])

    def f(x):
        val = c[0] + c[1] * x[..., 0] + c[2] * x[..., 1]
        if p >= 2:
            val = val + c[3] * x[..., 0] ** 2 + c[4] * x[..., 0] * x[..., 1] + c[5] * x[..., 1] ** 2
        return val

    def gf(x):
        gx = c[1] + (2 * c[3] * x[..., 0] + c[4] * x[..., 1] if p >= 2 else 0)
        gy = c[2] + (c[4] * x[..., 0] + 2 * c[5] * x[..., 1] if p >= 2 else 0)
        z = np.zeros_like(x[..., 0])
        return np.stack([gx + z, gy + z], axis=-1)

    pm = f(d.main_node_xy())
    g = solve.gradient(d, pm)
    dn = d.dual_node_xy()
    want = gf(dn).transpose(0, 2, 1)
    inner = d.mesh.interior
    assert np.abs(g[inner] - want[inner]).max() < 1e-11


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_divergence_of_polynomial_field(p):
    """eq. D by parts: for v a global polynomial field of degree <= p,
    (D v)_i = Mbar_i (div v at the main nodes) on triangles whose three edges are interior."""
    d = _walls(4, p)
    m = d.mesh

    def v(x):
        X, Y = x[..., 0], x[..., 1]
        return np.stack([X ** p - 0.5 * Y + 0.3, 0.25 * X * Y ** (p - 1) + Y], axis=-1)

    def divv(x):
        X, Y = x[..., 0], x[..., 1]
        return p * X ** (p - 1) + 0.25 * X * (p - 1) * Y ** max(p - 2, 0) + 1.0

    vd = v(d.dual_node_xy()).transpose(0, 2, 1)
    Dv = solve.divergence(d, vd)
    M = d.main_mass()
    want = np.einsum("ekl,el->ek", M, divv(d.main_node_xy()))
    full = m.interior[m.tri_edges].all(axis=1)
    assert full.sum() > 0
    assert np.abs(Dv[full] - want[full]).max() < 1e-12


@pytest.mark.parametrize("n", [3, 4])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_cg_matches_dense_bordered_solve(n, p):
    """Plain CG (Section 3.3) against a dense direct solve of the bordered system."""
    xy, tri, per = lattice_mesh(n, seed=13)
    d = OracleDisc(OracleMesh(xy, tri, per), p)
    K = solve.assemble_K(d)
    b = solve.project_mean(random_vector((d.mesh.ne, d.nphi), seed=17))
    x, info = solve.cg(K, b, tol=1e-14)
    xd = solve.dense_bordered_solve(K, b)
    x = solve.gauge(d, x)
    xd = solve.gauge(d, xd)
    assert info["converged"]
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    assert np.linalg.norm(K @ xd.ravel() - b.ravel()) <= 1e-11 * np.linalg.norm(b)


def _hodge_error(n, p):
    xy, tri, per = lattice_mesh(n, seed=19)
    d = OracleDisc(OracleMesh(xy, tri, per), p)
    K = solve.assemble_K(d)
    v = lambda x: np.stack([-2 * np.sin(2 * x[..., 0]), -2 * np.sin(2 * x[..., 1])], -1)
    phi_m = lambda x: np.cos(2 * x[..., 0]) + np.cos(2 * x[..., 1])
    b = solve.divergence(d, v(d.dual_node_xy()).transpose(0, 2, 1))
    x, info = solve.cg(K, b, tol=1e-13)
    x = solve.gauge(d, x)
    assert info["converged"]
    return np.sqrt(((x - phi_m(d.main_node_xy())) ** 2).mean())


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_pressure_of_gradient_field_converges(p):
    """Helmholtz-Hodge closed form: for v* = grad phi_m, phi_m = cos 2x + cos 2y (zero mean),
    the pressure of eq. pressure_final with b = D v* converges to phi_m at order about p + 1."""
    e1 = _hodge_error(6, p)
    e2 = _hodge_error(12, p)
    order = math.log2(e1 / e2)
    assert order > p + 0.5, (e1, e2, order)


@pytest.mark.parametrize("p", [1, 3])
def test_velocity_correction_is_divergence_free(p):
    """eq. ins.1 after eq. nc.2: v = v* - c Mhat^-1 Q p with K p = D v* / c gives D v = 0."""
    xy, tri, per = lattice_mesh(6, seed=23)
    d = OracleDisc(OracleMesh(xy, tri, per), p)
    K = solve.assemble_K(d)
    f = random_fourier_field(29, kmax=4)
    vs = f(d.dual_node_xy()).transpose(0, 2, 1)
    coef = 0.37
    b = solve.pressure_rhs(d, vs, 1.0 / coef)
    x, info = solve.cg(K, b, tol=1e-14)
    v = solve.velocity_correction(d, vs, x, coef)
    Dv = solve.divergence(d, v)
    assert np.linalg.norm(Dv) <= 1e-11 * np.linalg.norm(solve.divergence(d, vs))


def test_gauge_zero_mean():
    xy, tri, per = lattice_mesh(4, seed=31)
    d = OracleDisc(OracleMesh(xy, tri, per), 2)
    x = random_vector((d.mesh.ne, d.nphi), seed=37) + 5.0
    g = solve.gauge(d, x)
    assert abs((d.main_weights() * g).sum()) < 1e-12
    c = solve.gauge(d, np.full_like(x, 3.0))
    assert np.abs(c).max() < 1e-13


def test_mesh_rejects_bad_input():
    xy, tri, per = lattice_mesh(3, seed=1)
    bad = tri.copy()
    bad[0] = bad[0][::-1]
    with pytest.raises(MeshError):
        OracleMesh(xy, bad, per)


@pytest.mark.parametrize("n,periodic", [(3, True), (5, False)])
def test_mesh_counts(n, periodic):
    """Euler characteristic: periodic N_d = N_e + N_v; disk N_d = N_e + N_v - 1."""
    xy, tri, per = lattice_mesh(n, seed=1, periodic=periodic)
    m = OracleMesh(xy, tri, per)
    assert m.ne == 2 * n * n
    if periodic:
        assert m.nd == m.ne + m.nv and m.interior.all()
    else:
        assert m.nd == m.ne + m.nv - 1
    # every interior edge normal points from l to r: centroid difference has positive projection
    d = (m.centroid[m.right] - m.shift - m.centroid[m.left])[m.interior]
    assert ((d * m.normal[m.interior]).sum(axis=1) > 0).all()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gradient_of_piecewise_constant_pressure(p):
    """eq. ad4.2, distributional gradient across Gamma_j: for a pressure that is constant c_i
    on each triangle only the jump term survives, and integrating ghat_j over the dual cell
    gives the divergence-theorem value int_{R_j} ghat = (c_r - c_l) |Gamma_j| n_j."""
    xy, tri, per = lattice_mesh(4, seed=41)
    m = OracleMesh(xy, tri, per)
    d = OracleDisc(m, p)
    c = random_vector(m.ne, seed=43)
    pm = np.repeat(c[:, None], d.nphi, axis=1)
    g = solve.gradient(d, pm)  # [nd, 2, npsi]
    Mh = d.edge_blocks(np.arange(m.nd))["Mhat"]
    integral = np.einsum("ekl,eck->ec", Mh, g)  # sum_k (int psi_k) ghat_k
    want = (c[m.right] - c[m.left])[:, None] * m.edge_len[:, None] * m.normal
    assert np.abs(integral - want).max() < 1e-12


def test_planted_jump_sign_error_is_caught(monkeypatch):
    """A flipped edge normal (jump term of the wrong sign in both Q and D) keeps K symmetric
    and singular but must fail the piecewise-constant gradient pin."""
    xy, tri, per = lattice_mesh(4, seed=41)
    m = OracleMesh(xy, tri, per)
    m.normal = -m.normal
    d = OracleDisc(m, 1)
    c = random_vector(m.ne, seed=43)
    g = solve.gradient(d, np.repeat(c[:, None], d.nphi, axis=1))
    Mh = d.edge_blocks(np.arange(m.nd))["Mhat"]
    integral = np.einsum("ekl,eck->ec", Mh, g)
    want = (c[m.right] - c[m.left])[:, None] * m.edge_len[:, None] * (-m.normal)
    assert np.abs(integral - want).max() > 1e-3


@pytest.mark.parametrize("periodic", [True, False])
def test_schur_rows_equal_assembled_rows(periodic):
    """Sampled rows of K p, computed edge by edge without assembly (used at full size), equal
    the rows of the assembled K (itself pinned above)."""
    xy, tri, per = lattice_mesh(5, seed=9, periodic=periodic, length=(2 * np.pi if periodic else 1.0))
    d = OracleDisc(OracleMesh(xy, tri, per), 2)
    K = solve.assemble_K(d)
    x = np.random.default_rng(3).standard_normal((d.mesh.ne, d.nphi))
    ids = np.array([0, 7, 13, 21, d.mesh.ne - 1])
    want = (K @ x.ravel()).reshape(d.mesh.ne, d.nphi)[ids]
    got = solve.schur_rows(d, x, ids)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
