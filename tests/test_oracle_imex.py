"""Pins of the oracle's grid transfers (eqs. d2m, m2d) and of its R = 0 semi-Lagrangian IMEX
step (Section 4) against what the mathematics fixes:
  * a global polynomial of degree <= p lies in both spaces, so L_md reproduces its dual
    interpolant (wall cells included) and L_dm(L_md(.)) is the identity on it;
  * L_md and L_dm are L2 projections: the residual is orthogonal to every test function of the
    target space, checked with a finer quadrature than the operators use;
  * the viscous solve (Mbar - c K) x = Mbar f with c > 0 does not increase the mass-norm
    energy (fails for the wrong sign of K);
  * a fluid at rest stays at rest; the step's velocity is discretely divergence-free;
  * Taylor-Green vortex: first-order convergence in time at fixed CFL (R = 0 is Euler).
"""
import numpy as np
import pytest

from oracle import basis, imex, solve
from oracle.mesh import OracleMesh
from oracle.operators import OracleDisc
from oracle.quadrature import triangle_rule
from paper_2401_17806_amd.inputs import lattice_mesh, random_vector


def _disc(n, p, periodic=True, seed=3):
    xy, tri, per = lattice_mesh(n, seed=seed, periodic=periodic,
                                length=(2 * np.pi if periodic else 1.0))
    return OracleDisc(OracleMesh(xy, tri, per), p)


def _poly(p, seed):
    c = np.random.default_rng(seed).normal(size=(2, basis.n_phi(p)))

    def f(xy):
        x, y = xy[..., 0], xy[..., 1]
        mons = [x ** i * y ** j for j in range(p + 1) for i in range(p + 1 - j)]
        return np.stack([sum(c[k, m] * mons[m] for m in range(len(mons))) for k in range(2)], -1)
    return f


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_transfers_reproduce_global_polynomials(p):
    d = _disc(4, p, periodic=False)
    f = _poly(p, 10 + p)
    vm = np.ascontiguousarray(f(d.main_node_xy()).transpose(0, 2, 1))
    vd = imex.main_to_dual(d, vm)
    want = imex.dual_interpolant(d, f)
    inner = d.mesh.interior
    half = np.array([a + b <= p for (a, b) in basis.dual_node_ab(p)])
    scale = np.nanmax(np.abs(want))  # wall cells have no right-half nodes (NaN positions)
    assert np.abs(vd[inner] - want[inner]).max() <= 1e-12 * scale
    assert np.abs(vd[~inner][:, :, half] - want[~inner][:, :, half]).max() <= 1e-12 * scale
    assert np.all(vd[~inner][:, :, ~half] == 0.0)
    back = imex.dual_to_main(d, vd)
    assert np.abs(back - vm).max() <= 1e-12 * scale


def _sub_points(d, n_q):
    """Finer-rule points on both halves of every dual cell: (x [nd, q, 2] per side, psi, jac)."""
    m = d.mesh
    pts, w = triangle_rule(n_q)
    u, v = pts[:, 0], pts[:, 1]
    Rs = np.where(m.interior, m.right, m.left)
    out = []
    for side, b0 in ((0, m.centroid[m.left]), (1, m.centroid[Rs] - m.shift)):
        x = b0[:, None] + u[None, :, None] * (m.A - b0)[:, None] + v[None, :, None] * (m.B - b0)[:, None]
        dd, ee = m.A - b0, m.B - b0
        jac = np.abs(dd[:, 0] * ee[:, 1] - dd[:, 1] * ee[:, 0])
        if side == 0:
            ps = basis.psi(d.p, np.broadcast_to(u, (m.nd, u.size)), np.broadcast_to(v, (m.nd, v.size)))
            tri = m.left
        else:
            jac = jac * m.interior
            ps = basis.psi(d.p, np.broadcast_to(1.0 - v, (m.nd, v.size)),
                           np.broadcast_to(1.0 - u, (m.nd, u.size)))
            tri = Rs
            x = x + m.shift[:, None]  # r's own frame for its main polynomial
        out.append((x, ps, jac, tri, w))
    return out


@pytest.mark.parametrize("p,periodic", [(2, True), (3, False)])
def test_transfers_are_l2_projections(p, periodic):
    d = _disc(4, p, periodic=periodic)
    m = d.mesh
    vm = random_vector((m.ne, 2, d.nphi), seed=40 + p)
    vd = imex.main_to_dual(d, vm)
    # L_md: int_{R_j} psi_k (vhat_j - vbar) = 0 for every dual DOF k of cell j
    res = np.zeros((m.nd, 2, d.npsi))
    for x, ps, jac, tri, w in _sub_points(d, d.p + 4):
        ph = np.stack([d.phi_phys(int(i), x[e]) for e, i in enumerate(tri)])  # [nd, q, Nphi]
        diff = np.einsum("eqk,eck->eqc", ps, vd) - np.einsum("eql,ecl->eqc", ph, vm[tri])
        res += np.einsum("q,e,eqk,eqc->eck", w, jac, ps, diff)
    inner = m.interior
    half = np.array([a + b <= p for (a, b) in basis.dual_node_ab(p)])
    scale = np.abs(vm).max() * m.area.max()
    assert np.abs(res[inner]).max() <= 1e-12 * scale
    if (~inner).any():
        assert np.abs(res[~inner][:, :, half]).max() <= 1e-12 * scale
    # L_dm: int_{T_i} phi_k (vbar_i - vhat) = 0 for every main DOF k of triangle i
    vdr = random_vector((m.nd, 2, d.npsi), seed=50 + p)
    vdr[np.broadcast_to((~inner)[:, None, None] & (~half)[None, None, :], vdr.shape)] = 0.0
    vb = imex.dual_to_main(d, vdr)
    res2 = np.zeros((m.ne, 2, d.nphi))
    for x, ps, jac, tri, w in _sub_points(d, d.p + 4):
        for e in range(m.nd):
            if jac[e] == 0.0:
                continue
            i = int(tri[e])
            ph = d.phi_phys(i, x[e])  # [q, Nphi]
            diff = ph @ vb[i].T - ps[e] @ vdr[e].T  # [q, 2]
            res2[i] += np.einsum("q,qk,qc->ck", w * jac[e], ph, diff)
    assert np.abs(res2).max() <= 1e-12 * np.abs(vdr).max() * m.area.max()


@pytest.mark.parametrize("p", [1, 3])
def test_viscous_solve_dissipates(p):
    d = _disc(5, p)
    K = solve.assemble_K(d)
    f = random_vector((d.mesh.ne, 1, d.nphi), seed=7)
    x = imex.viscous_solve(d, K, f, 0.05)
    M = imex.mass_matrix(d)
    ef = float(f.reshape(-1) @ (M @ f.reshape(-1)))
    ex = float(x.reshape(-1) @ (M @ x.reshape(-1)))
    assert ex < ef
    # constants are in the kernel of K, so they pass unchanged
    one = np.ones_like(f)
    assert np.abs(imex.viscous_solve(d, K, one, 0.05) - 1.0).max() <= 1e-12


def test_rest_state_stays_at_rest():
    d = _disc(3, 2)
    K = solve.assemble_K(d)
    v = np.zeros((d.mesh.nd, 2, d.npsi))
    vn, pi, _ = imex.imex_step(d, K, v, 0.3, 1e-2)
    assert np.abs(vn).max() == 0.0 and np.abs(pi).max() <= 1e-14


@pytest.mark.parametrize("p", [1, 2])
def test_step_velocity_is_divergence_free(p):
    d = _disc(4, p)
    K = solve.assemble_K(d)
    v = imex.dual_interpolant(d, lambda xy: imex.tgv_velocity(xy, 0.0, 1e-2))
    vn, pi, st = imex.imex_step(d, K, v, 0.2, 1e-2)
    dv_star = np.linalg.norm(solve.divergence(d, st["vs"]))
    dv = np.linalg.norm(solve.divergence(d, vn))
    assert dv_star > 1e-3
    assert dv <= 1e-10 * dv_star


def test_tgv_first_order_in_time():
    """R = 0 at CFL 0.5 (dt = h / 2), nu = 1e-2, t_end = 2 pi / 6: the velocity error against
    the decaying vortex halves when h and dt halve (Euler in time dominates)."""
    nu, p = 1e-2, 2
    errs = []
    for n in (6, 12):
        d = _disc(n, p, seed=n)
        K = solve.assemble_K(d)
        dt = 0.5 * 2 * np.pi / n
        steps = n // 3
        v = imex.dual_interpolant(d, lambda xy: imex.tgv_velocity(xy, 0.0, nu))
        for _ in range(steps):
            v, _, _ = imex.imex_step(d, K, v, dt, nu)
        errs.append(imex.dual_l2_error(d, v, lambda xy: imex.tgv_velocity(xy, steps * dt, nu)))
    order = np.log2(errs[0] / errs[1])
    assert 0.8 <= order <= 1.4, (errs, order)
    assert errs[1] < 0.35


def _wall_side_masks(d):
    """Wall edges of the unit box: all walls, and the side walls x = 0, 1 only."""
    m = d.mesh
    wall = ~m.interior
    mid = 0.5 * (m.A + m.B)
    side = wall & ((np.abs(mid[:, 0]) < 1e-12) | (np.abs(mid[:, 0] - 1.0) < 1e-12))
    return wall, side


@pytest.mark.parametrize("p", [1, 2, 3])
def test_dirichlet_laplacian_pins(p):
    """Walls of diffusion solves (reading: Dirichlet cells take the jump to the data, zero-flux
    cells keep their sub-triangle stiffness): K_W is symmetric negative definite; a linear field
    with its own trace gives L(u) = K_W u + G_b = 0 with all walls Dirichlet, and also with
    Dirichlet side walls and zero flux on top and bottom for u = a + b x (zero normal derivative
    there); for p >= 2 a quadratic gives L(u) = (Delta u) int phi exactly (all walls
    Dirichlet), and with all walls zero-flux the constants span the kernel."""
    d = _disc(5, p, periodic=False, seed=13)
    m = d.mesh
    wall, side = _wall_side_masks(d)
    assert side.sum() > 0 and side.sum() < wall.sum()
    KD = imex.assemble_K_walls(d, wall)
    A = KD.toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).max() < 0.0
    lin = lambda q: 0.3 + 1.7 * q[..., 0] - 0.9 * q[..., 1]
    u = lin(d.main_node_xy()).reshape(-1)
    gb = imex.dirichlet_rhs(d, wall, lin).reshape(-1)
    assert np.abs(KD @ u + gb).max() <= 1e-12 * np.abs(gb).max()
    lx = lambda q: 0.25 - 0.5 * q[..., 0]
    KS = imex.assemble_K_walls(d, side)
    ux = lx(d.main_node_xy()).reshape(-1)
    gs = imex.dirichlet_rhs(d, side, lx).reshape(-1)
    assert np.abs(KS @ ux + gs).max() <= 1e-12 * np.abs(gs).max()
    if p >= 2:
        quad = lambda q: q[..., 0] ** 2 + q[..., 1] ** 2
        uq = quad(d.main_node_xy()).reshape(-1)
        gq = imex.dirichlet_rhs(d, wall, quad).reshape(-1)
        want = 4.0 * d.main_weights().reshape(-1)
        assert np.abs(KD @ uq + gq - want).max() <= 1e-12 * np.abs(want).max()
    KN = imex.assemble_K_walls(d, None).toarray()
    ev = np.linalg.eigvalsh(0.5 * (KN + KN.T))
    assert abs(ev[-1]) <= 1e-12 * abs(ev[0]) and ev[-2] < 0.0
    assert np.abs(KN @ np.ones(KN.shape[0])).max() <= 1e-12 * np.abs(KN).max()


def test_dirichlet_diffusion_keeps_the_linear_steady_state():
    """The implicit diffusion step with Dirichlet side walls leaves the conduction profile
    u = 0.5 - x unchanged (it is the steady state), for any time step."""
    d = _disc(6, 2, periodic=False, seed=14)
    _, side = _wall_side_masks(d)
    prof = lambda q: 0.5 - q[..., 0]
    KS = imex.assemble_K_walls(d, side)
    gb = imex.dirichlet_rhs(d, side, prof)
    u = prof(d.main_node_xy())[:, None, :]
    for c in (1e-3, 0.1, 10.0):
        out = imex.diffusion_solve(d, KS, u, c, gb)
        assert np.abs(out - u).max() <= 1e-11


def _cavity(n, p, jitter=0.0, seed=4):
    xy, tri, per = lattice_mesh(n, seed=seed, periodic=False, length=1.0, jitter=jitter)
    d = OracleDisc(OracleMesh(xy, tri, per), p)
    _, side = _wall_side_masks(d)
    ops = imex.cavity_operators(d, side, lambda q: 0.5 - q[..., 0])
    return d, ops


def test_cavity_conduction_state_is_steady():
    """Without buoyancy the conduction profile T = 0.5 - x at rest is a steady state."""
    d, ops = _cavity(5, 2, jitter=0.1)
    m = d.mesh
    T = 0.5 - d.main_node_xy()[..., 0]
    v = np.zeros((m.nd, 2, d.npsi))
    for _ in range(2):
        v, T2, pi = imex.cavity_step(d, ops, v, T, 0.1, 3e-3, 4e-3, 0.0)
        assert np.abs(T2 - T).max() <= 1e-11 and np.abs(v).max() <= 1e-12
        T = T2


@pytest.mark.parametrize("p", [1, 2, 3])
def test_cavity_first_step_symmetry_and_buoyancy(p):
    """The differentially heated cavity is symmetric under the point reflection about the box
    centre with T -> -T, v -> -v, p -> p.  From rest the walk is the identity, every other
    operator is an exact integral, and the unjittered mesh is symmetric, so the first step is
    symmetric to rounding; the hot fluid rises at the left wall and sinks at the right; the
    velocity is divergence-free and zero on the wall cells."""
    from scipy.spatial import cKDTree
    d, ops = _cavity(5, p)
    m = d.mesh
    v = np.zeros((m.nd, 2, d.npsi))
    T = np.zeros((m.ne, d.nphi))
    v, T, pi = imex.cavity_step(d, ops, v, T, 0.1, 2.7e-3, 3.7e-3, 1.0)
    xyn, cen = d.main_node_xy(), m.centroid
    _, ti = cKDTree(cen).query(1.0 - cen)
    for i in range(m.ne):
        nk = cKDTree(xyn[ti[i]]).query(1.0 - xyn[i])[1]
        assert np.abs(T[i] + T[ti[i]][nk]).max() <= 1e-13
        assert np.abs(pi[i] - pi[ti[i]][nk]).max() <= 1e-13 * max(np.abs(pi).max(), 1.0)
    dn = d.dual_node_xy()
    mid = 0.5 * (m.A + m.B)
    _, ej = cKDTree(mid).query(1.0 - mid)
    for j in np.nonzero(m.interior)[0]:
        nk = cKDTree(dn[ej[j]]).query(1.0 - dn[j])[1]
        assert np.abs(v[j] + v[ej[j]][:, nk]).max() <= 1e-13
    xs = dn[..., 0]
    inner = m.interior[:, None] & np.isfinite(xs)
    vy = v[:, 1, :]
    assert vy[inner & (xs < 0.3)].mean() > 0.0 > vy[inner & (xs > 0.7)].mean()
    assert np.abs(v[~m.interior]).max() == 0.0
    assert np.linalg.norm(solve.divergence(d, v)) <= 1e-12 * np.abs(v).max()


def test_walls_rows_equal_assembled_rows():
    """walls_rows (sampled rows, used at full size) equals the assembled K_W on every row."""
    d = _disc(5, 2, periodic=False, seed=15)
    _, side = _wall_side_masks(d)
    u = random_vector((d.mesh.ne, d.nphi), seed=77)
    want = (imex.assemble_K_walls(d, side) @ u.reshape(-1)).reshape(u.shape)
    ids = np.arange(d.mesh.ne)
    got = imex.walls_rows(d, u, ids, side)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def _ns_residual(vel, pres, xy, t, nu, h=1e-4):
    """dv/dt + (v.grad) v + grad p - nu lap v at points xy, by central differences of the
    closed-form fields (the incompressible momentum equation of Section 2 with g = 0)."""
    ex, ey = np.array([h, 0.0]), np.array([0.0, h])
    v = vel(xy, t, nu)
    dvdt = (vel(xy, t + h, nu) - vel(xy, t - h, nu)) / (2 * h)
    dvdx = (vel(xy + ex, t, nu) - vel(xy - ex, t, nu)) / (2 * h)
    dvdy = (vel(xy + ey, t, nu) - vel(xy - ey, t, nu)) / (2 * h)
    lap = (vel(xy + ex, t, nu) + vel(xy - ex, t, nu) + vel(xy + ey, t, nu) + vel(xy - ey, t, nu)
           - 4 * v) / h ** 2
    dpdx = (pres(xy + ex, t, nu) - pres(xy - ex, t, nu)) / (2 * h)
    dpdy = (pres(xy + ey, t, nu) - pres(xy - ey, t, nu)) / (2 * h)
    gradp = np.stack([dpdx, dpdy], axis=-1)
    adv = v[..., :1] * dvdx + v[..., 1:] * dvdy
    return dvdt + adv + gradp - nu * lap


def test_tgv_fields_solve_the_momentum_equation():
    """The Taylor-Green velocity and the oracle's pressure (Section 5, decay e^{-4 nu t}) satisfy
    the momentum and continuity equations; the printed pressure decay e^{-2 nu t} does not."""
    rng = np.random.default_rng(3)
    xy = rng.uniform(0, 2 * np.pi, size=(200, 2))
    for nu, t in [(1e-2, 0.7), (0.3, 1.9)]:
        res = _ns_residual(imex.tgv_velocity, imex.tgv_pressure, xy, t, nu)
        assert np.abs(res).max() <= 1e-6
        h = 1e-5
        div = ((imex.tgv_velocity(xy + [h, 0], t, nu) - imex.tgv_velocity(xy - [h, 0], t, nu))[:, 0]
               + (imex.tgv_velocity(xy + [0, h], t, nu) - imex.tgv_velocity(xy - [0, h], t, nu))[:, 1]) / (2 * h)
        assert np.abs(div).max() <= 1e-8

    def printed(q, t, nu):
        return 0.25 * (np.cos(2 * q[..., 0]) + np.cos(2 * q[..., 1])) * np.exp(-2.0 * nu * t)

    res = _ns_residual(imex.tgv_velocity, printed, xy, 1.9, 0.3)
    assert np.abs(res).max() > 1e-2
