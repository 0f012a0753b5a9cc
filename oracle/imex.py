"""Grid transfers and the semi-Lagrangian IMEX time step for the incompressible
Navier-Stokes equations (Section 4), first-order member R = 0.

Transfers (Section 4, eqs. d2m and m2d), with the operator U of eq. u,
U_ij[k, l] = int_{T_ij} psi_k^(j) phi_l^(i) dx over the sub-triangle T_ij of triangle i in
the dual cell of edge j, integrated here in physical space:
  * dual -> main  L_dm:  vbar_i = Mbar_i^{-1} sum_{j in S_i} U_ij^T vhat_j
  * main -> dual  L_md:  vhat_j = Mhat_j^{-1} (U_lj vbar_l + U_rj vbar_r)
A wall edge's dual cell is its left sub-triangle only: there U_rj is absent and L_md is solved
on the DOFs of the left half (the others are set to zero).

Time step, R = 0 (appendix tableau: one stage, explicit c = 0, implicit a_11 = 1, b = 1, so the
step is the stage; a_ss = 1):
  1. vbar^n = L_dm(vhat^n)                              (velocity on the main grid)
  2. vbar_F = SL projection of vbar^n at the feet x - dt vbar^n (Section 3.5, advect.py)
  3. (Mbar - a_ss dt nu K) vbar* = Mbar vbar_F per component (the advection-diffusion scheme of
     eq. ad5 with coefficient nu; K = D Mhat^{-1} Q is the main-grid discrete Laplacian of eq.
     pressure_final)
  4. vhat* = L_md(vbar*)
  5. K pi = (1/(a_ss dt)) D vhat*  (eq. pressure_IMEX with g = 0 and no buoyancy), int pi = 0
  6. vhat^{n+1} = vhat* - a_ss dt Mhat^{-1}(Q_l pi_l + Q_r pi_r)  (eq. nc.2 solved for vhat)

Readings (the paper leaves these to its references): the viscous operator is the same K as the
pressure operator (the main-grid Laplacian built from the staggered gradient and divergence);
initial data are the nodal interpolants of the exact fields at the dual nodes; the viscous solve
is skipped when nu = 0.

Test infrastructure only (imported by tests/ and never by the product path).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import advect, basis, solve
from .operators import OracleDisc


def transfer_blocks(disc: OracleDisc, J):
    """U_lj, U_rj [E, Npsi, Nphi] (eq. u) and Mhat_j [E, Npsi, Npsi] (eq. Mj) for edges J,
    by quadrature over the two physical sub-triangles of each dual cell (U_rj = 0 on walls)."""
    m = disc.mesh
    p = disc.p
    J = np.asarray(J, dtype=np.int64)
    E = J.size
    L = m.left[J]
    R = m.right[J]
    inner = R >= 0
    Rs = np.where(inner, R, L)
    A, B = m.A[J], m.B[J]
    shift = m.shift[J]
    bl = m.centroid[L]
    br = m.centroid[Rs] - shift
    u, v = disc.tri_pts[:, 0], disc.tri_pts[:, 1]
    w = disc.tri_w
    # left sub-triangle (b_l, A, B): x = b_l + u (A - b_l) + v (B - b_l), dual coords (u, v)
    xl = bl[:, None] + u[None, :, None] * (A - bl)[:, None] + v[None, :, None] * (B - bl)[:, None]
    dl, el = A - bl, B - bl
    jl = np.abs(dl[:, 0] * el[:, 1] - dl[:, 1] * el[:, 0])
    psi_l = basis.psi(p, np.broadcast_to(u, (E, u.size)), np.broadcast_to(v, (E, v.size)))
    # right sub-triangle (b_r, A, B): the same points seen from the upper half of R_ref
    xr = br[:, None] + u[None, :, None] * (A - br)[:, None] + v[None, :, None] * (B - br)[:, None]
    dr, er = A - br, B - br
    jr = np.abs(dr[:, 0] * er[:, 1] - dr[:, 1] * er[:, 0]) * inner
    psi_r = basis.psi(p, np.broadcast_to(1.0 - v, (E, v.size)), np.broadcast_to(1.0 - u, (E, u.size)))
    phi_l = disc.phi_phys(L, xl)                          # [E, q, Nphi]
    phi_r = disc.phi_phys(Rs, xr + shift[:, None])        # r's own frame
    Ul = np.einsum("q,e,eqk,eql->ekl", w, jl, psi_l, phi_l)
    Ur = np.einsum("q,e,eqk,eql->ekl", w, jr, psi_r, phi_r)
    Mhat = np.einsum("q,e,eqk,eql->ekl", w, jl, psi_l, psi_l) + \
        np.einsum("q,e,eqk,eql->ekl", w, jr, psi_r, psi_r)
    return Ul, Ur, Mhat


def _left_half(p: int) -> np.ndarray:
    """Dual DOFs of the lower half of R_ref (nodes with a + b <= p)."""
    return np.array([a + b <= p for (a, b) in basis.dual_node_ab(p)])


def main_to_dual(disc: OracleDisc, vm: np.ndarray) -> np.ndarray:
    """L_md (eq. m2d): vm [ne, nc, Nphi] -> [nd, nc, Npsi]."""
    m = disc.mesh
    J = np.arange(m.nd)
    Ul, Ur, Mhat = transfer_blocks(disc, J)
    R = np.maximum(m.right, 0)
    rhs = np.einsum("ekl,ecl->eck", Ul, vm[m.left]) + \
        np.einsum("ekl,ecl->eck", Ur, vm[R]) * m.interior[:, None, None]
    out = np.zeros((m.nd, vm.shape[1], disc.npsi))
    inner = m.interior
    if inner.any():
        out[inner] = np.linalg.solve(Mhat[inner][:, None], rhs[inner][..., None])[..., 0]
    if (~inner).any():
        h = _left_half(disc.p)
        Mw = Mhat[~inner][:, h][:, :, h]
        out_w = np.linalg.solve(Mw[:, None], rhs[~inner][:, :, h][..., None])[..., 0]
        tmp = np.zeros((out_w.shape[0], vm.shape[1], disc.npsi))
        tmp[:, :, h] = out_w
        out[~inner] = tmp
    return out


def dual_to_main(disc: OracleDisc, vd: np.ndarray) -> np.ndarray:
    """L_dm (eq. d2m): vd [nd, nc, Npsi] -> [ne, nc, Nphi]."""
    m = disc.mesh
    J = np.arange(m.nd)
    Ul, Ur, _ = transfer_blocks(disc, J)
    rhs = np.zeros((m.ne, vd.shape[1], disc.nphi))
    np.add.at(rhs, m.left, np.einsum("ekl,eck->ecl", Ul, vd))
    inner = np.nonzero(m.interior)[0]
    np.add.at(rhs, m.right[inner], np.einsum("ekl,eck->ecl", Ur[inner], vd[inner]))
    Mbar = disc.main_mass()
    return np.linalg.solve(Mbar[:, None], rhs[..., None])[..., 0]


# ---------------------------------------------------------------- walls of diffusion solves
# Reading (the paper leaves the boundary treatment of the diffusion solves to its references).
# The pressure operator K of eq. pressure_final has no wall cells: they carry prescribed
# velocity.  A diffusion operator keeps them.  On a wall edge j the dual cell is the left half
# alone, and its gradient follows eq. ad4.2 with the missing right-hand side replaced by the
# boundary condition:
#   * Dirichlet data u_b: the jump term takes u_l - u_b,
#       Mhat_j g_j = Q_lj u_l + int_{Gamma_j} psi u_b n ds;
#     the divergence block D_lj keeps its line term.
#   * zero flux: no jump term and no line term in D_lj (the flux through the wall is the data,
#     zero), so the cell contributes -int_{T_lj} grad phi . Mhat_j^{-1} int psi grad u_l, and the
#     projected gradient is grad u_l itself (a polynomial of the half's space):
#       -int_{T_lj} grad phi_k . grad phi_l.
# The Laplacian is L(u) = K_W u + G_b, with K_W = K plus these wall cells and
# G_b = sum_j D_lj Mhat_j^{-1} int_Gamma psi u_b n ds over the Dirichlet edges.  The data enter
# as their nodal interpolant of degree p along each wall edge (values at the p+1 equispaced
# edge nodes), as every field of the nodal scheme does.


def _wall_edges(disc: OracleDisc, mask) -> np.ndarray:
    m = disc.mesh
    mask = np.asarray(mask, dtype=bool)
    return np.nonzero(mask & ~m.interior)[0]


def _wall_stiffness(disc: OracleDisc, J) -> np.ndarray:
    """-int_{T_lj} grad phi_k . grad phi_l over the wall sub-triangles of edges J [E, N, N]."""
    m = disc.mesh
    L = m.left[J]
    bl = m.centroid[L]
    A, B = m.A[J], m.B[J]
    u, v = disc.tri_pts[:, 0], disc.tri_pts[:, 1]
    x = bl[:, None] + u[None, :, None] * (A - bl)[:, None] + v[None, :, None] * (B - bl)[:, None]
    d, e = A - bl, B - bl
    jac = np.abs(d[:, 0] * e[:, 1] - d[:, 1] * e[:, 0])
    g = disc.grad_phi_phys(L, x)  # [E, q, N, 2]
    return -np.einsum("q,e,eqkc,eqlc->ekl", disc.tri_w, jac, g, g)


def assemble_K_walls(disc: OracleDisc, dirichlet_mask=None) -> sp.csr_matrix:
    """K_W: K of eq. pressure_final plus a cell on every wall edge, Dirichlet where
    dirichlet_mask [nd] is set, zero flux elsewhere."""
    m = disc.mesh
    nphi = disc.nphi
    K = solve.assemble_K(disc)
    walls = np.nonzero(~m.interior)[0]
    if walls.size == 0:
        return K
    dmask = np.zeros(m.nd, dtype=bool) if dirichlet_mask is None else np.asarray(dirichlet_mask, bool)
    B = np.zeros((walls.size, nphi, nphi))
    isd = dmask[walls]
    if (~isd).any():
        B[~isd] = _wall_stiffness(disc, walls[~isd])
    if isd.any():
        J = walls[isd]
        h = _left_half(disc.p)
        blk = disc.edge_blocks(J)
        Mh = blk["Mhat"][:, h][:, :, h]
        Ql = blk["Ql"][:, h]
        Dl = blk["Dl"][:, :, h]
        E, nh = Mh.shape[0], Mh.shape[1]
        X = np.linalg.solve(Mh, Ql.reshape(E, nh, nphi * 2)).reshape(E, nh, nphi, 2)
        B[isd] = np.einsum("ekmc,emlc->ekl", Dl, X)
    kk, ll = np.meshgrid(np.arange(nphi), np.arange(nphi), indexing="ij")
    L = m.left[walls]
    rows = (L[:, None, None] * nphi + kk[None]).ravel()
    cols = (L[:, None, None] * nphi + ll[None]).ravel()
    n = m.ne * nphi
    Kw = sp.coo_matrix((B.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    return (K + Kw).tocsr()


def walls_rows(disc: OracleDisc, u: np.ndarray, tri_ids, dirichlet_mask=None) -> np.ndarray:
    """(K_W u)_i for the triangles in tri_ids only (rows of assemble_K_walls without assembling
    it), for checks on large meshes: the interior-edge rows of eq. pressure_final plus the wall
    cells of those triangles."""
    m = disc.mesh
    nphi = disc.nphi
    tri_ids = np.asarray(tri_ids, dtype=np.int64)
    out = solve.schur_rows(disc, u, tri_ids)
    J = np.unique(m.tri_edges[tri_ids].ravel())
    J = J[~m.interior[J]]
    if J.size == 0:
        return out
    dmask = np.zeros(m.nd, dtype=bool) if dirichlet_mask is None else np.asarray(dirichlet_mask, bool)
    B = np.zeros((J.size, nphi, nphi))
    isd = dmask[J]
    if (~isd).any():
        B[~isd] = _wall_stiffness(disc, J[~isd])
    if isd.any():
        h = _left_half(disc.p)
        blk = disc.edge_blocks(J[isd])
        Mh = blk["Mhat"][:, h][:, :, h]
        Ql = blk["Ql"][:, h]
        Dl = blk["Dl"][:, :, h]
        E, nh = Mh.shape[0], Mh.shape[1]
        X = np.linalg.solve(Mh, Ql.reshape(E, nh, nphi * 2)).reshape(E, nh, nphi, 2)
        B[isd] = np.einsum("ekmc,emlc->ekl", Dl, X)
    pos = {int(i): t for t, i in enumerate(tri_ids)}
    for e, j in enumerate(J):
        i = int(m.left[j])
        out[pos[i]] += B[e] @ u[i]
    return out


def dirichlet_rhs(disc: OracleDisc, dirichlet_mask, trace) -> np.ndarray:
    """G_b [ne, Nphi] for the data trace(xy [..., 2]) -> [...] on the masked wall edges (taken
    through its values at the edge nodes)."""
    m = disc.mesh
    out = np.zeros((m.ne, disc.nphi))
    J = _wall_edges(disc, dirichlet_mask)
    if J.size == 0:
        return out
    p = disc.p
    h = _left_half(p)
    blk = disc.edge_blocks(J)
    Mh = blk["Mhat"][:, h][:, :, h]
    Dl = blk["Dl"][:, :, h]
    t, wt = disc.line_t, disc.line_w
    A, B = m.A[J], m.B[J]
    xe = A[:, None] + t[None, :, None] * (B - A)[:, None]      # [E, q, 2]
    psi_e = basis.psi(p, np.broadcast_to(1.0 - t, (J.size, t.size)),
                      np.broadcast_to(t, (J.size, t.size)))[:, :, h]  # [E, q, nh]
    # the data's degree-p interpolant through the p+1 equispaced nodes of the edge
    tn = np.arange(p + 1) / p
    xn = A[:, None] + tn[None, :, None] * (B - A)[:, None]       # [E, p+1, 2]
    lag = np.ones((t.size, p + 1))
    for a in range(p + 1):
        for b in range(p + 1):
            if b != a:
                lag[:, a] *= (t - tn[b]) / (tn[a] - tn[b])
    ub = trace(xn) @ lag.T                                      # [E, q]
    line = np.einsum("q,e,eqk,eq,ec->ekc", wt, m.edge_len[J], psi_e, ub, m.normal[J])
    g = np.linalg.solve(Mh[:, None], line.transpose(0, 2, 1)[..., None])[..., 0]  # [E, 2, nh]
    np.add.at(out, m.left[J], np.einsum("ekmc,ecm->ek", Dl, g))
    return out


def diffusion_solve(disc: OracleDisc, KW: sp.csr_matrix, f: np.ndarray, c: float,
                    gb: np.ndarray | None = None) -> np.ndarray:
    """x with (Mbar - c K_W) x = Mbar f + c G_b for f [ne, nc, Nphi] (gb [ne, Nphi] or None)."""
    if c == 0.0:
        return f.copy()
    M = mass_matrix(disc)
    lu = spla.splu((M - c * KW).tocsc())
    ne, nc, n = f.shape
    out = np.empty_like(f)
    for comp in range(nc):
        rhs = M @ f[:, comp, :].reshape(-1)
        if gb is not None:
            rhs = rhs + c * gb.reshape(-1)
        out[:, comp, :] = lu.solve(rhs).reshape(ne, n)
    return out


def mass_matrix(disc: OracleDisc) -> sp.csr_matrix:
    """Block-diagonal Mbar (eq. Mi) as a sparse matrix over the main DOFs."""
    Mb = disc.main_mass()
    return sp.block_diag(list(Mb), format="csr")


def viscous_solve(disc: OracleDisc, K: sp.csr_matrix, f: np.ndarray, c: float) -> np.ndarray:
    """x with (Mbar - c K) x = Mbar f, for f [ne, nc, Nphi] component by component (sparse LU)."""
    if c == 0.0:
        return f.copy()
    M = mass_matrix(disc)
    A = (M - c * K).tocsc()
    lu = spla.splu(A)
    ne, nc, n = f.shape
    out = np.empty_like(f)
    for comp in range(nc):
        rhs = M @ f[:, comp, :].reshape(-1)
        out[:, comp, :] = lu.solve(rhs).reshape(ne, n)
    return out


def pressure_solve(disc: OracleDisc, K: sp.csr_matrix, b: np.ndarray, tol: float = 1e-13):
    """Zero-mean pi with K pi = b (dense bordered solve on tiny meshes, CG otherwise)."""
    if K.shape[0] <= 4000:
        p = solve.dense_bordered_solve(K, b)
    else:
        p, _ = solve.cg(K, b, tol=tol, maxit=200000)
    return solve.gauge(disc, p)


def imex_step(disc: OracleDisc, K: sp.csr_matrix, vhat: np.ndarray, dt: float, nu: float):
    """One R = 0 step of the semi-Lagrangian IMEX scheme.  vhat [nd, 2, Npsi] -> (vhat_new,
    pi [ne, Nphi], stages) with stages holding vbar, vbar_F, vbar*, vhat*, b."""
    a_ss = 1.0
    vbar = dual_to_main(disc, vhat)
    vF = advect.sl_advect(disc, vbar, vbar, dt)
    vs_bar = viscous_solve(disc, K, vF, a_ss * dt * nu)
    vs = main_to_dual(disc, vs_bar)
    b = solve.pressure_rhs(disc, vs, 1.0 / (a_ss * dt))
    pi = pressure_solve(disc, K, b)
    vnew = solve.velocity_correction(disc, vs, pi, a_ss * dt)
    return vnew, pi, {"vbar": vbar, "vF": vF, "vs_bar": vs_bar, "vs": vs, "b": b}


# ---------------------------------------------------------------- Boussinesq cavity
# R = 0 step of the natural-convection model (eqs. nc.1-nc.3, eq. pressure_IMEX), readings:
#   * nondimensional form with g beta = Delta T = L = 1: nu = sqrt(Pr / Ra), kappa =
#     1 / sqrt(Ra Pr); the momentum source (1 - beta dT) g keeps only its buoyancy part
#     (0, g beta T) -- the constant gravity is a hydrostatic pressure gradient, absorbed into p;
#   * no-slip walls: the wall dual cells carry zero velocity (prescribed), and the viscous solve
#     has Dirichlet cells with zero data on every wall;
#   * temperature: Dirichlet data on the flagged walls (the heated and cooled sides), zero flux
#     on the others (adiabatic);
#   * buoyancy enters with the new temperature: v* += dt g beta (0, L_md(T*)) on interior cells,
#     before the pressure projection (eq. nc.2 with the source of eq. pressure_IMEX).


def cavity_operators(disc: OracleDisc, temp_mask, temp_trace):
    """(K, K_V, K_T, G_T): pressure operator, no-slip viscous operator, temperature diffusion
    operator and its boundary-data vector."""
    m = disc.mesh
    K = solve.assemble_K(disc)
    KV = assemble_K_walls(disc, ~m.interior)
    KT = assemble_K_walls(disc, temp_mask)
    GT = dirichlet_rhs(disc, temp_mask, temp_trace)
    return K, KV, KT, GT


def cavity_step(disc: OracleDisc, ops, vhat: np.ndarray, T: np.ndarray, dt: float, nu: float,
                kappa: float, gbeta: float):
    """One R = 0 step.  vhat [nd, 2, Npsi], T [ne, Nphi] -> (vhat, T, pi)."""
    m = disc.mesh
    K, KV, KT, GT = ops
    vbar = dual_to_main(disc, vhat)
    vF = advect.sl_advect(disc, vbar, vbar, dt)
    TF = advect.sl_advect(disc, vbar, T[:, None, :], dt)
    Ts = diffusion_solve(disc, KT, TF, dt * kappa, GT)[:, 0]
    vsb = diffusion_solve(disc, KV, vF, dt * nu, None)
    vs = main_to_dual(disc, vsb)
    tb = main_to_dual(disc, Ts[:, None, :])[:, 0]
    vs[:, 1] += dt * gbeta * tb
    vs[~m.interior] = 0.0
    b = solve.pressure_rhs(disc, vs, 1.0 / dt)
    pi = pressure_solve(disc, K, b)
    vnew = solve.velocity_correction(disc, vs, pi, dt)
    return vnew, Ts, pi


# ---------------------------------------------------------------- Taylor-Green vortex
def tgv_velocity(xy: np.ndarray, t: float, nu: float) -> np.ndarray:
    """Exact Taylor-Green velocity (Section 5, with g = 0): [..., 2]."""
    x, y = xy[..., 0], xy[..., 1]
    e = np.exp(-2.0 * nu * t)
    return np.stack([np.sin(x) * np.cos(y) * e, -np.cos(x) * np.sin(y) * e], axis=-1)


def tgv_pressure(xy: np.ndarray, t: float, nu: float) -> np.ndarray:
    """Exact Taylor-Green pressure; the decay rate is e^{-4 nu t} (p is quadratic in the
    velocity amplitude; the printed e^{-2 nu t} does not satisfy the momentum equation)."""
    x, y = xy[..., 0], xy[..., 1]
    return 0.25 * (np.cos(2 * x) + np.cos(2 * y)) * np.exp(-4.0 * nu * t)


def dual_interpolant(disc: OracleDisc, field) -> np.ndarray:
    """Nodal interpolant [nd, 2, Npsi] of field(xy [..., 2]) -> [..., 2] at the dual nodes."""
    xy = disc.dual_node_xy()
    return np.ascontiguousarray(field(xy).transpose(0, 2, 1))


def dual_l2_error(disc: OracleDisc, vhat: np.ndarray, field) -> float:
    """sqrt(int_Omega |vhat - field|^2) over the dual cells (quadrature on both halves)."""
    m = disc.mesh
    p = disc.p
    u, v = disc.tri_pts[:, 0], disc.tri_pts[:, 1]
    w = disc.tri_w
    inner = m.interior
    Rs = np.where(inner, m.right, m.left)
    bl = m.centroid[m.left]
    br = m.centroid[Rs] - m.shift
    total = 0.0
    for side in (0, 1):
        b0 = bl if side == 0 else br
        xq = b0[:, None] + u[None, :, None] * (m.A - b0)[:, None] + v[None, :, None] * (m.B - b0)[:, None]
        d, e = m.A - b0, m.B - b0
        jac = np.abs(d[:, 0] * e[:, 1] - d[:, 1] * e[:, 0])
        if side == 0:
            ps = basis.psi(p, np.broadcast_to(u, (m.nd, u.size)), np.broadcast_to(v, (m.nd, v.size)))
        else:
            jac = jac * inner
            ps = basis.psi(p, np.broadcast_to(1.0 - v, (m.nd, v.size)),
                           np.broadcast_to(1.0 - u, (m.nd, u.size)))
        vh = np.einsum("eqk,eck->eqc", ps, vhat)
        diff = vh - field(xq)
        total += float(np.einsum("q,e,eqc->", w, jac, diff * diff))
    return float(np.sqrt(total))
