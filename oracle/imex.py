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
