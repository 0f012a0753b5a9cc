"""Semi-Lagrangian advection of main-grid DG fields (Section 3.5; its use in the SL-IMEX stages
is the Gauss-point projection of eq. intstage in Section 4).

For every triangle i and every Gauss point xi_g of the triangle rule:
  * the characteristic through x_g is followed backward in time over dt with straight
    segments (explicit Euler), one segment per cell: inside the current cell c the velocity
    is the cell's DG velocity at the segment's starting point, and the segment ends where the
    ray leaves c or the remaining time is used up;
  * on leaving c through an interior edge the walk continues in the neighbour from the same
    point (found through the edge, so periodic boxes need no coordinate wrap); on a wall edge
    it stops there;
  * the field is evaluated at the foot with the DG polynomial of the cell reached;
then q_new_i = M_ref^{-1} sum_g w_g phi(xi_g) q(foot_g) (the L2 projection onto the main
basis; the Jacobian of T_i cancels between the mass matrix and the load vector).

Readings (the paper leaves these details to its reference on trajectory tracing):
  * Gauss rule: collapsed Gauss-Legendre, p + 1 points per direction (exact for the degree 2p
    integrand of the projection, so a field at rest is reproduced exactly).
  * The walk is carried in barycentric coordinates lambda of the current cell.  The exit time
    is the smallest s > 0 with lambda_k - s dlambda_k = 0 over the coordinates that decrease
    (ties: lowest k); the exit edge is the edge opposite vertex k.  The exit point's
    coordinates are clamped to >= 0 and the crossed one is set to 0.
  * A walk that cannot move (the velocity of the cell just entered points straight back out
    through the entry edge, or out at a vertex) stops where it is.
  * At most `max_steps` segments per point (far more than any CFL-bounded step needs).

Test infrastructure only (imported by tests/ and never by the product path).
"""
from __future__ import annotations

import numpy as np

from . import basis
from .operators import OracleDisc
from .quadrature import triangle_rule


def sl_rule(p: int):
    """The Gauss rule of the projection: points [Ng, 2] on T_ref, weights [Ng] (sum 1/2)."""
    return triangle_rule(p + 1)


def projection_matrix(p: int) -> np.ndarray:
    """P [N, Ng] with q_new = P q_at_gauss_points: M_ref^{-1} Phi^T diag(w)."""
    pts, w = sl_rule(p)
    ph = basis.phi(p, pts[:, 0], pts[:, 1])  # [Ng, N]
    m_ref = ph.T @ (w[:, None] * ph)         # exact: the rule integrates degree 2p
    return np.linalg.solve(m_ref, ph.T * w[None, :])


def walk(disc: OracleDisc, vbar: np.ndarray, i: int, xi, dt: float, max_steps: int = 1024):
    """Foot of the backward characteristic from reference point xi of triangle i.

    vbar [ne, 2, N] nodal DG velocity.  Returns (cell, (xi, eta), segments)."""
    m = disc.mesh
    p = disc.p
    c = int(i)
    lam = np.array([1.0 - xi[0] - xi[1], xi[0], xi[1]])
    tau = float(dt)
    for step in range(max_steps):
        ph = basis.phi(p, np.array([lam[1]]), np.array([lam[2]]))[0]  # [N]
        u = vbar[c] @ ph                                              # physical velocity (2,)
        dxi = disc.Jinv[c] @ u                                        # reference velocity
        dlam = np.array([-(dxi[0] + dxi[1]), dxi[0], dxi[1]])
        # backward motion: lam(s) = lam - s dlam; a coordinate with dlam_k > 0 reaches 0
        s_star, k_star = np.inf, -1
        for k in range(3):
            if dlam[k] > 0.0:
                s = lam[k] / dlam[k]
                if s < s_star:
                    s_star, k_star = s, k
        if k_star < 0 or s_star >= tau:
            lam = lam - tau * dlam
            return c, (lam[1], lam[2]), step + 1
        if s_star <= 0.0:
            return c, (lam[1], lam[2]), step + 1
        lam = lam - s_star * dlam
        lam = np.maximum(lam, 0.0)
        lam[k_star] = 0.0
        tau -= s_star
        alpha = (k_star + 1) % 3                 # edge opposite vertex k_star
        j = int(m.tri_edges[c, alpha])
        if not m.interior[j]:
            return c, (lam[1], lam[2]), step + 1  # wall: the foot stays on the wall
        t = min(max(lam[(alpha + 1) % 3], 0.0), 1.0)  # position along v_alpha -> v_alpha+1
        if m.left[j] == c:
            r, ar = int(m.right[j]), int(m.alpha_r[j])
        else:
            r, ar = int(m.left[j]), int(m.alpha_l[j])
        # the neighbour's edge ar runs the other way: the point is t v'_ar + (1 - t) v'_ar+1
        lam = np.zeros(3)
        lam[ar] = t
        lam[(ar + 1) % 3] = 1.0 - t
        c = r
    return c, (lam[1], lam[2]), max_steps


def sl_advect(disc: OracleDisc, vbar: np.ndarray, q: np.ndarray, dt: float,
              max_steps: int = 1024) -> np.ndarray:
    """vbar [ne, 2, N], q [ne, nc, N] -> advected q [ne, nc, N]."""
    p = disc.p
    pts, _ = sl_rule(p)
    proj = projection_matrix(p)
    ne, nc, n = q.shape
    out = np.zeros_like(q)
    for i in range(ne):
        qf = np.zeros((pts.shape[0], nc))
        for g in range(pts.shape[0]):
            c, (a, b), _ = walk(disc, vbar, i, pts[g], dt, max_steps)
            ph = basis.phi(p, np.array([a]), np.array([b]))[0]
            qf[g] = q[c] @ ph
        out[i] = (proj @ qf).T
    return out


def nodal_velocity(disc: OracleDisc, field) -> np.ndarray:
    """Nodal DG velocity [ne, 2, N] of a callable field(x [..., 2]) -> [..., 2] at the main nodes."""
    xy = disc.main_node_xy()  # [ne, N, 2]
    return np.ascontiguousarray(field(xy).transpose(0, 2, 1))


def sl_advect_rows(disc: OracleDisc, vbar: np.ndarray, q: np.ndarray, dt: float, tri_ids,
                   max_steps: int = 1024) -> np.ndarray:
    """The advected coefficients of the triangles in tri_ids only, [len(tri_ids), nc, N]
    (the same computation as sl_advect, for checks on large meshes)."""
    p = disc.p
    pts, _ = sl_rule(p)
    proj = projection_matrix(p)
    nc = q.shape[1]
    out = np.zeros((len(tri_ids), nc, disc.nphi))
    for t, i in enumerate(tri_ids):
        qf = np.zeros((pts.shape[0], nc))
        for g in range(pts.shape[0]):
            c, (a, b), _ = walk(disc, vbar, int(i), pts[g], dt, max_steps)
            ph = basis.phi(p, np.array([a]), np.array([b]))[0]
            qf[g] = q[c] @ ph
        out[t] = (proj @ qf).T
    return out
