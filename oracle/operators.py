"""Per-edge operator blocks by physical-space quadrature (Sections 2.3, 2.4).

For every edge Gamma_j and each adjacent triangle i in {l(j), r(j)} the
oracle integrates the definitions directly in physical space:

* dual mass matrix (eq. Mj):        Mhat_j[k,l] = int_{R_j} psi_k psi_l dx
* gradient operator (eq. ad5.2):    Q_ij[k,l,:] = int_{T_ij} psi_k grad phi_l^(i) dx
                                                 - int_{Gamma_j} psi_k phi_l^(i) sigma_ij n_j ds
* divergence operator (eq. D):      D_ij[k,l,:] = int_{Gamma_j} phi_k^(i) psi_l sigma_ij n_j ds
                                                 - int_{T_ij} grad phi_k^(i) psi_l dx
* main mass matrix (eq. Mi):        Mbar_i[k,l] = int_{T_i} phi_k^(i) phi_l^(i) dx

with sigma_ij = +1 if i = l(j), -1 otherwise (eq. sigma).  phi^(i) is
evaluated through the inverse of the affine map of eq. linmap, and psi^(j)
through the two affine maps of the dual cell (eq. mapDual): the left
sub-triangle (b_l, A, B) is the image of the lower half of R_ref with
(1,0) -> A, (0,1) -> B, (0,0) -> b_l; the right sub-triangle (b_r, A, B) is
the image of the upper half with (1,0) -> A, (0,1) -> B, (1,1) -> b_r.  The
diagonal of R_ref is therefore Gamma_j traversed from A to B, as seen from
both sides, which is what makes the C0 dual space single valued on Gamma_j.

Nothing here uses the reference-operator factorisation of Section 3.4.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .quadrature import gauss_legendre_01, triangle_rule
from .mesh import OracleMesh


def _inv2(J):
    """Inverse of a batch of 2x2 matrices."""
    det = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
    inv = np.empty_like(J)
    inv[..., 0, 0] = J[..., 1, 1] / det
    inv[..., 1, 1] = J[..., 0, 0] / det
    inv[..., 0, 1] = -J[..., 0, 1] / det
    inv[..., 1, 0] = -J[..., 1, 0] / det
    return inv


class OracleDisc:
    """Degree-p discretisation on an OracleMesh."""

    def __init__(self, mesh: OracleMesh, p: int):
        if not (1 <= p <= 4):
            raise ValueError("degree p must be in 1..4")
        self.mesh = mesh
        self.p = p
        self.nphi = basis.n_phi(p)
        self.npsi = basis.n_psi(p)
        P = mesh.P
        # Jacobian of T_i^{-1} (eq. linmap): columns P1-P0, P2-P0
        J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)  # [ne, 2(x), 2(xi)]
        self.Jmain = J
        self.Jinv = _inv2(J)  # d xi / d x
        self.tri_pts, self.tri_w = triangle_rule(p + 2)
        self.line_t, self.line_w = gauss_legendre_01(p + 2)

    # ------------------------------------------------------------------ main grid
    def main_ref_coords(self, i, x):
        """xi = T_i(x) for points x (given in triangle i's unwrapped frame)."""
        d = x - self.mesh.P[i, 0][..., None, :]
        return np.einsum("...ab,...qb->...qa", self.Jinv[i], d)

    def phi_phys(self, i, x):
        xi = self.main_ref_coords(i, x)
        return basis.phi(self.p, xi[..., 0], xi[..., 1])

    def grad_phi_phys(self, i, x):
        xi = self.main_ref_coords(i, x)
        g = basis.grad_phi(self.p, xi[..., 0], xi[..., 1])  # [..., q, k, 2(xi)]
        # grad_x phi = J^{-T} grad_xi phi
        return np.einsum("...ab,...qka->...qkb", self.Jinv[i], g)

    def main_mass(self):
        """Mbar_i (eq. Mi) by quadrature over each physical triangle, [ne, Nphi, Nphi]."""
        m = self.mesh
        u, v = self.tri_pts[:, 0], self.tri_pts[:, 1]
        P = m.P
        x = P[:, None, 0] + u[None, :, None] * (P[:, None, 1] - P[:, None, 0]) + \
            v[None, :, None] * (P[:, None, 2] - P[:, None, 0])
        jac = 2.0 * m.area
        ph = self.phi_phys(np.arange(m.ne), x)  # [ne, q, k]
        return np.einsum("q,e,eqk,eql->ekl", self.tri_w, jac, ph, ph)

    def main_weights(self):
        """int_{T_i} phi_k^(i) dx, [ne, Nphi]."""
        m = self.mesh
        u, v = self.tri_pts[:, 0], self.tri_pts[:, 1]
        P = m.P
        x = P[:, None, 0] + u[None, :, None] * (P[:, None, 1] - P[:, None, 0]) + \
            v[None, :, None] * (P[:, None, 2] - P[:, None, 0])
        ph = self.phi_phys(np.arange(m.ne), x)
        return np.einsum("q,e,eqk->ek", self.tri_w, 2.0 * m.area, ph)

    def main_node_xy(self):
        """Physical position of every main DOF node, [ne, Nphi, 2] (unwrapped frames)."""
        nd = basis.main_nodes(self.p)
        P = self.mesh.P
        return P[:, None, 0] + nd[None, :, 0, None] * (P[:, None, 1] - P[:, None, 0]) + \
            nd[None, :, 1, None] * (P[:, None, 2] - P[:, None, 0])

    def dual_node_xy(self):
        """Physical position of every dual DOF node, [nd, Npsi, 2] (left triangle's frame)."""
        m = self.mesh
        p = self.p
        bl = m.centroid[m.left]
        br = np.where(m.interior[:, None], m.centroid[np.maximum(m.right, 0)] - m.shift, np.nan)
        out = np.empty((m.nd, self.npsi, 2))
        for k, (a, b) in enumerate(basis.dual_node_ab(p)):
            xi, eta = a / p, b / p
            if a + b <= p:
                out[:, k] = bl + xi * (m.A - bl) + eta * (m.B - bl)
            else:
                out[:, k] = br + (1 - eta) * (m.A - br) + (1 - xi) * (m.B - br)
        return out

    # ------------------------------------------------------------------ edge blocks
    def edge_blocks(self, J):
        """Blocks for the edges in index array J (all must be interior or all boundary
        edges are handled with the right half absent).

        Returns dict with
          Mhat [E, Npsi, Npsi]; Ql, Qr [E, Npsi, Nphi, 2]; Dl, Dr [E, Nphi, Npsi, 2].
        Qr, Dr are zero for boundary edges.
        """
        m = self.mesh
        p = self.p
        J = np.asarray(J, dtype=np.int64)
        E = J.size
        L = m.left[J]
        R = m.right[J]
        inner = R >= 0
        Rs = np.where(inner, R, L)  # placeholder index for boundary edges
        A, B = m.A[J], m.B[J]
        shift = m.shift[J]
        bl = m.centroid[L]
        br = m.centroid[Rs] - shift
        n = m.normal[J]
        glen = m.edge_len[J]
        u, v = self.tri_pts[:, 0], self.tri_pts[:, 1]
        w = self.tri_w

        # left half: x = b_l + u (A - b_l) + v (B - b_l), dual coords (xi, eta) = (u, v)
        xl = bl[:, None] + u[None, :, None] * (A - bl)[:, None] + v[None, :, None] * (B - bl)[:, None]
        dl = A - bl
        el = B - bl
        jl = np.abs(dl[:, 0] * el[:, 1] - dl[:, 1] * el[:, 0])
        psi_l = basis.psi(p, np.broadcast_to(u, (E, u.size)), np.broadcast_to(v, (E, v.size)))
        # right half: x = b_r + u (A - b_r) + v (B - b_r) = b_r + (1-eta)(A-b_r) + (1-xi)(B-b_r)
        xr = br[:, None] + u[None, :, None] * (A - br)[:, None] + v[None, :, None] * (B - br)[:, None]
        dr = A - br
        er = B - br
        jr = np.abs(dr[:, 0] * er[:, 1] - dr[:, 1] * er[:, 0]) * inner
        psi_r = basis.psi(p, np.broadcast_to(1.0 - v, (E, v.size)), np.broadcast_to(1.0 - u, (E, u.size)))

        Mhat = np.einsum("q,e,eqk,eql->ekl", w, jl, psi_l, psi_l) + \
            np.einsum("q,e,eqk,eql->ekl", w, jr, psi_r, psi_r)

        # edge points x(tau) = A + tau (B - A); on the diagonal (xi, eta) = (1 - tau, tau)
        t, wt = self.line_t, self.line_w
        xe = A[:, None] + t[None, :, None] * (B - A)[:, None]
        psi_e = basis.psi(p, np.broadcast_to(1.0 - t, (E, t.size)) - 0.0,
                          np.broadcast_to(t, (E, t.size)))

        # volume and line integrals for the left triangle (sigma = +1)
        gphi_l = self.grad_phi_phys(L, xl)                      # [E, q, Nphi, 2]
        phi_le = self.phi_phys(L, xe)                           # [E, qe, Nphi]
        vol_l = np.einsum("q,e,eqk,eqlc->eklc", w, jl, psi_l, gphi_l)
        line_l = np.einsum("q,e,eqk,eql,ec->eklc", wt, glen, psi_e, phi_le, n)
        Ql = vol_l - (+1.0) * line_l
        vol_lD = np.einsum("q,e,eqkc,eql->eklc", w, jl, gphi_l, psi_l)
        line_lD = np.einsum("q,e,eqk,eql,ec->eklc", wt, glen, phi_le, psi_e, n)
        Dl = (+1.0) * line_lD - vol_lD

        # right triangle (sigma = -1): evaluate phi^(r) in r's own frame (x + shift)
        gphi_r = self.grad_phi_phys(Rs, xr + shift[:, None])
        phi_re = self.phi_phys(Rs, xe + shift[:, None])
        vol_r = np.einsum("q,e,eqk,eqlc->eklc", w, jr, psi_r, gphi_r)
        line_r = np.einsum("q,e,eqk,eql,ec->eklc", wt, glen * inner, psi_e, phi_re, n)
        Qr = vol_r - (-1.0) * line_r
        vol_rD = np.einsum("q,e,eqkc,eql->eklc", w, jr, gphi_r, psi_r)
        line_rD = np.einsum("q,e,eqk,eql,ec->eklc", wt, glen * inner, phi_re, psi_e, n)
        Dr = (-1.0) * line_rD - vol_rD
        return {"Mhat": Mhat, "Ql": Ql, "Qr": Qr, "Dl": Dl, "Dr": Dr}
