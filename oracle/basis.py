"""Main and dual nodal bases (Section 3.2).

Main basis (Section 3.2, "simple nodal approach"): Lagrange polynomials of
total degree p on T_ref = {xi >= 0, eta >= 0, xi + eta <= 1}, N_phi =
(p+1)(p+2)/2.  Reading of the unspecified node set: the equispaced lattice
(a/p, b/p), a + b <= p, numbered with b outer and a inner.  The polynomials
are obtained by inverting the monomial Vandermonde matrix at the nodes.

Dual basis (Section 3.2, the p = 1 example and the split of R_ref into two
sub-triangles): nodes (a/p, b/p), a, b = 0..p on R_ref = [0,1]^2, numbered
k = b*(p+1) + a, N_psi = (p+1)^2.  On the lower sub-triangle xi + eta <= 1
psi_k equals the main basis function of node (a, b) (zero when the node lies
strictly above the diagonal).  On the upper sub-triangle psi_k equals the
main basis function of node rho(a, b) = (p-b, p-a) composed with the map
rho(xi, eta) = (1-eta, 1-xi) (zero when the node lies strictly below).
Reading of the garbled "1 - xi" of the p = 1 example: rho is the mirror
across the diagonal, which keeps the diagonal fixed pointwise and so gives
the C0 space the paper describes; point reflection would not.
"""
from __future__ import annotations

import numpy as np


def n_phi(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def n_psi(p: int) -> int:
    return (p + 1) * (p + 1)


def main_node_ab(p: int):
    """Integer lattice coordinates (a, b) of the main nodes, b outer, a inner."""
    return [(a, b) for b in range(p + 1) for a in range(p + 1 - b)]


def main_index(p: int):
    """Map (a, b) -> main node index."""
    return {ab: k for k, ab in enumerate(main_node_ab(p))}


def main_nodes(p: int) -> np.ndarray:
    return np.array(main_node_ab(p), dtype=np.float64) / p


def dual_node_ab(p: int):
    return [(a, b) for b in range(p + 1) for a in range(p + 1)]


def dual_nodes(p: int) -> np.ndarray:
    return np.array(dual_node_ab(p), dtype=np.float64) / p


def _exponents(p: int):
    return [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]


def _vander(p: int, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.stack([x ** i * y ** j for (i, j) in _exponents(p)], axis=-1)


def _vander_grad(p: int, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    cols = []
    for (i, j) in _exponents(p):
        dx = i * x ** max(i - 1, 0) * y ** j if i > 0 else np.zeros_like(x)
        dy = j * x ** i * y ** max(j - 1, 0) if j > 0 else np.zeros_like(x)
        cols.append(np.stack([dx, dy], axis=-1))
    return np.stack(cols, axis=-2)  # [..., nmono, 2]


_COEF_CACHE: dict = {}


def _coef(p: int) -> np.ndarray:
    if p not in _COEF_CACHE:
        nd = main_nodes(p)
        V = _vander(p, nd[:, 0], nd[:, 1])  # V[node, mono]
        _COEF_CACHE[p] = np.linalg.inv(V)  # phi_k = sum_m mono_m * C[m, k]
    return _COEF_CACHE[p]


def phi(p: int, xi, eta) -> np.ndarray:
    """Main basis values, shape [..., N_phi]."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    return _vander(p, xi, eta) @ _coef(p)


def grad_phi(p: int, xi, eta) -> np.ndarray:
    """Reference gradients d phi_k / d(xi, eta), shape [..., N_phi, 2]."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    G = _vander_grad(p, xi, eta)  # [..., nmono, 2]
    return np.einsum("...md,mk->...kd", G, _coef(p))


def psi(p: int, xi, eta) -> np.ndarray:
    """Dual basis values on R_ref, shape [..., N_psi] (definition of Section 3.2)."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    idx = main_index(p)
    lower = (xi + eta) <= 1.0
    ph_low = phi(p, xi, eta)
    ph_up = phi(p, 1.0 - eta, 1.0 - xi)
    out = np.zeros(xi.shape + (n_psi(p),))
    for k, (a, b) in enumerate(dual_node_ab(p)):
        if a + b <= p:
            out[..., k] += np.where(lower, ph_low[..., idx[(a, b)]], 0.0)
        if a + b >= p:
            out[..., k] += np.where(lower, 0.0, ph_up[..., idx[(p - b, p - a)]])
    return out
