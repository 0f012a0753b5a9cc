"""Gauss quadrature on [0, 1] and on triangles.

The paper integrates with "Gauss quadrature" without naming a rule
(Section 4, eq. intstage).  The oracle only needs rules that are exact for
the polynomial integrands of the operator definitions (degree <= 2p), so any
exact rule gives the same operators to rounding.

Triangle rule: collapsed (Duffy) tensor product of Gauss-Legendre rules.
With n points per direction it is exact for total degree <= 2n - 2.
"""
from __future__ import annotations

import numpy as np


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule on [0, 1]; exact to degree 2n - 1."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(n: int):
    """Points (u, v) and weights on T_ref = {u, v >= 0, u + v <= 1}; sum(w) = 1/2."""
    s, ws = gauss_legendre_01(n)
    t, wt = gauss_legendre_01(n)
    S, T = np.meshgrid(s, t, indexing="ij")
    WS, WT = np.meshgrid(ws, wt, indexing="ij")
    u = S
    v = (1.0 - S) * T
    w = WS * WT * (1.0 - S)
    return np.stack([u.ravel(), v.ravel()], axis=1), w.ravel()
