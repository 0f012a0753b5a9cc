"""Staggered mesh bookkeeping (Section 3.1).

From vertex coordinates and counter-clockwise triangles the oracle builds,
with its own loops:

* per-triangle vertex coordinates, unwrapped for periodic boxes so that each
  triangle is a compact set in the plane (image of every vertex nearest to
  the triangle's first vertex);
* the edge list Gamma_j with left/right triangles l(j), r(j).  The paper lets
  l and r be assigned arbitrarily; the convention used on both sides of the
  library boundary is: edges are numbered in order of first appearance while
  scanning triangles i = 0, 1, ... and their local edges alpha = 0, 1, 2
  (vertex pairs (v0,v1), (v1,v2), (v2,v0)); l(j) is the triangle that first
  references the edge, its endpoints A -> B follow l's counter-clockwise
  order (so l lies to the left of A -> B), and the unit normal n_j points
  from l to r (the right-hand normal of A -> B);
* the periodic shift s_j: r's copy of the edge equals l's copy plus s_j.

A boundary edge (walls) has r(j) = -1; its dual cell is the left
sub-triangle only (Section 3.1).
"""
from __future__ import annotations

import numpy as np


class MeshError(ValueError):
    pass


class OracleMesh:
    def __init__(self, xy, tri, period=None):
        xy = np.asarray(xy, dtype=np.float64)
        tri = np.asarray(tri, dtype=np.int64)
        self.xy = xy
        self.tri = tri
        self.period = None if period is None else np.asarray(period, dtype=np.float64)
        self.ne = tri.shape[0]
        self.nv = xy.shape[0]

        P = xy[tri]  # [ne, 3, 2]
        if self.period is not None:
            d = P - P[:, :1, :]
            P = P - np.round(d / self.period) * self.period
        self.P = P
        e1 = P[:, 1] - P[:, 0]
        e2 = P[:, 2] - P[:, 0]
        det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
        if np.any(det <= 0.0):
            raise MeshError("triangle with non-positive area (orientation must be ccw)")
        self.area = 0.5 * det  # |T_i|
        self.centroid = P.mean(axis=1)

        edge_of = {}
        left, right, al, ar = [], [], [], []
        tri_edges = np.empty((self.ne, 3), dtype=np.int64)
        for i in range(self.ne):
            for alpha in range(3):
                va = int(tri[i, alpha])
                vb = int(tri[i, (alpha + 1) % 3])
                key = (va, vb) if va < vb else (vb, va)
                j = edge_of.get(key)
                if j is None:
                    j = len(left)
                    edge_of[key] = j
                    left.append(i)
                    right.append(-1)
                    al.append(alpha)
                    ar.append(-1)
                else:
                    if right[j] != -1:
                        raise MeshError("non-manifold edge (shared by more than two triangles)")
                    lj, alj = left[j], al[j]
                    if (int(tri[lj, alj]), int(tri[lj, (alj + 1) % 3])) != (vb, va):
                        raise MeshError("inconsistent orientation across an edge")
                    if lj == i:
                        raise MeshError("edge joins a triangle to itself")
                    right[j] = i
                    ar[j] = alpha
                tri_edges[i, alpha] = j
        self.nd = len(left)
        self.left = np.array(left, dtype=np.int64)
        self.right = np.array(right, dtype=np.int64)
        self.alpha_l = np.array(al, dtype=np.int64)
        self.alpha_r = np.array(ar, dtype=np.int64)
        self.tri_edges = tri_edges
        self.interior = self.right >= 0

        L = self.left
        self.A = P[L, self.alpha_l]
        self.B = P[L, (self.alpha_l + 1) % 3]
        shift = np.zeros((self.nd, 2))
        m = self.interior
        R = self.right[m]
        # r's local edge runs B -> A in r's own frame
        Br = P[R, self.alpha_r[m]]
        shift[m] = Br - self.B[m]
        self.shift = shift
        if self.period is None and np.any(np.abs(shift) > 1e-12 * (1 + np.abs(self.B).max())):
            raise MeshError("edge endpoints disagree between neighbours")
        t = self.B - self.A
        self.edge_len = np.sqrt((t * t).sum(axis=1))
        self.normal = np.stack([t[:, 1], -t[:, 0]], axis=1) / self.edge_len[:, None]

    @property
    def domain_area(self) -> float:
        return float(self.area.sum())
