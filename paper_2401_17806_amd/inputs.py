"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This module only draws random numbers and lays out lattice coordinates; it
holds none of the discretisation's arithmetic (no basis, no quadrature, no
operators).  Both sides receive the arrays it returns.

Meshes follow the experiments' setting of a square box covered by n x n
squares, each split on its diagonal into two counter-clockwise triangles
(Section 5, Taylor-Green vortex on [0, 2*pi]^2 with periodic boundaries).
Vertices strictly inside the box are jittered i.i.d. uniformly in
[-jitter*h, +jitter*h] per coordinate; vertices on the box boundary stay on
the lattice so that periodic images are exact shifts.

Velocity fields are seeded Gaussian random Fourier series with wavenumbers
0 < |k| <= kmax on a half-plane and amplitude proportional to |k|^-2.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "lattice_mesh",
    "FourierField",
    "random_fourier_field",
    "random_vector",
]


def lattice_mesh(n: int, *, length: float = 2.0 * math.pi, periodic: bool = True,
                 jitter: float = 0.1, seed: int = 1):
    """Jittered split-square lattice on [0, length]^2.

    Returns ``(xy, tri, period)``:
      * ``xy``  float64 [nv, 2] vertex coordinates;
      * ``tri`` int32 [ne, 3] counter-clockwise vertex ids per triangle;
      * ``period`` float64 [2] (periodic) or ``None`` (walls).

    Periodic: nv = n^2, ne = 2 n^2, vertex (a, b) has id a + n*b and the
    triangles of square (a, b) reference vertex ids modulo n.  Walls:
    nv = (n+1)^2, vertex (a, b) has id a + (n+1)*b.  Square s = a + n*b owns
    triangles 2s (lower-right) and 2s+1 (upper-left) of the diagonal from
    (a, b) to (a+1, b+1).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = length / n
    rng = np.random.Generator(np.random.PCG64(seed))
    m = n if periodic else n + 1
    a = np.arange(m, dtype=np.float64)
    X, Y = np.meshgrid(a * h, a * h, indexing="xy")  # [b, a]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    jit = rng.uniform(-jitter * h, jitter * h, size=xy.shape)
    ia = np.tile(np.arange(m), m)
    ib = np.repeat(np.arange(m), m)
    if periodic:
        inside = (ia > 0) & (ib > 0)
    else:
        inside = (ia > 0) & (ib > 0) & (ia < n) & (ib < n)
    xy = xy + jit * inside[:, None]

    def vid(aa, bb):
        if periodic:
            return (aa % n) + n * (bb % n)
        return aa + (n + 1) * bb

    tri = np.empty((2 * n * n, 3), dtype=np.int32)
    s = 0
    for b in range(n):
        for aa in range(n):
            v00, v10 = vid(aa, b), vid(aa + 1, b)
            v01, v11 = vid(aa, b + 1), vid(aa + 1, b + 1)
            tri[2 * s] = (v00, v10, v11)
            tri[2 * s + 1] = (v00, v11, v01)
            s += 1
    period = np.array([length, length]) if periodic else None
    return xy, tri, period


class FourierField:
    """Vector field v(x) = sum_k a_k cos(w k.x) + b_k sin(w k.x), w = 2 pi / length."""

    def __init__(self, k: np.ndarray, a: np.ndarray, b: np.ndarray, length: float):
        self.k = np.asarray(k, dtype=np.float64)  # [nk, 2]
        self.a = np.asarray(a, dtype=np.float64)  # [nk, 2]
        self.b = np.asarray(b, dtype=np.float64)  # [nk, 2]
        self.length = float(length)

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        shp = pts.shape[:-1]
        x = pts.reshape(-1, 2)
        w = 2.0 * math.pi / self.length
        phase = w * (x @ self.k.T)  # [npts, nk]
        out = np.cos(phase) @ self.a + np.sin(phase) @ self.b
        return out.reshape(shp + (2,))


def random_fourier_field(seed: int, *, kmax: int = 8, length: float = 2.0 * math.pi):
    """Gaussian random Fourier velocity field, amplitude ~ |k|^-2, 0 < |k| <= kmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = []
    for kx in range(0, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if kx == 0 and ky <= 0:
                continue  # half-plane: one of each +-k pair, k != 0
            if kx * kx + ky * ky <= kmax * kmax:
                ks.append((kx, ky))
    k = np.array(ks, dtype=np.float64)
    mag = np.sqrt((k * k).sum(axis=1))
    std = mag ** -2.0
    a = rng.standard_normal((len(k), 2)) * std[:, None]
    b = rng.standard_normal((len(k), 2)) * std[:, None]
    return FourierField(k, a, b, length)


def random_vector(shape, seed: int) -> np.ndarray:
    """Seeded standard-normal float64 array."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape)
