"""Pressure Schur system and its solution (Section 3.3, eq. pressure_final).

K p |_i = sum_{j in S_i} D_ij Mhat_j^{-1} (Q_{l(j),j} p_l + Q_{r(j),j} p_r)

assembled as a block-sparse matrix from the physical-quadrature blocks of
``operators``.  Boundary (wall) edges carry no pressure coupling: K sums
over interior edges only (reading: wall dual cells hold prescribed velocity
and enter the right-hand side only).

Sign reading: with D = -Q^T (Section 3.3, after eq. ad5) K is symmetric
NEGATIVE semi-definite, a discrete Laplacian; the paper calls the pressure
system "symmetric and semi-positive definite", which holds for -K.  Plain
conjugate gradients (Section 3.3) are therefore run on -K p = -b.

Null space and gauge readings: on a periodic (or all-wall) connected mesh
K 1 = 0 for the nodal coefficient vector 1, and 1^T D v = 0.  The right-hand
side is projected onto 1^perp (Euclidean) and the returned pressure is the
unique solution with int_Omega p dx = 0.

Stopping rule reading: relative Euclidean residual ||r_k|| <= tol ||b|| on
coefficient vectors, x_0 = 0, true residual recomputed at exit.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse as sp

from .operators import OracleDisc


def _chunks(idx, size):
    for s in range(0, idx.size, size):
        yield idx[s:s + size]


def edge_solution_operators(disc: OracleDisc, J):
    """X = Mhat_j^{-1} [Q_lj | Q_rj] per velocity component, plus the D blocks."""
    blk = disc.edge_blocks(J)
    E = len(J)
    nphi, npsi = disc.nphi, disc.npsi
    Ql = blk["Ql"]  # [E, npsi, nphi, 2]
    Qr = blk["Qr"]
    rhs = np.concatenate([Ql.reshape(E, npsi, nphi * 2), Qr.reshape(E, npsi, nphi * 2)], axis=2)
    X = np.linalg.solve(blk["Mhat"], rhs)  # [E, npsi, 4 nphi]
    Xl = X[:, :, : 2 * nphi].reshape(E, npsi, nphi, 2)
    Xr = X[:, :, 2 * nphi:].reshape(E, npsi, nphi, 2)
    return Xl, Xr, blk


def assemble_K(disc: OracleDisc, chunk: int = 4096) -> sp.csr_matrix:
    """Block-sparse K of eq. pressure_final, [ne*Nphi, ne*Nphi]."""
    m = disc.mesh
    nphi = disc.nphi
    rows, cols, vals = [], [], []
    kk, ll = np.meshgrid(np.arange(nphi), np.arange(nphi), indexing="ij")
    interior = np.nonzero(m.interior)[0]
    for J in _chunks(interior, chunk):
        Xl, Xr, blk = edge_solution_operators(disc, J)
        tri = {"l": m.left[J], "r": m.right[J]}
        Dm = {"l": blk["Dl"], "r": blk["Dr"]}
        Xm = {"l": Xl, "r": Xr}
        for s in ("l", "r"):
            for t in ("l", "r"):
                B = np.einsum("ekmc,emlc->ekl", Dm[s], Xm[t])  # [E, nphi, nphi]
                rows.append((tri[s][:, None, None] * nphi + kk[None]).ravel())
                cols.append((tri[t][:, None, None] * nphi + ll[None]).ravel())
                vals.append(B.ravel())
    n = m.ne * nphi
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def gradient(disc: OracleDisc, p_main: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """ghat_j = Mhat_j^{-1} (Q_lj p_l + Q_rj p_r) (eq. ad4.2 with lambda = 1).

    p_main [ne, Nphi]  ->  [nd, 2, Npsi] (zero on boundary edges).
    """
    m = disc.mesh
    out = np.zeros((m.nd, 2, disc.npsi))
    interior = np.nonzero(m.interior)[0]
    for J in _chunks(interior, chunk):
        Xl, Xr, _ = edge_solution_operators(disc, J)
        g = np.einsum("ekmc,em->eck", Xl, p_main[m.left[J]]) + \
            np.einsum("ekmc,em->eck", Xr, p_main[m.right[J]])
        out[J] = g
    return out


def divergence(disc: OracleDisc, v_dual: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """(D v)_i = sum_{j in S_i} D_ij v_j (eq. D), v_dual [nd, 2, Npsi] -> [ne, Nphi].

    Interior edges only (wall cells excluded, as for K).
    """
    m = disc.mesh
    out = np.zeros((m.ne, disc.nphi))
    interior = np.nonzero(m.interior)[0]
    for J in _chunks(interior, chunk):
        blk = disc.edge_blocks(J)
        vj = v_dual[J]  # [E, 2, npsi]
        yl = np.einsum("ekmc,ecm->ek", blk["Dl"], vj)
        yr = np.einsum("ekmc,ecm->ek", blk["Dr"], vj)
        np.add.at(out, m.left[J], yl)
        np.add.at(out, m.right[J], yr)
    return out


def schur_apply(K: sp.csr_matrix, p_main: np.ndarray) -> np.ndarray:
    return (K @ p_main.reshape(-1)).reshape(p_main.shape)


def project_mean(b: np.ndarray) -> np.ndarray:
    """Euclidean projection onto the complement of the coefficient vector 1."""
    return b - b.mean()


def gauge(disc: OracleDisc, p_main: np.ndarray) -> np.ndarray:
    """Shift p by a constant so that int_Omega p dx = 0."""
    w = disc.main_weights()
    integral = float((w * p_main).sum())
    return p_main - integral / disc.mesh.domain_area


def cg(K: sp.csr_matrix, b: np.ndarray, tol: float = 1e-12, maxit: int = 100000,
       x0: np.ndarray | None = None, max_seconds: float | None = None, matvec=None):
    """Plain conjugate gradients on A = -K for A x = -b (b projected onto 1^perp).

    matvec: optional v -> K v (the same product by another library routine, e.g. a threaded
    sparse kernel); default K @ v.
    Returns (x, info) with info = {iters, rel_res, rel_res_true, converged, seconds}.
    """
    t0 = time.perf_counter()
    Kv = (lambda v: K @ v) if matvec is None else matvec
    shape = b.shape
    bb = -project_mean(b.reshape(-1))
    x = np.zeros_like(bb) if x0 is None else x0.reshape(-1).copy()
    r = bb - (-Kv(x))
    d = r.copy()
    rr = float(r @ r)
    nb = float(np.sqrt(bb @ bb))
    it = 0
    converged = nb == 0.0 or np.sqrt(rr) <= tol * nb
    while not converged and it < maxit:
        q = -Kv(d)
        alpha = rr / float(d @ q)
        x += alpha * d
        r -= alpha * q
        rr_new = float(r @ r)
        it += 1
        if np.sqrt(rr_new) <= tol * nb:
            converged = True
            rr = rr_new
            break
        beta = rr_new / rr
        rr = rr_new
        d = r + beta * d
        if max_seconds is not None and time.perf_counter() - t0 > max_seconds:
            break
    rt = bb - (-Kv(x))
    info = {
        "iters": it,
        "rel_res": float(np.sqrt(rr) / nb) if nb > 0 else 0.0,
        "rel_res_true": float(np.sqrt(rt @ rt) / nb) if nb > 0 else 0.0,
        "converged": bool(converged),
        "seconds": time.perf_counter() - t0,
    }
    return x.reshape(shape), info


def row_block_matvec(K: sp.csr_matrix, nthreads: int):
    """v -> K v computed as nthreads row blocks of K on a thread pool (scipy's sparse product
    releases the interpreter lock): the same per-row sums as K @ v, bitwise, on several cores."""
    from concurrent.futures import ThreadPoolExecutor
    n = K.shape[0]
    nb = max(1, int(nthreads))
    bounds = np.linspace(0, n, nb + 1).astype(np.int64)
    blocks = [K[bounds[i]:bounds[i + 1]] for i in range(nb)]
    pool = ThreadPoolExecutor(nb)

    def matvec(v):
        out = np.empty(n, dtype=np.result_type(K.dtype, v.dtype))

        def one(i):
            out[bounds[i]:bounds[i + 1]] = blocks[i] @ v
        list(pool.map(one, range(nb)))
        return out
    return matvec


def dense_bordered_solve(K: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """Tiny meshes: solve [[-K, 1], [1^T, 0]] [p; lam] = [-b; 0] by LU (numpy)."""
    n = K.shape[0]
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = -K.toarray()
    A[:n, n] = 1.0
    A[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[:n] = -project_mean(b.reshape(-1))
    sol = np.linalg.solve(A, rhs)
    return sol[:n].reshape(b.shape)


def pressure_rhs(disc: OracleDisc, v_star: np.ndarray, scale: float) -> np.ndarray:
    """b = scale * D v* (eq. pressure_IMEX without gravity/buoyancy sources; scale = 1/(a_ss dt))."""
    return scale * divergence(disc, v_star)


def velocity_correction(disc: OracleDisc, v_star: np.ndarray, p_main: np.ndarray,
                        coef: float) -> np.ndarray:
    """v = v* - coef * Mhat^{-1}(Q_l p_l + Q_r p_r), coef = a_ss dt (eq. nc.2 solved for v)."""
    return v_star - coef * gradient(disc, p_main)


def schur_rows(disc: OracleDisc, p_main: np.ndarray, tri_ids) -> np.ndarray:
    """(K p)_i for the triangles in tri_ids only, straight from eq. pressure_final:
    sum over the triangle's interior edges of D_ij Mhat_j^{-1} (Q_lj p_l + Q_rj p_r).
    Used to check large problems on a sample of rows without assembling K."""
    m = disc.mesh
    tri_ids = np.asarray(tri_ids, dtype=np.int64)
    J = np.unique(m.tri_edges[tri_ids].ravel())
    J = J[m.interior[J]]
    Xl, Xr, blk = edge_solution_operators(disc, J)
    g = np.einsum("ekmc,em->ekc", Xl, p_main[m.left[J]]) + \
        np.einsum("ekmc,em->ekc", Xr, p_main[m.right[J]])  # [E, npsi, 2]
    pos = {int(j): e for e, j in enumerate(J)}
    out = np.zeros((tri_ids.size, disc.nphi))
    for t, i in enumerate(tri_ids):
        for alpha in range(3):
            j = int(m.tri_edges[i, alpha])
            if not m.interior[j]:
                continue
            e = pos[j]
            Dm = blk["Dl"][e] if m.left[j] == i else blk["Dr"][e]
            out[t] += np.einsum("kmc,mc->k", Dm, g[e])
    return out
