"""FP64 CPU oracle for the staggered DG pressure Schur-complement path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product path (``paper_2401_17806_amd``) never imports it, and this package
never imports the product path: the two share no code.  Inputs reach both
sides as plain arrays from ``paper_2401_17806_amd.inputs``.

What the oracle computes is the plain definition of the method's objects
(Tavelli & Boscheri, "A new class of efficient high order semi-Lagrangian
IMEX discontinuous Galerkin methods on staggered unstructured meshes"):

* main nodal basis on T_ref and the C0 dual basis on the split reference
  square (Section 3.2);
* per-edge dual mass matrix (eq. Mj), gradient operator (eq. ad5.2) and
  divergence operator (eq. D), each integrated in PHYSICAL space by Gauss
  quadrature over the sub-triangles T_{l(j),j}, T_{r(j),j} and the edge
  Gamma_j (Section 3.3), not through the reference factorisation of
  Section 3.4;
* the pressure Schur operator K = sum_j D_ij Mhat_j^-1 (Q_lj p_l + Q_rj p_r)
  of eq. pressure_final, assembled block-sparse, and its solution by plain
  conjugate gradients (Section 3.3) or, on tiny meshes, a dense bordered
  direct solve.

Readings where the paper is silent or garbled are documented where used
(module docstrings) and listed in the repository's design notes.
"""
from . import basis, quadrature, mesh, operators, solve  # noqa: F401
