"""Writes c2_pressure_sample.txt: the oracle's pressure on the 128x128x2, p = 3 periodic
workload at sampled DOFs.  Calls only the oracle (and the seeded input generators).

Workload: inputs.lattice_mesh(128, seed=2); v* = random_fourier_field(102, kmax=8) at the
dual nodes; b = (1/(a_ss dt)) D v* with dt = 0.5 h, h = 2 pi / 128, a_ss = the SDIRK3
diagonal (eq. pressure_IMEX without sources); CG on -K to 1e-12 (eq. pressure_final, plain
matrix-free CG of Section 3.3 in its assembled oracle form); gauge int p = 0.

    python tests/golden/make_c2_sample.py     (about a minute on one core)
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import solve  # noqa: E402
from oracle.mesh import OracleMesh  # noqa: E402
from oracle.operators import OracleDisc  # noqa: E402
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field  # noqa: E402

A_SS = 0.43586652150845967
N, P, SEED, RHS_SEED, NSAMPLE = 128, 3, 2, 102, 512


def main():
    xy, tri, per = lattice_mesh(N, seed=SEED)
    od = OracleDisc(OracleMesh(xy, tri, per), P)
    coef = A_SS * 0.5 * (2 * math.pi / N)
    vs = random_fourier_field(RHS_SEED, kmax=8)(od.dual_node_xy()).transpose(0, 2, 1)
    b = solve.pressure_rhs(od, np.ascontiguousarray(vs), 1.0 / coef)
    K = solve.assemble_K(od)
    x, info = solve.cg(K, b, tol=1e-12, maxit=100000)
    x = solve.gauge(od, x)
    r = solve.project_mean(b).ravel() - K @ x.ravel()
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.sort(rng.choice(x.size, NSAMPLE, replace=False))
    with open(os.path.join(HERE, "c2_pressure_sample.txt"), "w") as f:
        f.write("# Oracle pressure, 128x128x2 periodic jittered mesh (seed 2), p = 3, rhs seed 102,\n")
        f.write("# CG to 1e-12 on -K (eq. pressure_final), gauge int p = 0; written by make_c2_sample.py\n")
        f.write(f"# cg_iters {info['iters']} rel_res_true {np.linalg.norm(r) / np.linalg.norm(solve.project_mean(b)):.3e}\n")
        f.write(f"# norm2_p {np.linalg.norm(x):.17e} maxabs_p {np.abs(x).max():.17e}\n")
        f.write("# flat_dof_index value\n")
        for i in idx:
            f.write(f"{i} {x.ravel()[i]:.17e}\n")
    print("cg iters", info["iters"], "rel_res_true", np.linalg.norm(r) / np.linalg.norm(b))


if __name__ == "__main__":
    main()
