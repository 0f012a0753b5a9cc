"""Writes c3_pressure_sample.txt: the oracle's pressure on the 512x512x2, p = 3 periodic
workload at sampled DOFs.  Calls only the oracle (and the seeded input generators).

Workload: inputs.lattice_mesh(512, seed=3); v* = random_fourier_field(103, kmax=8) at the
dual nodes; b = (1/(a_ss dt)) D v* with dt = 0.5 h, h = 2 pi / 512, a_ss = the SDIRK3
diagonal (eq. pressure_IMEX without sources); CG on -K to 1e-12 (eq. pressure_final, plain
matrix-free CG of Section 3.3 in its assembled oracle form); gauge int p = 0.

    python tests/golden/make_c3_sample.py [full_out.npy]   (about 20 GB of memory; the CG's
        sparse product K v runs as row blocks of the oracle's own product on every visible core,
        bitwise the same sums; about three hours on eight cores: 38058 CG iterations)
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import solve  # noqa: E402
from oracle.mesh import OracleMesh  # noqa: E402
from oracle.operators import OracleDisc  # noqa: E402
from paper_2401_17806_amd.inputs import lattice_mesh, random_fourier_field  # noqa: E402

A_SS = 0.43586652150845967
N, P, SEED, RHS_SEED, NSAMPLE = 512, 3, 3, 103, 1024


def main():
    t0 = time.perf_counter()
    xy, tri, per = lattice_mesh(N, seed=SEED)
    od = OracleDisc(OracleMesh(xy, tri, per), P)
    coef = A_SS * 0.5 * (2 * math.pi / N)
    vs = random_fourier_field(RHS_SEED, kmax=8)(od.dual_node_xy()).transpose(0, 2, 1)
    b = solve.pressure_rhs(od, np.ascontiguousarray(vs), 1.0 / coef)
    print(f"rhs done {time.perf_counter() - t0:.0f} s", flush=True)
    K = solve.assemble_K(od)
    print(f"K assembled, nnz {K.nnz}, {time.perf_counter() - t0:.0f} s", flush=True)
    x, info = solve.cg(K, b, tol=1e-12, maxit=400000,
                       matvec=solve.row_block_matvec(K, len(os.sched_getaffinity(0))))
    print(f"cg {info}, {time.perf_counter() - t0:.0f} s", flush=True)
    x = solve.gauge(od, x)
    bp = solve.project_mean(b).ravel()
    r = bp - K @ x.ravel()
    if len(sys.argv) > 1:
        np.save(sys.argv[1], x)
    rng = np.random.Generator(np.random.PCG64(11))
    idx = np.sort(rng.choice(x.size, NSAMPLE, replace=False))
    with open(os.path.join(HERE, "c3_pressure_sample.txt"), "w") as f:
        f.write("# Oracle pressure, 512x512x2 periodic jittered mesh (seed 3), p = 3, rhs seed 103,\n")
        f.write("# CG to 1e-12 on -K (eq. pressure_final), gauge int p = 0; written by make_c3_sample.py\n")
        f.write(f"# cg_iters {info['iters']} rel_res_true {np.linalg.norm(r) / np.linalg.norm(bp):.3e}\n")
        f.write(f"# norm2_p {np.linalg.norm(x):.17e} maxabs_p {np.abs(x).max():.17e}\n")
        f.write("# flat_dof_index value\n")
        for i in idx:
            f.write(f"{i} {x.ravel()[i]:.17e}\n")
    print("cg iters", info["iters"], "rel_res_true", np.linalg.norm(r) / np.linalg.norm(bp), flush=True)


if __name__ == "__main__":
    main()
