"""Write oracle-only expected values for the GPU parity tests.

    python tests/golden/make_golden.py [c3]

Calls only the seeded workload generator and the CPU oracle (never the GPU
library).  Output: c3_n8192_oracle_lambda.txt -- the eigenvalues of the plain
FP64 PFSM oracle for the N=8192 mixed-precision workload (2048 occupied +
6144 unoccupied levels, 3-fold clusters every 32 levels, ||K||_F = 5e-3,
32 slices of 256, halo 128, 3 folded-spectrum iterations, q = 2).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.pfsm_ref import pfsm_ref, eig_error  # noqa: E402
from pfsm_workloads import CONFIGS, prescribed_problem, uniform_layout  # noqa: E402


def make_c3():
    cfg = CONFIGS["c3_n8192"]
    t = time.time()
    A, V, lam_ex, _ = prescribed_problem(cfg.n, cfg.n_occ, cfg.kappa, cfg.seed_base, cfg.clusters)
    A, V = A.numpy(), V.numpy()
    print("generated in %.1f s" % (time.time() - t), flush=True)
    t = time.time()
    lam, _, info = pfsm_ref(A, V, uniform_layout(cfg.n, cfg.slice_size), cfg.halo, cfg.iterations, 2)
    print("oracle in %.1f s, info %d, error vs prescribed %.3e" % (time.time() - t, info, eig_error(lam, lam_ex)),
          flush=True)
    assert info == 0
    path = os.path.join(HERE, "c3_n8192_oracle_lambda.txt")
    with open(path, "w") as f:
        f.write("# oracle PFSM eigenvalues, workload c3_n8192 (see make_golden.py); one value per line\n")
        for x in lam:
            f.write("%.17e\n" % x)
    print("wrote", path)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3"]
    if "c3" in which:
        make_c3()
