"""Write oracle-only expected values for the GPU parity tests.

    python tests/golden/make_golden.py [c3] [c4]

Calls only the seeded workload generator and the CPU oracle (never the GPU
library).  Outputs, for the N=8192 mixed-precision workload (2048 occupied +
6144 unoccupied levels, 3-fold clusters every 32 levels, ||K||_F = 5e-3,
32 slices of 256, halo 128, 3 folded-spectrum iterations, q = 2):
  c3_n8192_oracle_lambda.txt -- the eigenvalues of the plain FP64 PFSM oracle;
  c3_n8192_oracle_vec_cols.txt, c3_n8192_oracle_vectors.npy -- the oracle's
    eigenvectors for 8 well separated eigenvalues (in each eighth of the
    spectrum the one with the widest gap to its neighbours; unique up to sign
    there, and the sign convention fixes the sign) and for one exactly
    degenerate 3-fold cluster (a subspace): the text file lists column index,
    group id (-1: single) and gap to the rest of the spectrum; the .npy holds
    the columns (11 x 8192, row-major, float64).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.pfsm_ref import pfsm_ref, eig_error  # noqa: E402
from pfsm_workloads import CONFIGS, batch_instance, batch_sizes, prescribed_problem, uniform_layout  # noqa: E402

SINGLE_COLS = 8


def make_c3():
    cfg = CONFIGS["c3_n8192"]
    t = time.time()
    A, V, lam_ex, _ = prescribed_problem(cfg.n, cfg.n_occ, cfg.kappa, cfg.seed_base, cfg.clusters)
    A, V = A.numpy(), V.numpy()
    print("generated in %.1f s" % (time.time() - t), flush=True)
    t = time.time()
    lam, Vn, info = pfsm_ref(A, V, uniform_layout(cfg.n, cfg.slice_size), cfg.halo, cfg.iterations, 2)
    print("oracle in %.1f s, info %d, error vs prescribed %.3e" % (time.time() - t, info, eig_error(lam, lam_ex)),
          flush=True)
    assert info == 0
    path = os.path.join(HERE, "c3_n8192_oracle_lambda.txt")
    with open(path, "w") as f:
        f.write("# oracle PFSM eigenvalues, workload c3_n8192 (see make_golden.py); one value per line\n")
        for x in lam:
            f.write("%.17e\n" % x)
    print("wrote", path)
    gaps = np.minimum(np.r_[np.inf, np.diff(lam)], np.r_[np.diff(lam), np.inf])
    rows = []
    for r in range(SINGLE_COLS):
        lo, hi = r * cfg.n // SINGLE_COLS, (r + 1) * cfg.n // SINGLE_COLS
        c = lo + int(np.argmax(gaps[lo:hi]))
        rows.append((c, -1, gaps[c]))
    # the exactly degenerate 3-fold cluster at the middle of the spectrum (its estimates
    # agree to the method error, far below the gap to the other levels)
    c0 = 32 * (cfg.n // 64)
    assert lam[c0 + 2] - lam[c0] <= 1e-6 * np.max(np.abs(lam))
    g = min(lam[c0] - lam[c0 - 1], lam[c0 + 3] - lam[c0 + 2])
    rows += [(c0 + t, 0, g) for t in range(3)]
    cols = [r[0] for r in rows]
    path = os.path.join(HERE, "c3_n8192_oracle_vec_cols.txt")
    with open(path, "w") as f:
        f.write("# oracle PFSM eigenvector columns stored in c3_n8192_oracle_vectors.npy (see make_golden.py)\n")
        f.write("# column group gap\n")
        for c, grp, gp in rows:
            f.write("%d %d %.17e\n" % (c, grp, gp))
    print("wrote", path)
    path = os.path.join(HERE, "c3_n8192_oracle_vectors.npy")
    np.save(path, np.ascontiguousarray(Vn[:, cols].T))
    print("wrote", path)


def make_c4():
    """c4_batch_oracle_lambda.txt: oracle eigenvalues of the first instance of every
    order in the 64-instance batched workload (slices of 128, halo 64, 3
    iterations, q = 2); one line per instance: index b, order n, n eigenvalues."""
    cfg = CONFIGS["c4_batched"]
    ns = batch_sizes(64)
    path = os.path.join(HERE, "c4_batch_oracle_lambda.txt")
    with open(path, "w") as f:
        f.write("# oracle PFSM eigenvalues of batched instances (see make_golden.py): b n lambda_0 .. lambda_{n-1}\n")
        for n in sorted(set(ns)):
            b = ns.index(n)
            A, V, lam_ex, _ = batch_instance(b, n, cfg.kappa, cfg.seed_base)
            t = time.time()
            lam, _, info = pfsm_ref(A.numpy(), V.numpy(), uniform_layout(n, cfg.slice_size), cfg.halo,
                                    cfg.iterations, 2)
            assert info == 0
            print("instance %d (n=%d): oracle in %.1f s, error vs prescribed %.3e" %
                  (b, n, time.time() - t, eig_error(lam, lam_ex)), flush=True)
            f.write("%d %d " % (b, n) + " ".join("%.17e" % x for x in lam) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c4"]
    if "c3" in which:
        make_c3()
    if "c4" in which:
        make_c4()
