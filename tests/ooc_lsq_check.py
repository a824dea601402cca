"""Host-side check of out-of-core solutions against the oracle's sparse A.

bench.py --save-check DIR writes, for each slice count of its out-of-core
leg, a few solutions X, their sinograms B and phantoms (DIR/<workload>_S<S>.npz).
This script rebuilds A with the oracle's Siddon ray tracer (independent of the
GPU build) and checks, per saved slice:
  * noisy slices: least-squares optimality ||A^T (b - A x)|| / (||A||_F ||b - A x||)
    below the bound of a backward-stable solution,
    100 u (||A||_F ||x|| / ||r|| + 1) with u = 2^-53 (Eq. 4: x is the
    least-squares solution);
  * noise-free slices: x equals the phantom to 1e-10 relative.
Usage: python tests/ooc_lsq_check.py DIR WORKLOAD.  Exit status 1 on a failure.
"""
import glob
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle.siddon import system_matrix_csr  # noqa: E402
from oracle import lsq  # noqa: E402
from synthetic import get_workload  # noqa: E402


def main(directory, workload):
    A = system_matrix_csr(get_workload(workload).geometry())
    nA = np.sqrt(A.multiply(A).sum())
    ok = True
    for f in sorted(glob.glob(os.path.join(directory, "%s_S*.npz" % workload))):
        d = np.load(f)
        X, B, Xt, clean = d["X"], d["B"], d["Xtrue"], d["noise_free"]
        for c in range(X.shape[1]):
            if clean[c]:
                e = lsq.rel_err(X[:, c:c + 1], Xt[:, c:c + 1])[0]
                good = e <= 1e-10
                print("%s slice %d (noise-free): recovery %.2e %s" % (os.path.basename(f), c, e, "ok" if good else "FAIL"))
            else:
                r = B[:, c] - A @ X[:, c]
                opt = lsq.ls_optimality(A, X[:, c:c + 1], B[:, c:c + 1])[0]
                bound = 100 * 2.0 ** -53 * (nA * np.linalg.norm(X[:, c]) / np.linalg.norm(r) + 1.0)
                good = opt <= bound
                print("%s slice %d: LS optimality %.2e (bound %.2e) %s" % (os.path.basename(f), c, opt, bound,
                                                                          "ok" if good else "FAIL"))
            ok = ok and good
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1], sys.argv[2]))
