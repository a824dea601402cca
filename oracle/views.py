"""Oracle: the smallest number of views that gives A full column rank.

Test infrastructure only: the product never imports this package.

The direct method needs A of full column rank (Section II-A: the number of
projections is adjusted to the resolution so that A has full rank, and Eq. 2
shifts the angles of each quarter turn to break the symmetry of the data and
raise the rank; Section IV).  For each candidate view count v in order, the
oracle builds A with the Siddon oracle, takes its singular values (LAPACK SVD)
and accepts v when A has at least as many rows as columns and
kappa(A) = sigma_max / sigma_min <= kappa_max.  Counts with fewer rays than
pixels are rejected without building A.
"""
import numpy as np

from .siddon import system_matrix_csr


def view_search(geom, v_min, v_max, v_step=1, kappa_max=1e8):
    """(v_best or 0, [(v, full_rank, kappa)]) for the geometry dict `geom`
    (its n_views is replaced by each candidate)."""
    side, bins = geom["side"], geom["n_bins"]
    n = side * side
    trials = []
    for v in range(v_min, v_max + 1, v_step):
        if v * bins < n:
            trials.append((v, False, np.inf))
            continue
        g = dict(geom)
        g["n_views"] = v
        s = np.linalg.svd(system_matrix_csr(g).toarray(), compute_uv=False)
        kappa = s[0] / s[-1] if s[-1] > 0 else np.inf
        ok = bool(kappa <= kappa_max)
        trials.append((v, ok, kappa))
        if ok:
            return v, trials
    return 0, trials
