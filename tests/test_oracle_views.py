"""Pins of the oracle's view-count search (CPU only).

The search accepts the first view count whose A has kappa <= kappa_max
(Section II-A, Eq. 2).  Pinned by: the closed-form rejection of counts with
fewer rays than pixels; LAPACK's matrix_rank and cond on the accepted and the
rejected matrices (accepted means numerically full rank, a rejected square-or-
taller matrix is rank deficient or ill-conditioned beyond kappa_max); and the
effect the paper attributes to Eq. 2 -- on a 16^2 grid with 24 bins, 12 views
at uniform angles give a rank-deficient A (the views' symmetry) while the
Eq. 2 shifts give full rank with the same 12 views.
"""
import numpy as np

from oracle.siddon import system_matrix_csr
from oracle.views import view_search
from synthetic.workloads import SCANNER, image_side_cm


def _geom(side, bins, sched):
    return {"side": side, "n_views": 1, "n_bins": bins, "src_iso_cm": SCANNER["src_iso_cm"],
            "src_det_cm": SCANNER["src_det_cm"], "fan_deg": SCANNER["fan_deg"], "fov_side_cm": image_side_cm(),
            "angle_schedule": sched}


def test_fewer_rays_than_pixels_rejected_without_build():
    v, trials = view_search(_geom(16, 24, 1), 1, 10)
    assert v == 0
    assert all(not ok and k == np.inf for _, ok, k in trials)     # 10 x 24 < 256 rays
    assert [t[0] for t in trials] == list(range(1, 11))


def test_accepted_and_rejected_against_lapack():
    for sched in (0, 1):
        g = _geom(16, 32, sched)
        v, trials = view_search(g, 8, 20, kappa_max=1e8)
        assert v > 0 and trials[-1][0] == v and trials[-1][1]
        for vv, ok, kappa in trials:
            gg = dict(g, n_views=vv)
            A = system_matrix_csr(gg).toarray()
            assert abs(np.linalg.cond(A) / kappa - 1.0) < 1e-6
            if ok:
                assert np.linalg.matrix_rank(A) == A.shape[1]
            else:
                # 8 x 32 = 256 rays for 256 pixels: square and singular
                assert np.linalg.matrix_rank(A) < A.shape[1] or kappa > 1e8


def test_eq2_shifts_restore_full_rank():
    # uniform angles: 12 views of a 16^2 grid with 24 bins leave A singular;
    # the Eq. 2 schedule reaches full rank with the same 12 views
    vu, tu = view_search(_geom(16, 24, 0), 12, 16)
    v2, t2 = view_search(_geom(16, 24, 1), 12, 16)
    assert (vu, v2) == (13, 12)
    A = system_matrix_csr(dict(_geom(16, 24, 0), n_views=12)).toarray()
    assert np.linalg.matrix_rank(A) < A.shape[1]
    A = system_matrix_csr(dict(_geom(16, 24, 1), n_views=12)).toarray()
    assert np.linalg.matrix_rank(A) == A.shape[1]
