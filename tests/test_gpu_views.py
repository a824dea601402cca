"""GPU view-count search (ctqr_view_search) against the oracle's
(oracle.views.view_search: SVD condition numbers of the oracle's A).

Both accept the first view count whose A has full column rank with
kappa <= 1e8 (Section II-A, Eq. 2).  The cases are chosen so that every
rejected count is either short of rows or singular (kappa > 1e15 in the SVD)
and every accepted one has kappa < 1e4, far from the threshold on both sides,
so the GPU's estimate (a lower bound of kappa, FP64 factor) and the SVD take
the same decision.  Each estimated kappa of an accepted count must lie within
10% below the SVD's value.
"""
import numpy as np
import pytest

from oracle.views import view_search as oracle_view_search
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import view_search
from synthetic.workloads import SCANNER, image_side_cm

pytestmark = pytest.mark.gpu


def _geom(side, bins, sched):
    return {"side": side, "n_views": 1, "n_bins": bins, "src_iso_cm": SCANNER["src_iso_cm"],
            "src_det_cm": SCANNER["src_det_cm"], "fan_deg": SCANNER["fan_deg"], "fov_side_cm": image_side_cm(),
            "angle_schedule": sched}


@pytest.mark.parametrize("side,bins,sched,v_min,v_max", [
    (16, 24, 0, 12, 18),    # uniform angles: singular at 12 (the views' symmetry), accepted at 13
    (16, 24, 1, 12, 18),    # Eq. 2: accepted at 12
    (16, 32, 0, 7, 14),     # short of rows at 7, square and singular at 8, accepted at 9
    (24, 36, 1, 16, 20),    # square and singular at 16, accepted at 17
    (4, 6, 0, 4, 8),        # uniform: singular at 4
    (4, 6, 1, 4, 8),        # Eq. 2: full rank at 4
])
def test_view_search_matches_oracle(gpu, side, bins, sched, v_min, v_max):
    print("[case] view search", side, bins, sched, flush=True)
    g = _geom(side, bins, sched)
    vo, to = oracle_view_search(g, v_min, v_max, kappa_max=1e8)
    vg, tg = view_search(g, v_min, v_max, kappa_max=1e8, iters=40)
    print("oracle", vo, [(v, ok, "%.2e" % k) for v, ok, k in to])
    print("gpu   ", vg, [(t.views, t.status, "%.2e" % t.kappa) for t in tg])
    assert vg == vo and vo > 0
    assert [t.views for t in tg] == [t[0] for t in to]
    for t, (v, ok, kappa) in zip(tg, to):
        assert (t.status == 0) == ok
        if ok:
            assert t.kappa <= kappa * (1 + 1e-9) and t.kappa >= 0.9 * kappa
