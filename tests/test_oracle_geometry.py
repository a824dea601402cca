"""Pins of the oracle's scanner geometry and system matrix (CPU only).

Each check ties the oracle to something other than itself: the paper's
printed sizes (Section III-B), closed forms of the angle schedule (Eq. 2),
an independent brute-force clipping derivation of A, and exact chord
lengths of rays through the image square.
"""
import math
import os

import numpy as np
import pytest

from synthetic import get_workload, WORKLOADS
from synthetic.workloads import image_side_cm, SCANNER
from oracle.geometry import projection_angles_deg, ray_endpoints, sizes, image_grid
from oracle.siddon import system_matrix_csr, siddon_ray
from oracle.clip import system_matrix_bruteforce, image_chord_lengths, chord_length


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_scanner.txt")


def _golden():
    kv = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = (t.strip() for t in line.split("=", 1))
            kv[k] = float(v)
    return kv


def test_paper_sizes():
    # Section III-B: detectors x projections rays, 512^2 pixels; the dense
    # FP64 A is about 560 GB (values as the paper prints them, golden file)
    t = _golden()
    w = get_workload("paper512")
    g = w.geometry()
    m, n = sizes(g)
    assert (w.n_bins, w.n_views, w.side) == (t["detectors"], t["projections"], t["image_side"])
    assert (m, n) == (t["A_rows"], t["A_cols"])
    assert abs(m * n * 8 / 1e9 - t["A_fp64_storage_gb_about"]) < 2.0


def test_table1_scanner():
    t = _golden()
    assert SCANNER == {"src_iso_cm": t["scan_radius_cm"], "src_det_cm": t["source_to_detector_cm"],
                       "fan_deg": t["fan_angle_deg"]}
    # a full turn: the uniform schedule spans 360 degrees in equal steps
    th = projection_angles_deg(int(t["projections"]), schedule=0)
    assert abs(th[1] - th[0] - t["trajectory_deg"] / t["projections"]) < 1e-12
    # image square circumscribing the circle R sin(15 deg) every fan covers
    L = image_side_cm()
    assert abs(L / 2 - 75.0 * math.sin(math.radians(15.0))) < 1e-12


@pytest.mark.parametrize("name", ["paper512", "ct512", "ct256"])
def test_every_ray_crosses_the_image(name):
    # QR of A needs full column rank, so at least n rays must cross the image:
    # the paper factors its 266,500 x 262,144 case (Section III-B), which only
    # holds if (nearly) all of its rays are informative
    w = get_workload(name)
    c = image_chord_lengths(w.geometry())
    assert (c > 0).all()
    assert w.m >= w.n
    # no chord is longer than the square's diagonal
    assert c.max() <= w.side * math.sqrt(2) + 1e-9


def test_undersampled_512_ratio_is_full_rank_small():
    # the 512^2 view/bin density (288 views, 2 bins per pixel across) at 32^2:
    # more crossing rays than pixels and a moderate condition number
    g = dict(get_workload("ct32").geometry(), n_views=18, n_bins=64)
    A = system_matrix_csr(g).toarray()
    assert A.shape == (1152, 1024)
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[-1] > 0 and sv[0] / sv[-1] < 1e5


def test_eq2_worked_values_v260():
    # Eq. 2 under the reading in the module docstring, v = 260 (Table I);
    # values computed by hand from the recurrence.
    th = projection_angles_deg(260)
    step = 360.0 / 260
    expect = {1: 0.0, 65: 64 * step, 66: 64 * step + 0.5 + step, 130: 64 * step + 0.5 + 65 * step,
              131: 64 * step + 0.5 + 65 * step - 0.75 + step}
    for i, v in expect.items():
        assert abs(th[i - 1] - v) < 1e-12
    assert abs(th[65] - 90.5) < 1e-12            # Theta_66
    assert abs(th[129] - 179.1153846153846) < 1e-9
    assert abs(th[195] - 269.5) < 1e-12          # Theta_196
    assert abs(th[259] - 358.1153846153846) < 1e-9


@pytest.mark.parametrize("v", [16, 64, 90, 120, 260, 288])
def test_eq2_quarter_offsets(v):
    # net offset from the uniform schedule: 0, +0.5, -0.25, -0.5 per quarter
    th = projection_angles_deg(v)
    uni = projection_angles_deg(v, schedule=0)
    q1, q2, q3 = v // 4, v // 2, (3 * v) // 4
    off = th - uni
    assert np.allclose(off[:q1], 0.0, atol=1e-12)
    assert np.allclose(off[q1:q2], 0.5, atol=1e-12)
    assert np.allclose(off[q2:q3], -0.25, atol=1e-12)
    assert np.allclose(off[q3:], -0.5, atol=1e-12)
    assert np.all(np.diff(th) > 0)


def test_rays_geometry():
    g = get_workload("ct32").geometry()
    src, dst = ray_endpoints(g)
    # source on the circle of radius 75, bins on the flat detector 150 away
    assert np.allclose(np.hypot(src[:, 0], src[:, 1]), 75.0)
    nb = g["n_bins"]
    mid = dst[(nb // 2 - 1)::nb] * 0.5 + dst[(nb // 2)::nb] * 0.5   # detector centre (even bin count)
    assert np.allclose(np.hypot(*(mid - src[::nb]).T), 150.0)
    # outermost bin centres sit half a pitch inside the 30 degree fan
    pitch = 2 * 150 * math.tan(math.radians(15)) / nb
    d0 = dst[0] - src[0]
    dc = mid[0] - src[0]
    ang = math.degrees(math.acos(d0 @ dc / np.linalg.norm(d0) / np.linalg.norm(dc)))
    assert abs(ang - math.degrees(math.atan((150 * math.tan(math.radians(15)) - pitch / 2) / 150))) < 1e-9


@pytest.mark.parametrize("name", ["ct4", "ct8"])
def test_siddon_matches_bruteforce(name):
    g = get_workload(name).geometry()
    A = system_matrix_csr(g).toarray()
    B = system_matrix_bruteforce(g)
    assert np.abs(A - B).max() <= 1e-13
    assert ((A > 0) == (B > 0)).all()


def test_siddon_matches_bruteforce_16():
    g = dict(get_workload("ct8").geometry(), side=16, n_views=20, n_bins=18)
    A = system_matrix_csr(g).toarray()
    B = system_matrix_bruteforce(g)
    assert np.abs(A - B).max() <= 1e-13


@pytest.mark.parametrize("name", ["ct24", "ct32", "ct40"])
def test_siddon_row_sums_are_chords(name):
    g = get_workload(name).geometry()
    A = system_matrix_csr(g)
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.abs(rs - image_chord_lengths(g)).max() <= 1e-12
    d = A.toarray()
    assert d.min() >= 0.0 and d.max() <= math.sqrt(2) + 1e-12
    assert (np.diff(A.indptr) <= 2 * g["side"] - 1).all()
    assert (d.sum(axis=0) > 0).all()          # every pixel seen (full-rank precondition)


def test_siddon_axis_aligned_ray():
    # a horizontal ray through the middle of a pixel row crosses every pixel
    # of that row with length exactly one pitch
    side, L = 8, 8.0
    x0 = y0 = -4.0
    cols, vals = siddon_ray((-10.0, 0.5), (10.0, 0.5), x0, y0, L / side, side)
    assert sorted(cols.tolist()) == list(range(4 * 8, 5 * 8))
    assert np.allclose(vals, 1.0, atol=1e-14)
    # on a grid line: the cell on the +y side (half-open cells)
    cols, vals = siddon_ray((-10.0, 0.0), (10.0, 0.0), x0, y0, L / side, side)
    assert sorted(cols.tolist()) == list(range(4 * 8, 5 * 8))
    # the same holds for the brute-force clipper
    assert abs(chord_length((-10.0, 0.0), (10.0, 0.0), -1, 0, 0, 1) - 1.0) < 1e-14
    assert chord_length((-10.0, 0.0), (10.0, 0.0), -1, 0, -1, 0) == 0.0


def test_siddon_diagonal_ray():
    # a diagonal through pixel corners: each pixel on the diagonal gets sqrt(2)
    side = 4
    cols, vals = siddon_ray((-3.0, -3.0), (3.0, 3.0), -2.0, -2.0, 1.0, side)
    assert sorted(cols.tolist()) == [0, 5, 10, 15]
    assert np.allclose(vals, math.sqrt(2), atol=1e-14)


def test_phantom_determinism():
    from synthetic import phantom_image, noise_vector, ellipse_params
    a = phantom_image(32, 3)
    b = phantom_image(32, 3)
    assert (a == b).all() and a.shape == (1024,)
    assert a.min() >= 0 and a.max() > 0
    e = ellipse_params(32, 3)
    assert e.shape == (8, 6) and (np.abs(e[:, :2]) <= 0.6).all() and (e[:, 5] <= 1).all()
    assert (noise_vector(32, 0, 10) == noise_vector(32, 0, 10)).all()
    assert not (noise_vector(32, 0, 10) == noise_vector(32, 1, 10)).all()
