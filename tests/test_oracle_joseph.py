"""Pins of the oracle's Joseph projector and SSIM (CPU only).

Joseph's projector samples each ray once per pixel column (row) and
interpolates linearly between pixel centres.  Pinned by:
  * the all-ones image: for every ray whose samples all fall between pixel
    centres of the image (both interpolation neighbours inside), the
    projection is the ray's chord through the image square, which the
    independent Siddon oracle's row sums give exactly;
  * a linear image a + b ix + c iy: on the same rays the sampled sum is the
    midpoint rule of a linear function, which is exact, so the projection is
    the chord length times the image's value at the chord's midpoint;
  * linearity in the image.
SSIM (Eq. 7): identical images give 1; two constant images give
(2ab + c1) / (a^2 + b^2 + c1) (the variance terms cancel); the window sums
match scipy.signal.correlate2d with the same Gaussian weights (an
independent evaluation of the same window statistics); the weights sum to 1.
"""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import joseph as J
from oracle.geometry import ray_endpoints, image_grid
from oracle.siddon import system_matrix_csr
from synthetic import get_workload, phantom_batch


def _interior_rays(g):
    """Rays whose every sample has both interpolation neighbours inside."""
    side = g["side"]
    x0, y0, delta = image_grid(g)
    src, dst = ray_endpoints(g)
    keep = []
    for i, (p0, p1) in enumerate(zip(src, dst)):
        dx, dy = p1[0] - p0[0], p1[1] - p0[1]
        if abs(dx) >= abs(dy):
            c = (x0 + (np.arange(side) + 0.5) * delta - p0[0]) / dx
            v = (p0[1] + c * dy - y0) / delta - 0.5
        else:
            c = (y0 + (np.arange(side) + 0.5) * delta - p0[1]) / dy
            v = (p0[0] + c * dx - x0) / delta - 0.5
        if v.min() >= 0.0 and v.max() <= side - 1:
            keep.append(i)
    return np.array(keep)


@pytest.mark.parametrize("name", ["ct8", "ct24"])
def test_constant_image_gives_chord_length(name):
    g = get_workload(name).geometry()
    side = g["side"]
    rows = _interior_rays(g)
    assert rows.size > 0.3 * g["n_views"] * g["n_bins"]
    B = J.joseph_project(g, np.ones((side * side, 1)))
    chord = np.asarray(system_matrix_csr(g).sum(axis=1)).ravel()
    assert np.abs(B[rows, 0] - chord[rows]).max() <= 1e-11 * side


@pytest.mark.parametrize("name", ["ct8", "ct24"])
def test_linear_image_exact(name):
    g = get_workload(name).geometry()
    side = g["side"]
    x0, y0, delta = image_grid(g)
    src, dst = ray_endpoints(g)
    a, b, c = 0.7, 0.05, -0.03
    iy, ix = np.divmod(np.arange(side * side), side)
    img = a + b * ix + c * iy
    B = J.joseph_project(g, img[:, None])
    A = system_matrix_csr(g)
    for i in _interior_rays(g):
        p0, p1 = src[i], dst[i]
        # chord through the square: the ray enters and leaves through the
        # two edges normal to its dominant axis
        dx, dy = p1[0] - p0[0], p1[1] - p0[1]
        if abs(dx) >= abs(dy):
            t0, t1 = (x0 - p0[0]) / dx, (x0 + side * delta - p0[0]) / dx
        else:
            t0, t1 = (y0 - p0[1]) / dy, (y0 + side * delta - p0[1]) / dy
        tm = 0.5 * (t0 + t1)
        u = (p0[0] + tm * dx - x0) / delta - 0.5
        v = (p0[1] + tm * dy - y0) / delta - 0.5
        length = abs(t1 - t0) * math.hypot(dx, dy) / delta
        assert abs(B[i, 0] - length * (a + b * u + c * v)) <= 1e-11 * length
        assert abs(length - A[i].sum()) <= 1e-11 * length


def test_linearity():
    g = get_workload("ct8").geometry()
    X = phantom_batch(8, 2)
    B = J.joseph_project(g, X)
    B2 = J.joseph_project(g, 2.0 * X[:, :1] - 3.0 * X[:, 1:])
    assert np.abs(B2[:, 0] - (2.0 * B[:, 0] - 3.0 * B[:, 1])).max() <= 1e-12 * np.abs(B).max()


def test_ssim_identity_and_constants():
    x = phantom_batch(24, 1)[:, 0].reshape(24, 24)
    assert abs(J.ssim(x, x) - 1.0) <= 1e-12
    L = 1.0
    c1 = (0.01 * L) ** 2
    a, b = 0.3, 0.5
    got = J.ssim(np.full((16, 16), a), np.full((16, 16), b), data_range=L)
    assert abs(got - (2 * a * b + c1) / (a * a + b * b + c1)) <= 1e-12
    w = J.gaussian_window()
    assert abs(w.sum() - 1.0) <= 1e-15 and np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])


def test_ssim_matches_correlate2d():
    rng = np.random.default_rng(3)
    x = phantom_batch(24, 1)[:, 0].reshape(24, 24)
    y = x + 0.05 * rng.standard_normal(x.shape)
    w = J.gaussian_window()
    mu_x, mu_y = correlate2d(x, w, "valid"), correlate2d(y, w, "valid")
    vx = correlate2d(x * x, w, "valid") - mu_x ** 2
    vy = correlate2d(y * y, w, "valid") - mu_y ** 2
    cxy = correlate2d(x * y, w, "valid") - mu_x * mu_y
    L = x.max() - x.min()
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    ref = np.mean((2 * mu_x * mu_y + c1) * (2 * cxy + c2) / ((mu_x ** 2 + mu_y ** 2 + c1) * (vx + vy + c2)))
    assert abs(J.ssim(x, y) - ref) <= 1e-12
    assert abs(J.ssim(x, y) - J.ssim(y, x, data_range=L)) <= 1e-12
