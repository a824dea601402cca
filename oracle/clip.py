"""Oracle cross-check: A by brute-force clipping of every ray against every pixel.

Test infrastructure only.  This is a second, independent derivation of the
intersection lengths of Section II-A (Eq. 1) for tiny images: each pixel
square is clipped against the ray segment with the Liang-Barsky parametric
test, with the same half-open cell convention as the Siddon oracle (a ray
lying exactly on a grid line counts for the cell on its +x/+y side).
"""
import math
import numpy as np

from .geometry import ray_endpoints, image_grid, sizes


def chord_length(p0, p1, xmin, xmax, ymin, ymax, half_open=True):
    """Length of the part of segment p0->p1 inside the box (Liang-Barsky)."""
    dx, dy = p1[0] - p0[0], p1[1] - p0[1]
    t0, t1 = 0.0, 1.0
    for p, q, upper in ((-dx, p0[0] - xmin, False), (dx, xmax - p0[0], True),
                        (-dy, p0[1] - ymin, False), (dy, ymax - p0[1], True)):
        if p == 0.0:
            if q < 0.0 or (half_open and upper and q == 0.0):
                return 0.0
        else:
            r = q / p
            if p < 0.0:
                t0 = max(t0, r)
            else:
                t1 = min(t1, r)
    return max(0.0, t1 - t0) * math.hypot(dx, dy)


def system_matrix_bruteforce(geom):
    """Dense A (units of the pixel pitch) by clipping every (ray, pixel) pair."""
    m, n = sizes(geom)
    x0, y0, delta = image_grid(geom)
    side = geom["side"]
    src, dst = ray_endpoints(geom)
    A = np.zeros((m, n), order="F")
    for i in range(m):
        for iy in range(side):
            for ix in range(side):
                ln = chord_length(src[i], dst[i], x0 + ix * delta, x0 + (ix + 1) * delta,
                                  y0 + iy * delta, y0 + (iy + 1) * delta)
                if ln > 1e-12 * delta:
                    A[i, iy * side + ix] = ln / delta
    return A


def image_chord_lengths(geom):
    """Length (in pixel pitches) of each ray inside the whole image square: the
    exact row sums of A."""
    x0, y0, delta = image_grid(geom)
    side = geom["side"]
    src, dst = ray_endpoints(geom)
    out = np.empty(src.shape[0])
    for i in range(src.shape[0]):
        out[i] = chord_length(src[i], dst[i], x0, x0 + side * delta, y0, y0 + side * delta,
                              half_open=False) / delta
    return out
