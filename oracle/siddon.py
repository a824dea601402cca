"""Oracle: the system matrix A by Siddon's parametric ray tracing.

Test infrastructure only: the product never imports this package.

a_ij is the contribution of ray i to pixel j (Section II-A, Eq. 1); here it is
the length of the straight ray from the source to the centre of detector bin
b inside pixel j, in units of the pixel pitch (so 0 <= a_ij <= sqrt(2)).  The
paper does not fix the projector used for A; the exact intersection length
is the reading taken.

Siddon's method (Siddon 1985): parametrise the ray as p0 + alpha (p1 - p0),
clip alpha to the image square, collect every alpha at which the ray crosses
a vertical or horizontal grid line, sort them, and give each consecutive pair
of crossings the pixel that contains their midpoint.  Cells are half-open
([x_k, x_{k+1}) x [y_l, y_{l+1})), so a ray running exactly along a grid line
belongs to the cell on its +x/+y side.  Segments shorter than 1e-12 pitches
are dropped.
"""
import math
import numpy as np
import scipy.sparse as sp

from .geometry import ray_endpoints, image_grid, sizes

ZERO_SEGMENT = 1e-12   # in pixel pitches


def siddon_ray(p0, p1, x0, y0, delta, side):
    """(columns, lengths/delta) of one ray, in traversal order."""
    dx = p1[0] - p0[0]
    dy = p1[1] - p0[1]
    length = math.hypot(dx, dy)
    xe, ye = x0 + side * delta, y0 + side * delta
    amin, amax = 0.0, 1.0
    if dx != 0.0:
        a0, a1 = (x0 - p0[0]) / dx, (xe - p0[0]) / dx
        amin, amax = max(amin, min(a0, a1)), min(amax, max(a0, a1))
    elif not (x0 <= p0[0] < xe):
        return np.empty(0, np.int64), np.empty(0)
    if dy != 0.0:
        a0, a1 = (y0 - p0[1]) / dy, (ye - p0[1]) / dy
        amin, amax = max(amin, min(a0, a1)), min(amax, max(a0, a1))
    elif not (y0 <= p0[1] < ye):
        return np.empty(0, np.int64), np.empty(0)
    if amax <= amin:
        return np.empty(0, np.int64), np.empty(0)
    parts = [np.array([amin, amax])]
    planes = np.arange(side + 1, dtype=np.float64)
    if dx != 0.0:
        ax = (x0 + planes * delta - p0[0]) / dx
        parts.append(ax[(ax > amin) & (ax < amax)])
    if dy != 0.0:
        ay = (y0 + planes * delta - p0[1]) / dy
        parts.append(ay[(ay > amin) & (ay < amax)])
    alphas = np.unique(np.concatenate(parts))          # sorted, exact duplicates merged
    seg = np.diff(alphas) * length
    mid = 0.5 * (alphas[:-1] + alphas[1:])
    ix = np.floor((p0[0] + mid * dx - x0) / delta).astype(np.int64)
    iy = np.floor((p0[1] + mid * dy - y0) / delta).astype(np.int64)
    keep = seg > ZERO_SEGMENT * delta
    ix = np.clip(ix[keep], 0, side - 1)
    iy = np.clip(iy[keep], 0, side - 1)
    return iy * side + ix, seg[keep] / delta


def system_matrix_csr(geom):
    """A as a scipy CSR matrix (FP64), rows view-major, columns iy*side+ix,
    column indices sorted within each row."""
    m, n = sizes(geom)
    x0, y0, delta = image_grid(geom)
    src, dst = ray_endpoints(geom)
    side = geom["side"]
    indptr = np.zeros(m + 1, np.int64)
    cols, vals = [], []
    for i in range(m):
        c, v = siddon_ray(src[i], dst[i], x0, y0, delta, side)
        cols.append(c)
        vals.append(v)
        indptr[i + 1] = indptr[i] + len(c)
    col = np.concatenate(cols) if cols else np.empty(0, np.int64)
    val = np.concatenate(vals) if vals else np.empty(0)
    A = sp.csr_matrix((val, col, indptr), shape=(m, n))
    A.sort_indices()
    return A


def system_matrix_dense(geom):
    """A as a dense FP64 array in Fortran (column-major) order."""
    return np.asfortranarray(system_matrix_csr(geom).toarray())
