"""Seeded random-ellipse phantoms, noise vectors and request streams.

Every draw comes from ``numpy.random.default_rng(SeedSequence([side, slice,
stream]))`` so the oracle, the tests and the benchmark see bit-identical
inputs on any machine.  Stream 0 draws the phantom, stream 1 the noise.

Phantom recipe (a reading: the paper uses the Forbild head phantom and
DeepLesion images, neither of which is available, Section III-A): 8 ellipses
in the normalised square [-1, 1]^2, drawn in the order
cx, cy ~ U(-0.6, 0.6); a, b ~ U(0.05, 0.4); phi ~ U(0, pi); d ~ U(0, 1),
summed and point-sampled at pixel centres.  Pixel (ix, iy) has column index
iy * side + ix, ix growing with x and iy with y, origin at the lower-left
corner.
"""
import numpy as np

N_ELLIPSES = 8
# Sinogram noise standard deviation relative to max|A x| (the paper ignores W
# in Eq. 1; the workloads add 1e-3 relative Gaussian noise).
NOISE_REL_LEVEL = 1e-3


def _rng(side, slice_idx, stream):
    return np.random.default_rng(np.random.SeedSequence([int(side), int(slice_idx), int(stream)]))


def ellipse_params(side, slice_idx, n_ellipses=N_ELLIPSES):
    """(n_ellipses, 6) array of (cx, cy, a, b, phi, density) in draw order."""
    rng = _rng(side, slice_idx, 0)
    out = np.empty((n_ellipses, 6))
    for e in range(n_ellipses):
        cx = rng.uniform(-0.6, 0.6)
        cy = rng.uniform(-0.6, 0.6)
        a = rng.uniform(0.05, 0.4)
        b = rng.uniform(0.05, 0.4)
        phi = rng.uniform(0.0, np.pi)
        d = rng.uniform(0.0, 1.0)
        out[e] = (cx, cy, a, b, phi, d)
    return out


def phantom_image(side, slice_idx):
    """FP64 vector of length side*side (column index iy*side + ix)."""
    c = (np.arange(side) + 0.5) * (2.0 / side) - 1.0
    xx, yy = np.meshgrid(c, c, indexing="xy")       # yy[iy, ix], xx[iy, ix]
    img = np.zeros((side, side))
    for cx, cy, a, b, phi, d in ellipse_params(side, slice_idx):
        cph, sph = np.cos(phi), np.sin(phi)
        u = (xx - cx) * cph + (yy - cy) * sph
        v = -(xx - cx) * sph + (yy - cy) * cph
        img += np.where((u / a) ** 2 + (v / b) ** 2 <= 1.0, d, 0.0)
    return img.reshape(-1)


def phantom_batch(side, n_slices, first=0):
    """(side*side, n_slices) column-major-friendly stack of phantoms (Fortran order)."""
    X = np.empty((side * side, n_slices), order="F")
    for s in range(n_slices):
        X[:, s] = phantom_image(side, first + s)
    return X


def noise_vector(side, slice_idx, m):
    """Standard-normal vector z of length m; the sinogram noise is sigma*z with
    sigma = NOISE_REL_LEVEL * max|A x| computed by whoever forms the sinogram."""
    return _rng(side, slice_idx, 1).standard_normal(m)


def noise_batch(side, m, n_slices, first=0):
    Z = np.empty((m, n_slices), order="F")
    for s in range(n_slices):
        Z[:, s] = noise_vector(side, first + s, m)
    return Z


def request_stream(n_requests=200, max_slices=512, seed=(4, 0, 2), geometries=("ct128", "ct256")):
    """Batched solve requests: geometry uniform over ``geometries``, slice count
    k = clip(round(exp(U(0, ln max_slices))), 1, max_slices) (log-uniform)."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    out = []
    for _ in range(n_requests):
        g = geometries[int(rng.integers(0, len(geometries)))]
        k = int(np.clip(np.round(np.exp(rng.uniform(0.0, np.log(max_slices)))), 1, max_slices))
        out.append((g, k))
    return out
