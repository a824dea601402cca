"""Oracle: Joseph's projector (sinogram simulation) and the image-quality
metrics of the evaluation (PSNR, SSIM).

Test infrastructure only: the product never imports this package.

The paper simulates its sinograms with Joseph's method (Section II-A, before
Eq. 2) and scores reconstructions with PSNR and SSIM (Section II-B, Eq. 5-7).

Joseph's method (Joseph 1982): a ray is sampled once per pixel column (when it
runs closer to the x axis) or per pixel row (otherwise), at the line through
the pixel centres; the image value there is linearly interpolated between the
two nearest pixel centres of that column (row), pixels outside the image
counting as zero; each sample is weighted by the ray length between
consecutive column (row) lines, 1 / |cos| of the ray's angle to that axis, in
pixel pitches.  Rays and pixels are those of the Siddon oracle (Table I
scanner, rows view-major, columns iy * side + ix).

SSIM (Eq. 7) is evaluated on every 11 x 11 window inside the image with the
Gaussian weights of standard deviation 1.5 pixels (normalised to sum 1) for
the window means, variances and covariance, c1 = (0.01 L)^2, c2 = (0.03 L)^2
with L the data range (default: max - min of the reference image), and
averaged over the windows.
"""
import math
import numpy as np

from .geometry import ray_endpoints, image_grid, sizes

SSIM_WIN = 11
SSIM_SIGMA = 1.5
SSIM_K1, SSIM_K2 = 0.01, 0.03


def joseph_ray(p0, p1, x0, y0, delta, side, img):
    """Line integral of the side x side image (img[iy, ix]) along the ray
    p0 -> p1, in pixel pitches."""
    dx, dy = p1[0] - p0[0], p1[1] - p0[1]
    total = 0.0
    if abs(dx) >= abs(dy):
        w = math.hypot(dx, dy) / abs(dx)
        for ix in range(side):
            x = x0 + (ix + 0.5) * delta
            t = (x - p0[0]) / dx
            v = (p0[1] + t * dy - y0) / delta - 0.5      # row coordinate of the sample
            iy = math.floor(v)
            f = v - iy
            a = img[iy, ix] if 0 <= iy < side else 0.0
            b = img[iy + 1, ix] if 0 <= iy + 1 < side else 0.0
            total += w * ((1.0 - f) * a + f * b)
    else:
        w = math.hypot(dx, dy) / abs(dy)
        for iy in range(side):
            y = y0 + (iy + 0.5) * delta
            t = (y - p0[1]) / dy
            u = (p0[0] + t * dx - x0) / delta - 0.5      # column coordinate of the sample
            ix = math.floor(u)
            f = u - ix
            a = img[iy, ix] if 0 <= ix < side else 0.0
            b = img[iy, ix + 1] if 0 <= ix + 1 < side else 0.0
            total += w * ((1.0 - f) * a + f * b)
    return total


def joseph_project(geom, X):
    """B = J X: the Joseph projections (m x S) of the images in the columns of
    X (n x S, pixel j = iy * side + ix)."""
    m, n = sizes(geom)
    side = geom["side"]
    x0, y0, delta = image_grid(geom)
    src, dst = ray_endpoints(geom)
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    B = np.zeros((m, X.shape[1]))
    for s in range(X.shape[1]):
        img = X[:, s].reshape(side, side)
        for i in range(m):
            B[i, s] = joseph_ray(src[i], dst[i], x0, y0, delta, side, img)
    return B


def gaussian_window(size=SSIM_WIN, sigma=SSIM_SIGMA):
    """size x size Gaussian weights (outer product of the 1-D profile), sum 1."""
    r = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-r * r / (2.0 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def ssim(ref, img, data_range=None):
    """Mean SSIM (Eq. 7) of img against ref (2-D arrays) over every 11 x 11
    window inside the image."""
    ref = np.asarray(ref, dtype=np.float64)
    img = np.asarray(img, dtype=np.float64)
    L = (ref.max() - ref.min()) if data_range is None else data_range
    c1, c2 = (SSIM_K1 * L) ** 2, (SSIM_K2 * L) ** 2
    w = gaussian_window()
    k = SSIM_WIN
    vals = []
    for p in range(ref.shape[0] - k + 1):
        for q in range(ref.shape[1] - k + 1):
            x = ref[p:p + k, q:q + k]
            y = img[p:p + k, q:q + k]
            mx, my = (w * x).sum(), (w * y).sum()
            vx = (w * (x - mx) ** 2).sum()
            vy = (w * (y - my) ** 2).sum()
            cxy = (w * (x - mx) * (y - my)).sum()
            vals.append((2 * mx * my + c1) * (2 * cxy + c2) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return float(np.mean(vals))
