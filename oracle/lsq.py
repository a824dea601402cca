"""Oracle: sinograms, the QR reconstruction X = R^-1 (Q^T B), and its checks.

Test infrastructure only.

* ``sinograms``: B = A X + W (Eq. 1) with W = sigma * z per slice,
  sigma = 1e-3 * max|A x| (the paper ignores W; the workloads add it).
* ``reconstruct``: factor once, then apply Q^T and back-substitute for all
  slices (Eq. 3, Eq. 4; the factorization does not depend on B and is reused,
  Section II-A).
* ``relative_residual``: ||AX - B||_F / ||A||_F, the paper's precision metric
  (Section III-A, Table II).
* ``ls_optimality``: ||A^T r|| / (||A||_F ||r||) per slice, zero exactly at
  the least-squares solution.
* ``cgls``: conjugate gradients on the normal equations for sizes whose dense
  factor the host cannot hold (matrix-free, FP64).
* ``psnr``: Eq. 5 and Eq. 6.
"""
import numpy as np

from synthetic import phantom_batch, noise_batch, NOISE_REL_LEVEL
from . import householder as hh


def sinograms(A, side, n_slices, first=0, noisy=True):
    """(X_true, B): phantoms and their sinograms A X (+ noise)."""
    X = phantom_batch(side, n_slices, first)
    B = np.asfortranarray(A @ X)
    if noisy:
        Z = noise_batch(side, A.shape[0], n_slices, first)
        sigma = NOISE_REL_LEVEL * np.abs(B).max(axis=0)
        B = np.asfortranarray(B + Z * sigma[None, :])
    return X, B


def reconstruct(A_dense, B):
    """X = R^-1 (Q^T B) with the unblocked oracle QR.  Returns (X, QR, tau)."""
    QR, tau = hh.geqr2(A_dense)
    C = hh.apply_qt(QR, tau, B)
    X = hh.backsub(QR, C)
    return X, QR, tau


def relative_residual(A, X, B):
    r = A @ X - B
    nA = np.sqrt((A.multiply(A)).sum()) if hasattr(A, "multiply") else np.linalg.norm(A)
    return np.linalg.norm(r) / nA


def ls_optimality(A, X, B):
    """Per-slice ||A^T (B - A X)||_2 / (||A||_F ||B - A X||_2)."""
    X = np.asarray(X).reshape(A.shape[1], -1)
    B = np.asarray(B).reshape(A.shape[0], -1)
    R = B - A @ X
    G = A.T @ R
    nA = np.sqrt((A.multiply(A)).sum()) if hasattr(A, "multiply") else np.linalg.norm(A)
    return np.linalg.norm(G, axis=0) / (nA * np.linalg.norm(R, axis=0))


def rel_err(X, Xref):
    """Per-slice ||X - Xref||_2 / ||Xref||_2."""
    X = np.asarray(X).reshape(Xref.shape[0], -1)
    Xref = np.asarray(Xref).reshape(Xref.shape[0], -1)
    return np.linalg.norm(X - Xref, axis=0) / np.linalg.norm(Xref, axis=0)


def cgls(A, B, tol=1e-14, max_iters=100000):
    """CGLS (Hestenes-Stiefel CG on A^T A x = A^T b) for every column of B,
    started from 0, stopped when ||A^T r|| <= tol * ||A||_F * ||r|| or when
    the normal-equation residual stops decreasing for 50 iterations."""
    B = np.asarray(B, dtype=np.float64).reshape(A.shape[0], -1)
    nA = np.sqrt((A.multiply(A)).sum())
    AT = A.T.tocsr()
    X = np.zeros((A.shape[1], B.shape[1]))
    iters = np.zeros(B.shape[1], dtype=np.int64)
    for s in range(B.shape[1]):
        x = np.zeros(A.shape[1])
        r = B[:, s].copy()
        g = AT @ r
        p = g.copy()
        gg = g @ g
        best, stall = np.inf, 0
        for it in range(max_iters):
            q = A @ p
            alpha = gg / (q @ q)
            x += alpha * p
            r -= alpha * q
            g = AT @ r
            gg_new = g @ g
            crit = np.sqrt(gg_new) / (nA * np.linalg.norm(r))
            if crit <= tol:
                break
            if gg_new < best:
                best, stall = gg_new, 0
            else:
                stall += 1
                if stall >= 50:
                    break
            p = g + (gg_new / gg) * p
            gg = gg_new
        X[:, s] = x
        iters[s] = it + 1
    return X, iters


def psnr(ref, img):
    """Eq. 5 and Eq. 6: 10 log10(max(I0)^2 / MSE) over the image."""
    mse = np.mean((np.asarray(ref) - np.asarray(img)) ** 2)
    return np.inf if mse == 0 else 10.0 * np.log10(np.max(ref) ** 2 / mse)
