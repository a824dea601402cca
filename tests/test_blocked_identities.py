"""Pins of the block-reflector algebra the factorization's updates rely on
(CPU only).

The GPU factorization applies groups of consecutive compact-WY blocks to the
trailing columns in one product: with W = V^T C over the group's Householder
vectors V = [V_0 V_1 ...], each block's rows of W' = T^T W are formed as
W'_j = T_j^T (W_j - G_{j,<j} W'_{<j}) with G = V^T V, and C -= V W'.  These
tests check that recurrence, with each block's T from the compact-WY
definition (Schreiber and Van Loan: H_1 ... H_k = I - V T V^T), against the
oracle's reflector-at-a-time application of the same reflectors.
"""
import numpy as np
import pytest

from oracle import householder as hh


def _t_factor(V, tau):
    # compact-WY T of reflectors (V[:, j], tau[j]) by its column recurrence
    k = V.shape[1]
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = tau[j]
        T[:j, j] = -tau[j] * T[:j, :j] @ (V[:, :j].T @ V[:, j])
    return T


def _group_apply_qt(V, tau, C, nb):
    # Q^T C for the group V (k columns) through the blockwise W' recurrence
    k = V.shape[1]
    G = V.T @ V
    W = V.T @ C
    Wp = np.zeros_like(W)
    for r0 in range(0, k, nb):
        r1 = min(k, r0 + nb)
        Tj = _t_factor(V[:, r0:r1], tau[r0:r1])
        Wp[r0:r1] = Tj.T @ (W[r0:r1] - G[r0:r1, :r0] @ Wp[:r0])
    return C - V @ Wp


@pytest.mark.parametrize("m,k,nb", [(200, 64, 16), (150, 56, 16), (90, 40, 8), (60, 16, 16), (120, 37, 8)])
def test_group_recurrence_equals_reflector_products(m, k, nb, oracle_lib):
    rng = np.random.default_rng(m * 100 + k)
    A = rng.standard_normal((m, k))
    QR, tau = hh.geqr2(A)
    V = hh.householder_vectors(QR)
    C = rng.standard_normal((m, 5))
    got = _group_apply_qt(V, tau, C, nb)
    want = hh.apply_qt(QR, tau, C)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_group_recurrence_reproduces_R(oracle_lib):
    # applying the group of the first 48 reflectors to A's columns yields R's
    # rows there (upper triangle) and zeros below the diagonal
    m, n, k, nb = 120, 80, 48, 16
    rng = np.random.default_rng(5)
    A = rng.standard_normal((m, n))
    QR, tau = hh.geqr2(A)
    V = hh.householder_vectors(QR)[:, :k]
    R = hh.r_factor(QR)
    out = _group_apply_qt(V, tau[:k], A, nb)
    assert np.abs(np.triu(out[:k, :k]) - R[:k, :k]).max() <= 1e-12 * np.abs(R).max()
    assert np.abs(np.tril(out[:, :k], -1)).max() <= 1e-12 * np.abs(R).max()
    # the rows of R to the right of the group's columns come out too
    assert np.abs(out[:k, k:] - R[:k, k:]).max() <= 1e-12 * np.abs(R).max()


def test_recurrence_needs_the_gram_correction(oracle_lib):
    # dropping G_{j,<j} W'_{<j} (applying every block to the original W) is
    # not the product of the reflectors: the correction carries the blocks'
    # coupling
    m, k, nb = 100, 32, 16
    rng = np.random.default_rng(9)
    QR, tau = hh.geqr2(rng.standard_normal((m, k)))
    V = hh.householder_vectors(QR)
    C = rng.standard_normal((m, 3))
    W = V.T @ C
    Wp = np.vstack([_t_factor(V[:, r0:r0 + nb], tau[r0:r0 + nb]).T @ W[r0:r0 + nb] for r0 in range(0, k, nb)])
    wrong = C - V @ Wp
    want = hh.apply_qt(QR, tau, C)
    assert np.abs(wrong - want).max() > 1e-3 * np.abs(want).max()
