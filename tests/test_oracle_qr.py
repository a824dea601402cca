"""Pins of the oracle's Householder QR and least-squares solve (CPU only).

The oracle (unblocked Householder QR, Eq. 3; X = R^-1 Q^T B, Eq. 4) is checked
against things it does not share code with: exact rational arithmetic on
tiny systems (the normal equations solved in fractions; R from an exact
LDL^T of A^T A), LAPACK (dgeqrf / dormqr / trtrs through SciPy, with the same
reflector convention), backward-error and orthogonality invariants, and
exact recovery of a phantom from consistent data.
"""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sl

from synthetic import get_workload, phantom_image
from oracle import householder as hh
from oracle import lsq
from oracle.siddon import system_matrix_csr


@pytest.fixture(scope="module")
def ct32(oracle_lib):
    g = get_workload("ct32").geometry()
    A = system_matrix_csr(g)
    d = A.toarray()
    QR, tau = hh.geqr2(d)
    return A, d, QR, tau


def _exact_lstsq(A, b):
    """x = (A^T A)^-1 A^T b in exact rationals (Gauss-Jordan)."""
    m, n = A.shape
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(m)]
    bf = [Fraction(float(v)) for v in b]
    N = [[sum(Af[k][i] * Af[k][j] for k in range(m) if Af[k][i] and Af[k][j]) for j in range(n)] for i in range(n)]
    r = [sum(Af[k][i] * bf[k] for k in range(m) if Af[k][i]) for i in range(n)]
    for c in range(n):
        p = next(i for i in range(c, n) if N[i][c] != 0)
        N[c], N[p] = N[p], N[c]
        r[c], r[p] = r[p], r[c]
        inv = 1 / N[c][c]
        N[c] = [v * inv for v in N[c]]
        r[c] *= inv
        for i in range(n):
            if i != c and N[i][c] != 0:
                f = N[i][c]
                N[i] = [a - f * bb for a, bb in zip(N[i], N[c])]
                r[i] -= f * r[c]
    return r


def _exact_abs_R(A):
    """|R| from an exact LDL^T of A^T A: R_ii = sqrt(D_i), R_ij = sqrt(D_i) L_ji
    (square roots in 40-digit decimal)."""
    m, n = A.shape
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(m)]
    N = [[sum(Af[k][i] * Af[k][j] for k in range(m)) for j in range(n)] for i in range(n)]
    L = [[Fraction(0)] * n for _ in range(n)]
    D = [Fraction(0)] * n
    for j in range(n):
        D[j] = N[j][j] - sum(L[j][k] ** 2 * D[k] for k in range(j))
        L[j][j] = Fraction(1)
        for i in range(j + 1, n):
            L[i][j] = (N[i][j] - sum(L[i][k] * L[j][k] * D[k] for k in range(j))) / D[j]
    getcontext().prec = 40
    R = np.zeros((n, n))
    for i in range(n):
        s = (Decimal(D[i].numerator) / Decimal(D[i].denominator)).sqrt()
        for j in range(i, n):
            R[i, j] = float(s * Decimal(L[j][i].numerator) / Decimal(L[j][i].denominator))
    return np.abs(R)


def test_exact_R_ct4(oracle_lib):
    g = get_workload("ct4").geometry()
    d = system_matrix_csr(g).toarray()
    QR, tau = hh.geqr2(d)
    R = hh.r_factor(QR)
    Rex = _exact_abs_R(d)
    assert np.abs(np.abs(R) - Rex).max() <= 1e-13 * Rex.max()


@pytest.mark.parametrize("name", ["ct4", "ct8"])
def test_exact_rational_lstsq(name, oracle_lib):
    g = get_workload(name).geometry()
    A = system_matrix_csr(g)
    d = A.toarray()
    X, B = lsq.sinograms(A, g["side"], 1)
    x = lsq.reconstruct(d, B)[0][:, 0]
    xe = np.array([float(v) for v in _exact_lstsq(d, B[:, 0])])
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) <= 1e-13


def test_matches_lapack_dgeqrf(ct32):
    _, d, QR, tau = ct32
    qr_l, tau_l, _, info = sl.lapack.dgeqrf(np.asfortranarray(d.copy()))
    assert info == 0
    # same reflector convention as LAPACK's larfg: tau, v and R agree to rounding
    assert np.abs(tau - tau_l).max() <= 1e-12
    assert np.abs(QR - qr_l).max() <= 1e-11 * np.abs(qr_l).max()


def test_qt_matches_lapack_dormqr(ct32):
    A, d, QR, tau = ct32
    rng = np.random.default_rng(0)
    B = np.asfortranarray(rng.standard_normal((d.shape[0], 3)))
    C = hh.apply_qt(QR, tau, B)
    Cl, _, info = sl.lapack.dormqr("L", "T", QR, tau, B.copy(), lwork=max(1, 64 * 3))
    assert info == 0
    assert np.abs(C - Cl).max() <= 1e-12 * np.abs(Cl).max()


def test_backsub_matches_trtrs(ct32):
    _, d, QR, tau = ct32
    R = hh.r_factor(QR)
    rng = np.random.default_rng(1)
    c = rng.standard_normal((R.shape[0], 2))
    x = hh.backsub(QR, c)
    xl = sl.solve_triangular(R, c, lower=False)
    assert np.abs(x - xl).max() <= 1e-11 * np.abs(xl).max()


def test_orthogonality_and_backward_error(ct32):
    _, d, QR, tau = ct32
    m, n = d.shape
    Q = hh.apply_q(QR, tau, np.eye(m)[:, :n])
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13 * n ** 0.5 * 10
    R = hh.r_factor(QR)
    assert np.linalg.norm(d - Q @ R) / np.linalg.norm(d) <= 1e-14
    assert np.allclose(np.tril(Q.T @ d, -1)[:n], 0, atol=1e-12)


def test_solution_matches_lstsq_and_optimality(ct32):
    A, d, QR, tau = ct32
    X, B = lsq.sinograms(A, 32, 1)
    x = hh.backsub(QR, hh.apply_qt(QR, tau, B))
    xl = np.linalg.lstsq(d, B, rcond=None)[0]
    assert lsq.rel_err(x, xl).max() <= 1e-12
    assert lsq.ls_optimality(A, x, B).max() <= 1e-13


@pytest.mark.parametrize("name", ["ct24", "ct32"])
def test_exact_recovery_noise_free(name, oracle_lib):
    # consistent data: the least-squares solution is the phantom itself
    g = get_workload(name).geometry()
    A = system_matrix_csr(g)
    X, B = lsq.sinograms(A, g["side"], 2, noisy=False)
    x = lsq.reconstruct(A.toarray(), B)[0]
    assert lsq.rel_err(x, X).max() <= 1e-12
    # the paper's Table II metric lands in its printed band for FP64 data
    assert lsq.relative_residual(A, x, B) <= 1e-11
    assert lsq.psnr(X[:, 0], x[:, 0]) > 200.0


def test_zero_column_tau_zero(oracle_lib):
    # x == 0 below the diagonal: tau = 0 and the column is left unchanged
    A = np.array([[3.0, 1.0], [0.0, 2.0], [0.0, 1.0]])
    QR, tau = hh.geqr2(A)
    assert tau[0] == 0.0 and QR[0, 0] == 3.0
    Rl = np.linalg.qr(A, mode="r")
    assert np.allclose(np.abs(hh.r_factor(QR)), np.abs(Rl), atol=1e-14)


def test_sign_convention(oracle_lib):
    # beta = -sign(alpha) ||x||: positive alpha gives a negative R_kk
    A = np.array([[3.0], [4.0]])
    QR, tau = hh.geqr2(A)
    assert QR[0, 0] == -5.0 and abs(tau[0] - 1.6) < 1e-15 and abs(QR[1, 0] - 0.5) < 1e-15
    QR, tau = hh.geqr2(-A)
    assert QR[0, 0] == 5.0


def test_condition_ct32(ct32):
    _, d, QR, tau = ct32
    s = np.linalg.svd(d, compute_uv=False)
    kappa = s[0] / s[-1]
    assert 10 < kappa < 1e2     # measured 32.3; full column rank


def _tiny_ls():
    """A 3 x 2 system whose least-squares solution and residual are known in
    closed form: A^T A = [[2, 1], [1, 2]], A^T b = [5, 6], x* = [4/3, 7/3],
    r* = b - A x* = [-1/3, -1/3, 1/3]."""
    import scipy.sparse as sps
    A = sps.csr_matrix(np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]]))
    b = np.array([[1.0], [2.0], [4.0]])
    return A, b, np.array([[4.0 / 3.0], [7.0 / 3.0]])


def test_ls_optimality_closed_form():
    A, b, xs = _tiny_ls()
    # zero (to rounding) at the least-squares solution
    assert lsq.ls_optimality(A, xs, b)[0] <= 1e-15
    # x = [1, 2]: r = [0, 0, 1], A^T r = [1, 1], ||A||_F = 2, ||r|| = 1
    assert abs(lsq.ls_optimality(A, np.array([[1.0], [2.0]]), b)[0] - np.sqrt(2.0) / 2.0) <= 1e-15


def test_ls_optimality_rejects_perturbed_solution(ct32):
    # the metric separates the least-squares solution from a solution moved
    # by 1e-6 relative: the check on noisy full-size solutions (bound of order
    # 1e-14) would fail for such an x
    A, d, QR, tau = ct32
    X, B = lsq.sinograms(A, 32, 2)
    x = hh.backsub(QR, hh.apply_qt(QR, tau, B))
    good = lsq.ls_optimality(A, x, B)
    rng = np.random.default_rng(5)
    xp = x * (1.0 + 1e-6 * rng.standard_normal(x.shape))
    bad = lsq.ls_optimality(A, xp, B)
    assert good.max() <= 1e-13
    assert bad.min() >= 1e-9, bad
    assert (bad > 1e4 * good).all()


def test_relative_residual_closed_form():
    # ||A x* - b||_F / ||A||_F = (1/sqrt(3)) / 2 for the tiny system
    A, b, xs = _tiny_ls()
    assert abs(lsq.relative_residual(A, xs, b) - 1.0 / (2.0 * np.sqrt(3.0))) <= 1e-15
    # dense input takes the same path
    assert abs(lsq.relative_residual(A.toarray(), xs, b) - 1.0 / (2.0 * np.sqrt(3.0))) <= 1e-15


def test_psnr_closed_form():
    # Eq. 5-6: a constant error of 0.1 on an image whose maximum is 1 gives
    # MSE = 0.01 and PSNR = 10 log10(1 / 0.01) = 20 dB; an exact image gives inf
    ref = np.array([[0.0, 1.0], [0.5, 0.25]])
    assert abs(lsq.psnr(ref, ref + 0.1) - 20.0) <= 1e-12
    assert abs(lsq.psnr(2.0 * ref, 2.0 * ref - 0.2) - 20.0) <= 1e-12   # scales with max(I0)
    assert lsq.psnr(ref, ref) == np.inf


@pytest.mark.parametrize("name", ["ct24", "ct32"])
def test_cgls_matches_qr_solve(name, oracle_lib):
    # the matrix-free CGLS used for sizes the dense oracle cannot hold reaches
    # the same least-squares solution as the Householder route (Eq. 4)
    g = get_workload(name).geometry()
    A = system_matrix_csr(g)
    X, B = lsq.sinograms(A, g["side"], 2)
    x_qr = lsq.reconstruct(A.toarray(), B)[0]
    x_cg, iters = lsq.cgls(A, B, tol=1e-14)
    assert lsq.rel_err(x_cg, x_qr).max() <= 1e-10
    assert lsq.ls_optimality(A, x_cg, B).max() <= 1e-13
    assert (iters < A.shape[1]).all()
