"""GPU parity of the benchmark's own factorization configuration, and the
status codes under forced numerical failures.

The benchmark factors the FP32 A with split-BF16 block-column products
(CTQR_PREC_BF16X3_MFMA) at nb = 256: groups of four block columns share one
trailing update of inner dimension K = 1024, and [G | W] = V^T [V | C] is
reduced over 1024-wide groups.  ct48 (n = 2304: two full groups and a
256-column tail) and ct64 (n = 4096: four groups, trailing updates of 3072,
2048 and 1024 columns) run that schedule at sizes the oracle's unblocked
Householder QR (Eq. 3) factors in seconds.

Tolerance of the split-BF16 factor: each FP32 operand is carried as a bf16
high part (8 significant bits) plus a bf16 low part, about 16 bits, and each
product drops the low-low term, so a product term is exact to about
3 * 2^-16 = 4.6e-5 relative; R, V and tau are compared with the oracle's at
1e-4 (relative to max|R| for R, absolute for V and tau, whose entries are at
most 1 in magnitude for V and in [1, 2] for tau).  Refined solutions (CSNE
with FP64 sparse residuals) must meet the 1e-10 bar against the oracle's
solution (Eq. 4).

Forced failures: every kernel runs to completion on these inputs (NaN
propagates through the arithmetic; no loop depends on data values), and the
status lands in the device-side ctqr_info.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import householder as hh
from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import SystemMatrix, QRFactor, to_colmajor
from synthetic import get_workload

from gpu_helpers import oracle_problem, oracle_factor, DeviceSparse, upload_dense, download

pytestmark = pytest.mark.gpu

U_SPLIT = 3.0 * 2.0 ** -16


def _case(*a):
    print("[case]", *a, flush=True)


def _factor(Ad, dtype, prec, nb):
    F = QRFactor(upload_dense(Ad, dtype), prec, nb=nb)
    F.factor()
    torch.cuda.synchronize()
    return F, F.info.read()


@pytest.mark.parametrize("name", ["ct48", "ct64"])
def test_bf16x3_nb256_grouped_factor_matches_oracle(gpu, name):
    _case("bf16x3 nb=256 grouped factor", name)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    m, n = A.shape
    assert n > 1024, "the case must hold at least one full group of four 256-wide blocks"
    Ad = A.toarray().astype(np.float32)
    F3, info = _factor(Ad, torch.float32, C.CTQR_PREC_BF16X3_MFMA, 256)
    assert info.status == 0, C.status_string(info.status)
    QRg = download(F3.A).astype(np.float64)
    taug = download(F3.tau)
    # R is unique up to the signs of its rows; where a pivot's sign agrees
    # (the reflector made the same choice), V and tau are unique too
    Rg, Ro = np.triu(QRg[:n, :n]), np.triu(QRo[:n, :n])
    sg, so = np.sign(np.diag(Rg)), np.sign(np.diag(Ro))
    same = sg == so
    assert same.mean() >= 0.99, same.mean()
    eR = np.abs(sg[:, None] * Rg - so[:, None] * Ro).max() / np.abs(Ro).max()
    Vg, Vo = np.tril(QRg, -1)[:, same], np.tril(QRo, -1)[:, same]
    eV = np.abs(Vg - Vo).max()
    et = np.abs(taug[same] - tauo[same]).max()
    print("split-BF16 nb=256 %s: R %.2e  V %.2e  tau %.2e  (sign agreement %.4f)" % (name, eR, eV, et, same.mean()))
    assert eR <= 1e-4 and eV <= 1e-4 and et <= 1e-4
    # the split products ran: the one-part BF16 factor of the same schedule is
    # far less accurate
    F1, _ = _factor(Ad, torch.float32, C.CTQR_PREC_BF16_MFMA, 256)
    R1 = np.triu(download(F1.A)[:n, :n]).astype(np.float64)
    e1 = np.abs(np.sign(np.diag(R1))[:, None] * R1 - so[:, None] * Ro).max() / np.abs(Ro).max()
    print("one-part BF16 nb=256 %s: R %.2e" % (name, e1))
    assert eR * 30 < e1
    # refined solve (the benchmark's solve) against the oracle's solution
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    spA = DeviceSparse(A)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    Xg = download(F3.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30))
    torch.cuda.synchronize()
    si = F3.sinfo.read()
    err = lsq.rel_err(Xg, Xo)
    print("refined: status %d iters %d err %.2e" % (si.status, si.iters, err.max()))
    assert si.status == 0, (si.status, si.iters, si.max_rel_update)
    assert si.x_iters == si.iters
    assert err.max() <= 1e-10


def test_nonfinite_in_A(gpu):
    _case("NaN in A")
    g, A, X, B = oracle_problem("ct24")
    Ad = A.toarray()
    Ad[37, 11] = np.nan
    for dt, prec in ((torch.float64, C.CTQR_PREC_FP64), (torch.float32, C.CTQR_PREC_BF16X3_MFMA)):
        F, info = _factor(Ad.astype(np.float64 if dt == torch.float64 else np.float32), dt, prec, 64)
        assert info.status == C.CTQR_NONFINITE, C.status_string(info.status)


def test_nonfinite_in_B_refined(gpu):
    _case("NaN in B")
    g, A, X, B = oracle_problem("ct24")
    F, info = _factor(A.toarray().astype(np.float32), torch.float32, C.CTQR_PREC_FP32_MFMA, 64)
    assert info.status == 0
    Bn = B.copy()
    Bn[100, 1] = np.nan
    spA = DeviceSparse(A)
    F.solve(to_colmajor(torch.as_tensor(Bn), dtype=torch.float64), sparse=spA.sp, tol=1e-12, max_iters=30)
    torch.cuda.synchronize()
    si = F.sinfo.read()
    assert si.status == C.CTQR_NONFINITE, C.status_string(si.status)
    assert si.iters == 1


def test_sparse_capacity_exceeded(gpu):
    _case("nnz capacity")
    g, A, _, _ = oracle_problem("ct24")
    small = A.nnz // 2
    S = SystemMatrix(g, C.CTQR_F64, dense=False, sparse=True, nnz_cap=small)
    torch.cuda.synchronize()
    info = S.info.read()
    assert info.status == C.CTQR_CAPACITY, C.status_string(info.status)
    assert info.nnz == A.nnz      # the count is still exact
    # the rows whose entries fit are complete and equal to the oracle's
    import scipy.sparse as sps
    rowptr = download(S.rowptr)
    assert (rowptr == A.indptr).all()
    rows = int(np.searchsorted(A.indptr, small, side="right") - 1)
    k = int(rowptr[rows])
    G = sps.csr_matrix((download(S.val)[:k], download(S.col)[:k], rowptr[:rows + 1]), shape=(rows, A.shape[1]))
    G.sort_indices()
    Ao = A[:rows]
    Ao.sort_indices()
    assert (G.indices == Ao.indices).all() and np.abs(G.data - Ao.data).max() <= 1e-12


def test_nearly_dependent_column_not_converged(gpu):
    # column 200 replaced by column 100 plus a 1e-7 relative perturbation:
    # kappa(A) is about 1e7, so the FP32 factor carries no information about
    # that direction (its R_jj is at the level of FP32 rounding) and the
    # corrections (R^T R)^-1 A^T r grow instead of contracting (the rate is
    # about u32 kappa^2 >> 1).  The refinement must report CTQR_NOT_CONVERGED
    # and return its best iterate.  (Scaling a column, by contrast, leaves
    # Householder QR's columnwise backward error and the refinement's rate
    # unchanged.)
    _case("nearly dependent column")
    g, A, X, B = oracle_problem("ct24")
    Ad = A.toarray()
    rng = np.random.default_rng(8)
    Ad[:, 200] = Ad[:, 100] + 1e-7 * np.linalg.norm(Ad[:, 100]) * rng.standard_normal(Ad.shape[0]) / np.sqrt(
        Ad.shape[0])
    import scipy.sparse as sps
    As = sps.csr_matrix(Ad)
    F, info = _factor(Ad.astype(np.float32), torch.float32, C.CTQR_PREC_FP32_MFMA, 64)
    assert info.status in (0, C.CTQR_RANK_DEFICIENT)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    X0 = download(F.solve(Bd))
    spA = DeviceSparse(As)
    Xr = download(F.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30))
    torch.cuda.synchronize()
    si = F.sinfo.read()
    print("nearly dependent column: factor status %d, refine status %d iters %d x_iters %d update %.2e "
          "contraction %.2e" % (info.status, si.status, si.iters, si.x_iters, si.max_rel_update, si.contraction))
    assert si.status == C.CTQR_NOT_CONVERGED
    assert 0 <= si.x_iters <= si.iters <= 30
    assert np.isfinite(Xr).all()
    if si.x_iters == 0:
        # the best iterate is the unrefined solution itself
        assert (Xr == X0).all()


def test_zero_subdiagonal_columns_tau_zero(gpu, oracle_lib):
    # columns 0..39 already upper triangular (zero below the diagonal): each
    # of their reflectors is the identity, tau = 0 and R_jj = A_jj with its
    # sign (beta = alpha), across the first inner panel's boundary
    _case("tau = 0 columns")
    rng = np.random.default_rng(21)
    m, n = 400, 150
    Ad = rng.standard_normal((m, n))
    for j in range(40):
        Ad[j + 1:, j] = 0.0
    QRo, tauo = hh.geqr2(Ad)
    assert (tauo[:40] == 0.0).all()
    F, info = _factor(Ad, torch.float64, C.CTQR_PREC_FP64, 64)
    assert info.status == 0, C.status_string(info.status)
    QRg, taug = download(F.A), download(F.tau)
    assert (taug[:40] == 0.0).all()
    assert (np.diag(QRg)[:40] == np.diag(Ad)[:40]).all()
    assert np.abs(taug - tauo).max() <= 1e-11
    assert np.abs(QRg - QRo).max() <= 1e-11 * np.abs(QRo).max()


def test_bf16x3_update_kernels_agree_bitwise(gpu, monkeypatch):
    # The trailing update runs on 256 x 256 tiles of eight waves when a launch
    # has enough tiles (CTQR_GEMM_W8=0 keeps the 128 x 128 form).  Both sum
    # every output's products in the same order, so the factors of the
    # benchmark's configuration are equal bit for bit.  ct128 (m = 23,040,
    # n = 16,384) has trailing updates of up to 86 x 60 tiles of 256.
    _case("bf16x3 update kernels ct128")
    w = get_workload("ct128")
    S = SystemMatrix(w.geometry(), C.CTQR_F32, dense=True, sparse=False)
    A0 = S.A.clone()
    outs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("CTQR_GEMM_W8", flag)
        S.A.copy_(A0)
        F = QRFactor(S.A, C.CTQR_PREC_BF16X3_MFMA, nb=256).factor()
        torch.cuda.synchronize()
        assert F.info.read().status == 0
        outs.append((F.A.clone(), F.T.clone(), F.tau.clone()))
        del F
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    del S, A0, outs
    torch.cuda.empty_cache()
