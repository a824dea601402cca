"""GPU parity of the libctqr hot path against the CPU oracle, at sizes the
oracle finishes in seconds (several 128-wide tiles, ragged edges).

Tolerances (FP64 path): the GPU and the oracle both run backward-stable
Householder QRs of the same matrix with different summation orders, so
their R, V and tau differ by O(kappa * u) relative to ||A|| (kappa <= ~500
here, u = 1.1e-16): 1e-11 relative is a bound with two orders of slack.
Solutions must agree to the 1e-10 relative bar of the mixed path and in
practice agree to ~1e-13.
"""
import ctypes

import numpy as np
import pytest
import torch

from synthetic import get_workload
from oracle import householder as hh
from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import SystemMatrix, QRFactor, colmajor, to_colmajor

from gpu_helpers import oracle_problem, oracle_factor, DeviceSparse, upload_dense, download

pytestmark = pytest.mark.gpu


def _print_case(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("name", ["ct8", "ct24", "ct32"])
def test_system_matrix_matches_oracle(gpu, name):
    _print_case("siddon", name)
    g, A, _, _ = oracle_problem(name)
    S = SystemMatrix(g, C.CTQR_F64, dense=True, sparse=True)
    torch.cuda.synchronize()
    info = S.info.read()
    assert info.status == 0, C.status_string(info.status)
    assert info.nnz == A.nnz
    Ad = download(S.A)
    assert np.abs(Ad - A.toarray()).max() <= 1e-12
    rowptr = download(S.rowptr)
    assert (rowptr == A.indptr).all()
    import scipy.sparse as sp
    nnz = A.nnz
    G = sp.csr_matrix((download(S.val)[:nnz], download(S.col)[:nnz], rowptr), shape=A.shape)
    G.sort_indices()
    assert (G.indices == A.indices).all()
    assert np.abs(G.data - A.data).max() <= 1e-12
    # CSC: the same values, rows ascending within each column
    Ac = A.tocsc()
    Ac.sort_indices()
    assert (download(S.colptr) == Ac.indptr).all()
    assert (download(S.row)[:nnz] == Ac.indices).all()
    Gc = sp.csc_matrix((download(S.cval)[:nnz], download(S.row)[:nnz], download(S.colptr)), shape=A.shape)
    assert (Gc != G.tocsc()).nnz == 0


def test_system_matrix_fp32_dense(gpu):
    _print_case("siddon f32")
    g, A, _, _ = oracle_problem("ct24")
    S64 = SystemMatrix(g, C.CTQR_F64, dense=True, sparse=False)
    S32 = SystemMatrix(g, C.CTQR_F32, dense=True, sparse=False)
    torch.cuda.synchronize()
    assert (download(S32.A) == download(S64.A).astype(np.float32)).all()


def _gpu_factor(Ad, dtype, prec, nb):
    A = upload_dense(Ad, dtype)
    F = QRFactor(A, prec, nb=nb)
    F.factor()
    torch.cuda.synchronize()
    info = F.info.read()
    return F, info


@pytest.mark.parametrize("name,nb", [("ct24", 32), ("ct24", 64), ("ct32", 256), ("ct32", 96), ("ct40", 128)])
def test_qr_fp64_matches_oracle(gpu, name, nb):
    _print_case("qr fp64", name, nb)
    g, A, _, _ = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    F, info = _gpu_factor(A.toarray(), torch.float64, C.CTQR_PREC_FP64, nb)
    assert info.status == 0, C.status_string(info.status)
    QRg = download(F.A)
    taug = download(F.tau)
    scale = np.abs(QRo).max()
    assert np.abs(taug - tauo).max() <= 1e-11
    assert np.abs(QRg - QRo).max() <= 1e-11 * scale
    assert abs(info.rdiag_max - np.abs(np.diag(QRo)).max()) <= 1e-11 * scale


@pytest.mark.parametrize("m,n,nb", [(1000, 333, 64), (517, 517, 256), (2000, 64, 32), (130, 33, 32),
                                    (64, 1, 32), (777, 300, 96)])
def test_qr_fp64_random_ragged(gpu, m, n, nb, oracle_lib):
    _print_case("qr random", m, n, nb)
    rng = np.random.default_rng(m * 1000 + n)
    Ad = rng.standard_normal((m, n))
    QRo, tauo = hh.geqr2(Ad)
    F, info = _gpu_factor(Ad, torch.float64, C.CTQR_PREC_FP64, nb)
    assert info.status == 0, C.status_string(info.status)
    QRg = download(F.A)
    assert np.abs(download(F.tau) - tauo).max() <= 1e-11
    assert np.abs(QRg - QRo).max() <= 1e-11 * np.abs(QRo).max()
    # backward error of the GPU factor, rebuilt by the oracle's reflector
    # application from the GPU's own V and tau
    R = np.triu(QRg[:n, :n])
    QR_rebuilt = hh.apply_q(QRg, download(F.tau), np.vstack([R, np.zeros((m - n, n))]))
    assert np.linalg.norm(QR_rebuilt - Ad) / np.linalg.norm(Ad) <= 1e-14


def _factor_route(monkeypatch, route, Ad, dtype, prec, nb):
    if route is None:
        monkeypatch.delenv("CTQR_PANEL_ROUTE", raising=False)
    else:
        monkeypatch.setenv("CTQR_PANEL_ROUTE", route)
    F, info = _gpu_factor(Ad, dtype, prec, nb)
    assert info.status == 0, C.status_string(info.status)
    return download(F.A), download(F.tau), download(F.T)


@pytest.mark.parametrize("m,n,nb", [(3000, 500, 128), (9000, 256, 256), (777, 300, 96), (64, 1, 32)])
def test_panel_routes_agree(gpu, monkeypatch, m, n, nb):
    # The inner panels run by default through Cholesky QR twice and the
    # Householder reconstruction (four grid barriers per panel);
    # CTQR_PANEL_ROUTE=columns forms the reflectors one column at a time.
    # Both give the Householder V, tau and R of the column route in exact
    # arithmetic: equal to the oracle's at the FP64 bound, to each other to
    # rounding, and not bit for bit (so the reconstruction did run).
    # 9000 rows: slabs of the minimum 64 rows, 141 workgroups, the last
    # slab ragged.
    _print_case("panel routes", m, n, nb)
    rng = np.random.default_rng(m + 7 * n)
    Ad = rng.standard_normal((m, n))
    QRo, tauo = hh.geqr2(Ad)
    scale = np.abs(QRo).max()
    a_c, t_c, T_c = _factor_route(monkeypatch, "columns", Ad, torch.float64, C.CTQR_PREC_FP64, nb)
    a_r, t_r, T_r = _factor_route(monkeypatch, None, Ad, torch.float64, C.CTQR_PREC_FP64, nb)
    for a, t in ((a_c, t_c), (a_r, t_r)):
        assert np.abs(t - tauo).max() <= 1e-11
        assert np.abs(a - QRo).max() <= 1e-11 * scale
    assert np.abs(a_r - a_c).max() <= 1e-12 * scale
    assert np.abs(T_r - T_c).max() <= 1e-12 * np.abs(T_c).max()
    if n > 1:
        assert not (a_r == a_c).all()


def test_panel_route_falls_back_bitwise(gpu, monkeypatch):
    # every 32-wide panel holds a column that nearly repeats another
    # (condition number ~1e8): one Cholesky QR pass leaves Q1^T Q1 far from
    # I, so each panel takes the column route, and the factor equals the
    # column route's bit for bit
    _print_case("panel route fallback")
    rng = np.random.default_rng(5)
    m, n = 2000, 96
    Ad = rng.standard_normal((m, n))
    for c0 in range(0, n, 32):
        Ad[:, c0 + 7] = Ad[:, c0 + 3] + 1e-8 * rng.standard_normal(m)
    a_c, t_c, T_c = _factor_route(monkeypatch, "columns", Ad, torch.float64, C.CTQR_PREC_FP64, 32)
    a_r, t_r, T_r = _factor_route(monkeypatch, None, Ad, torch.float64, C.CTQR_PREC_FP64, 32)
    assert (a_r == a_c).all() and (t_r == t_c).all() and (T_r == T_c).all()


def test_block_reflector_T(gpu, oracle_lib):
    """I - V T V^T applied to random vectors equals H_1 ... H_nb applied one
    reflector at a time (compact-WY definition of the S factors)."""
    _print_case("T check")
    m, n, nb = 700, 300, 128
    rng = np.random.default_rng(7)
    Ad = rng.standard_normal((m, n))
    F, info = _gpu_factor(Ad, torch.float64, C.CTQR_PREC_FP64, nb)
    QRg, tau, T = download(F.A), download(F.tau), download(F.T)
    for k0 in range(0, n, nb):
        w = min(nb, n - k0)
        sub = QRg[k0:, k0:k0 + w]
        V = np.tril(sub, -1)
        V[np.arange(w), np.arange(w)] = 1.0
        Tk = T[:w, k0:k0 + w]
        assert np.allclose(np.tril(Tk, -1), 0.0)
        z = rng.standard_normal((m - k0, 3))
        ref = hh.apply_q(sub, tau[k0:k0 + w], z)
        got = z - V @ (Tk @ (V.T @ z))
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name,nb", [("ct24", 64), ("ct32", 256), ("ct40", 128)])
def test_solve_fp64_matches_oracle(gpu, name, nb):
    _print_case("solve fp64", name, nb)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    F, info = _gpu_factor(A.toarray(), torch.float64, C.CTQR_PREC_FP64, nb)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    Xg = download(F.solve(Bd))
    torch.cuda.synchronize()
    assert F.sinfo.read().status == 0
    err = lsq.rel_err(Xg, Xo)
    assert err.max() <= 1e-10, err


@pytest.mark.parametrize("name", ["ct24", "ct32"])
def test_exact_recovery_fp64(gpu, name):
    _print_case("recovery", name)
    g, A, X, B = oracle_problem(name, noisy=False)
    F, info = _gpu_factor(A.toarray(), torch.float64, C.CTQR_PREC_FP64, 64)
    Xg = download(F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)))
    assert lsq.rel_err(Xg, X).max() <= 1e-11


@pytest.mark.parametrize("method", [C.CTQR_REFINE_CSNE, C.CTQR_REFINE_PCG])
@pytest.mark.parametrize("name,nb", [("ct24", 64), ("ct32", 256), ("ct40", 128)])
def test_mixed_fp32_refined_matches_oracle(gpu, name, nb, method):
    _print_case("mixed fp32", name, nb, "method", method)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    F, info = _gpu_factor(A.toarray().astype(np.float32), torch.float32, C.CTQR_PREC_FP32_MFMA, nb)
    assert info.status == 0, C.status_string(info.status)
    # the FP32 factor itself is an FP32-accurate QR
    R32 = np.triu(download(F.A)[:A.shape[1], :A.shape[1]]).astype(np.float64)
    Ro = np.triu(QRo[:A.shape[1], :A.shape[1]])
    assert np.abs(R32 - Ro).max() <= 1e-4 * np.abs(Ro).max()
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    Xu = download(F.solve(Bd))                   # unrefined FP32 solve
    spA = DeviceSparse(A)
    Xg = download(F.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30, method=method))
    torch.cuda.synchronize()
    si = F.sinfo.read()
    assert si.status == 0, (C.status_string(si.status), si.iters, si.max_rel_update)
    e_unref = lsq.rel_err(Xu, Xo).max()
    err = lsq.rel_err(Xg, Xo)
    print("unrefined %.3e refined %.3e iters %d" % (e_unref, err.max(), si.iters))
    assert err.max() <= 1e-10
    assert e_unref < 1e-2


def test_determinism(gpu):
    _print_case("determinism")
    g, A, X, B = oracle_problem("ct32")
    outs = []
    for _ in range(2):
        F, info = _gpu_factor(A.toarray(), torch.float64, C.CTQR_PREC_FP64, 64)
        Xg = download(F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)))
        outs.append((download(F.A), Xg))
    assert (outs[0][0] == outs[1][0]).all()
    assert (outs[0][1] == outs[1][1]).all()


def test_rank_deficient_reported(gpu):
    _print_case("rank deficiency")
    rng = np.random.default_rng(3)
    Ad = rng.standard_normal((300, 100))
    Ad[:, 57] = Ad[:, 10] * 2.0          # dependent column
    F, info = _gpu_factor(Ad, torch.float64, C.CTQR_PREC_FP64, 32)
    assert info.status == C.CTQR_RANK_DEFICIENT
    assert info.first_bad_col == 57


@pytest.mark.parametrize("name", ["ct24", "ct40"])
def test_bf16_trailing_update_factor(gpu, name):
    # BF16 MFMA for the block-column products (operands rounded to bf16, FP32
    # accumulation): R agrees with the oracle's to BF16 accuracy -- visibly
    # worse than the FP32 path, which shows the BF16 kernels ran -- and the
    # refined solve either converges or reports that it did not.
    _print_case("bf16 factor", name)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    n = A.shape[1]
    Ro = np.triu(QRo[:n, :n])
    F16, info = _gpu_factor(A.toarray().astype(np.float32), torch.float32, C.CTQR_PREC_BF16_MFMA, 64)
    F32, info32 = _gpu_factor(A.toarray().astype(np.float32), torch.float32, C.CTQR_PREC_FP32_MFMA, 64)
    assert info.status in (0, C.CTQR_RANK_DEFICIENT), C.status_string(info.status)
    # R is unique up to the signs of its rows: a pivot that BF16 rounding
    # moves across zero flips the reflector's sign choice, so compare
    # diag(sign R_ii) R
    sn = lambda R: np.sign(np.diag(R))[:, None] * R
    R16 = sn(np.triu(download(F16.A)[:n, :n]).astype(np.float64))
    R32 = sn(np.triu(download(F32.A)[:n, :n]).astype(np.float64))
    Ron = sn(Ro)
    e16 = np.abs(R16 - Ron).max() / np.abs(Ron).max()
    e32 = np.abs(R32 - Ron).max() / np.abs(Ron).max()
    print("R rel err: bf16 %.2e, fp32 %.2e" % (e16, e32))
    assert e16 <= 5e-2
    assert e16 > 10 * e32
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    spA = DeviceSparse(A)
    for method in (C.CTQR_REFINE_CSNE, C.CTQR_REFINE_PCG):
        Xg = download(F16.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30, method=method))
        torch.cuda.synchronize()
        si = F16.sinfo.read()
        err = lsq.rel_err(Xg, Xo).max()
        print("bf16 refined (method %d): status %d iters %d err %.2e" % (method, si.status, si.iters, err))
        assert si.status in (0, C.CTQR_NOT_CONVERGED)
        if si.status == 0:
            assert err <= 1e-10


@pytest.mark.parametrize("name", ["ct24", "ct40"])
def test_bf16x3_trailing_update_factor(gpu, name):
    # Split BF16 (high and low bf16 parts, three products, FP32 accumulation)
    # for the block-column products: R agrees with the oracle's far better
    # than the one-part BF16 path and close to the FP32 path, and the refined
    # solve reaches the oracle's solution with both refinement forms.
    _print_case("bf16x3 factor", name)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    n = A.shape[1]
    Ad = A.toarray().astype(np.float32)
    F3, info = _gpu_factor(Ad, torch.float32, C.CTQR_PREC_BF16X3_MFMA, 64)
    F16, _ = _gpu_factor(Ad, torch.float32, C.CTQR_PREC_BF16_MFMA, 64)
    F32, _ = _gpu_factor(Ad, torch.float32, C.CTQR_PREC_FP32_MFMA, 64)
    assert info.status == 0, C.status_string(info.status)
    sn = lambda R: np.sign(np.diag(R))[:, None] * R
    Ron = sn(np.triu(QRo[:n, :n]))
    err = {}
    for key, F in (("x3", F3), ("bf16", F16), ("fp32", F32)):
        R = sn(np.triu(download(F.A)[:n, :n]).astype(np.float64))
        err[key] = np.abs(R - Ron).max() / np.abs(Ron).max()
    print("R rel err: bf16x3 %.2e, bf16 %.2e, fp32 %.2e" % (err["x3"], err["bf16"], err["fp32"]))
    assert err["x3"] <= 1e-4
    assert err["x3"] * 30 < err["bf16"]
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    spA = DeviceSparse(A)
    for method in (C.CTQR_REFINE_CSNE, C.CTQR_REFINE_PCG):
        Xg = download(F3.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30, method=method))
        torch.cuda.synchronize()
        si = F3.sinfo.read()
        e = lsq.rel_err(Xg, Xo).max()
        print("bf16x3 refined (method %d): status %d iters %d err %.2e" % (method, si.status, si.iters, e))
        assert si.status == 0
        assert e <= 1e-10


def test_tune_nb_small_matrix(gpu):
    # n = 576 (fewer than 1024 columns, not a multiple of 256): every candidate
    # factors all columns, whole groups of block columns included
    name = "ct24"
    _print_case("tune nb small", name)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    Ad = A.toarray()
    F = QRFactor(upload_dense(Ad, torch.float64), C.CTQR_PREC_FP64, nb=256)
    nb, ms = F.tune_nb()
    torch.cuda.synchronize()
    assert nb in (64, 128, 256) and F.nb == nb and all(t > 0 for t in ms)
    F2, info = _gpu_factor(Ad, torch.float64, C.CTQR_PREC_FP64, nb)
    assert info.status == 0, C.status_string(info.status)
    assert np.abs(download(F2.A) - QRo).max() <= 1e-11 * np.abs(QRo).max()


def test_tune_nb_then_factor(gpu):
    # the block-width tuner times every candidate on the caller's matrix
    # (overwriting it); the matrix rebuilt and factored with the chosen width
    # meets the oracle
    name = "ct48"                       # n = 2304: the tuner factors 1024 columns per candidate
    _print_case("tune nb", name)
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    Ad = A.toarray()
    F = QRFactor(upload_dense(Ad, torch.float64), C.CTQR_PREC_FP64, nb=256)
    nb, ms = F.tune_nb()
    torch.cuda.synchronize()
    print("tuned nb %d, ms per column %s" % (nb, ms))
    assert nb in (64, 128, 256) and F.nb == nb
    assert all(t > 0 for t in ms)
    F.A.copy_(upload_dense(Ad, torch.float64))
    F.factor()
    torch.cuda.synchronize()
    assert F.info.read().status == 0
    n = A.shape[1]
    sn = lambda R: np.sign(np.diag(R))[:, None] * R
    R = np.triu(download(F.A)[:n, :n])
    assert np.abs(sn(R) - sn(np.triu(QRo[:n, :n]))).max() <= 1e-11 * np.abs(QRo[:n, :n]).max()
    Xg = download(F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)))
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    assert lsq.rel_err(Xg, Xo).max() <= 1e-10
