"""GPU tests of the persistent small-slice kernels (csrc/fused.hip): Q^T B and
the two block substitutions for at most 16 slices, one cooperative launch
each, selected by CTQR_FUSED=1 (every test here sets it).

They take the same blocks and the same products per block as the
launch-per-block path (Eq. 4; Section II-C, "System solving"), so they are
compared with the oracle's Householder solve (oracle/householder.py) at the
solve's bar, and with the launch-per-block path of the same factor (17
slices, which the persistent kernels do not take) to rounding.  Shapes span
several 2048-row diagonal blocks with a ragged last one, block reflectors
with a ragged last block, right-hand sides whose rows do not fill the last
64-row chunk, and grids where most workgroups own no row of R.  The
transposed substitution runs in the refinement (R^T y = A^T r): with an FP64
factor the corrections are exact to rounding, so the refinement must stop
after one or two iterations.
"""
import numpy as np
import pytest
import torch

from oracle import householder as hh
from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import QRFactor, to_colmajor

from gpu_helpers import oracle_problem, oracle_factor, DeviceSparse, upload_dense, download

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def fused_on(monkeypatch):
    # the persistent kernels are an option, selected per solve by CTQR_FUSED=1
    monkeypatch.setenv("CTQR_FUSED", "1")
    yield


def _case(*a):
    print("[case]", *a, flush=True)


def _dense_problem(m, n, S, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, S))
    QR, tau = hh.geqr2(A)
    Xo = hh.backsub(QR, hh.apply_qt(QR, tau, B))
    return A, B, Xo


def _factor(Ad, dtype, prec, nb):
    F = QRFactor(upload_dense(Ad.astype(np.float32) if dtype == torch.float32 else Ad, dtype), prec, nb=nb)
    F.factor()
    torch.cuda.synchronize()
    assert F.info.read().status == 0
    return F


@pytest.mark.parametrize("m,n,nb", [(3000, 2200, 256), (2600, 2304, 128), (700, 200, 64)])
def test_fused_fp64_direct_matches_oracle(gpu, m, n, nb):
    # 2200 = 2048 + 152: two diagonal blocks, the last ragged; block
    # reflectors of 256 with a ragged last one (152); m = 3000 leaves 56 rows
    # in the last chunk.  700 x 200: one diagonal block, 4 chunks of R
    A, B, Xo = _dense_problem(m, n, 17, seed=m + n)
    F = _factor(A, torch.float64, C.CTQR_PREC_FP64, nb)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    X17 = download(F.solve(Bd))                       # launch-per-block path (17 slices)
    for S in (1, 3, 16):
        _case("fused fp64 direct", m, n, nb, "S", S)
        X = download(F.solve(to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)))
        torch.cuda.synchronize()
        assert F.sinfo.read().status == 0
        assert lsq.rel_err(X, Xo[:, :S]).max() <= 1e-10
        assert lsq.rel_err(X, X17[:, :S]).max() <= 1e-12
    del F
    torch.cuda.empty_cache()


def test_fused_slices_independent(gpu):
    # a slice's result does not depend on the other slices of the call
    A, B, Xo = _dense_problem(3000, 2200, 16, seed=7)
    F = _factor(A, torch.float64, C.CTQR_PREC_FP64, 256)
    _case("fused independence")
    X16 = download(F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)))
    X5 = download(F.solve(to_colmajor(torch.as_tensor(B[:, 3:8]), dtype=torch.float64)))
    X1 = download(F.solve(to_colmajor(torch.as_tensor(B[:, 11:12]), dtype=torch.float64)))
    assert (X5 == X16[:, 3:8]).all()
    assert (X1 == X16[:, 11:12]).all()
    # and a repeated call gives the same bits
    X16b = download(F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)))
    assert (X16b == X16).all()
    del F
    torch.cuda.empty_cache()


def test_fused_fp32_unrefined_close_to_wide_path(gpu):
    A, B, Xo = _dense_problem(3000, 2200, 17, seed=3)
    F = _factor(A, torch.float32, C.CTQR_PREC_FP32_MFMA, 256)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    X17 = download(F.solve(Bd))
    _case("fused fp32 unrefined")
    X = download(F.solve(to_colmajor(torch.as_tensor(B[:, :16]), dtype=torch.float64)))
    # both FP32 solutions of a well-conditioned system: close to each other
    # (rounding order only) and to the oracle at the FP32 level
    assert lsq.rel_err(X, X17[:, :16]).max() <= 1e-5
    assert lsq.rel_err(X, Xo[:, :16]).max() <= 1e-3
    del F
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name,prec,nb", [("ct40", C.CTQR_PREC_FP32_MFMA, 128),
                                          ("ct48", C.CTQR_PREC_BF16X3_MFMA, 256),
                                          ("ct64", C.CTQR_PREC_BF16X3_MFMA, 256)])
def test_fused_refined_matches_oracle(gpu, name, prec, nb):
    # ct48: n = 2304 (a ragged second diagonal block); ct64: n = 4096 (two
    # full ones).  The refinement's substitutions (R^T y = s, R d = y) are
    # the persistent kernels at S <= 16.
    g, Asp, X, B = oracle_problem(name, n_slices=17)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    F = _factor(Asp.toarray(), torch.float32, prec, nb)
    spA = DeviceSparse(Asp)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    X17 = download(F.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30))
    it17 = F.sinfo.read().iters
    for S in (1, 5, 16):
        _case("fused refined", name, "S", S)
        Xs = download(F.solve(to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64), sparse=spA.sp,
                              tol=1e-12, max_iters=30))
        si = F.sinfo.read()
        assert si.status == 0, (C.status_string(si.status), si.iters)
        assert lsq.rel_err(Xs, Xo[:, :S]).max() <= 1e-10
        assert lsq.rel_err(Xs, X17[:, :S]).max() <= 1e-10
        assert si.iters <= it17 + 1
    del F
    torch.cuda.empty_cache()


def test_fused_fp64_refinement_exact_preconditioner(gpu):
    # with an FP64 factor, (R^T R)^-1 A^T r is the exact correction to
    # rounding: a wrong transposed substitution would not stop this early
    g, Asp, X, B = oracle_problem("ct40", n_slices=8)
    QRo, tauo = oracle_factor("ct40")
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    F = _factor(Asp.toarray(), torch.float64, C.CTQR_PREC_FP64, 128)
    spA = DeviceSparse(Asp)
    _case("fused fp64 refined")
    Xs = download(F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64), sparse=spA.sp, tol=1e-12,
                          max_iters=10))
    si = F.sinfo.read()
    assert si.status == 0 and si.iters <= 2, (si.status, si.iters)
    assert lsq.rel_err(Xs, Xo).max() <= 1e-10
    del F
    torch.cuda.empty_cache()


def test_fused_solver_buckets(gpu):
    # solver buckets of at most 16 slices enqueue the persistent kernels
    # directly: a padded request equals the direct solve bit for bit (slices
    # do not interact), and a refined bucket keeps the calibrated count
    from paper_1907_01891_amd.device import Solver
    g, Asp, X, B = oracle_problem("ct40", n_slices=20)
    QRo, tauo = oracle_factor("ct40")
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    F = _factor(Asp.toarray(), torch.float64, C.CTQR_PREC_FP64, 128)
    sv = Solver(F, max_slices=20)
    for S in (3, 16):
        _case("fused solver fp64", "S", S)
        Bd = to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)
        Xs = download(sv.solve(Bd))
        Xd = download(F.solve(Bd))
        assert sv.info.read().status == 0
        assert (Xs == Xd).all()
        assert lsq.rel_err(Xs, Xo[:, :S]).max() <= 1e-10
        assert sv.query(S)[2] == 0
    sv.close()
    F32 = _factor(Asp.toarray(), torch.float32, C.CTQR_PREC_FP32_MFMA, 128)
    spA = DeviceSparse(Asp)
    sv = Solver(F32, max_slices=20, sparse=spA.sp, tol=1e-12, max_iters=30)
    Bd = to_colmajor(torch.as_tensor(B[:, :5]), dtype=torch.float64)
    outs = []
    for rep in range(3):
        _case("fused solver mixed", "rep", rep)
        outs.append(download(sv.solve(Bd)))
        info = sv.info.read()
        assert info.status == 0, (C.status_string(info.status), info.iters)
        giters = sv.query(5)[2]
        if rep == 0:
            assert giters == -1                # calibration run: host-synchronised
            calib = info.iters
        else:
            assert giters == min(30, calib + 2)
            assert info.iters == calib
    assert (outs[1] == outs[0]).all() and (outs[2] == outs[0]).all()
    assert lsq.rel_err(outs[0], Xo[:, :5]).max() <= 1e-10
    sv.close()
    del F, F32
    torch.cuda.empty_cache()
