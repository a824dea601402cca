"""GPU tests of the out-of-core factorization (ctqr_qr_factor_ooc) and of the
FP32-slab panel of very tall matrices.

Pins: the out-of-core factor (resident columns in HBM, the rest streamed
from pinned host memory in tiles) is bit-identical to the all-in-HBM factor
of the same matrix -- factored matrix, T, tau and the diagonal-block
inverses -- since it performs the same arithmetic in another order of
blocks with every reduction split the same way.  The tall panel is pinned
to the oracle's FP64 Householder QR (R to FP32 accuracy).
"""
import numpy as np
import pytest
import torch

from oracle import householder as hh
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import QRFactor, OocFactor, to_colmajor

pytestmark = pytest.mark.gpu


def _print_case(*a):
    print("[case]", *a, flush=True)


def _random(m, n, seed, dtype):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    return torch.as_tensor(A, dtype=dtype)


@pytest.mark.parametrize("m,n,nb,n_dev,tile,dt", [
    (6000, 5000, 128, 2048, 2048, "f64"),     # resident part + two tiles (the last ragged)
    (6000, 5000, 256, 0, 2048, "f32"),        # everything streamed: three tiles, re-uploads
    (4500, 4096, 256, 2048, 4096, "f32"),     # one tile wider than the rest of the matrix
    (6000, 5000, 256, 2048, 2048, "bf16"),    # BF16 block-column products
    (6000, 5000, 256, 2048, 2048, "bf16x3"),  # split-BF16 block-column products
])
def test_ooc_factor_bitwise_equals_in_core(gpu, m, n, nb, n_dev, tile, dt):
    _print_case("ooc", m, n, nb, n_dev, tile, dt)
    dtype = torch.float64 if dt == "f64" else torch.float32
    cd = C.CTQR_F64 if dt == "f64" else C.CTQR_F32
    prec = {"f64": C.CTQR_PREC_FP64, "f32": C.CTQR_PREC_FP32_MFMA, "bf16": C.CTQR_PREC_BF16_MFMA,
            "bf16x3": C.CTQR_PREC_BF16X3_MFMA}[dt]
    A = _random(m, n, 11, dtype)
    Ad = to_colmajor(A, dtype=dtype)
    F = QRFactor(Ad, prec, nb=nb).factor()
    O = OocFactor(m, n, cd, prec, n_dev, tile, nb=nb)
    O.load(to_colmajor(A, dtype=dtype, device="cpu"))
    O.factor()
    torch.cuda.synchronize()
    fi, oi = F.info.read(), O.info.read()
    assert fi.status == 0 and oi.status == 0
    assert (fi.rdiag_min, fi.rdiag_max) == (oi.rdiag_min, oi.rdiag_max)
    assert torch.equal(O.factor_matrix(), F.A.cpu())
    # T: each block's nbk x nbk factor (rows below nbk of a ragged last block
    # are never written)
    To, Tf = O.T.cpu(), F.T.cpu()
    for k0 in range(0, n, nb):
        nbk = min(nb, n - k0)
        assert torch.equal(To[:nbk, k0:k0 + nbk], Tf[:nbk, k0:k0 + nbk]), k0
    assert torch.equal(O.tau.cpu(), F.tau.cpu())
    assert torch.equal(O.Rinv.cpu(), F.Rinv.cpu())


def test_tall_fp32_panel_matches_oracle(gpu, oracle_lib):
    # 160,000 rows: more rows per workgroup than an FP64 slab holds, so the
    # panel keeps its slab in FP32 (sums still in FP64)
    m, n = 160000, 320
    _print_case("tall panel", m, n)
    A = _random(m, n, 5, torch.float64)
    F = QRFactor(to_colmajor(A, dtype=torch.float32), C.CTQR_PREC_FP32_MFMA, nb=128).factor()
    torch.cuda.synchronize()
    assert F.info.read().status == 0
    QRo, tau_o = hh.geqr2(A.to(torch.float32).to(torch.float64).numpy())
    Rg = np.triu(F.A[:n, :].cpu().numpy().astype(np.float64))
    Ro = np.triu(QRo[:n, :])
    err = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    print("tall panel R rel err %.2e" % err)
    assert err <= 2e-5
    assert np.abs(F.tau.cpu().numpy() - tau_o).max() <= 1e-5


def test_sparse_to_dense_matches_build(gpu):
    from synthetic import get_workload
    from paper_1907_01891_amd.device import SystemMatrix, colmajor
    g = get_workload("ct32").geometry()
    S = SystemMatrix(g, C.CTQR_F32, dense=True, sparse=True)
    out = colmajor(S.m, S.n, torch.float32)
    S.dense_cols(0, S.n, out, C.CTQR_F32)
    part = colmajor(S.m, 600, torch.float32)
    S.dense_cols(100, 700, part, C.CTQR_F32)
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), S.A.cpu())
    assert torch.equal(part.cpu(), S.A[:, 100:700].cpu())


@pytest.mark.parametrize("name,n_dev,dt,method", [("ct48", 0, "f64", 0), ("ct48", 0, "f32", 0),
                                                  ("ct64", 2048, "f32", 0), ("ct64", 2048, "f32", 1)])
def test_ooc_solve_matches_in_core_and_oracle(gpu, name, n_dev, dt, method):
    from gpu_helpers import oracle_problem, oracle_factor, DeviceSparse
    from oracle import lsq
    g, A, X, B = oracle_problem(name, n_slices=40)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    m, n = A.shape
    dtype = torch.float64 if dt == "f64" else torch.float32
    cd = C.CTQR_F64 if dt == "f64" else C.CTQR_F32
    prec = C.CTQR_PREC_FP64 if dt == "f64" else C.CTQR_PREC_FP32_MFMA
    Ad = torch.as_tensor(A.toarray(), dtype=dtype)
    F = QRFactor(to_colmajor(Ad, dtype=dtype), prec, nb=256).factor()
    O = OocFactor(m, n, cd, prec, n_dev, 2048, nb=256)
    O.load(to_colmajor(Ad, dtype=dtype, device="cpu"))
    O.factor()
    spA = DeviceSparse(A)
    kw = {} if dt == "f64" else dict(sparse=spA.sp, tol=1e-12, max_iters=30, method=method)
    for S in (4, 40):
        _print_case("ooc solve", name, n_dev, dt, "S", S)
        Bd = to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)
        Xg = O.solve(Bd, **kw).cpu().numpy()
        Xi = F.solve(Bd, **kw).cpu().numpy()
        torch.cuda.synchronize()
        si = O.sinfo.read()
        assert si.status == 0, (C.status_string(si.status), si.iters)
        e_in, e_or = lsq.rel_err(Xg, Xi).max(), lsq.rel_err(Xg, Xo[:, :S]).max()
        print("%s S %d vs in-core %.2e vs oracle %.2e iters %d" % (dt, S, e_in, e_or, si.iters))
        assert e_or <= 1e-10
        assert e_in <= (1e-12 if dt == "f64" else 1e-10)
