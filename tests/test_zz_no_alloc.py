"""ctqr_qr_solve_slices_noalloc, the solve for callers that cannot allocate,
against ctqr_qr_solve_slices on the same factor and right-hand sides.

Both run the same kernels over the same workspace layout (the no-alloc call
carves it from the library's device scratch array), so their solutions are
compared bit for bit, and against the oracle's least-squares solution at the
1e-10 bar (Eq. 4).  Two calls in a row, the second with a smaller input (fewer
slices, and a smaller problem), check that the scratch array's leftover
contents from the first call do not leak into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import householder as hh
from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import QRFactor, Info, colmajor, ld_of, stream_handle, to_colmajor

from gpu_helpers import oracle_problem, oracle_factor, DeviceSparse, upload_dense, download

pytestmark = pytest.mark.gpu


def _case(*a):
    print("[case]", *a, flush=True)


def _noalloc(F, B, sparse=None, tol=1e-12, max_iters=0):
    S = B.shape[1]
    X = colmajor(F.n, S, torch.float64, B.device)
    info = Info(B.device)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = C.lib().ctqr_qr_solve_slices_noalloc(F.m, F.n, F.dtype, p(F.A), ld_of(F.A), p(F.T), p(F.tau), p(F.Rinv),
                                              F.nb, p(B), ld_of(B), S, p(X), ld_of(X),
                                              ctypes.byref(sparse) if sparse is not None else None, tol,
                                              max_iters, C.CTQR_REFINE_CSNE, info.ptr, stream_handle())
    C.check(st, "ctqr_qr_solve_slices_noalloc")
    torch.cuda.synchronize()
    return X, info.read()


def _setup(name, dtype, prec):
    g, A, X, B = oracle_problem(name)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    Ad = A.toarray() if dtype == torch.float64 else A.toarray().astype(np.float32)
    F = QRFactor(upload_dense(Ad, dtype), prec, nb=64).factor()
    torch.cuda.synchronize()
    assert F.info.read().status == 0
    return A, B, Xo, F


@pytest.mark.parametrize("dtype,prec,refine", [(torch.float64, C.CTQR_PREC_FP64, False),
                                               (torch.float32, C.CTQR_PREC_BF16X3_MFMA, True)])
def test_noalloc_matches_workspace_solve(gpu, dtype, prec, refine):
    # first call: ct40 (5 slices); second call: ct24 with 2 slices
    for name, nsl in (("ct40", 5), ("ct24", 2)):
        _case("noalloc", name, nsl, dtype, "refine" if refine else "")
        A, B, Xo, F = _setup(name, dtype, prec)
        Bd = to_colmajor(torch.as_tensor(B[:, :nsl]), dtype=torch.float64)
        spA = DeviceSparse(A) if refine else None
        kw = dict(sparse=spA.sp, tol=1e-12, max_iters=30) if refine else {}
        Xw = download(F.solve(Bd, **kw))
        torch.cuda.synchronize()
        iw = F.sinfo.read()
        Xn, inn = _noalloc(F, Bd, **kw)
        Xn = download(Xn)
        assert inn.status == iw.status == 0, (inn.status, iw.status)
        assert inn.iters == iw.iters
        assert (Xn == Xw).all()
        assert lsq.rel_err(Xn, Xo[:, :nsl]).max() <= 1e-10


def test_noalloc_rejects_beyond_scratch(gpu):
    # 256^2 with 256 slices needs far more than the scratch: refused, with
    # nothing enqueued
    _case("noalloc limit")
    p = ctypes.c_void_p(256)
    st = C.lib().ctqr_qr_solve_slices_noalloc(88320, 65536, C.CTQR_F32, p, 88320, p, p, p, 256, p, 88320, 256,
                                              p, 65536, None, 1e-12, 0, C.CTQR_REFINE_CSNE, p, None)
    assert st == C.CTQR_ENOMEM
    assert b"CTQR_NOALLOC_SCRATCH_BYTES" in C.lib().ctqr_last_error()
