"""ctqr_cond_estimate against the oracle's SVD, and the refinement's
reported contraction against the corrected semi-normal-equations rate.

kappa(A) = sigma_max / sigma_min (2-norm).  The estimate runs power iteration
on A^T A (FP64 sparse A) and inverse iteration on R^T R (the factor's R, A = QR,
Eq. 3): each Rayleigh quotient is a lower bound of its target, so with an FP64
factor the estimates never exceed the SVD's values (beyond rounding) and
approach them as the iterations proceed.
"""
import numpy as np
import pytest
import torch

from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import QRFactor, to_colmajor

from gpu_helpers import oracle_problem, DeviceSparse, upload_dense

pytestmark = pytest.mark.gpu


def _case(*a):
    print("[case]", *a, flush=True)


def _factor(Ad, dtype, prec, nb=64):
    F = QRFactor(upload_dense(Ad, dtype), prec, nb=nb)
    F.factor()
    torch.cuda.synchronize()
    assert F.info.read().status == 0
    return F


@pytest.mark.parametrize("name", ["ct24", "ct32", "ct40"])
def test_cond_estimate_matches_svd(gpu, name):
    _case("cond", name)
    g, A, _, _ = oracle_problem(name)
    Ad = A.toarray()
    sv = np.linalg.svd(Ad, compute_uv=False)
    F = _factor(Ad, torch.float64, C.CTQR_PREC_FP64)
    spA = DeviceSparse(A)
    smax, smin, kappa = F.cond_estimate(spA.sp, nvec=8, iters=40)
    print("%s: sigma_max %.6e (svd %.6e)  sigma_min %.6e (svd %.6e)  kappa %.4e (svd %.4e)"
          % (name, smax, sv[0], smin, sv[-1], kappa, sv[0] / sv[-1]))
    assert smax <= sv[0] * (1 + 1e-10) and smax >= 0.999 * sv[0]
    assert smin >= sv[-1] * (1 - 1e-10) and smin <= 1.1 * sv[-1]
    assert kappa <= sv[0] / sv[-1] * (1 + 1e-9) and kappa >= 0.9 * sv[0] / sv[-1]


def test_cond_estimate_known_spectrum(gpu):
    # A = U diag(s) V^T with s geometric from 1 to 1e-4: kappa = 1e4 exactly;
    # the FP32 factor's R gives sigma_min to about kappa * u32 relative
    _case("cond known spectrum")
    rng = np.random.default_rng(4)
    m, n = 700, 300
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.geomspace(1.0, 1e-4, n)
    Ad = (U * s) @ V.T
    spA = DeviceSparse(Ad)
    for dt, prec, tol in ((torch.float64, C.CTQR_PREC_FP64, 1e-9), (torch.float32, C.CTQR_PREC_FP32_MFMA, 1e-2)):
        A_in = Ad if dt == torch.float64 else Ad.astype(np.float32)
        F = _factor(A_in, dt, prec)
        smax, smin, kappa = F.cond_estimate(spA.sp, nvec=8, iters=60)
        print("known spectrum (%s): sigma_max %.6e sigma_min %.6e kappa %.6e" % (dt, smax, smin, kappa))
        assert abs(smax - 1.0) <= 1e-3
        assert abs(smin / 1e-4 - 1.0) <= max(tol, 1e-3)
        assert abs(kappa / 1e4 - 1.0) <= max(tol, 2e-3)


def test_refinement_contraction_reported(gpu):
    # corrected semi-normal equations contract the error by about
    # c eps kappa^2 per iteration, eps the factor's relative backward error
    # (about sqrt(m) u32 for the FP32 factor, as in the full-size Gram check);
    # the info reports the mean rate
    _case("contraction")
    g, A, X, B = oracle_problem("ct40")
    F = _factor(A.toarray().astype(np.float32), torch.float32, C.CTQR_PREC_FP32_MFMA)
    spA = DeviceSparse(A)
    _, _, kappa = F.cond_estimate(spA.sp, nvec=8, iters=40)
    F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64), sparse=spA.sp, tol=1e-12, max_iters=30)
    torch.cuda.synchronize()
    si = F.sinfo.read()
    u32 = 2.0 ** -24
    print("kappa %.3e, iters %d, contraction %.3e, u32 kappa^2 %.3e" % (kappa, si.iters, si.contraction,
                                                                      u32 * kappa ** 2))
    assert si.status == 0 and si.iters >= 2 and si.x_iters == si.iters
    assert 0.0 < si.contraction < 1.0
    assert si.contraction <= 10.0 * np.sqrt(A.shape[0]) * u32 * kappa ** 2
