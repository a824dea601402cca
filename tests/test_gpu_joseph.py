"""GPU Joseph projector and image-quality metrics against the oracle
(oracle.joseph: Joseph's method ray by ray, PSNR of Eq. 5-6, SSIM of Eq. 7
over 11 x 11 Gaussian windows).

Tolerances: the projections are FP64 sums of at most `side` interpolated
samples on both sides, with the same sample positions computed in a different
order: 1e-12 relative to the largest projection.  PSNR and SSIM are FP64
reductions in different orders: 1e-9 absolute on PSNR (dB), 1e-12 on SSIM.
"""
import numpy as np
import pytest
import torch

from oracle import joseph as J
from oracle import lsq
from paper_1907_01891_amd.device import project_joseph, image_quality, to_colmajor
from synthetic import get_workload, phantom_batch

from gpu_helpers import download

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,schedule", [("ct8", 1), ("ct24", 1), ("ct24", 0), ("ct40", 1)])
def test_joseph_matches_oracle(gpu, name, schedule):
    print("[case] joseph", name, schedule, flush=True)
    g = dict(get_workload(name).geometry(), angle_schedule=schedule)
    X = phantom_batch(g["side"], 3)
    Bo = J.joseph_project(g, X)
    Bg = download(project_joseph(g, to_colmajor(torch.as_tensor(X), dtype=torch.float64)))
    assert np.abs(Bg - Bo).max() <= 1e-12 * np.abs(Bo).max()


def test_image_quality_matches_oracle(gpu):
    print("[case] quality", flush=True)
    side, S = 32, 4
    rng = np.random.default_rng(9)
    Xr = phantom_batch(side, S)
    Xn = Xr + 10.0 ** -rng.uniform(1, 6, S)[None, :] * rng.standard_normal(Xr.shape)
    Xn[:, 3] = Xr[:, 3]                      # an exact image: PSNR inf, SSIM 1
    dr = lambda a: to_colmajor(torch.as_tensor(a), dtype=torch.float64)
    ps, ss = image_quality(side, dr(Xr), dr(Xn))
    for s in range(S):
        ref, img = Xr[:, s].reshape(side, side), Xn[:, s].reshape(side, side)
        po, so = lsq.psnr(ref, img), J.ssim(ref, img)
        print("slice %d: psnr %.6f (oracle %.6f)  ssim %.12f (oracle %.12f)" % (s, ps[s], po, ss[s], so))
        if np.isinf(po):
            assert np.isinf(ps[s]) and abs(ss[s] - 1.0) <= 1e-12
        else:
            assert abs(ps[s] - po) <= 1e-9 and abs(ss[s] - so) <= 1e-12
    # an explicit data range
    ps2, ss2 = image_quality(side, dr(Xr[:, :1]), dr(Xn[:, :1]), data_range=2.0)
    assert abs(ss2[0] - J.ssim(Xr[:, 0].reshape(side, side), Xn[:, 0].reshape(side, side), data_range=2.0)) <= 1e-12
