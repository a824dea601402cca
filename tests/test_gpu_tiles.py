"""GPU algorithm-by-blocks QR and solve (ctqr_tile_qr_factor/_solve) against
the oracle's task-by-task execution (oracle.tiles, Section II-C).

Both run the same tasks with the same arithmetic per task (the GPU groups
independent tasks into dependency levels; each block still sees its tasks in
the table's order), so the factored blocks, the S factors and the solutions
agree element by element up to summation order: 1e-12 relative for the
factor and S (FP64; the matrices here are well conditioned), 1e-10 for the
solutions against the unblocked oracle's least-squares solution (the mixed
path's bar, Eq. 4).  Sizes cover square and ragged block grids, b from 16 to
64, and more right-hand sides than one solve workgroup takes (64).
"""
import numpy as np
import pytest
import torch

from oracle import tiles as T
from oracle import lsq
from paper_1907_01891_amd.device import TileQR, to_colmajor

from gpu_helpers import oracle_problem, download

pytestmark = pytest.mark.gpu


def _s_blocks(Sg, m, n, b):
    mt, nt = -(-m // b), -(-n // b)
    out = {}
    for k in range(nt):
        c = min(b, n - k * b)
        for i in range(k, mt):
            blk = Sg[(k * mt + i) * b * b:(k * mt + i + 1) * b * b].reshape(b, b).T   # column-major
            out[(i, k)] = blk[:c, :c]
    return out


@pytest.mark.parametrize("m,n,b", [(96, 96, 32), (100, 70, 32), (130, 33, 16), (200, 150, 48), (64, 64, 64),
                                   (300, 200, 64), (40, 40, 64)])
def test_tile_qr_matches_oracle(gpu, m, n, b):
    print("[case] tile qr", m, n, b, flush=True)
    rng = np.random.default_rng(m * 31 + n + b)
    A = rng.standard_normal((m, n))
    Fo, So = T.tile_qr(A, b)
    G = TileQR(to_colmajor(torch.as_tensor(A), dtype=torch.float64), b).factor()
    torch.cuda.synchronize()
    Fg = download(G.A)
    scale = np.abs(Fo).max()
    assert np.abs(Fg - Fo).max() <= 1e-12 * scale, np.abs(Fg - Fo).max()
    Sg = _s_blocks(download(G.S), m, n, b)
    for key, So_k in So.items():
        assert np.abs(Sg[key] - So_k).max() <= 1e-12 * max(1.0, np.abs(So_k).max()), key


@pytest.mark.parametrize("name,b,nsl", [("ct24", 64, 3), ("ct32", 64, 70), ("ct40", 48, 5)])
def test_tile_solve_matches_oracle(gpu, name, b, nsl):
    print("[case] tile solve", name, b, nsl, flush=True)
    g, A, X, B = oracle_problem(name, n_slices=nsl)
    Ad = A.toarray()
    Xo = lsq.reconstruct(Ad, B)[0]
    G = TileQR(to_colmajor(torch.as_tensor(Ad), dtype=torch.float64), b).factor()
    Xg = download(G.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)))
    torch.cuda.synchronize()
    err = lsq.rel_err(Xg, Xo)
    print("tile solve %s b=%d: max rel err %.2e" % (name, b, err.max()))
    assert err.max() <= 1e-10
    # the oracle's task-by-task solve agrees more tightly
    Fo, So = T.tile_qr(Ad, b)
    Xt = T.tile_solve(Fo, So, b, B)
    assert lsq.rel_err(Xg, Xt).max() <= 1e-11
