"""GPU tests of the batched solver (ctqr_solver_*): graph-replayed solves of
padded slice buckets against the direct solve and the CPU oracle.

Pins: a request padded into its bucket gives the direct solve's result (the
extra slices are zero; bitwise when both use the same slice tile, since
every product then has the same tiling and the same split of the reduction);
the oracle's solution to the 1e-10 bar of the mixed path; replays of a
captured bucket are bitwise identical to its first run, with other GPU work
and host synchronisations between them.
"""
import numpy as np
import pytest
import torch

from oracle import householder as hh
from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import QRFactor, Solver, to_colmajor

from gpu_helpers import oracle_problem, oracle_factor, DeviceSparse, upload_dense, download

pytestmark = pytest.mark.gpu

NAME = "ct40"          # m = 3744, n = 1600: 13 block columns at nb = 128, ragged edges
N_SLICES = 130


def _print_case(*a):
    print("[case]", *a, flush=True)


def _problem():
    g, A, X, B = oracle_problem(NAME, n_slices=N_SLICES)
    QRo, tauo = oracle_factor(NAME)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    return A, B, Xo


def _factor(A, dtype, prec, nb=128):
    Ad = A.toarray()
    if dtype == torch.float32:
        Ad = Ad.astype(np.float32)
    F = QRFactor(upload_dense(Ad, dtype), prec, nb=nb)
    F.factor()
    torch.cuda.synchronize()
    assert F.info.read().status == 0
    return F


def _other_gpu_work():
    # unrelated eager work and a synchronisation between graph replays
    a = torch.randn(512, 512, device="cuda", dtype=torch.float32)
    (a @ a).sum().item()
    torch.cuda.synchronize()


def test_solver_fp64_matches_direct_and_oracle(gpu):
    A, B, Xo = _problem()
    F = _factor(A, torch.float64, C.CTQR_PREC_FP64)
    sv = Solver(F, max_slices=130)             # buckets 1 .. 64, 128, 192
    for S in (1, 3, 5, 8, 17, 32, 40, 70, 130):
        _print_case("solver fp64", NAME, "S", S)
        Bd = to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)
        Xd = download(F.solve(Bd))
        Xs = download(sv.solve(Bd))
        torch.cuda.synchronize()
        assert sv.info.read().status == 0
        bucket, tile, giters = sv.query(S)
        if S <= 64:
            assert bucket >= S and bucket & (bucket - 1) == 0 and bucket < 2 * S
        else:
            assert bucket % 64 == 0 and S <= bucket < S + 64
        assert giters == 0                      # captured, no refinement
        if S <= 32:
            assert tile == 32
            assert (Xs == Xd).all(), S          # same tiles: padding changes nothing
        else:
            assert lsq.rel_err(Xs, Xd).max() <= 1e-12
        assert lsq.rel_err(Xs, Xo[:, :S]).max() <= 1e-10
    sv.close()


def test_solver_replays_bitwise(gpu):
    A, B, Xo = _problem()
    F = _factor(A, torch.float64, C.CTQR_PREC_FP64)
    sv = Solver(F, max_slices=16)
    Bd = to_colmajor(torch.as_tensor(B[:, :6]), dtype=torch.float64)
    ref = None
    for rep in range(4):
        _print_case("solver replay", rep)
        X = download(sv.solve(Bd))
        torch.cuda.synchronize()
        if ref is None:
            ref = X
        assert (X == ref).all(), rep
        _other_gpu_work()
    # a different request in between leaves the bucket's results unchanged
    sv.solve(to_colmajor(torch.as_tensor(B[:, 10:15]), dtype=torch.float64))
    assert (download(sv.solve(Bd)) == ref).all()
    sv.close()


@pytest.mark.parametrize("method", [C.CTQR_REFINE_CSNE, C.CTQR_REFINE_PCG])
def test_solver_mixed_refined(gpu, method):
    A, B, Xo = _problem()
    F = _factor(A, torch.float32, C.CTQR_PREC_FP32_MFMA)
    spA = DeviceSparse(A)
    sv = Solver(F, max_slices=64, sparse=spA.sp, tol=1e-12, max_iters=30, method=method)
    for S in (5, 40):
        Bd = to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)
        outs = []
        for rep in range(3):
            _print_case("solver mixed", NAME, "method", method, "S", S, "rep", rep)
            outs.append(download(sv.solve(Bd)))
            torch.cuda.synchronize()
            info = sv.info.read()
            assert info.status == 0, (C.status_string(info.status), info.iters)
            bucket, tile, giters = sv.query(S)
            if rep == 0:
                assert giters == -1             # calibration run: eager
                calib = info.iters
            else:
                assert giters == min(30, calib + 2)
                assert info.iters == calib      # the graph stops where the eager run stopped
            _other_gpu_work()
        assert (outs[1] == outs[0]).all() and (outs[2] == outs[0]).all()
        err = lsq.rel_err(outs[0], Xo[:, :S])
        print("S %d iters %d err %.3e" % (S, calib, err.max()))
        assert err.max() <= 1e-10
        # the direct refined solve converges to the same least-squares solution
        Xd = download(F.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=30, method=method))
        assert lsq.rel_err(outs[0], Xd).max() <= 1e-10
    sv.close()


def test_solver_tune(gpu):
    A, B, Xo = _problem()
    F = _factor(A, torch.float64, C.CTQR_PREC_FP64)
    sv = Solver(F, max_slices=N_SLICES)
    _print_case("solver tune")
    sv.tune(reps=1)
    torch.cuda.synchronize()
    for S in (2, 33, 40):
        bucket, tile, _ = sv.query(S)
        assert tile in (32, 128)
        Bd = to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)
        Xs = download(sv.solve(Bd))
        assert lsq.rel_err(Xs, download(F.solve(Bd))).max() <= 1e-12
        assert lsq.rel_err(Xs, Xo[:, :S]).max() <= 1e-10
    sv.close()


def test_narrow_and_wide_tiles_agree(gpu):
    # 40 slices: the direct solve uses the 128-wide tile; a solver bucket of
    # 64 forced onto the 32-wide tile by tuning or not, both meet the oracle
    A, B, Xo = _problem()
    F = _factor(A, torch.float32, C.CTQR_PREC_FP32_MFMA)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    Xw = download(F.solve(Bd))
    Xn = np.concatenate([download(F.solve(to_colmajor(torch.as_tensor(B[:, i:i + 8]), dtype=torch.float64)))
                         for i in range(0, N_SLICES, 8)], axis=1)
    # unrefined FP32 solves: both are FP32-accurate solutions of the same
    # problem, equal to each other far below the FP32 error level
    e = lsq.rel_err(Xn, Xw).max()
    e_or = lsq.rel_err(Xw, Xo).max()
    print("narrow vs wide %.3e, wide vs oracle %.3e" % (e, e_or))
    assert e <= 1e-5 and e_or < 1e-2


def test_solver_calls_on_two_streams(gpu):
    # calls from two streams, enqueued back to back without host waits, share
    # the solver's request buffer and workspace: each call's stream waits for
    # the previous call's work, so every result equals the direct solve
    A, B, Xo = _problem()
    F = _factor(A, torch.float64, C.CTQR_PREC_FP64)
    sv = Solver(F, max_slices=64)
    reqs = [(0, 6), (6, 40), (46, 3), (49, 64), (0, 6)]
    Bs = [to_colmajor(torch.as_tensor(B[:, a:a + k]), dtype=torch.float64) for a, k in reqs]
    ref = [download(F.solve(b)) for b in Bs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    _print_case("solver two streams")
    outs = [sv.solve(b, stream=streams[i % 2]) for i, b in enumerate(Bs)]
    torch.cuda.synchronize()
    for i, (x, r) in enumerate(zip(outs, ref)):
        assert lsq.rel_err(download(x), r).max() <= 1e-12, i
    sv.close()


def test_solver_batch_of_requests(gpu):
    # three queued requests packed into one bucket give each request's own
    # solution (and, refined, the oracle's)
    A, B, Xo = _problem()
    F = _factor(A, torch.float32, C.CTQR_PREC_FP32_MFMA)
    spA = DeviceSparse(A)
    sv = Solver(F, max_slices=64, sparse=spA.sp, tol=1e-12, max_iters=30)
    cuts = [(0, 3), (3, 10), (10, 27)]
    Bs = [to_colmajor(torch.as_tensor(B[:, a:b]), dtype=torch.float64) for a, b in cuts]
    for rep in range(2):
        _print_case("solver batch", rep)
        Xs = [download(x) for x in sv.solve_batch(Bs)]
        torch.cuda.synchronize()
        assert sv.info.read().status == 0
        for (a, b), Xg in zip(cuts, Xs):
            assert Xg.shape == (A.shape[1], b - a)
            assert lsq.rel_err(Xg, Xo[:, a:b]).max() <= 1e-10
        if rep == 0:
            first = Xs
        else:
            assert all((x == y).all() for x, y in zip(Xs, first))
    sv.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_block_substitution_orders(gpu, dtype):
    # n = 2304: two diagonal blocks of the block substitution (2048 + a ragged
    # 256).  Few slices take the left-looking order, 40 slices the
    # right-looking one; both must reach the oracle's solution.
    name = "ct48"
    g, A, X, B = oracle_problem(name, n_slices=40)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    if dtype == "f64":
        F = _factor(A, torch.float64, C.CTQR_PREC_FP64, nb=256)
        kw = {}
    else:
        F = _factor(A, torch.float32, C.CTQR_PREC_FP32_MFMA, nb=256)
        spA = DeviceSparse(A)
        kw = dict(sparse=spA.sp, tol=1e-12, max_iters=30)
    for S in (4, 40):
        _print_case("two-block trsm", dtype, "S", S)
        Bd = to_colmajor(torch.as_tensor(B[:, :S]), dtype=torch.float64)
        Xg = download(F.solve(Bd, **kw))
        torch.cuda.synchronize()
        si = F.sinfo.read()
        assert si.status == 0, (C.status_string(si.status), si.iters)
        err = lsq.rel_err(Xg, Xo[:, :S]).max()
        print("%s S %d err %.3e iters %d" % (dtype, S, err, si.iters))
        assert err <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("method", [C.CTQR_REFINE_CSNE, C.CTQR_REFINE_PCG])
def test_wide_refinement_with_split_substitutions(gpu, prec, method):
    # 130 slices (>= 128) of an n = 2304 problem (two diagonal blocks): the
    # corrected semi-normal-equations refinement's right-looking
    # substitutions take split-BF16 off-diagonal products (the
    # conjugate-gradient form keeps FP32 ones), directly and through the
    # batched solver (bucket 192); the refined solution meets the oracle
    name = "ct48"
    g, A, X, B = oracle_problem(name, n_slices=130)
    QRo, tauo = oracle_factor(name)
    Xo = hh.backsub(QRo, hh.apply_qt(QRo, tauo, B))
    code = {"fp32": C.CTQR_PREC_FP32_MFMA, "bf16x3": C.CTQR_PREC_BF16X3_MFMA}[prec]
    F = _factor(A, torch.float32, code, nb=128)
    spA = DeviceSparse(A)
    Bd = to_colmajor(torch.as_tensor(B), dtype=torch.float64)
    _print_case("wide refinement", name, prec, "method", method)
    Xg = download(F.solve(Bd, sparse=spA.sp, tol=1e-12, max_iters=40, method=method))
    torch.cuda.synchronize()
    si = F.sinfo.read()
    err = lsq.rel_err(Xg, Xo).max()
    print("direct: status %d iters %d err %.2e" % (si.status, si.iters, err))
    assert si.status == 0 and err <= 1e-10
    sv = Solver(F, max_slices=130, sparse=spA.sp, tol=1e-12, max_iters=40, method=method)
    for rep in range(2):
        _print_case("wide refinement solver", prec, method, rep)
        Xs = download(sv.solve(Bd))
        torch.cuda.synchronize()
        info = sv.info.read()
        assert info.status == 0, (C.status_string(info.status), info.iters)
        assert lsq.rel_err(Xs, Xo).max() <= 1e-10
    assert sv.query(130)[0] == 192
    sv.close()
