"""Pins of the algorithm-by-blocks oracle (Section II-C), CPU only.

  * The task lists for m = n = 3b equal the paper's two task tables
    (tests/golden/tasks_*_ab_3x3.txt, transcribed with their operands): the
    operands each generated task writes and reads are derived here from the
    task's type and indices, so the order, the types and the blocks are all
    checked.
  * The factor's R equals the unblocked Householder R of the same matrix up to
    the signs of its rows (R is unique up to them for full column rank), on
    square and ragged block grids; the product of the tasks' reflectors
    reproduces A (backward error).
  * The solve equals the least-squares solution of the unblocked oracle and
    LAPACK's lstsq.
"""
import os

import numpy as np
import pytest

from oracle import householder as hh
from oracle import tiles as T
from oracle import lsq
from oracle.siddon import system_matrix_csr
from synthetic import get_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NAMES = {T.DENSE_QR: "Comp_dense_QR", T.TD_QR: "Comp_TD_QR", T.APPLY_DENSE: "Apply_left_Qt_of_dense_QR",
         T.APPLY_TD: "Apply_left_Qt_of_TD_QR", T.TRSM: "Trsm_lunn", T.GEMM: "Gemm_nn_mo"}


def _read(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        lhs, rhs = line.split("|")
        op, *outs = lhs.split()
        rows.append((op, outs, rhs.split()))
    return rows


def _operands_qr(t):
    typ, i, k, j = t
    A = lambda r, c: "A%d%d" % (r, c)
    Sf = lambda r, c: "S%d%d" % (r, c)
    if typ == T.DENSE_QR:
        return [A(k, k), Sf(k, k)], [A(k, k)]
    if typ == T.TD_QR:
        return [A(k, k), A(i, k), Sf(i, k)], [A(k, k), A(i, k)]
    if typ == T.APPLY_DENSE:
        return [A(k, j)], [A(k, k), Sf(k, k), A(k, j)]
    return [A(k, j), A(i, j)], [A(i, k), Sf(i, k), A(k, j), A(i, j)]


def _operands_solve(t):
    typ, i, k, j = t
    A = lambda r, c: "A%d%d" % (r, c)
    Bb = lambda r: "B%d0" % r
    if typ == T.APPLY_DENSE:
        return [Bb(k)], [A(k, k), "S%d%d" % (k, k), Bb(k)]
    if typ == T.APPLY_TD:
        return [Bb(k), Bb(i)], [A(i, k), "S%d%d" % (i, k), Bb(k), Bb(i)]
    if typ == T.GEMM:
        return [Bb(i)], [Bb(i), A(i, j), Bb(j)]
    return [Bb(i)], [A(i, i), Bb(i)]


def test_qr_task_table():
    got = [(NAMES[t[0]], *_operands_qr(t)) for t in T.qr_tasks(3, 3)]
    assert got == [(op, o, i) for op, o, i in _read("tasks_qr_ab_3x3.txt")]
    assert len(got) == 14


def test_solve_task_table():
    got = [(NAMES[t[0]], *_operands_solve(t)) for t in T.solve_tasks(3, 3)]
    assert got == [(op, o, i) for op, o, i in _read("tasks_solve_ab_3x3.txt")]
    assert len(got) == 12


@pytest.mark.parametrize("m,n,b", [(96, 96, 32), (100, 70, 32), (130, 33, 16), (64, 64, 64), (200, 150, 48)])
def test_tile_qr_matches_householder(m, n, b, oracle_lib):
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((m, n))
    F, S = T.tile_qr(A, b)
    QR, tau = hh.geqr2(A)
    Rt, Ro = np.triu(F[:n, :n]), np.triu(QR[:n, :n])
    sn = lambda R: np.sign(np.diag(R))[:, None] * R
    assert np.abs(sn(Rt) - sn(Ro)).max() <= 1e-12 * np.abs(Ro).max()
    # Q^T A = [R; 0] with the tasks' own reflectors (apply every transformation to A)
    QtA = np.array(A)
    rb, cb = T.tile_bounds(m, b), T.tile_bounds(n, b)
    row = lambda i: QtA[rb[i][0]:rb[i][1]]
    blk = lambda i, j: F[rb[i][0]:rb[i][1], cb[j][0]:cb[j][1]]
    for typ, i, k, j in T.solve_tasks(len(rb), len(cb)):
        if typ == T.APPLY_DENSE:
            T.apply_dense(blk(k, k), S[(k, k)], row(k))
        elif typ == T.APPLY_TD:
            T.apply_td(blk(i, k), S[(i, k)], row(k), row(i))
    assert np.abs(QtA[:n] - Rt).max() <= 1e-12 * np.abs(A).max() * np.sqrt(m)
    if m > n:
        assert np.abs(QtA[n:]).max() <= 1e-12 * np.abs(A).max() * np.sqrt(m)


@pytest.mark.parametrize("name,b", [("ct24", 64), ("ct24", 100), ("ct32", 128)])
def test_tile_solve_matches_reconstruction(name, b, oracle_lib):
    g = get_workload(name).geometry()
    A = system_matrix_csr(g)
    X, B = lsq.sinograms(A, g["side"], 2)
    Ad = A.toarray()
    F, S = T.tile_qr(Ad, b)
    Xt = T.tile_solve(F, S, b, B)
    Xo = lsq.reconstruct(Ad, B)[0]
    Xl = np.linalg.lstsq(Ad, B, rcond=None)[0]
    assert lsq.rel_err(Xt, Xo).max() <= 1e-12
    assert lsq.rel_err(Xt, Xl).max() <= 1e-12
