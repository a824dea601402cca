"""Full-size parity at the benchmark's workload (256x256 image, m = 88,320,
n = 65,536, nb = 256, 256 slices) and launch configuration.

The dense oracle QR of this A would take hours, so the HIP path is compared
with what the oracle computes at this size (section references are to the
paper):
  * A itself (Section II-A, Eq. 1): the GPU CSR/CSC against the oracle's
    Siddon matrix, elementwise;
  * the first 64 columns of the factor: Householder QR is column-by-column,
    so R[0:64, 0:64], V[:, 0:64] and tau[0:64] depend only on A[:, 0:64],
    which the oracle factors exactly (Eq. 3);
  * R^T R = A^T A (Eq. 3) on sampled column pairs across the whole matrix,
    with a_i^T a_j from the oracle's sparse A;
  * exact recovery: consistent (noise-free) sinograms must reconstruct the
    phantom (Eq. 4), for the FP64 path and the refined FP32 path;
  * least-squares optimality ||A^T (b - A x)|| / (||A||_F ||b - A x||) of the
    noisy reconstructions, evaluated with the oracle's sparse A.

Tolerances: FP64 factor entries 1e-11 relative to max|R| (kappa ~ 1e5 at this
size bounds the forward difference of two stable QRs by ~kappa*u); FP32
factor 1e-4; R^T R vs A^T A: 2 sqrt(m) u_storage ||a_i|| ||a_j||; reconstructions
1e-10 relative (the mixed path's bar).  Optimality: a solution that is the
exact least-squares solution of (A + dA, b) with ||dA|| <= c u ||A|| has
||A^T r|| / (||A|| ||r||) <= c u (||A|| ||x|| / ||r|| + 1); the test allows
c = 100 with u = 2^-53 and the measured ||A||_F, ||x||, ||r||.
"""
import numpy as np
import pytest
import torch

from synthetic import get_workload, phantom_batch, noise_batch, NOISE_REL_LEVEL
from oracle.siddon import system_matrix_csr
from oracle import householder as hh
from oracle import lsq
from paper_1907_01891_amd import ctqr as C
from paper_1907_01891_amd.device import SystemMatrix, QRFactor, colmajor, to_colmajor

pytestmark = pytest.mark.gpu

NAME = "ct256"
NB = 256
N_SLICES = 8


def _case(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def oracle_A():
    _case("oracle Siddon ct256")
    return system_matrix_csr(get_workload(NAME).geometry())


@pytest.fixture(scope="module")
def gpu_sparse(gpu):
    g = get_workload(NAME).geometry()
    sp = SystemMatrix(g, C.CTQR_F64, dense=False, sparse=True)
    torch.cuda.synchronize()
    return sp


@pytest.fixture(scope="module")
def rhs(oracle_A):
    w = get_workload(NAME)
    X = phantom_batch(w.side, N_SLICES)
    B0 = np.asfortranarray(oracle_A @ X)
    Z = noise_batch(w.side, w.m, N_SLICES)
    B = np.asfortranarray(B0 + Z * (NOISE_REL_LEVEL * np.abs(B0).max(axis=0))[None, :])
    return X, B0, B


def _factor(gpu_sparse, dtype, prec):
    w = get_workload(NAME)
    A = colmajor(w.m, w.n, dtype)
    import ctypes
    from paper_1907_01891_amd.device import ld_of, stream_handle, Workspace
    ws = Workspace()
    wp, wb = ws.get(C.ctqr_build_workspace(gpu_sparse.geom))
    C.check(C.ctqr_build_system_matrix(gpu_sparse.geom, C.CTQR_F64 if dtype == torch.float64 else C.CTQR_F32,
                                       ctypes.c_void_p(A.data_ptr()), ld_of(A), None, wp, wb,
                                       gpu_sparse.info.ptr, stream_handle()), "build")
    F = QRFactor(A, prec, nb=NB).factor()
    torch.cuda.synchronize()
    return F


@pytest.fixture(scope="module")
def factor32(gpu_sparse):
    _case("factor fp32 ct256")
    return _factor(gpu_sparse, torch.float32, C.CTQR_PREC_FP32_MFMA)


def test_system_matrix_fullsize(gpu_sparse, oracle_A):
    _case("A ct256")
    A = oracle_A
    sp = gpu_sparse
    assert sp.info.read().status == 0
    assert sp.nnz() == A.nnz
    import scipy.sparse as sps
    rowptr = sp.rowptr.cpu().numpy()
    assert (rowptr == A.indptr).all()
    G = sps.csr_matrix((sp.val[:A.nnz].cpu().numpy(), sp.col[:A.nnz].cpu().numpy(), rowptr), shape=A.shape)
    G.sort_indices()
    assert (G.indices == A.indices).all()
    assert np.abs(G.data - A.data).max() <= 1e-12
    Ac = A.tocsc()
    Ac.sort_indices()
    assert (sp.colptr.cpu().numpy() == Ac.indptr).all()
    assert (sp.row[:A.nnz].cpu().numpy() == Ac.indices).all()
    assert np.abs(sp.cval[:A.nnz].cpu().numpy() - Ac.data).max() <= 1e-12


def _check_leading_columns(F, A, tol):
    k = 64
    QRo, tauo = hh.geqr2(A.tocsc()[:, :k].toarray())
    QRg = F.A[:, :k].double().cpu().numpy()
    scale = np.abs(QRo).max()
    assert np.abs(F.tau[:k].cpu().numpy() - tauo).max() <= tol
    assert np.abs(QRg - QRo).max() <= tol * scale


def _check_gram(F, A, u):
    # Householder QR's backward error on a column grows like sqrt(m) u in
    # practice (the worst-case bound is O(m n u)); allow 2 sqrt(m) u.
    worst = _gram_worst(F, A)
    assert worst <= 2.0 * np.sqrt(A.shape[0]) * u, worst


def _gram_worst(F, A):
    """max |r_a^T r_b - a_a^T a_b| / (||a_a|| ||a_b||) over sampled column pairs."""
    Acsc = A.tocsc()
    rng = np.random.default_rng(11)
    n = A.shape[1]
    cols = np.unique(np.concatenate([rng.integers(0, n, 40), [0, 1, 255, 256, 257, n - 2, n - 1]]))
    R = {}
    for j in cols:
        colj = F.A[:, int(j)].double().cpu().numpy()
        R[j] = colj[:j + 1]                       # R[0:j+1, j]
    norms = {j: np.sqrt(Acsc[:, j].multiply(Acsc[:, j]).sum()) for j in cols}
    worst = 0.0
    for a in cols:
        for b in cols:
            if b < a:
                continue
            rr = R[a] @ R[b][:a + 1]
            aa = (Acsc[:, a].T @ Acsc[:, b]).toarray()[0, 0]
            worst = max(worst, abs(rr - aa) / (norms[a] * norms[b]))
    return worst


def _check_optimality(A, X, B):
    nA = np.sqrt(A.multiply(A).sum())
    r = B - A @ X
    bound = 100 * 2.0 ** -53 * (nA * np.linalg.norm(X, axis=0) / np.linalg.norm(r, axis=0) + 1.0)
    opt = lsq.ls_optimality(A, X, B)
    assert (opt <= bound).all(), (opt, bound)


def test_fp32_factor_leading_columns(factor32, oracle_A):
    _case("fp32 leading columns")
    assert factor32.info.read().status == 0
    _check_leading_columns(factor32, oracle_A, 1e-4)


def test_fp32_factor_gram(factor32, oracle_A):
    _case("fp32 gram")
    _check_gram(factor32, oracle_A, 6e-8)


def test_fp32_refined_solutions(factor32, gpu_sparse, oracle_A, rhs):
    _case("fp32 refined solve")
    X, B0, B = rhs
    Xc = factor32.solve(to_colmajor(torch.as_tensor(B0), dtype=torch.float64), sparse=gpu_sparse.sp,
                        tol=1e-12, max_iters=30).cpu().numpy()
    si = factor32.sinfo.read()
    assert si.status == 0, (si.status, si.iters, si.max_rel_update)
    assert lsq.rel_err(Xc, X).max() <= 1e-10
    Xn = factor32.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64), sparse=gpu_sparse.sp,
                        tol=1e-12, max_iters=30).cpu().numpy()
    assert factor32.sinfo.read().status == 0
    _check_optimality(oracle_A, Xn, B)


@pytest.fixture(scope="module")
def factorx3(gpu_sparse):
    _case("factor split-bf16 ct256")
    return _factor(gpu_sparse, torch.float32, C.CTQR_PREC_BF16X3_MFMA)


# Split-BF16 products: each FP32 operand as a bf16 high part plus a bf16 low
# part (about 16 significant bits), the low-low product dropped, so one product
# term is exact to about 3 * 2^-16 relative.  A column's backward error then
# grows with the number of block-reflector applications it receives (64 group
# updates at nb = 256 with groups of four), each contributing two products
# ([G | W] and C -= V W'): |r_a^T r_b - a_a^T a_b| <= 2 * 2 sqrt(64) u_split
# ||a_a|| ||a_b||.
U_SPLIT = 3.0 * 2.0 ** -16


def test_bf16x3_factor_leading_columns(factorx3, oracle_A):
    # the leading 64 columns sit inside the first block column: panel (FP64
    # arithmetic, FP32 storage) and FP32 inner updates only
    _case("split-bf16 leading columns")
    assert factorx3.info.read().status == 0
    _check_leading_columns(factorx3, oracle_A, 1e-4)


def test_bf16x3_factor_gram(factorx3, oracle_A):
    _case("split-bf16 gram")
    worst = _gram_worst(factorx3, oracle_A)
    bound = 2.0 * 2.0 * np.sqrt(get_workload(NAME).n / (4 * NB)) * U_SPLIT
    print("split-bf16 R^T R vs A^T A: %.2e (bound %.2e)" % (worst, bound))
    assert worst <= bound


def test_bf16x3_refined_solutions(factorx3, gpu_sparse, oracle_A, rhs):
    _case("split-bf16 refined solve")
    X, B0, B = rhs
    Xc = factorx3.solve(to_colmajor(torch.as_tensor(B0), dtype=torch.float64), sparse=gpu_sparse.sp,
                        tol=1e-12, max_iters=30).cpu().numpy()
    si = factorx3.sinfo.read()
    assert si.status == 0, (si.status, si.iters, si.max_rel_update)
    assert lsq.rel_err(Xc, X).max() <= 1e-10
    Xn = factorx3.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64), sparse=gpu_sparse.sp,
                        tol=1e-12, max_iters=30).cpu().numpy()
    assert factorx3.sinfo.read().status == 0
    _check_optimality(oracle_A, Xn, B)


def test_fp64_factor_and_solve(gpu_sparse, oracle_A, rhs):
    _case("fp64 factor ct256")
    F = _factor(gpu_sparse, torch.float64, C.CTQR_PREC_FP64)
    assert F.info.read().status == 0
    _check_leading_columns(F, oracle_A, 1e-11)
    _check_gram(F, oracle_A, 1.1e-16)
    X, B0, B = rhs
    Xc = F.solve(to_colmajor(torch.as_tensor(B0), dtype=torch.float64)).cpu().numpy()
    assert lsq.rel_err(Xc, X).max() <= 1e-10
    Xn = F.solve(to_colmajor(torch.as_tensor(B), dtype=torch.float64)).cpu().numpy()
    _check_optimality(oracle_A, Xn, B)
    del F
    torch.cuda.empty_cache()
