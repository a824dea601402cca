"""Oracle: the algorithm-by-blocks QR factorization and solve (Section II-C).

Test infrastructure only: the product never imports this package.

The matrix is cut into b x b blocks A_ij (the last block row and column may be
smaller).  Four task types factor it and apply the factorization:

  dense_qr(k)          Compute_dense_QR(A_kk, S_kk): Householder QR of A_kk;
                       R on and above its diagonal, the reflectors below, S_kk
                       their compact-WY factor (H_1 ... H_c = I - V S V^T).
  td_qr(i, k)          Compute_TD_QR(A_kk, A_ik, S_ik): QR of the triangle
                       R_kk stacked on the dense A_ik; each reflector is
                       [e_p; v_p] (a unit vector in the triangle, v_p in A_ik),
                       v_p replaces column p of A_ik, R_kk is updated, S_ik is
                       the compact-WY factor of U = [I; V].
  apply_dense(k, C)    Apply_left_Qt_of_dense_QR(A_kk, S_kk, C):
                       C <- (I - V S V^T)^T C.
  apply_td(i, k, F, G) Apply_left_Qt_of_TD_QR(A_ik, S_ik, F, G):
                       [F; G] <- (I - U S U^T)^T [F; G], U = [I; A_ik].

The factorization runs them in the left-looking order of the paper's task
table: for each block column j, first the transformations of every earlier
block column k (apply_dense(k, A_kj), then apply_td(i, k, A_kj, A_ij) for each
block row i > k), then dense_qr(j) and td_qr(i, j) for i > j.  The solve
X = R^-1 (Q^T B) applies the same transformations to the block rows of B
(apply_dense(k, B_k), apply_td(i, k, B_k, B_i) for each k, then i > k), then
substitutes by block rows from the last: B_i -= A_ij X_j for j > i in
increasing j (Gemm_nn_mo), X_i = R_ii^-1 B_i (Trsm_lunn).

Every Householder vector follows the larfg convention of householder.py
(beta = -sign(alpha) ||[alpha; x]||, sign(0) = +1, tau = (beta - alpha) / beta,
v = x / (alpha - beta); tau = 0 when x = 0), and each compact-WY factor is
built by the larft recurrence S_pp = tau_p,
S_{0:p, p} = -tau_p S_{0:p, 0:p} (U_{:, 0:p}^T u_p).
"""
import math
import numpy as np

DENSE_QR, TD_QR, APPLY_DENSE, APPLY_TD = 0, 1, 2, 3
TRSM, GEMM = 4, 5


def qr_tasks(mt, nt):
    """The factorization's tasks in the paper's order: tuples (type, i, k, j)
    (apply tasks: block row i (or k), reflector block column k, target block
    column j; factor tasks: j = k)."""
    out = []
    for j in range(nt):
        for k in range(min(j, mt)):
            out.append((APPLY_DENSE, k, k, j))
            for i in range(k + 1, mt):
                out.append((APPLY_TD, i, k, j))
        if j < mt:
            out.append((DENSE_QR, j, j, j))
            for i in range(j + 1, mt):
                out.append((TD_QR, i, j, j))
    return out


def solve_tasks(mt, nt):
    """The solve's tasks in the paper's order: (type, i, k, j) with apply tasks
    on block rows of B (j = -1), then TRSM (i = k = j) and GEMM (B_i -= A_ij X_j)."""
    out = []
    for k in range(min(mt, nt)):
        out.append((APPLY_DENSE, k, k, -1))
        for i in range(k + 1, mt):
            out.append((APPLY_TD, i, k, -1))
    for i in range(nt - 1, -1, -1):
        for j in range(i + 1, nt):
            out.append((GEMM, i, i, j))
        out.append((TRSM, i, i, i))
    return out


def _larfg(alpha, x):
    s = float(x @ x)
    if s == 0.0:
        return alpha, 0.0, np.zeros_like(x)
    beta = -math.copysign(math.sqrt(alpha * alpha + s), alpha if alpha != 0.0 else 1.0)
    return beta, (beta - alpha) / beta, x / (alpha - beta)


def _larft(tau, U):
    """S with H_1 ... H_c = I - U S U^T (U's columns the full reflector vectors)."""
    c = len(tau)
    G = U.T @ U
    S = np.zeros((c, c))
    for p in range(c):
        S[p, p] = tau[p]
        if p:
            S[:p, p] = -tau[p] * (S[:p, :p] @ G[:p, p])
    return S


def dense_qr(T):
    """Householder QR of the tile T (r x c, r >= c or not) in place; returns S."""
    r, c = T.shape
    tau = np.zeros(min(r, c))
    for p in range(min(r, c)):
        beta, tau[p], v = _larfg(T[p, p], T[p + 1:, p].copy())
        T[p + 1:, p] = v
        T[p, p] = beta
        u = np.concatenate([[1.0], v])
        w = u @ T[p:, p + 1:]
        T[p:, p + 1:] -= tau[p] * np.outer(u, w)
    U = np.tril(T[:, :len(tau)], -1)
    U[np.arange(len(tau)), np.arange(len(tau))] = 1.0
    return _larft(tau, U)


def td_qr(Rt, D):
    """QR of [upper triangle of Rt (c x c); D (r x c)] in place: Rt's upper
    triangle becomes the new R (its strict lower part is not touched), D the
    reflectors' dense parts; returns S."""
    c = Rt.shape[1]
    tau = np.zeros(c)
    for p in range(c):
        beta, tau[p], v = _larfg(Rt[p, p], D[:, p].copy())
        D[:, p] = v
        Rt[p, p] = beta
        if p + 1 < c:
            w = Rt[p, p + 1:] + v @ D[:, p + 1:]
            Rt[p, p + 1:] -= tau[p] * w
            D[:, p + 1:] -= tau[p] * np.outer(v, w)
    U = np.vstack([np.eye(c), D])
    return _larft(tau, U)


def apply_dense(Vt, S, C):
    """C <- (I - V S V^T)^T C, V the unit lower trapezoid of Vt (its c = S's size columns)."""
    c = S.shape[0]
    V = np.tril(Vt[:, :c], -1)
    V[np.arange(c), np.arange(c)] = 1.0
    C -= V @ (S.T @ (V.T @ C))


def apply_td(D, S, F, G):
    """[F; G] <- (I - U S U^T)^T [F; G] with U = [I; D] (F's first c rows)."""
    c = S.shape[0]
    W = F[:c] + D.T @ G
    W = S.T @ W
    F[:c] -= W
    G -= D @ W


def tile_bounds(m, b):
    return [(i0, min(m, i0 + b)) for i0 in range(0, m, b)]


def tile_qr(A, b):
    """Algorithm-by-blocks QR of A (m x n, m >= n): returns (F, S) with F the
    factored A (R in the upper triangle of the diagonal and above-diagonal
    blocks, the reflectors below) and S[(i, k)] the compact-WY factors."""
    F = np.array(A, dtype=np.float64, order="F")
    m, n = F.shape
    rb, cb = tile_bounds(m, b), tile_bounds(n, b)
    blk = lambda i, j: F[rb[i][0]:rb[i][1], cb[j][0]:cb[j][1]]
    S = {}
    for typ, i, k, j in qr_tasks(len(rb), len(cb)):
        if typ == DENSE_QR:
            S[(k, k)] = dense_qr(blk(k, k))
        elif typ == TD_QR:
            S[(i, k)] = td_qr(blk(k, k), blk(i, k))
        elif typ == APPLY_DENSE:
            apply_dense(blk(k, k), S[(k, k)], blk(k, j))
        else:
            apply_td(blk(i, k), S[(i, k)], blk(k, j), blk(i, j))
    return F, S


def tile_solve(F, S, b, B):
    """X = R^-1 (Q^T B) with the output of tile_qr (B: m x s)."""
    m, n = F.shape
    rb, cb = tile_bounds(m, b), tile_bounds(n, b)
    Bw = np.array(B, dtype=np.float64).reshape(m, -1).copy()
    row = lambda i: Bw[rb[i][0]:rb[i][1]]
    blk = lambda i, j: F[rb[i][0]:rb[i][1], cb[j][0]:cb[j][1]]
    for typ, i, k, j in solve_tasks(len(rb), len(cb)):
        if typ == APPLY_DENSE:
            apply_dense(blk(k, k), S[(k, k)], row(k))
        elif typ == APPLY_TD:
            apply_td(blk(i, k), S[(i, k)], row(k), row(i))
        elif typ == GEMM:
            c_i = cb[i][1] - cb[i][0]
            row(i)[:c_i] -= blk(i, j)[:c_i] @ row(j)[:cb[j][1] - cb[j][0]]
        else:
            c = cb[i][1] - cb[i][0]
            Rii = np.triu(blk(i, i)[:c, :c])
            xi = row(i)[:c]
            for p in range(c - 1, -1, -1):      # back substitution in the block
                xi[p] = (xi[p] - Rii[p, p + 1:] @ xi[p + 1:]) / Rii[p, p]
    return Bw[:n]
