"""Oracle: ctypes front end of the unblocked FP64 Householder QR in qr_oracle.c.

Test infrastructure only.  ``build()`` compiles qr_oracle.c with gcc into
oracle/libqr_oracle.so (OpenMP, -ffp-contract=off so the arithmetic is the
plain one written in the C source).

Functions follow Eq. 3 (A = QR) and Eq. 4 (X = R^-1 Q^T B) of the paper; see
qr_oracle.c for the reflector convention.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qr_oracle.c")
_LIB = os.path.join(_HERE, "libqr_oracle.so")
_lib = None


def build(force=True):
    """Compile the C oracle (always, when force=True)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.oracle_geqr2.argtypes = [i64, i64, dp, i64, dp]
        lib.oracle_apply_qt.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_apply_q.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_backsub.argtypes = [i64, dp, i64, i64, dp, i64]
        for f in (lib.oracle_geqr2, lib.oracle_apply_qt, lib.oracle_apply_q, lib.oracle_backsub):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran64(a):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return np.array(a, dtype=np.float64, order="F", copy=True)


def geqr2(A):
    """Unblocked Householder QR (Eq. 3).  Returns (QR, tau): QR holds R in its
    upper triangle and the reflector tails v_k(1:) below the diagonal."""
    QR = _fortran64(A)
    m, n = QR.shape
    if m < n:
        raise ValueError("need m >= n")
    tau = np.zeros(n)
    _load().oracle_geqr2(m, n, _ptr(QR), m, _ptr(tau))
    return QR, tau


def apply_qt(QR, tau, B):
    """Q^T B, applying the stored reflectors one at a time (Eq. 4, first step)."""
    QR = np.asfortranarray(QR, dtype=np.float64)
    m, n = QR.shape
    C = _fortran64(B)
    if C.shape[0] != m:
        raise ValueError("B must have m rows")
    _load().oracle_apply_qt(m, n, _ptr(QR), m, _ptr(tau), C.shape[1], _ptr(C), m)
    return C


def apply_q(QR, tau, B):
    """Q B (used to rebuild A = QR in tests)."""
    QR = np.asfortranarray(QR, dtype=np.float64)
    m, n = QR.shape
    C = _fortran64(B)
    _load().oracle_apply_q(m, n, _ptr(QR), m, _ptr(tau), C.shape[1], _ptr(C), m)
    return C


def backsub(R, C):
    """X = R^-1 C by backward substitution (Eq. 4, second step); R is the
    upper triangle of the leading n x n block of its argument."""
    R = np.asfortranarray(R, dtype=np.float64)
    n = R.shape[1]
    X = _fortran64(np.asarray(C)[:n])
    _load().oracle_backsub(n, _ptr(R), R.shape[0], X.shape[1], _ptr(X), n)
    return X


def r_factor(QR):
    """The upper-triangular R (n x n) held in a factored matrix."""
    n = QR.shape[1]
    return np.triu(QR[:n, :n])


def householder_vectors(QR):
    """V (m x n), unit lower trapezoidal, from a factored matrix."""
    m, n = QR.shape
    V = np.tril(QR, -1)[:, :n]
    V[np.arange(n), np.arange(n)] = 1.0
    return V
