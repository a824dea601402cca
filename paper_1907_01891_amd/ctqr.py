"""ctypes binding of libctqr.so (the C ABI in include/ctqr.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name.  The library is loaded from this package directory; if it
is missing or cannot be loaded, ``lib()`` raises -- there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctqr.so")

c_i32, c_i64, c_dbl, c_sz, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p

# status codes
CTQR_OK = 0
CTQR_EINVAL = -1
CTQR_ENOMEM = -2
CTQR_EHIP = -3
CTQR_EUNSUPPORTED = -4
CTQR_RANK_DEFICIENT = 1
CTQR_NOT_CONVERGED = 2
CTQR_NONFINITE = 3
CTQR_CAPACITY = 4
CTQR_BARRIER_TIMEOUT = 5
# dtypes / precisions
CTQR_F64 = 0
CTQR_F32 = 1
CTQR_PREC_FP64 = 0
CTQR_PREC_FP32_MFMA = 1
CTQR_PREC_BF16_MFMA = 2
CTQR_PREC_BF16X3_MFMA = 3
CTQR_REFINE_CSNE = 0
CTQR_REFINE_PCG = 1


class ctqr_geometry(ctypes.Structure):
    _fields_ = [("side", c_i32), ("n_views", c_i32), ("n_bins", c_i32), ("angle_schedule", c_i32),
                ("src_iso_cm", c_dbl), ("src_det_cm", c_dbl), ("fan_deg", c_dbl), ("fov_side_cm", c_dbl)]


class ctqr_sparse(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("nnz_cap", c_i64),
                ("rowptr", c_vp), ("col", c_vp), ("val", c_vp),
                ("colptr", c_vp), ("row", c_vp), ("cval", c_vp)]


class ctqr_view_trial(ctypes.Structure):
    _fields_ = [("views", c_i32), ("status", c_i32), ("kappa", c_dbl), ("rdiag_min", c_dbl), ("rdiag_max", c_dbl)]


class ctqr_tile_task(ctypes.Structure):
    _fields_ = [("type", c_i32), ("i", c_i32), ("k", c_i32), ("j", c_i32)]


class ctqr_info(ctypes.Structure):
    _fields_ = [("status", c_i32), ("first_bad_col", c_i32), ("iters", c_i32), ("x_iters", c_i32),
                ("max_rel_update", c_dbl), ("rdiag_max", c_dbl), ("rdiag_min", c_dbl), ("nnz", c_i64),
                ("contraction", c_dbl)]


class ctqr_solver_desc(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("dtype", c_i32), ("nb", c_i32), ("QR", c_vp), ("lda", c_i64),
                ("T", c_vp), ("tau", c_vp), ("Rinv", c_vp), ("A64", ctypes.POINTER(ctqr_sparse)),
                ("tol", c_dbl), ("max_iters", c_i32), ("max_slices", c_i32), ("refine_method", c_i32),
                ("pad", c_i32)]


CTQR_PROGRESS_FACTOR = 1
CTQR_PROGRESS_SOLVE = 2
ctqr_progress_fn = ctypes.CFUNCTYPE(None, c_i32, c_i64, c_i64, c_vp)

_P = ctypes.POINTER
_SIGNATURES = {
    "ctqr_status_string": (ctypes.c_char_p, [c_i32]),
    "ctqr_version": (ctypes.c_char_p, []),
    "ctqr_last_error": (ctypes.c_char_p, []),
    "ctqr_geometry_sizes": (c_i32, [_P(ctqr_geometry), _P(c_i64), _P(c_i64), _P(c_i64)]),
    "ctqr_build_workspace": (c_i32, [_P(ctqr_geometry), _P(c_sz)]),
    "ctqr_build_system_matrix": (c_i32, [_P(ctqr_geometry), c_i32, c_vp, c_i64, _P(ctqr_sparse),
                                         c_vp, c_sz, c_vp, c_vp]),
    "ctqr_qr_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, c_i32, _P(c_sz)]),
    "ctqr_qr_factor": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, c_vp,
                               c_vp, c_sz, c_vp, c_vp]),
    "ctqr_qr_tune_nb": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp,
                                _P(c_i32), _P(ctypes.c_float), c_vp]),
    "ctqr_sparse_to_dense": (c_i32, [_P(ctqr_sparse), c_i32, c_i64, c_i64, c_vp, c_i64, c_vp]),
    "ctqr_qr_factor_ooc_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, c_i32, c_i64, c_i64, _P(c_sz)]),
    "ctqr_qr_factor_ooc": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_vp, c_i64, c_i64, c_i64, c_i32, c_i32, c_vp, c_vp,
                                   c_vp, c_vp, c_sz, c_vp, c_vp]),
    "ctqr_solve_ooc_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, c_i32, c_i32, c_i64, c_i64, _P(c_sz)]),
    "ctqr_qr_solve_ooc": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_i32,
                                  c_vp, c_i64, c_i32, c_vp, c_i64, _P(ctqr_sparse), c_dbl, c_i32, c_i32, c_vp, c_sz,
                                  c_vp, c_vp]),
    "ctqr_qr_rinv_bytes": (c_i32, [c_i64, c_i32, _P(c_sz)]),
    "ctqr_solve_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, c_i32, c_i32, _P(c_sz)]),
    "ctqr_qr_solve_slices": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_i64, c_vp, c_vp, c_vp, c_i32,
                                     c_vp, c_i64, c_i32, c_vp, c_i64, _P(ctqr_sparse), c_dbl, c_i32, c_i32,
                                     c_vp, c_sz, c_vp, c_vp]),
    "ctqr_qr_solve_slices_noalloc": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_i64, c_vp, c_vp, c_vp, c_i32,
                                             c_vp, c_i64, c_i32, c_vp, c_i64, _P(ctqr_sparse), c_dbl, c_i32,
                                             c_i32, c_vp, c_vp]),
    "ctqr_solver_workspace": (c_i32, [_P(ctqr_solver_desc), _P(c_sz)]),
    "ctqr_solver_create": (c_i32, [_P(ctqr_solver_desc), c_vp, c_sz, _P(c_vp)]),
    "ctqr_solver_tune": (c_i32, [c_vp, c_i32, c_vp]),
    "ctqr_solver_solve": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_vp, c_vp]),
    "ctqr_solver_solve_batch": (c_i32, [c_vp, c_i32, _P(c_vp), _P(c_i64), _P(c_i32), _P(c_vp), _P(c_i64),
                                        c_vp, c_vp]),
    "ctqr_solver_query": (c_i32, [c_vp, c_i32, _P(c_i32), _P(c_i32), _P(c_i32)]),
    "ctqr_solver_destroy": (c_i32, [c_vp]),
    "ctqr_cond_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, _P(c_sz)]),
    "ctqr_cond_estimate": (c_i32, [c_i64, c_i64, c_i32, c_vp, c_i64, c_vp, _P(ctqr_sparse), c_i32, c_i32, c_vp,
                                   c_sz, c_vp, c_vp]),
    "ctqr_tile_tasks": (c_i32, [c_i32, c_i32, c_i32, _P(ctqr_tile_task), c_i64, _P(c_i64)]),
    "ctqr_tile_qr_sizes": (c_i32, [c_i64, c_i64, c_i32, _P(c_i64), _P(c_sz)]),
    "ctqr_tile_qr_factor": (c_i32, [c_i64, c_i64, c_vp, c_i64, c_i32, c_vp, c_vp, c_sz, c_vp]),
    "ctqr_tile_qr_solve": (c_i32, [c_i64, c_i64, c_vp, c_i64, c_i32, c_vp, c_vp, c_i64, c_i32, c_vp, c_sz, c_vp]),
    "ctqr_project_joseph": (c_i32, [_P(ctqr_geometry), c_i32, c_vp, c_i64, c_vp, c_i64, c_vp]),
    "ctqr_image_quality": (c_i32, [c_i32, c_i32, c_vp, c_i64, c_vp, c_i64, c_dbl, c_vp, c_vp]),
    "ctqr_view_search_workspace": (c_i32, [_P(ctqr_geometry), c_i32, _P(c_sz)]),
    "ctqr_view_search": (c_i32, [_P(ctqr_geometry), c_i32, c_i32, c_i32, c_dbl, c_i32, c_vp, c_sz,
                                 _P(ctqr_view_trial), c_i32, _P(c_i32), _P(c_i32), c_vp]),
    "ctqr_spmm": (c_i32, [_P(ctqr_sparse), c_i32, c_dbl, c_vp, c_i64, c_dbl, c_vp, c_i64, c_vp]),
    "ctqr_set_progress": (c_i32, [ctqr_progress_fn, c_vp]),
    "ctqr_profile_enable": (c_i32, [c_i32]),
    "ctqr_profile_read": (c_i32, [_P(c_i64), _P(c_dbl), _P(c_dbl)]),
    "ctqr_profile_read_reduction": (c_i32, [_P(c_i64), _P(c_dbl), _P(c_dbl)]),
    "ctqr_profile_phases": (c_i32, [_P(c_dbl), _P(c_i64)]),
    "ctqr_release": (c_i32, []),
}
EXPORTS = tuple(_SIGNATURES)

_lib = None


def lib():
    """The loaded libctqr (raises OSError/RuntimeError if it is absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libctqr.so is not built (%s); run paper_1907_01891_amd.build.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class CtqrError(RuntimeError):
    def __init__(self, code, where):
        msg = "%s returned %d (%s)" % (where, code, status_string(code))
        last = lib().ctqr_last_error()
        if last:
            msg += ": " + last.decode()
        super().__init__(msg)
        self.code = code


def ctqr_release():
    """ctqr_release: the library's process-lifetime state (pinned flag words,
    timing events, progress hook) freed after the device has finished."""
    return lib().ctqr_release()


def check(code, where):
    if code != CTQR_OK:
        raise CtqrError(code, where)
    return code


def status_string(code):
    return lib().ctqr_status_string(int(code)).decode()


def ctqr_version():
    return lib().ctqr_version().decode()


def ctqr_geometry_sizes(geom):
    m, n, nnz = c_i64(), c_i64(), c_i64()
    check(lib().ctqr_geometry_sizes(ctypes.byref(geom), ctypes.byref(m), ctypes.byref(n), ctypes.byref(nnz)),
          "ctqr_geometry_sizes")
    return m.value, n.value, nnz.value


def ctqr_build_workspace(geom):
    b = c_sz()
    check(lib().ctqr_build_workspace(ctypes.byref(geom), ctypes.byref(b)), "ctqr_build_workspace")
    return b.value


def ctqr_build_system_matrix(geom, dtype, A_ptr, lda, sparse, work_ptr, work_bytes, info_ptr, stream):
    return lib().ctqr_build_system_matrix(ctypes.byref(geom), dtype, A_ptr, lda,
                                          ctypes.byref(sparse) if sparse is not None else None,
                                          work_ptr, work_bytes, info_ptr, stream)


def ctqr_qr_workspace(m, n, dtype, prec, nb):
    b = c_sz()
    check(lib().ctqr_qr_workspace(m, n, dtype, prec, nb, ctypes.byref(b)), "ctqr_qr_workspace")
    return b.value


def ctqr_qr_factor(m, n, dtype, A_ptr, lda, prec, nb, T_ptr, tau_ptr, rinv_ptr, work_ptr, work_bytes, info_ptr,
                   stream):
    return lib().ctqr_qr_factor(m, n, dtype, A_ptr, lda, prec, nb, T_ptr, tau_ptr, rinv_ptr, work_ptr, work_bytes,
                                info_ptr, stream)


def ctqr_qr_tune_nb(m, n, dtype, A_ptr, lda, prec, T_ptr, tau_ptr, work_ptr, work_bytes, info_ptr, stream):
    """(status, nb_best, [ms per column for nb = 64, 128, 256]); overwrites A."""
    nb = c_i32()
    ms = (ctypes.c_float * 3)()
    st = lib().ctqr_qr_tune_nb(m, n, dtype, A_ptr, lda, prec, T_ptr, tau_ptr, work_ptr, work_bytes, info_ptr,
                               ctypes.byref(nb), ms, stream)
    return st, nb.value, list(ms)


def ctqr_sparse_to_dense(sparse, dtype, c0, c1, A_ptr, lda, stream):
    return lib().ctqr_sparse_to_dense(ctypes.byref(sparse), dtype, c0, c1, A_ptr, lda, stream)


def ctqr_qr_factor_ooc_workspace(m, n, dtype, prec, nb, lda, tile_cols):
    b = c_sz()
    check(lib().ctqr_qr_factor_ooc_workspace(m, n, dtype, prec, nb, lda, tile_cols, ctypes.byref(b)),
          "ctqr_qr_factor_ooc_workspace")
    return b.value


def ctqr_qr_factor_ooc(m, n, dtype, A_dev, A_host, lda, n_dev, tile_cols, prec, nb, T_ptr, tau_ptr, rinv_ptr,
                       work_ptr, work_bytes, info_ptr, stream):
    return lib().ctqr_qr_factor_ooc(m, n, dtype, A_dev, A_host, lda, n_dev, tile_cols, prec, nb, T_ptr, tau_ptr,
                                    rinv_ptr, work_ptr, work_bytes, info_ptr, stream)


def ctqr_solve_ooc_workspace(m, n, dtype, nb, nslices, refine, lda, tile_cols):
    b = c_sz()
    check(lib().ctqr_solve_ooc_workspace(m, n, dtype, nb, nslices, refine, lda, tile_cols, ctypes.byref(b)),
          "ctqr_solve_ooc_workspace")
    return b.value


def ctqr_qr_solve_ooc(m, n, dtype, QR_dev, QR_host, lda, n_dev, tile_cols, T_ptr, tau_ptr, rinv_ptr, nb, B_ptr, ldb,
                      nslices, X_ptr, ldx, sparse, tol, max_iters, refine_method, work_ptr, work_bytes, info_ptr,
                      stream):
    return lib().ctqr_qr_solve_ooc(m, n, dtype, QR_dev, QR_host, lda, n_dev, tile_cols, T_ptr, tau_ptr, rinv_ptr, nb,
                                   B_ptr, ldb, nslices, X_ptr, ldx, ctypes.byref(sparse) if sparse is not None else None,
                                   tol, max_iters, refine_method, work_ptr, work_bytes, info_ptr, stream)


def ctqr_qr_rinv_bytes(n, dtype):
    b = c_sz()
    check(lib().ctqr_qr_rinv_bytes(n, dtype, ctypes.byref(b)), "ctqr_qr_rinv_bytes")
    return b.value


def ctqr_solve_workspace(m, n, dtype, nb, nslices, refine):
    b = c_sz()
    check(lib().ctqr_solve_workspace(m, n, dtype, nb, nslices, refine, ctypes.byref(b)), "ctqr_solve_workspace")
    return b.value


def ctqr_qr_solve_slices(m, n, dtype, QR_ptr, lda, T_ptr, tau_ptr, rinv_ptr, nb, B_ptr, ldb, nslices, X_ptr, ldx,
                         sparse, tol, max_iters, refine_method, work_ptr, work_bytes, info_ptr, stream):
    return lib().ctqr_qr_solve_slices(m, n, dtype, QR_ptr, lda, T_ptr, tau_ptr, rinv_ptr, nb, B_ptr, ldb, nslices,
                                      X_ptr, ldx, ctypes.byref(sparse) if sparse is not None else None,
                                      tol, max_iters, refine_method, work_ptr, work_bytes, info_ptr, stream)


def ctqr_solver_workspace(desc):
    b = c_sz()
    check(lib().ctqr_solver_workspace(ctypes.byref(desc), ctypes.byref(b)), "ctqr_solver_workspace")
    return b.value


def ctqr_solver_create(desc, work_ptr, work_bytes):
    h = c_vp()
    check(lib().ctqr_solver_create(ctypes.byref(desc), work_ptr, work_bytes, ctypes.byref(h)), "ctqr_solver_create")
    return h


def ctqr_solver_tune(solver, reps, stream):
    return lib().ctqr_solver_tune(solver, reps, stream)


def ctqr_solver_solve(solver, B_ptr, ldb, nslices, X_ptr, ldx, info_ptr, stream):
    return lib().ctqr_solver_solve(solver, B_ptr, ldb, nslices, X_ptr, ldx, info_ptr, stream)


def ctqr_solver_solve_batch(solver, B_ptrs, ldbs, nslices, X_ptrs, ldxs, info_ptr, stream):
    k = len(B_ptrs)
    return lib().ctqr_solver_solve_batch(solver, k, (c_vp * k)(*B_ptrs), (c_i64 * k)(*ldbs), (c_i32 * k)(*nslices),
                                         (c_vp * k)(*X_ptrs), (c_i64 * k)(*ldxs), info_ptr, stream)


def ctqr_solver_query(solver, nslices):
    b, t, g = c_i32(), c_i32(), c_i32()
    check(lib().ctqr_solver_query(solver, nslices, ctypes.byref(b), ctypes.byref(t), ctypes.byref(g)),
          "ctqr_solver_query")
    return b.value, t.value, g.value


def ctqr_solver_destroy(solver):
    return lib().ctqr_solver_destroy(solver)


def ctqr_cond_workspace(m, n, dtype, nvec):
    b = c_sz()
    check(lib().ctqr_cond_workspace(m, n, dtype, nvec, ctypes.byref(b)), "ctqr_cond_workspace")
    return b.value


def ctqr_cond_estimate(m, n, dtype, QR_ptr, lda, rinv_ptr, sparse, nvec, iters, work_ptr, work_bytes, out_ptr,
                       stream):
    return lib().ctqr_cond_estimate(m, n, dtype, QR_ptr, lda, rinv_ptr, ctypes.byref(sparse), nvec, iters, work_ptr,
                                    work_bytes, out_ptr, stream)


CTQR_TASK_DENSE_QR, CTQR_TASK_TD_QR, CTQR_TASK_APPLY_DENSE, CTQR_TASK_APPLY_TD, CTQR_TASK_TRSM, CTQR_TASK_GEMM = range(6)


def ctqr_tile_tasks(mt, nt, solve):
    """[(type, i, k, j)] of the factorization (solve=0) or the solve (solve=1)."""
    cnt = c_i64()
    check(lib().ctqr_tile_tasks(mt, nt, solve, None, 0, ctypes.byref(cnt)), "ctqr_tile_tasks")
    arr = (ctqr_tile_task * max(1, cnt.value))()
    check(lib().ctqr_tile_tasks(mt, nt, solve, arr, cnt.value, ctypes.byref(cnt)), "ctqr_tile_tasks")
    return [(t.type, t.i, t.k, t.j) for t in arr[:cnt.value]]


def ctqr_tile_qr_sizes(m, n, b):
    se, wb = c_i64(), c_sz()
    check(lib().ctqr_tile_qr_sizes(m, n, b, ctypes.byref(se), ctypes.byref(wb)), "ctqr_tile_qr_sizes")
    return se.value, wb.value


def ctqr_tile_qr_factor(m, n, A_ptr, lda, b, S_ptr, work_ptr, work_bytes, stream):
    return lib().ctqr_tile_qr_factor(m, n, A_ptr, lda, b, S_ptr, work_ptr, work_bytes, stream)


def ctqr_tile_qr_solve(m, n, QR_ptr, lda, b, S_ptr, B_ptr, ldb, nslices, work_ptr, work_bytes, stream):
    return lib().ctqr_tile_qr_solve(m, n, QR_ptr, lda, b, S_ptr, B_ptr, ldb, nslices, work_ptr, work_bytes, stream)


def ctqr_project_joseph(geom, nslices, X_ptr, ldx, B_ptr, ldb, stream):
    return lib().ctqr_project_joseph(ctypes.byref(geom), nslices, X_ptr, ldx, B_ptr, ldb, stream)


def ctqr_image_quality(side, nslices, Xref_ptr, ldr, X_ptr, ldx, data_range, out_ptr, stream):
    return lib().ctqr_image_quality(side, nslices, Xref_ptr, ldr, X_ptr, ldx, data_range, out_ptr, stream)


def ctqr_view_search_workspace(geom, v_max):
    b = c_sz()
    check(lib().ctqr_view_search_workspace(ctypes.byref(geom), v_max, ctypes.byref(b)), "ctqr_view_search_workspace")
    return b.value


def ctqr_view_search(geom, v_min, v_max, v_step, kappa_max, iters, work_ptr, work_bytes, stream):
    """Returns (status, v_best, [ctqr_view_trial])."""
    cap = (v_max - v_min) // v_step + 1
    trials = (ctqr_view_trial * cap)()
    nt, vb = c_i32(), c_i32()
    st = lib().ctqr_view_search(ctypes.byref(geom), v_min, v_max, v_step, kappa_max, iters, work_ptr, work_bytes,
                                trials, cap, ctypes.byref(nt), ctypes.byref(vb), stream)
    return st, vb.value, list(trials[:nt.value])


def ctqr_spmm(sparse, nslices, alpha, X_ptr, ldx, beta, Y_ptr, ldy, stream):
    return lib().ctqr_spmm(ctypes.byref(sparse), nslices, alpha, X_ptr, ldx, beta, Y_ptr, ldy, stream)


_progress_keep = None


def ctqr_set_progress(fn):
    """Install a Python hook fn(stage, done, total) (None removes it)."""
    global _progress_keep
    cb = ctqr_progress_fn(lambda st, d, t, u: fn(st, d, t)) if fn is not None else ctqr_progress_fn()
    _progress_keep = cb
    return lib().ctqr_set_progress(cb, None)


CTQR_PROFILE_UPDATE = 1
CTQR_PROFILE_PHASES = 2
PHASES = ("panel", "inner", "reduction", "update", "group_update", "rinv",
          "qtb", "trsm", "residual", "refine_trsm", "refine_other")
CTQR_NPHASES = len(PHASES)


def ctqr_profile_enable(on):
    """on: True (= CTQR_PROFILE_UPDATE), False, or a bit set of the CTQR_PROFILE_* flags."""
    return lib().ctqr_profile_enable(int(on))


def ctqr_profile_phases():
    """{phase name: (total ms, intervals)} of the phase timing."""
    ms = (c_dbl * CTQR_NPHASES)()
    cnt = (c_i64 * CTQR_NPHASES)()
    check(lib().ctqr_profile_phases(ms, cnt), "ctqr_profile_phases")
    return {PHASES[i]: (ms[i], cnt[i]) for i in range(CTQR_NPHASES)}


def ctqr_profile_read():
    n, ms, fl = c_i64(), c_dbl(), c_dbl()
    check(lib().ctqr_profile_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)), "ctqr_profile_read")
    return n.value, ms.value, fl.value


def ctqr_profile_read_reduction():
    n, ms, fl = c_i64(), c_dbl(), c_dbl()
    check(lib().ctqr_profile_read_reduction(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)),
          "ctqr_profile_read_reduction")
    return n.value, ms.value, fl.value
