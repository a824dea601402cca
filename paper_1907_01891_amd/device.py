"""Device memory for the libctqr calls, allocated through PyTorch.

PyTorch supplies HBM buffers and the current HIP stream; every computation is
a libctqr call (ctqr.py).  Matrices are column-major: an m x n matrix with
leading dimension ld is a torch tensor of shape (m, n) and strides (1, ld),
carved from a (n, ld) row-major allocation.
"""
import atexit
import ctypes
import weakref

import torch

from . import ctqr as C

_live_solvers = weakref.WeakSet()


@atexit.register
def _release_at_exit():
    """At interpreter exit, before torch's own exit handlers (registered
    earlier, so run later): destroy the solvers still alive (their graphs and
    capture streams) and release the library's process-lifetime HIP state,
    so nothing of libctqr is left for the HIP runtime's teardown."""
    if not torch.cuda.is_initialized():
        return
    for sv in list(_live_solvers):
        try:
            sv.close()
        except Exception:
            pass
    try:
        C.ctqr_release()
    except Exception:
        pass

_DT = {C.CTQR_F64: torch.float64, C.CTQR_F32: torch.float32}


def round_up(a, b):
    return (a + b - 1) // b * b


def colmajor(rows, cols, dtype, device="cuda", ld=None, fill=None):
    """(rows x cols) column-major tensor with leading dimension ld (default
    rows rounded up to 64 elements), 256-byte aligned columns."""
    ld = ld or round_up(max(rows, 1), 64)
    base = torch.empty((cols, ld), dtype=dtype, device=device)
    if fill is not None:
        base.fill_(fill)
    return base.t()[:rows, :]


def ld_of(t):
    """Leading dimension of a column-major 2-D tensor."""
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor")
    return t.stride(1) if t.shape[1] > 1 else max(t.stride(1), t.shape[0])


def to_colmajor(x, dtype=None, device="cuda", ld=None):
    x = torch.as_tensor(x)
    if x.dim() == 1:
        x = x[:, None]
    out = colmajor(x.shape[0], x.shape[1], dtype or x.dtype, device, ld=ld)
    out.copy_(x.to(device=device, dtype=dtype or x.dtype))
    return out


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def geometry(d):
    """ctqr_geometry from a dict with the keys of synthetic.Workload.geometry()."""
    return C.ctqr_geometry(int(d["side"]), int(d["n_views"]), int(d["n_bins"]), int(d.get("angle_schedule", 1)),
                           float(d["src_iso_cm"]), float(d["src_det_cm"]), float(d["fan_deg"]),
                           float(d["fov_side_cm"]))


class Info:
    """Device-side ctqr_info."""

    def __init__(self, device="cuda"):
        self.buf = torch.zeros(ctypes.sizeof(C.ctqr_info), dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())

    def read(self):
        return C.ctqr_info.from_buffer_copy(bytes(self.buf.cpu().numpy()))


class Workspace:
    """Grow-only device workspace."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            torch.cuda.empty_cache()
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return ctypes.c_void_p(self.buf.data_ptr()), self.buf.numel()


class SystemMatrix:
    """A for one geometry: dense (optional, FP64 or FP32) and the FP64 sparse
    copy (CSR + CSC, optional), built on the GPU by ctqr_build_system_matrix."""

    def __init__(self, geom_dict, dtype=C.CTQR_F64, dense=True, sparse=True, device="cuda", stream=None,
                 nnz_cap=None):
        self.geom = geometry(geom_dict)
        self.m, self.n, self.nnz_cap = C.ctqr_geometry_sizes(self.geom)
        if nnz_cap is not None:          # a smaller capacity than the geometry's upper bound
            self.nnz_cap = int(nnz_cap)
        self.dtype = dtype
        self.device = device
        self.A = colmajor(self.m, self.n, _DT[dtype], device) if dense else None
        self.sp = None
        if sparse:
            cap = self.nnz_cap
            self.rowptr = torch.empty(self.m + 1, dtype=torch.int64, device=device)
            self.col = torch.empty(cap, dtype=torch.int32, device=device)
            self.val = torch.empty(cap, dtype=torch.float64, device=device)
            self.colptr = torch.empty(self.n + 1, dtype=torch.int64, device=device)
            self.row = torch.empty(cap, dtype=torch.int32, device=device)
            self.cval = torch.empty(cap, dtype=torch.float64, device=device)
            self.sp = C.ctqr_sparse(self.m, self.n, cap, self.rowptr.data_ptr(), self.col.data_ptr(),
                                    self.val.data_ptr(), self.colptr.data_ptr(), self.row.data_ptr(),
                                    self.cval.data_ptr())
        self.info = Info(device)
        self.work = Workspace(device)
        self.build(stream)

    def build(self, stream=None):
        wp, wb = self.work.get(C.ctqr_build_workspace(self.geom))
        A_ptr = ctypes.c_void_p(self.A.data_ptr()) if self.A is not None else None
        lda = ld_of(self.A) if self.A is not None else 0
        C.check(C.ctqr_build_system_matrix(self.geom, self.dtype, A_ptr, lda, self.sp, wp, wb, self.info.ptr,
                                           stream_handle(stream)), "ctqr_build_system_matrix")

    def nnz(self):
        return int(self.info.read().nnz)

    def dense_cols(self, c0, c1, out, dtype=C.CTQR_F32, stream=None):
        """Columns [c0, c1) of the dense A into the column-major device tensor out."""
        C.check(C.ctqr_sparse_to_dense(self.sp, dtype, c0, c1, ctypes.c_void_p(out.data_ptr()), ld_of(out),
                                       stream_handle(stream)), "ctqr_sparse_to_dense")
        return out

    def spmm(self, X, alpha=1.0, beta=0.0, Y=None, stream=None):
        """Y = alpha A X + beta Y (FP64, column-major), with the sparse copy."""
        S = X.shape[1]
        if Y is None:
            Y = colmajor(self.m, S, torch.float64, self.device, fill=0.0)
        C.check(C.ctqr_spmm(self.sp, S, alpha, ctypes.c_void_p(X.data_ptr()), ld_of(X), beta,
                            ctypes.c_void_p(Y.data_ptr()), ld_of(Y), stream_handle(stream)), "ctqr_spmm")
        return Y


class QRFactor:
    """A = QR in place on a column-major dense A (ctqr_qr_factor), plus the
    stored T blocks and tau for ctqr_qr_solve_slices."""

    def __init__(self, A, prec, nb=0, device="cuda"):
        self.A = A
        self.m, self.n = A.shape
        self.dtype = C.CTQR_F64 if A.dtype == torch.float64 else C.CTQR_F32
        self.prec = prec
        self.nb = nb or 256
        self.T = colmajor(self.nb, self.n, A.dtype, device, ld=self.nb)
        self.tau = torch.zeros(self.n, dtype=torch.float64, device=device)
        rb = C.ctqr_qr_rinv_bytes(self.n, self.dtype)
        self.Rinv = torch.empty(rb // A.element_size(), dtype=A.dtype, device=device)
        self.info = Info(device)
        self.work = Workspace(device)
        self.swork = Workspace(device)
        self.sinfo = Info(device)

    def factor(self, stream=None):
        wp, wb = self.work.get(C.ctqr_qr_workspace(self.m, self.n, self.dtype, self.prec, self.nb))
        C.check(C.ctqr_qr_factor(self.m, self.n, self.dtype, ctypes.c_void_p(self.A.data_ptr()), ld_of(self.A),
                                 self.prec, self.nb, ctypes.c_void_p(self.T.data_ptr()),
                                 ctypes.c_void_p(self.tau.data_ptr()), ctypes.c_void_p(self.Rinv.data_ptr()),
                                 wp, wb, self.info.ptr, stream_handle(stream)), "ctqr_qr_factor")
        return self

    def tune_nb(self, stream=None):
        """Pick the outer block width by timing on this A (ctqr_qr_tune_nb);
        A is overwritten and must be rebuilt before factor().  Sets self.nb
        and returns (nb, ms per column for 64, 128, 256)."""
        wp, wb = self.work.get(C.ctqr_qr_workspace(self.m, self.n, self.dtype, self.prec, 256))
        Tt = colmajor(256, self.n, self.A.dtype, self.A.device, ld=256)
        st, nb, ms = C.ctqr_qr_tune_nb(self.m, self.n, self.dtype, ctypes.c_void_p(self.A.data_ptr()),
                                       ld_of(self.A), self.prec, ctypes.c_void_p(Tt.data_ptr()),
                                       ctypes.c_void_p(self.tau.data_ptr()), wp, wb, self.info.ptr,
                                       stream_handle(stream))
        C.check(st, "ctqr_qr_tune_nb")
        del Tt
        if nb != self.nb:
            self.nb = nb
            self.T = colmajor(self.nb, self.n, self.A.dtype, self.A.device, ld=self.nb)
        return nb, ms

    def solve(self, B, X=None, sparse=None, tol=1e-12, max_iters=0, method=C.CTQR_REFINE_CSNE, stream=None):
        """X = R^-1 Q^T B (FP64, column-major), refined with the sparse A if given."""
        S = B.shape[1]
        if X is None:
            X = colmajor(self.n, S, torch.float64, B.device)
        refine = (2 if method == C.CTQR_REFINE_PCG else 1) if (sparse is not None and max_iters > 0) else 0
        wp, wb = self.swork.get(C.ctqr_solve_workspace(self.m, self.n, self.dtype, self.nb, S, refine))
        C.check(C.ctqr_qr_solve_slices(self.m, self.n, self.dtype, ctypes.c_void_p(self.A.data_ptr()),
                                       ld_of(self.A), ctypes.c_void_p(self.T.data_ptr()),
                                       ctypes.c_void_p(self.tau.data_ptr()),
                                       ctypes.c_void_p(self.Rinv.data_ptr()), self.nb,
                                       ctypes.c_void_p(B.data_ptr()), ld_of(B), S,
                                       ctypes.c_void_p(X.data_ptr()), ld_of(X), sparse, tol, max_iters, method,
                                       wp, wb, self.sinfo.ptr, stream_handle(stream)),
                "ctqr_qr_solve_slices")
        return X


    def cond_estimate(self, sparse, nvec=8, iters=30, stream=None):
        """(sigma_max(A), sigma_min(R), kappa) by ctqr_cond_estimate: power and
        inverse iteration, lower bounds of the true values."""
        ws = Workspace(self.A.device)
        wp, wb = ws.get(C.ctqr_cond_workspace(self.m, self.n, self.dtype, nvec))
        out = torch.zeros(3, dtype=torch.float64, device=self.A.device)
        C.check(C.ctqr_cond_estimate(self.m, self.n, self.dtype, ctypes.c_void_p(self.A.data_ptr()), ld_of(self.A),
                                     ctypes.c_void_p(self.Rinv.data_ptr()), sparse, nvec, iters, wp, wb,
                                     ctypes.c_void_p(out.data_ptr()), stream_handle(stream)), "ctqr_cond_estimate")
        return tuple(float(v) for v in out.cpu().tolist())


class OocFactor:
    """Out-of-core factor (ctqr_qr_factor_ooc): columns [0, n_dev) of A in
    device memory, the rest in pinned host memory, streamed in tiles."""

    def __init__(self, m, n, dtype, prec, n_dev, tile_cols, nb=0, device="cuda"):
        tdt = _DT[dtype]
        self.m, self.n, self.dtype, self.prec = m, n, dtype, prec
        self.nb = nb or 256
        self.lda = round_up(m, 64)
        self.n_dev, self.tile_cols = n_dev, tile_cols
        self.A_dev = colmajor(m, n_dev, tdt, device, ld=self.lda) if n_dev > 0 else None
        # host part: pinned (hipHostMalloc) rows of lda elements, one per column
        self.host_base = torch.empty((n - n_dev, self.lda), dtype=tdt, pin_memory=True) if n_dev < n else None
        self.A_host = self.host_base.t()[:m, :] if n_dev < n else None
        self.T = colmajor(self.nb, n, tdt, device, ld=self.nb)
        self.tau = torch.zeros(n, dtype=torch.float64, device=device)
        self.Rinv = torch.empty(C.ctqr_qr_rinv_bytes(n, dtype) // self.T.element_size(), dtype=tdt, device=device)
        self.info = Info(device)
        self.work = Workspace(device)

    def load(self, A):
        """Copy a column-major (m x n) matrix (host or device tensor) into the two parts."""
        if self.A_dev is not None:
            self.A_dev.copy_(A[:, :self.n_dev])
        if self.A_host is not None:
            self.A_host.copy_(A[:, self.n_dev:])

    def factor(self, stream=None):
        wp, wb = self.work.get(C.ctqr_qr_factor_ooc_workspace(self.m, self.n, self.dtype, self.prec, self.nb,
                                                              self.lda, self.tile_cols))
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        C.check(C.ctqr_qr_factor_ooc(self.m, self.n, self.dtype, ptr(self.A_dev), ptr(self.A_host), self.lda,
                                     self.n_dev, self.tile_cols, self.prec, self.nb, ptr(self.T), ptr(self.tau),
                                     ptr(self.Rinv), wp, wb, self.info.ptr, stream_handle(stream)),
                "ctqr_qr_factor_ooc")
        return self

    def solve(self, B, X=None, sparse=None, tol=1e-12, max_iters=0, method=C.CTQR_REFINE_CSNE, stream=None):
        """X = R^-1 Q^T B with the out-of-core factor (ctqr_qr_solve_ooc)."""
        S = B.shape[1]
        if X is None:
            X = colmajor(self.n, S, torch.float64, B.device)
        refine = (2 if method == C.CTQR_REFINE_PCG else 1) if (sparse is not None and max_iters > 0) else 0
        if not hasattr(self, "swork"):
            self.swork, self.sinfo = Workspace(self.T.device), Info(self.T.device)
        wp, wb = self.swork.get(C.ctqr_solve_ooc_workspace(self.m, self.n, self.dtype, self.nb, S, refine, self.lda,
                                                           self.tile_cols))
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        C.check(C.ctqr_qr_solve_ooc(self.m, self.n, self.dtype, ptr(self.A_dev), ptr(self.A_host), self.lda,
                                    self.n_dev, self.tile_cols, ptr(self.T), ptr(self.tau), ptr(self.Rinv), self.nb,
                                    ptr(B), ld_of(B), S, ptr(X), ld_of(X), sparse, tol, max_iters, method, wp, wb,
                                    self.sinfo.ptr, stream_handle(stream)), "ctqr_qr_solve_ooc")
        return X

    def factor_matrix(self):
        """The whole factored matrix as one host tensor (m x n, column-major)."""
        out = torch.empty((self.n, self.lda), dtype=self.T.dtype).t()[:self.m, :]
        if self.A_dev is not None:
            out[:, :self.n_dev].copy_(self.A_dev.cpu())
        if self.A_host is not None:
            out[:, self.n_dev:].copy_(self.A_host)
        return out


class Solver:
    """Batched solver over a stored factor (ctqr_solver_*): requests of 1 ..
    max_slices slices, one HIP graph per slice bucket (powers of two up to 64, multiples of 64 above)."""

    def __init__(self, qr, max_slices, sparse=None, tol=1e-12, max_iters=0, method=C.CTQR_REFINE_CSNE,
                 device="cuda"):
        self.qr = qr
        self.sparse = sparse    # ctqr_sparse (kept alive: the solver copies the struct only)
        self.desc = C.ctqr_solver_desc(qr.m, qr.n, qr.dtype, qr.nb, qr.A.data_ptr(), ld_of(qr.A), qr.T.data_ptr(),
                                       qr.tau.data_ptr(), qr.Rinv.data_ptr(),
                                       ctypes.pointer(sparse) if sparse is not None else None,
                                       float(tol), int(max_iters) if sparse is not None else 0, int(max_slices),
                                       int(method), 0)
        nbytes = C.ctqr_solver_workspace(self.desc)
        self.work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.h = C.ctqr_solver_create(self.desc, ctypes.c_void_p(self.work.data_ptr()), self.work.numel())
        self.info = Info(device)
        self.device = device
        _live_solvers.add(self)

    def tune(self, reps=2, stream=None):
        C.check(C.ctqr_solver_tune(self.h, reps, stream_handle(stream)), "ctqr_solver_tune")

    def solve(self, B, X=None, stream=None):
        S = B.shape[1]
        if X is None:
            X = colmajor(self.qr.n, S, torch.float64, self.device)
        C.check(C.ctqr_solver_solve(self.h, ctypes.c_void_p(B.data_ptr()), ld_of(B), S,
                                    ctypes.c_void_p(X.data_ptr()), ld_of(X), self.info.ptr, stream_handle(stream)),
                "ctqr_solver_solve")
        return X

    def solve_batch(self, Bs, Xs=None, stream=None):
        """Queued requests packed into one bucket (sum of slices <= max_slices)."""
        if Xs is None:
            Xs = [colmajor(self.qr.n, b.shape[1], torch.float64, self.device) for b in Bs]
        C.check(C.ctqr_solver_solve_batch(self.h, [b.data_ptr() for b in Bs], [ld_of(b) for b in Bs],
                                          [b.shape[1] for b in Bs], [x.data_ptr() for x in Xs],
                                          [ld_of(x) for x in Xs], self.info.ptr, stream_handle(stream)),
                "ctqr_solver_solve_batch")
        return Xs

    def query(self, nslices):
        """(bucket, slice_tile, graph_iters) for a request of nslices."""
        return C.ctqr_solver_query(self.h, nslices)

    def close(self):
        if self.h is not None:
            C.ctqr_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def view_search(geom_dict, v_min, v_max, v_step=1, kappa_max=1e8, iters=30, stream=None):
    """ctqr_view_search for a geometry dict (its n_views is replaced by each
    candidate): (v_best or 0, [ctqr_view_trial]).  The workspace is allocated
    here for the largest candidate."""
    g = geometry(dict(geom_dict, n_views=v_max))
    ws = Workspace()
    wp, wb = ws.get(C.ctqr_view_search_workspace(g, v_max))
    st, vb, trials = C.ctqr_view_search(g, v_min, v_max, v_step, kappa_max, iters, wp, wb, stream_handle(stream))
    C.check(st, "ctqr_view_search")
    return vb, trials


def project_joseph(geom_dict, X, B=None, stream=None):
    """B = J X (ctqr_project_joseph): Joseph-projector sinograms of the images
    in the columns of the column-major FP64 device tensor X."""
    g = geometry(geom_dict)
    m = g.n_views * g.n_bins
    if B is None:
        B = colmajor(m, X.shape[1], torch.float64, X.device)
    C.check(C.ctqr_project_joseph(g, X.shape[1], ctypes.c_void_p(X.data_ptr()), ld_of(X),
                                  ctypes.c_void_p(B.data_ptr()), ld_of(B), stream_handle(stream)),
            "ctqr_project_joseph")
    return B


def image_quality(side, Xref, X, data_range=0.0, stream=None):
    """(PSNR per slice, SSIM per slice) as host lists (ctqr_image_quality)."""
    S = X.shape[1]
    out = torch.empty(2 * S, dtype=torch.float64, device=X.device)
    C.check(C.ctqr_image_quality(side, S, ctypes.c_void_p(Xref.data_ptr()), ld_of(Xref),
                                 ctypes.c_void_p(X.data_ptr()), ld_of(X), float(data_range),
                                 ctypes.c_void_p(out.data_ptr()), stream_handle(stream)), "ctqr_image_quality")
    o = out.cpu().tolist()
    return o[:S], o[S:]


class TileQR:
    """Algorithm-by-blocks QR (ctqr_tile_qr_factor) of a column-major FP64
    device matrix, in place, with block size b, and its solve."""

    def __init__(self, A, b):
        self.A, self.b = A, b
        self.m, self.n = A.shape
        se, wb = C.ctqr_tile_qr_sizes(self.m, self.n, b)
        self.S = torch.zeros(max(se, 1), dtype=torch.float64, device=A.device)
        self.work = torch.empty(wb, dtype=torch.uint8, device=A.device)

    def factor(self, stream=None):
        C.check(C.ctqr_tile_qr_factor(self.m, self.n, ctypes.c_void_p(self.A.data_ptr()), ld_of(self.A), self.b,
                                      ctypes.c_void_p(self.S.data_ptr()), ctypes.c_void_p(self.work.data_ptr()),
                                      self.work.numel(), stream_handle(stream)), "ctqr_tile_qr_factor")
        return self

    def solve(self, B, stream=None):
        """X = R^-1 Q^T B (B is copied; returns the n x S solution)."""
        Bw = colmajor(self.m, B.shape[1], torch.float64, B.device)
        Bw.copy_(B)
        C.check(C.ctqr_tile_qr_solve(self.m, self.n, ctypes.c_void_p(self.A.data_ptr()), ld_of(self.A), self.b,
                                     ctypes.c_void_p(self.S.data_ptr()), ctypes.c_void_p(Bw.data_ptr()), ld_of(Bw),
                                     B.shape[1], ctypes.c_void_p(self.work.data_ptr()), self.work.numel(),
                                     stream_handle(stream)), "ctqr_tile_qr_solve")
        return Bw[:self.n]

