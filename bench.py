"""Benchmark of the QR least-squares CT reconstruction hot path on one MI355X.

Workload (default ct256): 256x256 image (n = 65,536 pixels), fan-beam scanner
of Table I with 120 views x 736 bins (m = 88,320 rays), A stored in FP32 for
the factorization, 256 seeded ellipse-phantom sinograms with 1e-3 relative
Gaussian noise.  One step is the whole hot path on resident inputs:
  1. build the dense FP32 system matrix A on the GPU (Siddon),
  2. blocked Householder QR (A = QR, Eq. 3) whose block-column products run
     on split-BF16 MFMA (each FP32 operand as a high and a low bf16 part,
     three products, FP32 accumulation; --prec fp32 for FP32 MFMA), panel
     norms and reflectors in FP64,
  3. X = R^-1 Q^T B for all 256 slices (Eq. 4), refined by corrected
     semi-normal equations with FP64 residuals against the FP64 sparse A.
value = QR TFLOP/s of step 2 ((2 m n^2 - 2 n^3 / 3) / t_QR); slices/s of
step 3 are reported beside it, as are the same two figures for the plain FP64
GPU path (FP64 A, FP64 MFMA, no refinement) and for the other FP32-storage
product modes (FP32 MFMA, one-part BF16), each timed once after the K steps.

The "roofline" object covers the dominant kernel (the trailing-update product
C -= V W'), timed per launch with HIP events on the stream it runs on.  The
"cpu_baseline" leg times the CPU oracle (unblocked FP64 Householder QR) on a
bounded column sample of the same A.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0}
REFINE = {"csne": 0, "pcg": 1}
CHECK_CHUNK = 256          # slices per chunk of the out-of-core optimality check


def prec_codes(C):
    """Product mode name -> ctqr_prec of an FP32-storage factorization."""
    return {"bf16x3": C.CTQR_PREC_BF16X3_MFMA, "fp32": C.CTQR_PREC_FP32_MFMA, "bf16": C.CTQR_PREC_BF16_MFMA}
HBM_PEAK_GBS = 8000.0


def qr_flops(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def solve_flops(m, n):
    return 4.0 * m * n - 2.0 * n * n + n * n


def solve_phase_model(m, n, S, nnz, iters, store_bytes, split_refine, mfma_tflops=PEAK_TFLOPS["f32"]):
    """Per-phase algorithmic work of one refined solve of S slices: flops and
    HBM bytes, and the floor time max(flops / peak, bytes / HBM) of each phase.
      qtb          Q^T B: 4 m n S - 2 n^2 S flops; reads V (the factor below
                   the diagonal, m n - n^2 / 2 elements) and T, B in FP64,
                   the working copy written and read back.
      trsm         R X = C: n^2 S flops; reads R (n^2 / 2 elements) and the
                   stored diagonal-block inverses (2 x 2048 n elements).
      residual     per iteration r = B - A x, s = A^T r: 4 nnz S flops; the CSR
                   and CSC values and indices (12 B per nonzero each) and the
                   FP64 vectors.
      refine_trsm  per iteration R^T y = s, R d = y: 2 n^2 S flops; R read twice.
    MFMA phases are priced at the MFMA peak of the factor's precision
    (mfma_tflops), or at a third of the BF16 peak for the refinement's
    split-BF16 products (three BF16 products each); the sparse products at the
    HBM rate only (FP64 gathers, no MFMA)."""
    b = store_bytes
    bw = HBM_PEAK_GBS * 1e9
    f32 = mfma_tflops * 1e12
    ph = {}
    fl = S * (4.0 * m * n - 2.0 * n * n)
    by = (m * n - n * n / 2.0) * b + 256.0 * n * b + 8.0 * m * S + 2 * 4.0 * m * S
    ph["qtb"] = (fl, by, max(fl / f32, by / bw))
    fl = S * float(n) * n
    by = (n * n / 2.0 + 2 * 2048.0 * n) * b + 2 * 4.0 * n * S
    ph["trsm"] = (fl, by, max(fl / f32, by / bw))
    fl = iters * 4.0 * nnz * S
    by = iters * (24.0 * nnz + 8.0 * S * (3 * m + 2 * n))
    ph["residual"] = (fl, by, by / bw)
    fl = iters * 2.0 * n * n * S
    by = iters * (2 * (n * n / 2.0 + 2 * 2048.0 * n) * b + 4 * 4.0 * n * S)
    peak = PEAK_TFLOPS["bf16"] * 1e12 / 3.0 if split_refine else f32
    ph["refine_trsm"] = (fl, by, max(fl / peak, by / bw))
    return ph


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="ct256")
    p.add_argument("--nb", type=int, default=0,
                   help="outer block width; 0 = picked by ctqr_qr_tune_nb on the benchmark's own A (untimed)")
    p.add_argument("--max-iters", type=int, default=30)
    p.add_argument("--tol", type=float, default=1e-10,
                   help="refinement tolerance on the relative update, the accuracy bar itself (the error that "
                        "remains after the last update is about the contraction rate times it)")
    p.add_argument("--prec", choices=["bf16x3", "fp32"], default="bf16x3",
                   help="block-column products of the mixed path: split-BF16 MFMA or FP32 MFMA")
    p.add_argument("--refine", choices=["csne", "pcg"], default="csne",
                   help="refinement form: corrected semi-normal equations or their conjugate-gradient form")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison run")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-stream", action="store_true", help="skip the batched request-stream leg")
    p.add_argument("--no-bf16", action="store_true", help="skip the BF16-MFMA factorization leg")
    p.add_argument("--ooc", action="store_true",
                   help="out-of-core factorization (default for workloads whose dense FP32 A exceeds HBM)")
    p.add_argument("--ooc-tile", type=int, default=8192, help="columns per streamed host tile")
    p.add_argument("--ooc-dev-cols", type=int, default=0,
                   help="cap on the HBM-resident columns (0: as many as fit)")
    p.add_argument("--ooc-slices", default="",
                   help="out of core: comma-separated slice counts, each solved in one pass after one "
                        "factorization (default: the workload's count)")
    p.add_argument("--save-check", default="",
                   help="out of core: directory for .npz files of a few solutions and their sinograms, for the "
                        "host-side least-squares check against the oracle's sparse A")
    p.add_argument("--no-phases", action="store_true",
                   help="skip the untimed phase breakdown, condition estimate and solve roofline (profiled runs)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run 3 device-to-device copies of 1 GiB (counter calibration) and exit")
    return p.parse_args()


# committed HBM-counter summaries of the trailing-update kernel, per product mode
TRAFFIC_FILES = {"bf16x3": os.path.join(ROOT, "profiles", "gemm_nn_bf16x3_trailing_update_ct256_traffic.txt")}
# the trailing-update kernel of each mode, as rocprofv3 names it
TRAILING_KERNEL = {"fp32": "gemm_nn_kernel<float, 1, 128, false, 0>",
                   "bf16x3": "gemm_nn_bf16x3_w8_kernel"}


def trailing_launches(m, n, nb):
    """(rows, columns, inner dimension) of every trailing-update launch of the
    factorization.  With nb dividing 512, groups of four block columns share
    one update: each block's reflector updates only the rest of its group, and
    the group's block reflector (up to 4 nb wide) updates the remaining columns
    in one launch."""
    out, k0 = [], 0
    g = 4 if 512 % nb == 0 else 1
    while k0 < n:
        w = min(g * nb, n - k0)
        if n - k0 - w > 0:
            out.append((m - k0, n - k0 - w, w))
        k0 += w
    return out


def gemm_source_hash(src=None):
    """Hash of the code of gemm.hip (comments and blank lines removed) without the host-side
    split-count rule of the TN products (gemm_tn_splits), which the
    trailing-update kernels and their launchers do not use: the key of the
    committed HBM-counter summaries.  src: the file's text (read if None)."""
    import hashlib
    import re
    if src is None:
        with open(os.path.join(ROOT, "paper_1907_01891_amd", "csrc", "gemm.hip")) as f:
            src = f.read()
    src = re.sub(r"\nint gemm_tn_splits\(int M, int N, int K\)\n\{.*?\n\}\n", "\n", src, count=1, flags=re.S)
    src = re.sub(r"[ \t]*//[^\n]*", "", src)
    src = "\n".join(l.strip() for l in src.splitlines() if l.strip())   # comment-only edits keep the key
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic(workload, prec, launches):
    """HBM bytes per launch of the trailing-update kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE scaled by a copy kernel), or None
    if there is none for this workload and launch count (the factorization's
    schedule) or the kernel source changed since."""
    try:
        kv = dict(l.strip().split("=", 1) for l in open(TRAFFIC_FILES[prec])
                  if "=" in l and not l.lstrip().startswith("#"))
    except (OSError, KeyError):
        return None
    if kv.get("workload") != workload or kv.get("gemm_hip_sha256") != gemm_source_hash():
        return None
    if kv.get("launches") != str(launches):
        return None
    return float(kv["bytes_per_launch"])


def calibrate_copy():
    """Three 1 GiB device-to-device copies (a plain copy kernel of known size)."""
    import torch
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": x.numel() * 4, "calibrate_copy_bytes_written": y.numel() * 4,
                      "copies": 3}))


def cpu_baseline(workload, target_s):
    """Oracle QR (unblocked FP64 Householder, OpenMP) on A[:, :k] of the same
    geometry, k chosen for about target_s seconds; TFLOP/s by the flop count of
    that k-column factorization."""
    import numpy as np
    from synthetic import get_workload
    from oracle.siddon import system_matrix_csr
    from oracle import householder as hh
    g = get_workload(workload).geometry()
    A = system_matrix_csr(g).tocsc()
    m = A.shape[0]
    hh.build(force=False)
    k = 128
    t0 = time.perf_counter()
    hh.geqr2(A[:, :k].toarray())
    t = time.perf_counter() - t0
    rate = qr_flops(m, k) / max(t, 1e-6)
    # flops grow ~ k^2: pick k for the target time
    k = int(min(A.shape[1], max(k, (target_s * rate / (2.0 * m)) ** 0.5)))
    k = max(128, k // 32 * 32)
    Ad = A[:, :k].toarray()
    t0 = time.perf_counter()
    QR, tau = hh.geqr2(Ad)
    t = time.perf_counter() - t0
    # the oracle's solve of the sample (Q^T B and back substitution) for a few
    # slices, and LAPACK's blocked dgeqrf on the same columns as the tuned
    # CPU library reference
    import numpy as np
    import scipy.linalg as sl
    S = 16
    Bs = np.asfortranarray(np.random.default_rng(0).standard_normal((m, S)))
    t1 = time.perf_counter()
    hh.backsub(QR, hh.apply_qt(QR, tau, Bs))
    ts = time.perf_counter() - t1
    t2 = time.perf_counter()
    sl.lapack.dgeqrf(np.asfortranarray(Ad))
    tl = time.perf_counter() - t2
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": qr_flops(m, k) / t / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "unblocked FP64 Householder QR of A[:, :%d] (%d x %d) of the %s geometry, %.1f s"
                      % (k, m, k, workload, t),
            "solve": {"value": S / ts, "unit": "slices/s (of the %d-column sample)" % k,
                      "tflops": S * solve_flops(m, k) / ts / 1e12, "slices": S, "seconds": ts},
            "lapack_dgeqrf": {"value": qr_flops(m, k) / tl / 1e12, "unit": "TFLOP/s", "seconds": tl,
                              "note": "SciPy LAPACK dgeqrf (blocked, multithreaded BLAS) on the same sample"}}


def request_stream_bench(args, log, F256, sp256, B256):
    """Batched serving of 200 solve requests (slice counts log-uniform in
    [1, 512], geometry uniform over 128^2 and 256^2) on two resident factors:
    128^2 FP64 (plain FP64 path) and 256^2 FP32 (mixed path, CSNE-refined).
    Right-hand sides are drawn cyclically from each geometry's slice pool.
    Closed loop (one request in flight): per-request latency, host clock
    around the call and a stream synchronisation.  All queued: requests of
    one geometry packed in arrival order into solves of at most 512 slices."""
    import numpy as np
    import torch
    from synthetic import get_workload, phantom_batch, noise_batch, NOISE_REL_LEVEL, request_stream
    from paper_1907_01891_amd import ctqr as C
    from paper_1907_01891_amd.device import SystemMatrix, QRFactor, Solver, colmajor, to_colmajor
    dev = B256.device
    w128 = get_workload("ct128")
    s128 = SystemMatrix(w128.geometry(), C.CTQR_F64, dense=True, sparse=True)
    X128 = to_colmajor(torch.as_tensor(phantom_batch(w128.side, w128.n_slices)), dtype=torch.float64)
    B128 = s128.spmm(X128)
    torch.cuda.synchronize()
    B128.add_(torch.as_tensor(noise_batch(w128.side, w128.m, w128.n_slices), device=dev)
              * (NOISE_REL_LEVEL * B128.abs().amax(dim=0))[None, :])
    F128 = QRFactor(s128.A, C.CTQR_PREC_FP64, nb=256).factor()
    torch.cuda.synchronize()
    assert F128.info.read().status == 0
    solvers = {"ct128": Solver(F128, 512),
               "ct256": Solver(F256, 512, sparse=sp256.sp, tol=args.tol, max_iters=args.max_iters)}
    pools = {"ct128": B128, "ct256": B256}
    t0 = time.perf_counter()
    for sv in solvers.values():
        sv.tune(reps=1)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    reqs = request_stream()
    cursor = {"ct128": 0, "ct256": 0}

    def cyclic(pool, c0, k):
        cols = torch.tensor([(c0 + j) % pool.shape[1] for j in range(k)], device=dev)
        b = colmajor(pool.shape[0], k, torch.float64, dev)
        b.copy_(pool.index_select(1, cols))
        return b
    Bs = []
    for g, k in reqs:
        Bs.append(cyclic(pools[g], cursor[g], k))
        cursor[g] = (cursor[g] + k) % pools[g].shape[1]
    Xs = [colmajor(solvers[g].qr.n, k, torch.float64, dev) for g, k in reqs]
    # warm-up: every bucket of both solvers calibrated and captured
    buckets = {g: sorted({sv.query(k)[0] for k in range(1, 513)}) for g, sv in solvers.items()}
    t0 = time.perf_counter()
    for g, sv in solvers.items():
        for b in buckets[g]:
            Bw = cyclic(pools[g], 0, b)
            for _ in range(2):
                sv.solve(Bw)
            del Bw
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    log("stream: tuned in %.1f s, buckets captured in %.1f s" % (t_tune, t_warm))

    lat = []
    status = 0
    tc0 = time.perf_counter()
    for (g, k), b, x in zip(reqs, Bs, Xs):
        t0 = time.perf_counter()
        solvers[g].solve(b, X=x)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        status = max(status, solvers[g].info.read().status)
    t_closed = time.perf_counter() - tc0
    total = sum(k for _, k in reqs)
    lat_ms = np.array(lat) * 1e3

    tq0 = time.perf_counter()
    for g in solvers:
        batch, nsl = [], 0
        idx = [i for i, (gg, _) in enumerate(reqs) if gg == g]
        for i in idx + [None]:
            k = reqs[i][1] if i is not None else 0
            if batch and (i is None or nsl + k > 512):
                solvers[g].solve_batch([Bs[j] for j in batch], [Xs[j] for j in batch])
                batch, nsl = [], 0
            if i is not None:
                batch.append(i)
                nsl += k
    torch.cuda.synchronize()
    t_queued = time.perf_counter() - tq0
    per = {}
    nnz256 = sp256.nnz()
    for g in solvers:
        l = np.array([lat_ms[i] for i, (gg, _) in enumerate(reqs) if gg == g])
        per[g] = {"requests": int(l.size), "slices": int(sum(k for gg, k in reqs if gg == g)),
                  "p50_ms": float(np.percentile(l, 50)), "p99_ms": float(np.percentile(l, 99)),
                  "slice_tiles": {str(b): solvers[g].query(b)[1] for b in buckets[g]},
                  "graph_refine_iters": {str(b): solvers[g].query(b)[2] for b in buckets[g]}}
        # closed-loop latency of each bucket against the floor of its work
        # (the phase model of solve_phase_model at the bucket's width and its
        # graph's refinement count): factor and sparse reads for narrow
        # buckets, MFMA work for wide ones
        sv = solvers[g]
        qr = sv.qr
        fl = {}
        for b in buckets[g]:
            li = [lat_ms[i] for i, (gg, k) in enumerate(reqs) if gg == g and sv.query(k)[0] == b]
            if not li:
                continue
            gi = sv.query(b)[2]
            it = max(0, gi - 2) if gi > 0 else 0   # the graph holds the calibrated count + 2
            if g == "ct128":
                mod = solve_phase_model(qr.m, qr.n, b, 0, 0, 8, False, PEAK_TFLOPS["f64"])
            else:
                mod = solve_phase_model(qr.m, qr.n, b, nnz256, it, 4, args.prec == "bf16x3" and b >= 128)
            floor = sum(v[2] for v in mod.values()) * 1e3
            med = float(np.median(li))
            fl[str(b)] = {"requests": len(li), "median_ms": med, "floor_ms": floor, "frac": floor / med}
        per[g]["bucket_floor"] = fl
    out = {"requests": len(reqs), "slices": int(total),
           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
           "closed_loop_slices_per_s": total / t_closed, "queued_slices_per_s": total / t_queued,
           "queued_s": t_queued, "worst_status": int(status), "per_geometry": per}
    log("stream: %d requests, %d slices; closed loop p50 %.1f ms p99 %.1f ms (%.0f slices/s); "
        "all queued %.0f slices/s" % (len(reqs), total, out["p50_ms"], out["p99_ms"],
                                     out["closed_loop_slices_per_s"], out["queued_slices_per_s"]))
    for sv in solvers.values():
        sv.close()
    return out


def ooc_bench(args, log):
    """Out-of-core leg (a matrix whose dense FP32 copy does not fit in HBM):
    the sparse FP64 A and the sinograms are built on the GPU; as many leading
    columns of the dense FP32 A as leave room for the largest solve stay in
    HBM, the rest go to pinned host memory in tiles (dense column tiles rebuilt
    from the sparse copy); the factorization streams the host tiles
    (ctqr_qr_factor_ooc) once, then each slice count S is solved in one pass
    group that streams them once per substitution (ctqr_qr_solve_ooc), refined
    with FP64 sparse residuals (the paper's Table V times this solve for
    S = 256 ... 2048, Section III-B).  Checks per S: least-squares optimality
    of the noisy slices and exact recovery of two noise-free slices."""
    import numpy as np
    import torch
    from synthetic import get_workload, phantom_batch, noise_batch, NOISE_REL_LEVEL
    from paper_1907_01891_amd import ctqr as C
    from paper_1907_01891_amd.device import (SystemMatrix, OocFactor, colmajor, to_colmajor, round_up, ld_of,
                                             stream_handle)
    w = get_workload(args.workload)
    m, n = w.m, w.n
    slist = [int(v) for v in args.ooc_slices.split(",")] if args.ooc_slices else [w.n_slices]
    S_max = max(slist)
    n_clean = 2
    dev = torch.device("cuda:0")
    args.nb = args.nb or 256   # the out-of-core factorization is not tuned (tiles are multiples of 256)
    log("workload %s m=%d n=%d slices=%s (out of core)" % (w.name, m, n, slist))
    C.ctqr_set_progress(lambda st, d, t: log("%s %d/%d" % ("factor columns" if st == 1 else "solve iterations",
                                                          d, t)))
    t0 = time.perf_counter()
    sp = SystemMatrix(w.geometry(), C.CTQR_F64, dense=False, sparse=True)
    torch.cuda.synchronize()
    nnz = sp.nnz()
    log("sparse A: nnz %d (%.1f s)" % (nnz, time.perf_counter() - t0))
    # the inputs of the largest solve: S_max phantoms (the last n_clean
    # noise-free) and their sinograms, kept in host memory between solves
    Xtrue_h = torch.as_tensor(phantom_batch(w.side, S_max))
    B_h = torch.empty((m, S_max), dtype=torch.float64)
    for c0 in range(0, S_max, 256):
        c1 = min(S_max, c0 + 256)
        Xd = to_colmajor(Xtrue_h[:, c0:c1], dtype=torch.float64)
        Bd = sp.spmm(Xd)
        torch.cuda.synchronize()
        sigma = NOISE_REL_LEVEL * Bd.abs().amax(dim=0)
        Z = torch.as_tensor(noise_batch(w.side, m, c1 - c0, first=c0), device=dev)
        B_h[:, c0:c1] = (Bd + Z * sigma[None, :]).cpu()
        del Xd, Bd, Z
    lda = round_up(m, 64)
    col_bytes = lda * 4
    tile = args.ooc_tile
    free, total = torch.cuda.mem_get_info()
    solve_ws = C.ctqr_solve_ooc_workspace(m, n, C.CTQR_F32, args.nb, S_max, REFINE[args.refine] + 1, lda, tile)
    # the factorization's three tiles and the solve's workspace are never live
    # together (the factor's workspace is freed before the first solve)
    io = 8 * S_max * (m + 2 * n) + 8 * CHECK_CHUNK * (m + n)   # B, phantoms, X; the check's chunk buffers
    reserve = (max(3 * tile * col_bytes, solve_ws + io) + 2 * 2048 * round_up(n, 2048) * 4 + 4 * 256 * n * 4
               + int(5e9))
    n_dev = max(0, (free - reserve) // col_bytes // tile * tile)
    n_dev = min(n_dev, (n // tile) * tile)
    if args.ooc_dev_cols:
        n_dev = min(n_dev, args.ooc_dev_cols)
    host_gb = (n - n_dev) * col_bytes / 1e9
    log("HBM free %.1f GB of %.1f: %d resident columns (%.1f GB), %d host columns (%.1f GB pinned), tiles of %d; "
        "solve workspace for %d slices %.1f GB" % (free / 1e9, total / 1e9, n_dev, n_dev * col_bytes / 1e9, n - n_dev,
                                                   host_gb, tile, S_max, solve_ws / 1e9))
    O = OocFactor(m, n, C.CTQR_F32, prec_codes(C)[args.prec], n_dev, tile, nb=args.nb)
    t0 = time.perf_counter()
    if n_dev > 0:
        sp.dense_cols(0, n_dev, O.A_dev, C.CTQR_F32)
    if n_dev < n:
        stage = torch.empty((tile, lda), dtype=torch.float32, device=dev)
        for c0 in range(n_dev, n, tile):
            c1 = min(n, c0 + tile)
            sp.dense_cols(c0, c1, stage.t()[:m, :c1 - c0], C.CTQR_F32)
            O.host_base[c0 - n_dev:c1 - n_dev].copy_(stage[:c1 - c0])
        del stage
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    t_fill = time.perf_counter() - t0
    log("dense A in place (%.1f s)" % t_fill)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1 = ev(), ev()
    e0.record()
    O.factor()
    e1.record()
    torch.cuda.synchronize()
    t_qr = e0.elapsed_time(e1)
    finfo = O.info.read()
    qr_tf = qr_flops(m, n) / (t_qr * 1e-3) / 1e12
    log("ooc qr: %.1f s, %.2f TFLOP/s, status %d" % (t_qr * 1e-3, qr_tf, finfo.status))
    O.work.buf = None
    torch.cuda.empty_cache()
    spT = C.ctqr_sparse(n, m, sp.sp.nnz_cap, sp.colptr.data_ptr(), sp.row.data_ptr(), sp.cval.data_ptr(),
                        sp.rowptr.data_ptr(), sp.col.data_ptr(), sp.val.data_ptr())
    normA = sp.val[:nnz].pow(2).sum().sqrt().item()
    solves = []
    for S in slist:
        # the first S - n_clean noisy slices and the n_clean noise-free ones
        cols = list(range(S - n_clean)) + list(range(S_max - n_clean, S_max))
        B = to_colmajor(B_h[:, cols], dtype=torch.float64)
        Xt = to_colmajor(Xtrue_h[:, cols], dtype=torch.float64)
        Bc = sp.spmm(Xt[:, S - n_clean:])                 # noise-free sinograms of the last slices
        B[:, S - n_clean:].copy_(Bc)
        del Bc
        torch.cuda.synchronize()
        e2, e3 = ev(), ev()
        e2.record()
        X = O.solve(B, sparse=sp.sp, tol=args.tol, max_iters=args.max_iters, method=REFINE[args.refine])
        e3.record()
        torch.cuda.synchronize()
        t_solve = e2.elapsed_time(e3)
        sinfo = O.sinfo.read()
        # least-squares optimality ||A^T r|| / (||A||_F ||r||), r = b - A x (FP64,
        # sparse), over the noisy slices in chunks
        opt = 0.0
        for c0 in range(0, S - n_clean, CHECK_CHUNK):
            c1 = min(S - n_clean, c0 + CHECK_CHUNK)
            R = colmajor(m, c1 - c0, torch.float64, dev)
            R.copy_(B[:, c0:c1])
            sp.spmm(X[:, c0:c1], alpha=-1.0, beta=1.0, Y=R)
            G = colmajor(n, c1 - c0, torch.float64, dev)
            C.check(C.ctqr_spmm(spT, c1 - c0, 1.0, ctypes.c_void_p(R.data_ptr()), ld_of(R), 0.0,
                                ctypes.c_void_p(G.data_ptr()), ld_of(G), stream_handle()), "ctqr_spmm")
            torch.cuda.synchronize()
            opt = max(opt, (G.norm(dim=0) / (normA * R.norm(dim=0))).max().item())
            del R, G
        rec = ((X[:, S - n_clean:] - Xt[:, S - n_clean:]).norm(dim=0) / Xt[:, S - n_clean:].norm(dim=0)).max().item()
        log("ooc solve S=%d: %.1f s (%.4f s per slice), refine iters %d status %d, ls optimality %.2e, "
            "noise-free recovery %.2e" % (S, t_solve * 1e-3, t_solve * 1e-3 / S, sinfo.iters, sinfo.status, opt, rec))
        solves.append({"slices": S, "solve_ms": t_solve, "s_per_slice": t_solve * 1e-3 / S,
                       "slices_per_s": S / (t_solve * 1e-3), "refine_iters": int(sinfo.iters),
                       "refine_status": int(sinfo.status), "ls_optimality_max": opt, "recovery_rel_err_max": rec})
        if args.save_check:
            os.makedirs(args.save_check, exist_ok=True)
            keep = [0, 1, S - 2, S - 1]
            np.savez(os.path.join(args.save_check, "%s_S%d.npz" % (w.name, S)), X=X[:, keep].cpu().numpy(),
                     B=B[:, keep].cpu().numpy(), Xtrue=Xt[:, keep].cpu().numpy(), noise_free=np.array([0, 0, 1, 1]))
        del B, Xt, X
        torch.cuda.empty_cache()
    C.ctqr_set_progress(None)
    head = solves[0]
    return {
        "metric": "QR TFLOP/s + slices/s at %d^2, out of core (A larger than HBM)" % w.side,
        "value": qr_tf, "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": t_qr + head["solve_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if args.prec == "bf16x3" else "f32", "data": "synthetic",
        "config": {"workload": "%s: %dx%d image, %d views x %d bins (m=%d, n=%d), ellipse-phantom slices "
                               "(%d noise-free per solve); FP32 A %.1f GB: %d columns in HBM, %d in pinned host "
                               "memory, tiles of %d" % (w.name, w.side, w.side, w.n_views, w.n_bins, m, n, n_clean,
                                                        m * n * 4 / 1e9, n_dev, n - n_dev, tile),
                   "nb": args.nb, "slices": slist, "parallelism": "single GPU"},
        "qr_ms": t_qr, "fill_s": t_fill, "qr_info_status": int(finfo.status),
        "rdiag_min_max": [finfo.rdiag_min, finfo.rdiag_max], "refine_method": args.refine, "tol": args.tol,
        "solves": solves, "nnz": nnz, "resident_columns": int(n_dev), "host_columns": int(n - n_dev),
        "host_gb": host_gb,
    }


def phase_and_conditioning(args, log, C, F, A32, B, sp, Xmixed, sinfo, t_solve, build_dense, m, n, S, dev):
    """Untimed extras of the mixed path: the phase breakdown of one more
    factorization and refined solve (HIP events per phase), the condition
    estimate kappa(A) with the least-squares perturbation bound, and the solve
    roofline from the per-phase work model."""
    import torch
    from paper_1907_01891_amd.device import colmajor
    build_dense(A32, C.CTQR_F32)
    torch.cuda.synchronize()
    C.ctqr_profile_enable(C.CTQR_PROFILE_PHASES)
    F.factor()
    Xp = F.solve(B, sparse=sp.sp, tol=args.tol, max_iters=args.max_iters, method=REFINE[args.refine])
    torch.cuda.synchronize()
    phases = C.ctqr_profile_phases()
    C.ctqr_profile_enable(False)
    del Xp
    phase_ms = {k: v[0] for k, v in phases.items()}
    log("phases (ms): " + ", ".join("%s %.1f" % (k, v) for k, v in phase_ms.items()))

    # ---- condition estimate and the least-squares perturbation bound
    smax, smin, kappa = F.cond_estimate(sp.sp, nvec=8, iters=30)
    Rr = colmajor(m, S, torch.float64, dev)
    Rr.copy_(B)
    sp.spmm(Xmixed, alpha=-1.0, beta=1.0, Y=Rr)
    AX = sp.spmm(Xmixed)
    torch.cuda.synchronize()
    tan_theta = (Rr.norm(dim=0) / AX.norm(dim=0)).max().item()
    del Rr, AX
    u64, u32 = 2.0 ** -53, 2.0 ** -24
    ls_bound64 = u64 * (2.0 * kappa + kappa ** 2 * tan_theta)
    log("kappa estimate %.4e (sigma_max %.4e, sigma_min %.4e); tan(theta) %.3e; LS bound u64 (2k + k^2 tan) %.2e; "
        "contraction %.3e (u32 kappa^2 %.3e)" % (kappa, smax, smin, tan_theta, ls_bound64, sinfo.contraction,
                                                 u32 * kappa ** 2))
    nnz = sp.nnz()
    split_refine = args.prec == "bf16x3" and S >= 128
    model = solve_phase_model(m, n, S, nnz, int(sinfo.iters), 4, split_refine)
    floor_ms = sum(v[2] for v in model.values()) * 1e3
    solve_roof = {
        "bound": "per phase: MFMA (Q^T B, substitutions) and HBM (sparse residuals)",
        "floor_ms": floor_ms, "measured_ms": t_solve, "frac": floor_ms / t_solve,
        "refine_iters": int(sinfo.iters),
        "phases": {k: {"flops": v[0], "bytes": v[1], "floor_ms": v[2] * 1e3,
                       "measured_ms": phase_ms[k]} for k, v in model.items()},
        "refine_other_ms": phase_ms["refine_other"],
        "model": "floor = sum over phases of max(flops / MFMA peak, bytes / 8 TB/s); FP32 MFMA peak, a third of "
                 "the BF16 peak for split-BF16 substitution products; per-phase measured = HIP events of an "
                 "untimed profiled solve",
    }
    return {
        "refine_contraction": sinfo.contraction,
        "kappa_est": kappa, "sigma_max_est": smax, "sigma_min_est": smin,
        "kappa_note": "lower-bound estimates: power iteration on A^T A (FP64 sparse A), inverse iteration on R^T R "
                      "(the factor's R), 8 vectors x 30 steps",
        "ls_tan_theta_max": tan_theta,
        "ls_perturbation_bound_fp64": ls_bound64,
        "u32_kappa2": u32 * kappa ** 2,
        "qr_phases_ms": {k: phase_ms[k] for k in ("panel", "inner", "reduction", "update", "group_update", "rinv")},
        "solve_roofline": solve_roof,
    }


def tile_qr_leg(log, name="ct64", b=64, nsl=8):
    """The algorithm-by-blocks QR and solve (Section II-C; ctqr_tile_qr_*) on
    the FP64 A of a smaller workload, timed, beside the blocked FP64 GPU path
    on the same matrix (their solutions compared).  The tile tasks run FP64
    arithmetic on the vector ALUs, one workgroup per b x b task."""
    import torch
    from synthetic import get_workload, phantom_batch
    from paper_1907_01891_amd import ctqr as C
    from paper_1907_01891_amd.device import SystemMatrix, QRFactor, TileQR, to_colmajor
    w = get_workload(name)
    S = SystemMatrix(w.geometry(), C.CTQR_F64, dense=True, sparse=True)
    X = to_colmajor(torch.as_tensor(phantom_batch(w.side, nsl)), dtype=torch.float64)
    B = S.spmm(X)
    A0 = S.A.clone()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    G = TileQR(S.A, b)
    G.factor()                                     # warm-up (A overwritten)
    S.A.copy_(A0)
    torch.cuda.synchronize()
    e0, e1, e2 = ev(), ev(), ev()
    e0.record()
    G.factor()
    e1.record()
    Xt = G.solve(B)
    e2.record()
    torch.cuda.synchronize()
    t_f, t_s = e0.elapsed_time(e1), e1.elapsed_time(e2)
    Ab = A0.clone()
    Fb = QRFactor(Ab, C.CTQR_PREC_FP64, nb=256)
    torch.cuda.synchronize()
    e0.record()
    Fb.factor()
    e1.record()
    Xb = Fb.solve(B)
    e2.record()
    torch.cuda.synchronize()
    tb_f = e0.elapsed_time(e1)
    diff = ((Xt - Xb).norm(dim=0) / Xb.norm(dim=0)).max().item()
    rec = ((Xt - X).norm(dim=0) / X.norm(dim=0)).max().item()
    fl = qr_flops(w.m, w.n)
    tf = fl / (t_f * 1e-3) / 1e12
    mt, nt = -(-w.m // b), -(-w.n // b)
    out = {"workload": "%s: %d x %d FP64, blocks of %d (%d x %d blocks, %d tasks)"
                       % (name, w.m, w.n, b, mt, nt, len(C.ctqr_tile_tasks(mt, nt, 0))),
           "qr_ms": t_f, "qr_tflops": tf, "frac_of_fp64_peak": tf / PEAK_TFLOPS["f64"],
           "solve_ms": t_s, "slices": nsl, "blocked_fp64_qr_ms": tb_f,
           "blocked_fp64_qr_tflops": fl / (tb_f * 1e-3) / 1e12,
           "rel_diff_vs_blocked_solution": diff, "recovery_rel_err": rec}
    log("tile QR %s: %.1f ms (%.3f TFLOP/s, blocked FP64 %.1f ms), solve %.1f ms, vs blocked %.2e, recovery %.2e"
        % (name, t_f, tf, tb_f, t_s, diff, rec))
    return out


def image_quality_leg(args, log, w, F, sp, Xtrue, Xc, n_clean):
    """The evaluation around the solve (Section II-A, II-B): sinograms of the
    phantoms simulated with Joseph's projector (ctqr_project_joseph, timed),
    reconstructed with the mixed factor and the Siddon A (refined), and scored
    with PSNR and SSIM (ctqr_image_quality, timed) against the phantoms; the
    noise-free Siddon sinograms' reconstructions are scored the same way (the
    setting of the paper's quality table: data consistent with A)."""
    import numpy as np
    import torch
    from paper_1907_01891_amd.device import project_joseph, image_quality
    g = w.geometry()
    S = Xtrue.shape[1]
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1, e2, e3 = ev(), ev(), ev(), ev()
    project_joseph(g, Xtrue)                       # warm-up
    e0.record()
    BJ = project_joseph(g, Xtrue)
    e1.record()
    torch.cuda.synchronize()
    t_j = e0.elapsed_time(e1)
    XJ = F.solve(BJ, sparse=sp.sp, tol=args.tol, max_iters=args.max_iters, method=REFINE[args.refine])
    torch.cuda.synchronize()
    sj = F.sinfo.read()
    image_quality(w.side, Xtrue, XJ)               # warm-up
    e2.record()
    pj, qj = image_quality(w.side, Xtrue, XJ)
    e3.record()
    torch.cuda.synchronize()
    t_q = e2.elapsed_time(e3)
    pc, qc = image_quality(w.side, Xtrue[:, :n_clean], Xc)
    out = {"joseph_ms": t_j, "joseph_ray_slices_per_s": w.m * S / (t_j * 1e-3), "quality_ms": t_q,
           "joseph_recon_refine_status": int(sj.status), "joseph_recon_refine_iters": int(sj.iters),
           "joseph_psnr_db_mean": float(np.mean(pj)), "joseph_psnr_db_min": float(np.min(pj)),
           "joseph_ssim_mean": float(np.mean(qj)), "joseph_ssim_min": float(np.min(qj)),
           "consistent_psnr_db_min": float(np.min(pc)), "consistent_ssim_min": float(np.min(qc)),
           "note": "Joseph sinograms reconstructed with the Siddon A carry a projector mismatch; the consistent "
                   "(noise-free Siddon) reconstructions are the analogue of the paper's quality table"}
    log("joseph: %.1f ms for %d x %d rays x slices; reconstructions PSNR mean %.2f dB, SSIM mean %.4f; consistent "
        "data PSNR min %.1f dB, SSIM min %.6f; quality kernel %.2f ms"
        % (t_j, w.m, S, out["joseph_psnr_db_mean"], out["joseph_ssim_mean"], out["consistent_psnr_db_min"],
           out["consistent_ssim_min"], t_q))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    import numpy as np
    import torch
    from synthetic import get_workload, phantom_batch, noise_batch, NOISE_REL_LEVEL
    from paper_1907_01891_amd import ctqr as C
    from paper_1907_01891_amd.device import SystemMatrix, QRFactor, colmajor, to_colmajor

    C.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = get_workload(args.workload)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    free, _ = torch.cuda.mem_get_info()
    # out of core unless the dense FP32 A, its factorization and the refined
    # solve of all slices (workspaces as the library reports them) fit in HBM
    from paper_1907_01891_amd.device import round_up
    nb_q, refine_q = args.nb or 256, REFINE[args.refine] + 1
    need = (round_up(w.m, 64) * w.n * 4 + nb_q * w.n * 4 + C.ctqr_qr_rinv_bytes(w.n, C.CTQR_F32)
            + C.ctqr_qr_workspace(w.m, w.n, C.CTQR_F32, prec_codes(C)[args.prec], nb_q)
            + C.ctqr_solve_workspace(w.m, w.n, C.CTQR_F32, nb_q, w.n_slices, refine_q)
            + 24 * w.m * (2 * w.side - 1) + 4 * 8 * w.m * w.n_slices)   # sparse copies, B / X
    if args.ooc or need > 0.95 * free:
        print(json.dumps(ooc_bench(args, log)))
        return
    g = w.geometry()
    m, n, S = w.m, w.n, w.n_slices
    log("workload %s m=%d n=%d slices=%d" % (w.name, m, n, S))

    # ---- untimed input synthesis: sparse FP64 A, phantoms, noisy sinograms
    sp = SystemMatrix(g, C.CTQR_F64, dense=False, sparse=True)
    Xtrue = to_colmajor(torch.as_tensor(phantom_batch(w.side, S)), dtype=torch.float64)
    B = sp.spmm(Xtrue)
    torch.cuda.synchronize()
    sigma = NOISE_REL_LEVEL * B.abs().amax(dim=0)
    Z = torch.as_tensor(noise_batch(w.side, m, S), device=dev)
    n_clean = 4
    Bclean = colmajor(m, n_clean, torch.float64, dev)
    Bclean.copy_(B[:, :n_clean])
    B.add_(Z * sigma[None, :])
    del Z
    log("inputs ready, nnz=%d" % sp.nnz())

    A32 = colmajor(m, n, torch.float32, dev)
    stream = torch.cuda.current_stream()

    def build_dense(A, dtype):
        from paper_1907_01891_amd.device import Workspace, stream_handle, ld_of
        import ctypes
        ws = build_dense.ws
        wp, wb = ws.get(C.ctqr_build_workspace(sp.geom))
        C.check(C.ctqr_build_system_matrix(sp.geom, dtype, ctypes.c_void_p(A.data_ptr()), ld_of(A), None,
                                           wp, wb, sp.info.ptr, stream_handle()), "build")
    from paper_1907_01891_amd.device import Workspace
    build_dense.ws = Workspace()

    tuned = None
    if args.nb == 0:
        # block width by timing on this A (overwrites it; every step rebuilds A)
        build_dense(A32, C.CTQR_F32)
        Ft = QRFactor(A32, prec_codes(C)[args.prec], nb=256)
        nb_t, ms_col = Ft.tune_nb()
        torch.cuda.synchronize()
        del Ft
        args.nb = nb_t
        tuned = {"nb": nb_t, "ms_per_column": {"64": ms_col[0], "128": ms_col[1], "256": ms_col[2]}}
        log("tuned nb = %d (ms per column: 64: %.3f, 128: %.3f, 256: %.3f)" % (nb_t, *ms_col))
    F = QRFactor(A32, prec_codes(C)[args.prec], nb=args.nb)
    X = colmajor(n, S, torch.float64, dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(profile):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record()
        build_dense(A32, C.CTQR_F32)
        e1.record()
        if profile:
            C.ctqr_profile_enable(True)
        F.factor()
        e2.record()
        F.solve(B, X=X, sparse=sp.sp, tol=args.tol, max_iters=args.max_iters, method=REFINE[args.refine])
        e3.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2), e2.elapsed_time(e3)

    for i in range(args.warmup):
        t = step(False)
        log("warmup %d: build %.1f ms, qr %.1f ms, solve %.1f ms" % (i, *t))
    torch.cuda.synchronize()
    times = []
    tw0 = time.perf_counter()
    for i in range(args.steps):
        t = step(True)
        times.append(t)
        log("step %d: build %.1f ms, qr %.1f ms, solve %.1f ms" % (i, *t))
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw0
    launches, kern_ms, kern_flops = C.ctqr_profile_read()
    red_launches, red_ms, red_flops = C.ctqr_profile_read_reduction()
    C.ctqr_profile_enable(False)
    finfo, sinfo = F.info.read(), F.sinfo.read()
    t_build = np.mean([t[0] for t in times])
    t_qr = np.mean([t[1] for t in times])
    t_solve = np.mean([t[2] for t in times])
    qr_tf = qr_flops(m, n) / (t_qr * 1e-3) / 1e12
    slices_s = S / (t_solve * 1e-3)

    # accuracy: exact recovery on noise-free slices (the least-squares solution
    # of consistent data is the phantom itself)
    Xc = F.solve(Bclean, sparse=sp.sp, tol=args.tol, max_iters=args.max_iters, method=REFINE[args.refine])
    torch.cuda.synchronize()
    rec_err = ((Xc - Xtrue[:, :n_clean]).norm(dim=0) / Xtrue[:, :n_clean].norm(dim=0)).max().item()
    Xmixed = X.clone()
    log("mixed (%s products): qr %.2f TFLOP/s, %.0f slices/s, refine iters %d (status %d), recovery err %.2e"
        % (args.prec, qr_tf, slices_s, sinfo.iters, sinfo.status, rec_err))

    extras = {}
    if not args.no_phases:
        extras = phase_and_conditioning(args, log, C, F, A32, B, sp, Xmixed, sinfo, t_solve, build_dense,
                                        m, n, S, dev)
        extras["image_quality"] = image_quality_leg(args, log, w, F, sp, Xtrue, Xc, n_clean)
    log("mixed path done")

    stream_out = None
    if not args.no_stream and args.workload == "ct256":
        stream_out = request_stream_bench(args, log, F, sp, B)
        torch.cuda.empty_cache()
    bf16 = {}
    if not args.no_bf16:
        # the other product modes of the FP32-storage factorization (FP32
        # MFMA, one-part BF16, split BF16), each factored once; errors are
        # reported against the refined solution of the headline mode
        for key in [k for k in ("fp32", "bf16", "bf16x3") if k != args.prec]:
            build_dense(A32, C.CTQR_F32)
            F16 = QRFactor(A32, prec_codes(C)[key], nb=args.nb)
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            C.ctqr_profile_enable(True)
            e0.record()
            F16.factor()
            e1.record()
            torch.cuda.synchronize()
            t16 = e0.elapsed_time(e1)
            tl, tms, tfl = C.ctqr_profile_read()
            C.ctqr_profile_enable(False)
            if tl:
                bf16[key + "_trailing_update_avg_ms"] = tms / tl
                bf16[key + "_trailing_update_tflops"] = tfl / (tms * 1e-3) / 1e12
                if key == "fp32":
                    bf16["fp32_trailing_update_frac_of_fp32_mfma_peak"] = tfl / (tms * 1e-3) / 1e12 / PEAK_TFLOPS["f32"]
            Xu = F16.solve(B)
            torch.cuda.synchronize()
            e_unref = ((Xu - Xmixed).norm(dim=0) / Xmixed.norm(dim=0)).max().item()
            e0.record()
            Xr = F16.solve(B, sparse=sp.sp, tol=args.tol, max_iters=args.max_iters, method=REFINE[args.refine])
            e1.record()
            torch.cuda.synchronize()
            ts16 = e0.elapsed_time(e1)
            si16 = F16.sinfo.read()
            e_ref = ((Xr - Xmixed).norm(dim=0) / Xmixed.norm(dim=0)).max().item()
            bf16.update({key + "_qr_tflops": qr_flops(m, n) / (t16 * 1e-3) / 1e12, key + "_qr_ms": t16,
                         key + "_unrefined_rel_err_vs_headline": e_unref, key + "_refined_rel_err_vs_headline": e_ref,
                         key + "_refine_status": int(si16.status), key + "_refine_iters": int(si16.iters),
                         key + "_refined_slices_per_s": S / (ts16 * 1e-3),
                         key + "_qr_info_status": int(F16.info.read().status)})
            log("%s: qr %.2f TFLOP/s (%.0f ms; trailing update %.2f ms per launch); error vs headline: unrefined "
                "%.2e, refined %.2e (status %d, %d iters, %.0f slices/s)"
                % (key, bf16[key + "_qr_tflops"], t16, bf16.get(key + "_trailing_update_avg_ms", 0.0), e_unref,
                   e_ref, si16.status, si16.iters, S / (ts16 * 1e-3)))
            del F16, Xu, Xr
            torch.cuda.empty_cache()
    del A32, F
    torch.cuda.empty_cache()

    tile = None
    if not args.no_phases:
        tile = tile_qr_leg(log)
        torch.cuda.empty_cache()

    fp64 = {}
    if not args.no_fp64:
        A64 = colmajor(m, n, torch.float64, dev)
        build_dense(A64, C.CTQR_F64)
        F64 = QRFactor(A64, C.CTQR_PREC_FP64, nb=args.nb)
        torch.cuda.synchronize()
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        F64.factor()
        e1.record()
        X64 = F64.solve(B)
        e2.record()
        torch.cuda.synchronize()
        t64_qr, t64_solve = e0.elapsed_time(e1), e1.elapsed_time(e2)
        diff = ((Xmixed - X64).norm(dim=0) / X64.norm(dim=0)).max().item()
        Xc64 = F64.solve(Bclean)
        torch.cuda.synchronize()
        rec64 = ((Xc64 - Xtrue[:, :n_clean]).norm(dim=0) / Xtrue[:, :n_clean].norm(dim=0)).max().item()
        fp64 = {"fp64_qr_tflops": qr_flops(m, n) / (t64_qr * 1e-3) / 1e12,
                "fp64_slices_per_s": S / (t64_solve * 1e-3), "fp64_qr_ms": t64_qr, "fp64_solve_ms": t64_solve,
                "fp64_recovery_err": rec64, "mixed_vs_fp64_rel_diff": diff,
                "fp64_info_status": F64.info.read().status}
        log("fp64: qr %.2f TFLOP/s (%.0f ms), %.0f slices/s, mixed-vs-fp64 %.2e, recovery %.2e"
            % (fp64["fp64_qr_tflops"], t64_qr, fp64["fp64_slices_per_s"], diff, rec64))
        del A64, F64
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        log("cpu baseline ...")
        cpu = cpu_baseline(args.workload, args.cpu_seconds)
        log("cpu baseline %.4f TFLOP/s (%s)" % (cpu["value"], cpu["sample"]))

    achieved = kern_flops / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    # algorithmic HBM bytes of one trailing update C -= V W' (FP32): read and
    # write C (m_k x n_k), read V (m_k x K) and W' (K x n_k) once
    launches_k = trailing_launches(m, n, args.nb)
    alg = sum(8.0 * mk * nc + 4.0 * kk * (mk + nc) for mk, nc, kk in launches_k)
    alg_bytes = alg / len(launches_k) if launches_k else None
    avg_ms = kern_ms / launches if launches else None
    if args.prec == "fp32":
        roof = {"bound": "mfma", "kernel": TRAILING_KERNEL["fp32"] + " (trailing update C -= V W', FP32 MFMA)",
                "achieved": achieved, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                "frac": (achieved / PEAK_TFLOPS["f32"]) if achieved else None}
    else:
        # The split-BF16 update executes three BF16 products per FP32-equivalent
        # product (high-high, high-low, low-high).  The method's own work is one
        # product, 2 m_k n_k K flops per launch: that is what `achieved` and
        # `frac` count, against the BF16 MFMA peak the products run on.  The
        # executed three-product rate and the HBM figures are reported beside it.
        gbs = alg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms else None
        exec_tf = 3 * achieved if achieved else None
        flops_method = sum(2.0 * mk * nc * kk for mk, nc, kk in launches_k)
        ridge = PEAK_TFLOPS["bf16"] * 1e12 / (HBM_PEAK_GBS * 1e9)
        roof = {"bound": "mfma", "kernel": TRAILING_KERNEL["bf16x3"] + " (split-BF16 trailing update C -= V W'; "
                                           "launches of fewer than 512 tiles of 256 run gemm_nn_bf16x3_kernel<1>)",
                "achieved": achieved, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS["bf16"] if achieved else None,
                "achieved_counts": "method flops 2 m_k n_k K per launch (one FP32-equivalent product)",
                "method_flop_per_byte": flops_method / alg if alg else None, "ridge_flop_per_byte": ridge,
                "mfma_tflops_executed_bf16": exec_tf,
                "executed_frac_of_bf16_peak": exec_tf / PEAK_TFLOPS["bf16"] if exec_tf else None,
                "hbm_gbs_algorithmic": gbs, "hbm_frac": gbs / HBM_PEAK_GBS if gbs else None}
    roof.update({
        "traffic": measured_traffic(args.workload, args.prec, launches) if args.nb == 256 else None,
        "traffic_unit": "bytes per launch (HBM, FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_bytes_per_launch": alg_bytes,
        "launches": launches,
        "avg_launch_ms": avg_ms,
        "flops_per_launch": kern_flops / launches if launches else None,
        "flops_per_launch_counts": "2 rows cols K (one FP32-equivalent product; the split-BF16 "
                                   "update executes three BF16 products of this size)",
    })
    # The other large product of the factorization: the reductions
    # [G | W] = V^T [V | C] (every block column and group), timed the same way
    # on the last timed step.  Method flops 2 M N K per launch.
    red_tf = red_flops / (red_ms * 1e-3) / 1e12 if red_ms > 0 else None
    red_peak = PEAK_TFLOPS["f32"] if args.prec == "fp32" else PEAK_TFLOPS["bf16"]
    roof_red = {"bound": "mfma",
                "kernel": ("gemm_tn_kernel (FP32 MFMA)" if args.prec == "fp32" else
                           "gemm_tn_bf16x3_kernel (split-BF16, C split while staged)") + ": [G | W] = V^T [V | C]",
                "achieved": red_tf, "peak": red_peak, "unit": "TFLOP/s",
                "frac": red_tf / red_peak if red_tf else None,
                "achieved_counts": "method flops 2 M N K per launch (one FP32-equivalent product)",
                "mfma_tflops_executed_bf16": 3 * red_tf if (red_tf and args.prec == "bf16x3") else None,
                "launches": red_launches, "avg_launch_ms": red_ms / red_launches if red_launches else None,
                "total_ms": red_ms, "flops_per_launch": red_flops / red_launches if red_launches else None}
    products = {"bf16x3": "split-BF16 MFMA block-column products (high + low bf16 parts, three products, FP32 "
                          "accumulation)",
                "fp32": "FP32-MFMA block-column products"}[args.prec]
    out = {
        "metric": "QR TFLOP/s + slices/s at 256^2 (mixed vs FP64 GPU, rel err <= 1e-10)",
        "value": qr_tf,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean([sum(t) for t in times])),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if args.prec == "bf16x3" else "f32",
        "dtype_detail": "FP32 storage of A and the factor; the dominant contractions (block-column products) on %s "
                        "with FP32 accumulation; FP64 panel norms and reflectors; FP64 sparse residuals in the "
                        "refinement" % ("split-BF16 MFMA (three BF16 products per FP32 product)"
                                        if args.prec == "bf16x3" else "FP32 MFMA"),
        "data": "synthetic",
        "config": {
            "workload": "%s: %dx%d image, %d views x %d bins (m=%d, n=%d), %d ellipse-phantom slices, "
                        "1e-3 relative noise; FP32 A, %s, FP64 panel, %s refinement with FP64 sparse "
                        "residuals" % (w.name, w.side, w.side, w.n_views, w.n_bins, m, n, S, products,
                                       args.refine.upper()),
            "nb": args.nb, "nb_tuning": tuned, "slices": S, "products": args.prec, "parallelism": "single GPU",
        },
        "slices_per_s": slices_s,
        "qr_ms": t_qr, "solve_ms": t_solve, "build_ms": t_build,
        "solve_tflops": S * solve_flops(m, n) / (t_solve * 1e-3) / 1e12,
        "refine_method": args.refine,
        "refine_iters": int(sinfo.iters), "refine_status": int(sinfo.status),
        "refine_last_rel_update": sinfo.max_rel_update,
        "recovery_rel_err_max": rec_err,
        "refine_contraction": sinfo.contraction,
        **extras,
        "qr_info_status": int(finfo.status),
        "rdiag_min_max": [finfo.rdiag_min, finfo.rdiag_max],
        "roofline": roof,
        "roofline_reduction": roof_red,
        "cpu_baseline": cpu,
        "request_stream": stream_out,
        "tile_qr": tile,
        "wall_s_timed": wall,
    }
    out.update(fp64)
    out.update(bf16)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
