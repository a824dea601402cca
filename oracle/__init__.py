"""CPU oracle for the QR least-squares CT reconstruction path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import, call, link or execute anything in this package;
the product path (the HIP library and its Python binding) never does.  It
shares no code with the HIP path: only the seeded input generators in
``synthetic`` serve both.

Everything is plain FP64 and follows the paper's definitions:
  geometry.py   scanner and projection angles (Section II-A, Table I, Eq. 2)
  siddon.py     system matrix A by Siddon ray tracing (Section II-A, Eq. 1)
  clip.py       A again by brute-force pixel clipping (independent cross-check)
  householder.py + qr_oracle.c
                unblocked Householder QR A = QR, Q^T B and back substitution
                (Eq. 3, Eq. 4; Section II-C "System solving")
  lsq.py        the reconstruction X = R^-1 (Q^T B), residual metrics, CGLS,
                PSNR (Eq. 5-6)
  views.py      the smallest view count giving A full column rank (Section
                II-A, Eq. 2), by SVD condition numbers
"""
