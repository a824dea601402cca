"""MI355X-native QR least-squares CT reconstruction.

The hot path of algebraic CT reconstruction by a direct QR solve (Chillaron,
Quintana-Orti, Vidal, Verdu): build the fan-beam system matrix A, factor it
once with a blocked Householder QR (A = QR, Eq. 3), and reconstruct many
sinogram slices as X = R^-1 (Q^T B) (Eq. 4).  All arithmetic runs in the
gfx950 HIP library libctqr.so behind the C ABI of include/ctqr.h; ``ctqr`` is
its ctypes binding and ``device`` allocates device buffers with PyTorch.
Importing this package does not load the library; ``ctqr.lib()`` does, and
raises if it has not been built.
"""
__all__ = ["ctqr", "device", "build"]
