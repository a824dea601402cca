/*
 * Oracle: unblocked FP64 Householder QR, Q^T B and back substitution.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; the product never links it.  Plain C +
 * OpenMP, compiled with gcc, sharing nothing with the HIP library.
 *
 * The paper factors A = QR (Eq. 3) and reconstructs X = R^-1 (Q^T B) (Eq. 4),
 * with Q applied implicitly from the Householder reflectors stored below the
 * diagonal and R in the upper triangle (Section II-C, "QR factorization":
 * the output of Compute_dense_QR), and R^-1 applied by backward substitution
 * (Section II-C, "System solving").  This file is the textbook unblocked form:
 * one reflector per column, applied at once to every column to its right.
 *
 * Reflector convention (a reading: the paper does not fix one), that of
 * LAPACK's larfg: for the column [alpha; x],
 *   beta = -sign(alpha) * ||[alpha; x]||   (sign(0) = +1),
 *   tau  = (beta - alpha) / beta,
 *   v    = [1; x / (alpha - beta)],
 * and H = I - tau v v^T maps [alpha; x] to [beta; 0].  If x == 0 then
 * tau = 0 and the column is left as is.  Norms are a plain sum of squares.
 *
 * All matrices are column-major with a leading dimension.
 */
#include <math.h>
#include <stdint.h>

/* QR in place: on exit the upper triangle of A[0:n,0:n] holds R, the strict
 * lower part of column k holds v_k(1:), tau[k] holds tau_k. */
void oracle_geqr2(int64_t m, int64_t n, double *A, int64_t lda, double *tau)
{
    for (int64_t k = 0; k < n; ++k) {
        double *ak = A + k * lda;
        double alpha = ak[k];
        double ss = 0.0;
        for (int64_t i = k + 1; i < m; ++i) ss += ak[i] * ak[i];
        if (ss == 0.0) {
            tau[k] = 0.0;
            continue;
        }
        double norm = sqrt(alpha * alpha + ss);
        double beta = alpha >= 0.0 ? -norm : norm;
        double t = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        for (int64_t i = k + 1; i < m; ++i) ak[i] *= scale;
        ak[k] = beta;
        tau[k] = t;
        /* apply H_k = I - t v v^T to every later column */
        #pragma omp parallel for schedule(static)
        for (int64_t c = k + 1; c < n; ++c) {
            double *ac = A + c * lda;
            double w = ac[k];
            for (int64_t i = k + 1; i < m; ++i) w += ak[i] * ac[i];
            w *= t;
            ac[k] -= w;
            for (int64_t i = k + 1; i < m; ++i) ac[i] -= w * ak[i];
        }
    }
}

/* B <- Q^T B = H_{n-1} ... H_0 B for nrhs columns, using the reflectors of
 * oracle_geqr2. */
void oracle_apply_qt(int64_t m, int64_t n, const double *QR, int64_t lda,
                     const double *tau, int64_t nrhs, double *B, int64_t ldb)
{
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nrhs; ++s) {
        double *b = B + s * ldb;
        for (int64_t k = 0; k < n; ++k) {
            const double *v = QR + k * lda;
            if (tau[k] == 0.0) continue;
            double w = b[k];
            for (int64_t i = k + 1; i < m; ++i) w += v[i] * b[i];
            w *= tau[k];
            b[k] -= w;
            for (int64_t i = k + 1; i < m; ++i) b[i] -= w * v[i];
        }
    }
}

/* B <- Q B = H_0 ... H_{n-1} B (used by the tests to rebuild A = QR). */
void oracle_apply_q(int64_t m, int64_t n, const double *QR, int64_t lda,
                    const double *tau, int64_t nrhs, double *B, int64_t ldb)
{
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nrhs; ++s) {
        double *b = B + s * ldb;
        for (int64_t k = n - 1; k >= 0; --k) {
            const double *v = QR + k * lda;
            if (tau[k] == 0.0) continue;
            double w = b[k];
            for (int64_t i = k + 1; i < m; ++i) w += v[i] * b[i];
            w *= tau[k];
            b[k] -= w;
            for (int64_t i = k + 1; i < m; ++i) b[i] -= w * v[i];
        }
    }
}

/* Backward substitution R x = c for nrhs columns: x_i = (c_i - sum_{j>i}
 * R_ij x_j) / R_ii, i = n-1 .. 0.  C (n rows used) is overwritten by X. */
void oracle_backsub(int64_t n, const double *R, int64_t ldr, int64_t nrhs,
                    double *C, int64_t ldc)
{
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nrhs; ++s) {
        double *c = C + s * ldc;
        for (int64_t i = n - 1; i >= 0; --i) {
            double acc = c[i];
            for (int64_t j = i + 1; j < n; ++j) acc -= R[i + j * ldr] * c[j];
            c[i] = acc / R[i + i * ldr];
        }
    }
}
