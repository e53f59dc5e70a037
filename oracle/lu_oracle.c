/*
 * Oracle for the shifted systems (A - sigma_j I) X_j = B,  G_j = C X_j.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU reference that the GPU path is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * library never links, loads or calls it, and it shares no code with it.
 *
 * What it computes (Section 1, the transfer function and the shifted systems
 * it needs; Section 2, where the paper rewrites the transfer function through
 * the controller-Hessenberg form): for every shift sigma_j,
 *     X_j = (A - sigma_j I)^{-1} B         (n x m, complex)
 *     G_j = C X_j                          (p x m, complex)
 * The paper's own transfer function is C (sigma I - A)^{-1} B = -G_j; this
 * oracle returns G_j = C (A - sigma_j I)^{-1} B and leaves the sign to the
 * caller, the same convention the GPU path uses.
 *
 * How: Gaussian elimination with partial pivoting on the complex matrix
 * A - sigma_j I, applied to the right-hand sides as it goes, then column
 * oriented back substitution.  This is the textbook definition of the
 * solution; the paper's RQ-based method reaches the same X_j up to rounding
 * because it is a direct method with no approximation.
 *
 *  - pivot: the first row of largest modulus |z| = hypot(Re z, Im z) in the
 *    current column;
 *  - a multiplier that is exactly zero skips its row update (for an
 *    m-Hessenberg matrix this is what keeps the cost at O(n^2 m));
 *  - a zero pivot marks the shift SINGULAR (status 1) and leaves NaNs in its
 *    outputs; other shifts are unaffected.
 *
 * A second entry point, oracle_solve_rhs, solves op(A - sigma_j I) X_j = F_j
 * with a right-hand side block F_j of its own for every shift and op either
 * the identity or the transpose (not the conjugate transpose).  These are the
 * two families of systems Section 3.3 needs for the interpolation method of
 * Section 1: (A - sigma I) x = B b_hat with a per-shift direction b_hat, and
 * the transposed systems (A - sigma I)^T x = C^T c_hat.  The same elimination
 * runs on the explicitly formed matrix op(A) - sigma I.
 *
 * All matrices are column-major double precision; complex arrays are
 * interleaved (re, im) pairs, i.e. C99 `double complex`.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

static double zabs(zc z) { return hypot(creal(z), cimag(z)); }

/* One shift: op(A) - sigma I is eliminated with the n x m right-hand side F0
 * (complex, ld ldf) or, if F0 is NULL, the real B (ld ldb).  Returns 0 on
 * success, 1 if a pivot was exactly zero, -1 if the work arrays could not be
 * allocated.  The solution goes to X (ld ldx). */
static int solve_one(int64_t n, int64_t m, const double *A, int64_t lda, int trans,
                     const double *B, int64_t ldb, const zc *F0, int64_t ldf,
                     zc sigma, zc *X, int64_t ldx)
{
    zc *M = (zc *)malloc(sizeof(zc) * (size_t)n * (size_t)n);
    zc *F = (zc *)malloc(sizeof(zc) * (size_t)n * (size_t)(m > 0 ? m : 1));
    if (!M || !F) { free(M); free(F); return -1; }

    /* M = op(A) - sigma I, F = B or F0 */
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) M[i + j * n] = trans ? A[j + i * lda] : A[i + j * lda];
        M[j + j * n] -= sigma;
    }
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = 0; i < n; ++i) F[i + c * n] = F0 ? F0[i + c * ldf] : B[i + c * ldb];

    int status = 0;
    for (int64_t k = 0; k < n; ++k) {
        /* partial pivoting: first index of largest modulus */
        int64_t r = k;
        double best = zabs(M[k + k * n]);
        for (int64_t i = k + 1; i < n; ++i) {
            double v = zabs(M[i + k * n]);
            if (v > best) { best = v; r = i; }
        }
        if (best == 0.0) { status = 1; break; }
        if (r != k) {
            for (int64_t j = k; j < n; ++j) {
                zc t = M[k + j * n]; M[k + j * n] = M[r + j * n]; M[r + j * n] = t;
            }
            for (int64_t c = 0; c < m; ++c) {
                zc t = F[k + c * n]; F[k + c * n] = F[r + c * n]; F[r + c * n] = t;
            }
        }
        zc piv = M[k + k * n];
        /* multipliers l_i = M(i,k) / M(k,k); remember the last nonzero one */
        int64_t last = k;
        for (int64_t i = k + 1; i < n; ++i) {
            if (M[i + k * n] != 0.0) {
                M[i + k * n] /= piv;
                last = i;
            }
        }
        if (last == k) continue;
        /* trailing update M(i, j) -= l_i M(k, j) and F(i, :) -= l_i F(k, :) */
        for (int64_t j = k + 1; j < n; ++j) {
            zc mkj = M[k + j * n];
            if (mkj == 0.0) continue;
            for (int64_t i = k + 1; i <= last; ++i) M[i + j * n] -= M[i + k * n] * mkj;
        }
        for (int64_t c = 0; c < m; ++c) {
            zc fk = F[k + c * n];
            if (fk == 0.0) continue;
            for (int64_t i = k + 1; i <= last; ++i) F[i + c * n] -= M[i + k * n] * fk;
        }
    }

    if (status != 0) {
        for (int64_t c = 0; c < m; ++c)
            for (int64_t i = 0; i < n; ++i) X[i + c * ldx] = NAN + NAN * I;
        free(M); free(F);
        return status;
    }

    /* column oriented back substitution with the upper triangle of M */
    for (int64_t c = 0; c < m; ++c) {
        zc *f = F + c * n;
        for (int64_t k = n - 1; k >= 0; --k) {
            zc xk = f[k] / M[k + k * n];
            f[k] = xk;
            if (xk == 0.0) continue;
            for (int64_t i = 0; i < k; ++i) f[i] -= M[i + k * n] * xk;
        }
        for (int64_t i = 0; i < n; ++i) X[i + c * ldx] = f[i];
    }

    free(M); free(F);
    return 0;
}

/*
 * Solve all s shifts with the shared right-hand side B.  X is n x (s*m) with
 * X(:, j*m:(j+1)*m) = X_j, G is p x (s*m) likewise (G_j = C X_j; NaN for a
 * singular shift); status (length s) is per shift.  nthreads <= 0 uses the
 * OpenMP default.  Returns 0, or -1 if any shift ran out of memory.
 */
int oracle_solve(int64_t n, int64_t m, int64_t p,
                 const double *A, int64_t lda,
                 const double *B, int64_t ldb,
                 const double *C, int64_t ldc,
                 int64_t s, const double *shifts_ri,
                 double *X_ri, int64_t ldx,
                 double *G_ri, int64_t ldg,
                 int32_t *status, int nthreads)
{
    const zc *shifts = (const zc *)shifts_ri;
    zc *X = (zc *)X_ri;
    zc *G = (zc *)G_ri;
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(min : rc)
    for (int64_t j = 0; j < s; ++j) {
        zc *Xj = X + j * m * ldx, *Gj = G + j * m * ldg;
        int st = solve_one(n, m, A, lda, 0, B, ldb, NULL, 0, shifts[j], Xj, ldx);
        status[j] = st < 0 ? -1 : st;
        if (st < 0) rc = -1;
        /* G_j = C X_j (NaN columns stay NaN) */
        for (int64_t c = 0; c < m; ++c)
            for (int64_t i = 0; i < p; ++i) {
                zc acc = 0.0;
                for (int64_t k = 0; k < n; ++k) acc += C[i + k * ldc] * Xj[k + c * ldx];
                Gj[i + c * ldg] = acc;
            }
    }
    return rc;
}

/*
 * Per-shift right-hand sides: op(A - sigma_j I) X_j = F_j for j = 0..s-1,
 * with op the identity (trans = 0) or the transpose (trans = 1).  F is
 * n x (s*r) complex with F(:, j*r:(j+1)*r) = F_j (ld ldf); X likewise (ld
 * ldx).  status as for oracle_solve.
 */
int oracle_solve_rhs(int64_t n, const double *A, int64_t lda, int trans,
                     int64_t s, const double *shifts_ri, int64_t r,
                     const double *F_ri, int64_t ldf,
                     double *X_ri, int64_t ldx,
                     int32_t *status, int nthreads)
{
    const zc *shifts = (const zc *)shifts_ri;
    const zc *F = (const zc *)F_ri;
    zc *X = (zc *)X_ri;
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(min : rc)
    for (int64_t j = 0; j < s; ++j) {
        int st = solve_one(n, r, A, lda, trans != 0, NULL, 0, F + j * r * ldf, ldf, shifts[j],
                           X + j * r * ldx, ldx);
        status[j] = st < 0 ? -1 : st;
        if (st < 0) rc = -1;
    }
    return rc;
}

/* Number of threads an OpenMP parallel region would use here. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
