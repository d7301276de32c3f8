/*
 * Oracle for sigma_min(C - z I) on a grid of points z.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it is built and run by the tests, by the smoke check and
 * by the CPU-baseline leg of the benchmark.  It shares no code with the HIP
 * path.
 *
 * What it computes (paper, Sec. 1, eqs. (defSquare)/(defSquareSVD)): the
 * epsilon-pseudospectrum is the set of z with sigma_min(C - zI) < epsilon,
 * where for a rectangular C (m >= n) the identity is the m x n matrix
 * [I_n; 0].  The oracle is that definition written out: form A = C - z I and
 * take its smallest singular value, by two independent plain methods.
 *
 *  O1  dense one-sided (Hestenes) Jacobi SVD of A.  Published method:
 *      Hestenes (1958); the convergence test and the 2x2 rotation follow
 *      Demmel & Veselic (1992).  Cost O(sweeps * m n^2) per point.
 *
 *  O2  banded inputs (C with lower bandwidth kl and upper bandwidth ku):
 *      Givens QR of A to an upper band R of width kl + ku, Givens bulge
 *      chasing of R to upper bidiagonal form (the band reduction of
 *      Golub & Van Loan, Matrix Computations, Sec. 8.6 / Schwarz's band
 *      reduction), removal of the phases, and Sturm-count bisection on the
 *      Golub-Kahan tridiagonal [0 B; B^T 0] (Kahan's bisection).  Every step
 *      is a unitary transformation, so the result is backward stable;
 *      cost O((kl+ku) n^2) per point.
 *
 * Complex numbers are stored as interleaved (re, im) doubles; dense matrices
 * are column-major with a leading dimension; band storage is row-major,
 * band[i * (kl + ku + 1) + (j - i + kl)] = C[i][j].
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

/* 2-norm of a complex vector with scaling against overflow/underflow
 * (the classical scaled sum of squares). */
static double znrm2(const zc* x, int64_t m)
{
    double scale = 0.0, ssq = 1.0;
    for (int64_t i = 0; i < m; ++i) {
        double parts[2] = {creal(x[i]), cimag(x[i])};
        for (int k = 0; k < 2; ++k) {
            double v = fabs(parts[k]);
            if (v == 0.0) continue;
            if (scale < v) {
                ssq = 1.0 + ssq * (scale / v) * (scale / v);
                scale = v;
            } else {
                ssq += (v / scale) * (v / scale);
            }
        }
    }
    return scale * sqrt(ssq);
}

/* One Jacobi rotation of the column pair (p, q) given the Gram entries
 * a = ||A_p||^2, b = ||A_q||^2, c = A_p^* A_q with |c| > 0.
 * The phase of c is moved onto column q so that the pair's Gram matrix is
 * real, then the real symmetric 2x2 Jacobi rotation with the smaller angle
 * annihilates the off-diagonal.  Afterwards ||A_p||^2 = a - t|c| and
 * ||A_q||^2 = b + t|c| in exact arithmetic. */
static void jacobi_rotate(zc* ap, zc* aq, int64_t m, double a, double b, zc c, double* t_out)
{
    double ca = cabs(c);
    zc ph = conj(c) / ca;                 /* e^{-i arg c} */
    double zeta = (b - a) / (2.0 * ca);
    double sgn = (zeta >= 0.0) ? 1.0 : -1.0;
    double t = sgn / (fabs(zeta) + hypot(1.0, zeta));
    double cs = 1.0 / sqrt(1.0 + t * t);
    double sn = t * cs;
    for (int64_t i = 0; i < m; ++i) {
        zc x = ap[i];
        zc y = aq[i] * ph;
        ap[i] = cs * x - sn * y;
        aq[i] = sn * x + cs * y;
    }
    if (t_out) *t_out = t;
}

/* Exported single rotation (c given as its real and imaginary parts). */
void oracle_jacobi_rotate(double* ap, double* aq, int64_t m, double a, double b,
                          double cr, double ci, double* t_out)
{
    jacobi_rotate((zc*)ap, (zc*)aq, m, a, b, cr + I * ci, t_out);
}

/*
 * O1: one-sided Jacobi on the columns of A (m x n, column-major, lda).
 * Sweeps visit the pairs p < q in cyclic-by-row order; a pair is rotated
 * when |A_p^* A_q| > m * eps * ||A_p|| ||A_q||.  The iteration stops after
 * a sweep with no rotation.  On return sv[j] = ||A_j||_2 (unsorted).
 * Returns the number of sweeps used, or -1 if max_sweeps passed without
 * convergence (sv is still filled).
 */
int oracle_jacobi_columns(zc* A, int64_t m, int64_t n, int64_t lda, double* sv, int max_sweeps)
{
    const double tol = (double)m * DBL_EPSILON;
    int converged = 0, sweep;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        int64_t rotations = 0;
        for (int64_t p = 0; p + 1 < n; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                zc* ap = A + p * lda;
                zc* aq = A + q * lda;
                double a = 0.0, b = 0.0;
                zc c = 0.0;
                for (int64_t i = 0; i < m; ++i) {
                    a += creal(ap[i]) * creal(ap[i]) + cimag(ap[i]) * cimag(ap[i]);
                    b += creal(aq[i]) * creal(aq[i]) + cimag(aq[i]) * cimag(aq[i]);
                    c += conj(ap[i]) * aq[i];
                }
                double ca = cabs(c);
                if (ca == 0.0 || ca <= tol * sqrt(a) * sqrt(b)) continue;
                ++rotations;
                jacobi_rotate(ap, aq, m, a, b, c, NULL);
            }
        }
        if (rotations == 0) { converged = 1; break; }
    }
    for (int64_t j = 0; j < n; ++j) sv[j] = znrm2(A + j * lda, m);
    return converged ? sweep + 1 : -1;
}

static int cmp_desc(const void* x, const void* y)
{
    double a = *(const double*)x, b = *(const double*)y;
    return (a < b) - (a > b);
}

/* All singular values (descending) of a dense m x n complex matrix by O1. */
int oracle_singular_values_dense(const double* A_in, int64_t m, int64_t n, int64_t lda,
                                 double* sv, int max_sweeps)
{
    zc* A = (zc*)malloc(sizeof(zc) * (size_t)(m * n));
    if (!A) return -2;
    for (int64_t j = 0; j < n; ++j)
        memcpy(A + j * m, (const zc*)A_in + j * lda, sizeof(zc) * (size_t)m);
    int s = oracle_jacobi_columns(A, m, n, m, sv, max_sweeps);
    qsort(sv, (size_t)n, sizeof(double), cmp_desc);
    free(A);
    return s;
}

/*
 * O1 over a list of points: sigma[k] = sigma_min(C - z_k I_{m x n}),
 * sweeps[k] = sweeps used (-1 when the cap was hit).  One point per thread.
 * Returns 0, or -2 if memory ran out.
 */
int oracle_sigma_min_dense(const double* C_in, int64_t m, int64_t n, int64_t ldc,
                           const double* zre, const double* zim, int64_t npts,
                           int max_sweeps, double* sigma, int32_t* sweeps)
{
    const zc* C = (const zc*)C_in;
    int err = 0;
#pragma omp parallel
    {
        zc* A = (zc*)malloc(sizeof(zc) * (size_t)(m * n));
        double* sv = (double*)malloc(sizeof(double) * (size_t)n);
        if (!A || !sv) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < npts; ++k) {
            if (!A || !sv) continue;
            zc z = zre[k] + I * zim[k];
            for (int64_t j = 0; j < n; ++j) {
                memcpy(A + j * m, C + j * ldc, sizeof(zc) * (size_t)m);
                A[j * m + j] -= z;
            }
            int s = oracle_jacobi_columns(A, m, n, m, sv, max_sweeps);
            double mn = INFINITY;
            for (int64_t j = 0; j < n; ++j) mn = sv[j] < mn ? sv[j] : mn;
            sigma[k] = mn;
            if (sweeps) sweeps[k] = s;
        }
        free(A);
        free(sv);
    }
    return err;
}

/* ------------------------------------------------------------------ O2 -- */

/* Complex Givens rotation G = [c s; -conj(s) c], c real, with
 * G [f; g] = [r; 0]. */
static void zgivens(zc f, zc g, double* c, zc* s)
{
    double af = cabs(f), ag = cabs(g);
    if (ag == 0.0) { *c = 1.0; *s = 0.0; return; }
    if (af == 0.0) { *c = 0.0; *s = conj(g) / ag; return; }
    double rho = hypot(af, ag);
    *c = af / rho;
    *s = (f / af) * conj(g) / rho;
}

/* Rows x, y <- G [x; y] for G = [c s; -conj(s) c]. */
static inline void rot_rows(zc* x, zc* y, double c, zc s)
{
    zc a = *x, b = *y;
    *x = c * a + s * b;
    *y = -conj(s) * a + c * b;
}

/* Sturm count: number of eigenvalues < x of the symmetric tridiagonal
 * matrix with zero diagonal and off-diagonal e[0..len-2] (order len). */
static int64_t sturm_count(const double* e, int64_t len, double x)
{
    int64_t cnt = 0;
    double q = -x;
    const double tiny = DBL_MIN / DBL_EPSILON;
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++cnt;
    for (int64_t k = 1; k < len; ++k) {
        q = -x - (e[k - 1] * e[k - 1]) / q;
        if (q == 0.0) q = -tiny;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

/* k-th smallest singular value (k = 1..n) of the real upper bidiagonal
 * matrix with diagonal d[0..n-1] >= 0 and superdiagonal f[0..n-2] >= 0, by
 * bisection on the Golub-Kahan tridiagonal, whose eigenvalues are +-sigma_i
 * and whose off-diagonal is d0, f0, d1, f1, ..., d_{n-1}. */
static double bidiag_kth_sigma(const double* d, const double* f, int64_t n, int64_t k, double* work)
{
    int64_t len = 2 * n;
    double bound = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        work[2 * i] = d[i];
        if (i + 1 < n) work[2 * i + 1] = f[i];
    }
    for (int64_t i = 0; i + 1 < len; ++i) {
        double left = (i > 0) ? work[i - 1] : 0.0;
        double v = left + work[i];
        if (v > bound) bound = v;
    }
    if (len >= 2 && work[len - 2] > bound) bound = work[len - 2];
    double lo = 0.0, hi = bound * (1.0 + 4.0 * DBL_EPSILON) + DBL_MIN;
    /* sigma_k is the (n + k)-th smallest eigenvalue: the smallest x with
     * count(x) >= n + k is just above it. */
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(work, len, mid) >= n + k) hi = mid; else lo = mid;
        if (hi - lo <= 2.0 * DBL_EPSILON * hi) break;
    }
    return 0.5 * (lo + hi);
}

/*
 * Reduce A = C - z I_{m x n} (band storage, see header) to a real upper
 * bidiagonal matrix with the same singular values.  d, f receive the
 * absolute values of the diagonal and superdiagonal.  Returns 0 or -2.
 */
static int banded_to_bidiag(const zc* band, int64_t m, int64_t n, int kl, int ku, zc z,
                            double* d, double* f)
{
    const int64_t wq = 2 * kl + ku + 1;  /* QR window: columns [i-kl, i+kl+ku] */
    zc* X = (zc*)calloc((size_t)(m * wq), sizeof(zc));
    if (!X) return -2;
#define XQ(i, c) X[(i) * wq + ((c) - (i) + kl)]
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = i - kl; j <= i + ku; ++j) {
            if (j < 0 || j >= n) continue;
            XQ(i, j) = band[i * (kl + ku + 1) + (j - i + kl)];
        }
        if (i < n) XQ(i, i) -= z;
    }
    /* Givens QR, column by column: zero the kl entries below the diagonal. */
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = j + 1; i < m && i <= j + kl; ++i) {
            double c; zc s;
            zgivens(XQ(j, j), XQ(i, j), &c, &s);
            int64_t cend = j + kl + ku;
            if (cend > n - 1) cend = n - 1;
            for (int64_t col = j; col <= cend; ++col) rot_rows(&XQ(j, col), &XQ(i, col), c, s);
            XQ(i, j) = 0.0;
        }
    }
    /* R: n x n upper band of width b.  Chasing window: columns [i-1, i+b+1]. */
    const int b = kl + ku;
    const int64_t wr = b + 3;
    zc* R = (zc*)calloc((size_t)(n * wr), sizeof(zc));
    if (!R) { free(X); return -2; }
#define RR(i, c) R[(i) * wr + ((c) - (i) + 1)]
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = i; c <= i + b && c < n; ++c) RR(i, c) = XQ(i, c);
    free(X);
#undef XQ
    /* Eliminate the outermost superdiagonal d = b, b-1, ..., 2 one entry at
     * a time; each column rotation leaves a bulge below the diagonal which
     * is chased down and out of the matrix. */
    for (int dd = b; dd >= 2; --dd) {
        for (int64_t i = 0; i + dd <= n - 1; ++i) {
            /* column rotation on (i+dd-1, i+dd) zeroing R[i][i+dd] */
            int64_t c1 = i + dd - 1, c2 = i + dd;
            {
                double c; zc s;
                /* For row vector [x y], choose G so [x y] G^* ... : use the
                 * conjugated Givens on the transposed pair. */
                zgivens(conj(RR(i, c1)), conj(RR(i, c2)), &c, &s);
                /* columns: [col1 col2] <- [col1 col2] G^H with G from the
                 * conjugated entries; row i becomes [conj(r), 0]. */
                int64_t r0 = i, r1 = c2;
                for (int64_t r = r0; r <= r1 && r < n; ++r) {
                    zc a = RR(r, c1), bb = RR(r, c2);
                    RR(r, c1) = c * a + conj(s) * bb;
                    RR(r, c2) = -s * a + c * bb;
                }
                RR(i, c2) = 0.0;
            }
            int64_t j = i + dd; /* bulge at (j, j-1) */
            while (1) {
                /* row rotation on (j-1, j) zeroing R[j][j-1] */
                double c; zc s;
                zgivens(RR(j - 1, j - 1), RR(j, j - 1), &c, &s);
                int64_t cend = j + dd;
                if (cend > n - 1) cend = n - 1;
                for (int64_t col = j - 1; col <= cend; ++col) rot_rows(&RR(j - 1, col), &RR(j, col), c, s);
                RR(j, j - 1) = 0.0;
                if (j + dd > n - 1) break;
                /* column rotation on (j+dd-1, j+dd) zeroing R[j-1][j+dd] */
                int64_t k1 = j + dd - 1, k2 = j + dd;
                zgivens(conj(RR(j - 1, k1)), conj(RR(j - 1, k2)), &c, &s);
                int64_t rend = k2;
                if (rend > n - 1) rend = n - 1;
                for (int64_t r = j - 1; r <= rend; ++r) {
                    zc a = RR(r, k1), bb = RR(r, k2);
                    RR(r, k1) = c * a + conj(s) * bb;
                    RR(r, k2) = -s * a + c * bb;
                }
                RR(j - 1, k2) = 0.0;
                j = k2;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        d[i] = cabs(RR(i, i));
        if (i + 1 < n) f[i] = cabs(RR(i, i + 1));
    }
#undef RR
    free(R);
    return 0;
}

/*
 * O2: the kk smallest singular values (ascending) of A = C - z I_{m x n}
 * for a banded C.  Returns 0, -1 for bad arguments, -2 if memory ran out.
 */
int oracle_banded_smallest(const double* band_in, int64_t m, int64_t n, int kl, int ku,
                           double zr, double zi, int64_t kk, double* out)
{
    if (m < n || n < 1 || kl < 0 || ku < 0 || kk < 1 || kk > n) return -1;
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    double* f = (double*)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    double* w = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    if (!d || !f || !w) { free(d); free(f); free(w); return -2; }
    int rc = banded_to_bidiag((const zc*)band_in, m, n, kl, ku, zr + I * zi, d, f);
    if (rc == 0)
        for (int64_t k = 1; k <= kk; ++k) out[k - 1] = bidiag_kth_sigma(d, f, n, k, w);
    free(d); free(f); free(w);
    return rc;
}

/* O2 over a list of points (one point per thread). */
int oracle_sigma_min_banded(const double* band_in, int64_t m, int64_t n, int kl, int ku,
                            const double* zre, const double* zim, int64_t npts, double* sigma)
{
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < npts; ++k) {
        int rc = oracle_banded_smallest(band_in, m, n, kl, ku, zre[k], zim[k], 1, sigma + k);
        if (rc != 0) {
#pragma omp atomic write
            err = rc;
        }
    }
    return err;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
