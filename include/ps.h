/*
 * ps.h - C ABI of the recycled pseudospectra library for AMD Instinct MI355X
 * (gfx950).
 *
 * The library evaluates sigma_min(C - z I) at every point z of a Cartesian
 * grid, for a complex matrix C (m x n, m >= n, dense or CSR), where I is the
 * m x n matrix [I_n; 0] (Deng & Xu, "Recycling singular and projection
 * subspaces for pseudospectra computation", Sec. 1, eqs. (defSquare) and
 * (defSquareSVD)).  It reports sigma_min and the membership of each point in
 * the epsilon-pseudospectrum, sigma_min < epsilon (strict), for a list of
 * epsilon levels.
 *
 * The method is the paper's Alg. 5 (psPrecRecy).  A point is first tried
 * against the recycled singular subspace: Ritz singular pairs by the
 * one-step Rayleigh-Ritz-SVD of Sec. 2.2 (Alg. 1, recySing), evaluated from
 * cached R factors of the subspace's auxiliary blocks, and the residual test
 * of eq. (tolC).  A rejected point runs a block LOBPCG-SVD (supplement,
 * Alg. SM1.1) and its result enters the subspace by the adaptive update of
 * Alg. 2.  The LOBPCG preconditioner is chosen by ps_params.precond:
 *  - 1 (dense default): base preconditioner K = F^* F = N(z_dag) + delta I,
 *    an exact Cholesky factor at sites z_dag placed by a base-only form of
 *    the rebuild rule (eq. (tauRecycle) with the projection part empty);
 *  - 2 (CSR default): the two-level preconditioner of eq.
 *    (twolevel): an incomplete-Cholesky base of N(z_dag) (CSR) or a
 *    regularised Cholesky base
 *    (dense), plus a projection subspace recycled by Alg. 4 (recyProj) and
 *    eq. (tolTz), refined by LOBPCG-SVD on Mbar(z) = C(z) F^{-1} when the
 *    test fails, and the full rebuild rule of eq. (tauRecycle);
 *  - 0: K = I.
 * Every numerical step runs in HIP kernels on the GPU in complex128.
 *
 * Conventions
 *  - Complex numbers are interleaved (re, im) doubles.  Dense matrices are
 *    column-major with a leading dimension.
 *  - Grid: x_i = re_lo + i (re_hi - re_lo)/(nx - 1), y_j likewise, both
 *    ends included (x_0 = re_lo when nx = 1); point (i, j) has index
 *    j * nx + i in every per-point array.
 *  - Ownership: input arrays are borrowed for the duration of the call (and
 *    copied to the device unless on_device = 1, in which case they must stay
 *    valid and unchanged until ps_destroy).  Handles belong to the library
 *    until the matching *_destroy.  Output arrays are caller-allocated host
 *    memory.
 *  - Errors: negative return values are errors and leave outputs undefined;
 *    PS_WARN_UNCERTIFIED (positive) means every output was written but some
 *    points hit the LOBPCG iteration cap (see flags).
 *  - Threading: a ps_matrix must not be used from two threads at once.
 *    Calls on different handles may run concurrently on different streams.
 */
#ifndef PS_H
#define PS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_matrix ps_matrix; /* device copy of C + recycled stores + preconditioner */
typedef struct ps_gridh ps_gridh;   /* grid points and traversal plan */

typedef enum {
    PS_OK = 0,
    PS_WARN_UNCERTIFIED = 1,
    PS_EINVAL = -1,
    PS_ENOMEM = -2,
    PS_EDEVICE = -3,
    PS_EBREAKDOWN = -4,
    PS_EUNSUPPORTED = -5
} ps_status;

typedef enum { PS_DENSE = 0, PS_CSR = 1 } ps_kind;

/* Number of event-timed kernel classes in ps_stats. */
#define PS_NCLASS 9

/* Input matrix C (m x n, m >= n >= 1). */
typedef struct {
    int32_t kind;           /* PS_DENSE or PS_CSR */
    int64_t m, n;
    const double* dense;    /* PS_DENSE: 2 * ld * n doubles, column-major */
    int64_t ld;             /* PS_DENSE: leading dimension >= m */
    const int64_t* rowptr;  /* PS_CSR: m + 1 entries, rowptr[0] = 0 */
    const int32_t* colind;  /* PS_CSR: nnz column indices, sorted within each row */
    const double* vals;     /* PS_CSR: 2 * nnz doubles */
    int64_t nnz;
    int32_t on_device;      /* 1: the pointers above are device memory */
} ps_matrix_desc;

/* Tunables; ps_default_params fills in the defaults.  Symbols follow the
 * paper (Sec. 4 lists its own values). */
typedef struct {
    int32_t r;          /* singular LOBPCG block size r (default 8) */
    int32_t k_max;      /* cap on the recycled singular dimension p r (default 32) */
    int32_t rbar;       /* projection block size rbar (Sec. 3.2); with the
                           two-level preconditioner it must equal r, because
                           the projection LOBPCG shares the singular one's
                           block layout (default 8) */
    int32_t kbar_max;   /* cap on the recycled projection dimension kbar
                           per preconditioner site, a multiple of rbar,
                           <= 64 (default 64) */
    int32_t max_iters;  /* LOBPCG iteration cap (default 300) */
    int32_t precond;    /* LOBPCG preconditioner (Sec. 3): 0: K = I;
                           1: base preconditioner alone, K = F^* F with F
                           the Cholesky factor of N(z_dag) + delta I, a site
                           serving z while ((1 + g) / (1 - g))^2 <= tau_max,
                           g = ||F^{-1}|| |z - z_dag|;
                           2: the two-level preconditioner of eq. (twolevel)
                           with a recycled projection subspace per site
                           (Alg. 4 and 5), K = F^* F with F the Cholesky
                           factor of N(z_dag) + (reg_base (||C|| + |z_dag|))^2 I,
                           rebuilt by the rule of eq. (tauRecycle);
                           For CSR C, K = L D L^* is instead the
                           incomplete Cholesky factorization (no fill, on
                           the pattern of C^* C in a colour ordering of its
                           graph) of N(z_dag) + alpha I, alpha starting at
                           (reg_base (||C|| + |z_dag|))^2 and raised 4x
                           until every pivot is positive; F = D^{1/2} L^* P.
                           -1 (default): 1 for dense C, 2 for CSR */
    int32_t tiles_x;    /* grid-front partition: tiles along x (0 = auto) */
    int32_t tiles_y;    /* tiles along y (0 = auto) */
    int32_t tile_points;/* auto partition: points per tile (default 80) */
    int32_t tile_mem_gb;/* auto partition: device memory for per-tile state
                           (default 48) */
    int32_t site_mem_gb;/* device memory for preconditioner sites and their
                           staging (dense: explicit inverse factors; sparse:
                           incomplete-Cholesky values and projection
                           stores)
                           (default 128) */
    int32_t batch;      /* b of the batch-zigzag traversal (default 20) */
    int32_t traversal;  /* order of the points inside a tile: 0 batch zigzag
                           (Sec. 2.3, default); 1 Hilbert curve; 2 Morton
                           (Z) order -- the locality-preserving alternatives
                           of Sec. 5.4 */
    int32_t recycle;    /* 1: recycled path; 0: plain per-point LOBPCG from a
                           seeded random start (the comparison solver) */
    double eta;         /* acceptance tolerance of eq. (tolC) (default 1e-6) */
    double eta_svd;     /* LOBPCG convergence tolerance, eq. (tolSVD) (1e-9) */
    double eta_proj;    /* relaxed tolerance of eq. (tolTz) for projection
                           Ritz pairs and the projection LOBPCG (1e-4) */
    double omega;       /* pruning threshold of eq. (omegaCond) (1.6) */
    double tau_min;     /* eq. (tauRecycle): rebuild the base preconditioner
                           when lambda_bar_rbar < tau_min; projection columns
                           with sigma_bar^2 <= tau_min enter the omega test
                           (1e-3) */
    double tau_max;     /* eq. (tauRecycle): a site serves z while
                           (sqrt(lambda_n^dagger) + gamma |z - z_dag|)^2 <=
                           tau_max (30) */
    double zdag_re;     /* first base-preconditioner site; NaN = region centre */
    double zdag_im;
    uint64_t seed;      /* seed of random start blocks */
    double eta_abs;     /* absolute acceptance: a smallest Ritz value xi_1 <=
                           eta_abs ||C||_2 is accepted, because sigma_min lies
                           in [0, xi_1] (Ritz values bound it from above)
                           (default 8e-9; 0 disables; at most 1e-8) */
    double rho_small;   /* refined points whose recycled Ritz value is below
                           rho_small ||M(z)|| run LOBPCG with K = I and build no
                           base preconditioner (default 1e-5) */
    int32_t profile;    /* 1: time the operator-apply and matrix-core GEMM
                           kernels with HIP events (fills the k_* stats) */
    int32_t verbose;    /* 1: progress lines on stderr */
    double tol_abs;     /* certification half-width tau as a fraction of
                           ||C||_2 (default 8e-9): a refinement still running
                           after esc_iters iterations is accepted when
                           N(z) - mu I, mu = (xi - tau)^2 + rounding slack, is
                           positive definite (then xi - tau <= sigma_min <= xi);
                           0 disables.  The test factors N(z) - mu I exactly:
                           dense C, and CSR C whose N has bandwidth <= 63
                           in the natural order (a band Cholesky); other CSR
                           matrices get no certificate */
    int32_t esc_iters;  /* escalation period of slow refinements: the
                           inertia test above, then (dense C) a shifted
                           preconditioner N(z) - (xi - 64 tau)^2 I, else
                           N(z) - (xi - 4096 tau)^2 I, else an exact site at
                           z (default 30; 0 disables) */
    int32_t cert_recycled; /* 1: in a cluster regime, test a recycled Ritz
                           value that failed eq. (tolC) with the inertia test
                           before starting LOBPCG (default 0: on the dense
                           Toeplitz workload half of those tests fail and the
                           sweep is 27% slower) */
    double reg_base;    /* relative regularisation of the base
                           preconditioner (dense with precond = 2, and the
                           starting shift of the sparse incomplete
                           Cholesky), which bounds gamma = ||F^{-1}|| by
                           1 / (reg_base (||C|| + |z_dag|)) so that a site
                           serves a region even near the spectrum (0.02) */
    int32_t lipschitz;  /* 1 (default): after the sweep, points whose value
                           exceeds an upper bound from a finished grid
                           neighbour (the norm of C(z) on the neighbour's
                           singular vector, or the 1-Lipschitz bound) are
                           refined again from a random start */
    int32_t fact_blas;  /* dense base sites and inertia tests: 1 runs the
                           plain products of the blocked Cholesky (the
                           rank-128 trailing Hermitian updates and the F^{-1}
                           block products) as rocBLAS strided-batched
                           ZHERK / ZGEMM; 0 (default) on this library's
                           matrix-core kernels, which are faster on these
                           shapes */
} ps_params;

typedef struct {
    int64_t points;        /* grid points evaluated */
    int64_t accepted;      /* accepted by the recycled Ritz test (tolC) */
    int64_t refined;       /* LOBPCG-SVD refinements (recycling points, and
                              points refined again by the Lipschitz pass) */
    int64_t uncertified;   /* LOBPCG hit max_iters */
    int64_t lobpcg_iters;  /* singular LOBPCG iterations, summed over points */
    int64_t proj_accepted; /* projection Ritz vectors accepted (tolTz) */
    int64_t proj_refined;  /* projection LOBPCG runs */
    int64_t proj_iters;
    int64_t rebuilds;      /* base-preconditioner constructions */
    int64_t mv_M;          /* operator column-applies of C or C^* */
    int64_t sv_F;          /* column solves / applies with F^{-1}, F^{-*} */
    int64_t rounds;        /* scheduler rounds */
    int64_t certified;     /* refinements ended by the inertia test (tol_abs) */
    int64_t lipschitz_redo;/* points refined again by the neighbour pass */
    int64_t guard_rejects; /* points that passed eq. (tolC) above a neighbour bound */
    int64_t cert_tests;    /* inertia tests (Cholesky of N(z) - mu I) run */
    int64_t builds_shared; /* preconditioner sites built for sharing (rebuild rule) */
    int64_t builds_private;/* sites built for one slow refinement (shifted or exact) */
    int64_t ritz_jobs;     /* Ritz extractions from a recycled store (points tested) */
    int64_t store_updates; /* updateRecy calls that appended a block (Alg. 2) */
    int64_t precond_iters; /* LOBPCG iterations that applied K^{-1} != I */
    int64_t repairs;       /* LOBPCG steps whose search space lost rank and was rebuilt */
    int64_t mv_update;     /* operator column-applies made by updateRecy (3 r per
                              singular update with S = [I_n; 0]: C Q, C^* C Q, C^* S Q) */
    int64_t ic_retries;    /* sparse sites refactored with a 4x larger shift after a
                              non-positive incomplete-Cholesky pivot */
    double t_total_ms;     /* wall time of ps_eval */
    double t_ritz_ms, t_lobpcg_ms, t_update_ms, t_precond_ms;
    /* with profile >= 1: event-timed kernel classes (launches, device ms,
     * algorithmic flops and bytes per class).  Class 0: operator applies
     * C X, C^* Y (dense: matrix-core GEMM + split-K reduction; CSR: SpMM);
     * class 1: preconditioner applies K^{-1} W; class 2: Ritz extraction
     * (per-point QR + Jacobi SVD + residual); class 3: matrix-core products
     * at least 64 columns wide inside factorizations (preconditioner sites,
     * inertia tests: the trailing updates and the F^{-1} block columns, on
     * 64 x 64 tiles); class 4: the diagonal-block steps of those
     * factorizations and the forming of N(z); class 8: the narrower
     * products inside factorizations (64 x 32 tiles).  With profile >= 2
     * also class 5: per-tile small dense kernels (Rayleigh-Ritz-SVD,
     * Cholesky of Gram matrices, SVQB, rotations); class 6: tall-skinny
     * Gram, product and norm kernels; class 7: the rest (copies, fills). */
    int64_t k_launches[PS_NCLASS];
    double k_ms[PS_NCLASS];
    double k_flops[PS_NCLASS];
    double k_bytes[PS_NCLASS];
} ps_stats;

/* Per-point flag bits written to `flags`. */
#define PS_FLAG_ACCEPTED 1u     /* sigma from the recycled Ritz value */
#define PS_FLAG_REFINED 2u      /* sigma from LOBPCG-SVD */
#define PS_FLAG_UNCERTIFIED 4u  /* LOBPCG hit the iteration cap */
#define PS_FLAG_PROJ_REFINED 8u /* projection subspace refined here */
#define PS_FLAG_REBUILD 16u     /* base preconditioner rebuilt here */
#define PS_FLAG_CERTIFIED 32u   /* sigma certified by the inertia test */
#define PS_FLAG_LIPSCHITZ 64u   /* refined again after a neighbour-bound violation */

void ps_default_params(ps_params* p);

/* Upload C (Sec. 1: the m x n matrix whose pseudospectra are computed,
 * m >= n, with C(z) = C - z I, eq. (defSquare)), prepare the operators
 * (C and C^*; for dense C with a preconditioner also C^* C) and the empty
 * recycled stores.  desc is read during the call only (unless on_device).
 * hip_stream: the hipStream_t all work is issued on (NULL = default).
 * Errors: PS_EINVAL (m < n, n < 1, bad CSR, NULL pointers, bad params),
 * PS_ENOMEM, PS_EDEVICE; *out is NULL on error. */
ps_status ps_create(const ps_matrix_desc* desc, const ps_params* params, void* hip_stream,
                    ps_matrix** out);

/* The equispaced Cartesian grid of the experiments (Sec. 4) over
 * [re_lo, re_hi] x [im_lo, im_hi] with nx x ny points (ends included), and
 * its traversal plan: tiles of neighbouring points in batch-zigzag order
 * (Sec. 2.3).  Errors: PS_EINVAL (nx < 1, ny < 1, non-finite bounds). */
ps_status ps_grid(double re_lo, double re_hi, double im_lo, double im_hi, int32_t nx,
                  int32_t ny, ps_gridh** out);

/* Evaluate sigma_min(C - z I) on every grid point (eq. (defSquareSVD):
 * the smallest singular value, whose sublevel sets are the
 * epsilon-pseudospectra of eq. (defSquare)), by Alg. 5.
 * sigma:  nx*ny doubles (host), sigma[j*nx+i].
 * member: n_eps*nx*ny bytes (host) or NULL; member[e*nx*ny + p] = sigma[p] < eps[e].
 * flags:  nx*ny bytes (host) or NULL; PS_FLAG_* bits.
 * stats:  or NULL.
 * Each call starts from empty recycled stores, so results do not depend on
 * earlier calls.  Errors: PS_EINVAL, PS_ENOMEM, PS_EDEVICE, PS_EBREAKDOWN. */
ps_status ps_eval(ps_matrix* h, const ps_gridh* g, const double* eps, int32_t n_eps,
                  double* sigma, uint8_t* member, uint8_t* flags, ps_stats* stats);

void ps_grid_destroy(ps_gridh* g);
void ps_destroy(ps_matrix* h);
const char* ps_strerror(ps_status s);

/* Text of the last error raised on this thread (empty if none). */
const char* ps_last_error(void);

/* Operator apply without allocation, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same operation as
 * ps_debug_apply: Y = C(z) X (herm = 0; X n x w, Y m x w) or
 * Y = C(z)^* X (herm = 1; X m x w, Y n x w), C(z) = C - z [I_n; 0], but X
 * and Y are DEVICE column-major complex arrays with leading dimensions ldx,
 * ldy (in complex elements), owned by the caller, and the call only
 * enqueues the work on the handle's stream (Y is valid once that stream has
 * reached this point).  Its workspace (the dense split-K partial products
 * and a small header) is a static 32 MiB device array, one per GPU, set up
 * by ps_create; it calls no hipMalloc / hipFree and no allocating library
 * routine.  Limits: 1 <= w <= 64 and, for dense C, rows(Y) * w * 16 bytes
 * <= 32 MiB - 256.  All calls on one GPU share the array: calls that
 * overlap in time on one GPU (different handles or streams) race and must
 * be serialised by the caller.  Errors: PS_EINVAL (NULL pointers, w, ld or
 * size out of range, non-finite z), PS_EDEVICE. */
ps_status ps_apply_noalloc(ps_matrix* h, int32_t herm, double z_re, double z_im, const double* X,
                           int64_t ldx, int32_t w, double* Y, int64_t ldy);

#ifdef __cplusplus
}
#endif
#endif /* PS_H */
