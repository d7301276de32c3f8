/*
 * ps_debug.h - test hooks of the pseudospectra library (not needed by
 * applications).  They run single building blocks of the method on the
 * device so that tests can compare each against a plain reference.
 */
#ifndef PS_DEBUG_H
#define PS_DEBUG_H
#include "ps.h"
#ifdef __cplusplus
extern "C" {
#endif

/* Y = C(z) X (herm = 0; X n x w, Y m x w) or Y = C(z)^* X (herm = 1; X m x w,
 * Y n x w), with C(z) = C - z [I_n; 0]; host column-major complex arrays
 * (ld = rows).  This is the operator apply of LOBPCG-SVD (supplement,
 * Alg. SM1.1) on the matrix cores (dense) or CSR kernel (sparse).  w <= 64.
 * Errors: PS_EINVAL (NULL pointers, w out of range), PS_EDEVICE. */
ps_status ps_debug_apply(ps_matrix* h, int32_t herm, double z_re, double z_im, const double* X, int32_t w,
                         double* Y);

/* Build the dense base preconditioner F (F^* F = N(z) + delta I, eq.
 * (twolevel) with K = F^* F) at z in tile slot 0 and copy F^{-1} (n x n,
 * column-major, host) out; gamma receives the ||F^{-1}||_2 estimate.
 * Errors: PS_EUNSUPPORTED if the handle has no dense preconditioner. */
ps_status ps_debug_precond(ps_matrix* h, double z_re, double z_im, double* Finv, double* gamma);

/* Two-level preconditioner (eq. (twolevel), Lemma 3.1): builds a
 * regularised base site K = N(z_dag) + d I at z_dag, runs the projection
 * LOBPCG-SVD on Mbar(z) = C(z) F^{-1} (Sec. 3.2) at z from a seeded random
 * block, forms Ebar = F^{-1} Xbar (n x r, host, column-major) and
 * Lambda_bar = Sigma_bar^2 (r values), and applies
 * Y = K_Ebar^{-1} W = F^{-1} F^{-*} W + Ebar Lambda_bar^{-1} Ebar^* W to the
 * n x r host block W.  iters (nullable) receives the LOBPCG iterations.
 * Errors: PS_EUNSUPPORTED without precond = 2, PS_EINVAL, PS_EDEVICE. */
ps_status ps_debug_twolevel(ps_matrix* h, double zd_re, double zd_im, double z_re, double z_im, const double* W,
                            double* Y, double* Ebar, double* lam, int32_t* iters);

/* Regularisation shift d and gamma = ||F^{-1}||_2 of the site built by the
 * last ps_debug_twolevel call. */
ps_status ps_debug_site(ps_matrix* h, double* dreg, double* gamma);

/* Build the sparse base site at z (square CSR handle with a
 * preconditioner): K = F^* F the incomplete Cholesky factorization of
 * N(z) + alpha I (Sec. 3 and 4), and return Y = F^{-1} X (trans 0) or
 * Y = F^{-*} X (trans 1) for host column-major n x w X (w <= 64), with the
 * shift alpha used.  Errors: PS_EINVAL, PS_EUNSUPPORTED (dense handle or
 * no preconditioner), PS_EDEVICE. */
ps_status ps_debug_sparse_site(ps_matrix* h, double z_re, double z_im, int32_t trans, const double* X, int32_t w,
                               double* Y, double* alpha);

/* One inertia test (the certificate of a clustered refinement): pd = 1 when
 * every pivot of the Cholesky factorization of N(z) - mu I is positive,
 * i.e. sigma_min(C - z I)^2 > mu; dense handles factor N(z) - mu I densely,
 * CSR handles whose N = C^* C has bandwidth <= 63 by a band Cholesky.
 * Errors: PS_EUNSUPPORTED (no preconditioner, or a CSR matrix without a
 * narrow band), PS_EDEVICE. */
ps_status ps_debug_inertia(ps_matrix* h, double z_re, double z_im, double mu, int32_t* pd);

/* The recycled singular store of `tile` as the last ps_eval left it (Sec.
 * 2.2): its dimension k, the orthonormal basis V (n x k_max), W1 = C V
 * (m x k_max), W3 = C^* C V and W4 = C^* S V (n x k_max), and the cached R
 * factors R_A of [W1 W2] (2k_max square) and R_res of [W3 W4 W5 W6]
 * (4k_max square); host column-major, the leading k columns valid.
 * Errors: PS_EINVAL (tile out of range), PS_EDEVICE. */
ps_status ps_debug_store(ps_matrix* h, int32_t tile, int32_t* k, double* V, double* W1, double* W3, double* W4,
                         double* RA, double* Rres);

/* The Ritz stage of recySing (Alg. 1 in its cached-R form) on that store at
 * z: the k Ritz singular values xi (ascending), the residual norms
 * ||T(z) V g_j - xi_j^2 V g_j|| of eq. (fastresidual) and the right vectors
 * G (k_max x k, column-major).  Errors: PS_EINVAL (empty store). */
ps_status ps_debug_ritz(ps_matrix* h, int32_t tile, double z_re, double z_im, double* xi, double* res, double* G);

/* The ||C||_2 estimate used in the acceptance tests (power iteration). */
double ps_debug_norm(const ps_matrix* h);

/* Host only (no device call): the traversal plan of an nx x ny grid cut
 * into tx x ty tiles (Sec. 2.3 batch zigzag with band height b, or the
 * Hilbert / Morton orders of Sec. 5.4 for traversal 1 / 2).  order receives
 * the nx*ny point indices (j*nx + i) tile after tile, tile_start the
 * tx*ty + 1 offsets of the tiles in it.  Errors: PS_EINVAL. */
ps_status ps_debug_order(int32_t nx, int32_t ny, int32_t tx, int32_t ty, int32_t b, int32_t traversal,
                         int32_t* order, int32_t* tile_start);

#ifdef __cplusplus
}
#endif
#endif
