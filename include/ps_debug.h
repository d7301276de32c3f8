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

/* The ||C||_2 estimate used in the acceptance tests (power iteration). */
double ps_debug_norm(const ps_matrix* h);

#ifdef __cplusplus
}
#endif
#endif
