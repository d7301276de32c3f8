// Kernel argument blocks and host launchers (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "zdev.h"

// ---- small per-workgroup kernels (k_small.hip) ----------------------------
struct RitzArgs {
    int njobs;
    const int* job_tile;   // per job: tile index
    const int* kdim;       // per tile: current recycled dimension k
    const zd* z;           // per job: grid point
    const double* nrm;     // per job: ||M(z)|| (mode 0) or ||Tbar(z)|| (mode 1)
    const zd* RA; int64_t strideRA; int ldRA;
    const zd* Rres; int64_t strideRres; int ldRres; int nres;
    int nv, ng, max_sweeps, mode;
    double eta;
    double floor_c;        // floor of tolC: floor_c * eps * nrm^2
    double floor_tol;      // a residual accepted on the floor alone must also be
                           // <= floor_tol * xi_0 (0: no such test)
    double eta_abs;        // accept when xi_0 <= eta_abs * normC (upper-bound certificate)
    double normC;
    double* xi; double* res; int ldxi;     // per job nv values
    zd* Gout; int64_t strideG; int ldG;    // per job k x ng right vectors
    uint8_t* accept;
};
struct CholArgs {
    const int* list;       // tile list (NULL: identity)
    const int* cdim;       // per tile dimension (NULL: use c); c = cdim[t] * cmul
    int cmul, c;
    zdd* G; int64_t strideG; int ldG;
    zd* R; int64_t strideR; int ldR;
    int* nzero;            // per tile: pivots treated as zero (NULL: not reported)
};
struct RRArgs {
    const int* list;
    const int* cdim;       // per tile: 2r or 3r
    int r, max_sweeps;
    const zd* R; int64_t strideR; int ldR;
    zd* GX; zd* GP; int64_t strideGX; int ldGX;
    double* xi; int ldxi;
    int* status;
};
struct SvqbArgs {
    const int* list;
    int r, max_sweeps;
    double drop;
    const zd* R; int64_t strideR; int ldR;
    zd* T; int64_t strideT; int ldT;
    uint32_t* mask;
};
struct RotArgs {
    const int* list;
    const int* qdim;       // per tile: number of kept blocks q
    int r;
    const zd* U; int64_t strideU; int ldU;       // q r x r
    const zd* Upp; int64_t strideUpp; int ldUpp; // r x r
    zd* Qt; int64_t strideQt; int ldQt;          // (q+1) r square
};
void launch_ritz(const RitzArgs& a, int kmax, hipStream_t s);
void launch_chol_dd(const CholArgs& a, int nb, hipStream_t s);
void launch_rr_hl(const RRArgs& a, int nb, int cmax, hipStream_t s);
void launch_svqb(const SvqbArgs& a, int nb, hipStream_t s);
void launch_rotations(const RotArgs& a, int nb, int qmax, hipStream_t s);
void small_kernels_init();
int small_kernels_max_lds();
// k_svqb: T = U S^{-1} from the SVD of R (columns of the block already scaled)

// ---- tall-skinny batched kernels (k_ts.hip) --------------------------------
// A "block list" describes a tall matrix made of up to 5 column blocks that
// live in different arrays: block b starts at ptr[b] + tile * stride[b], has
// ld[b] and ncols[b] (or ncols from a per-tile dims array times mul).
#define TS_MAXB 5
struct BlockList {
    int nb;
    const zd* ptr[TS_MAXB];
    int64_t stride[TS_MAXB];
    int64_t ld[TS_MAXB];
    int ncols[TS_MAXB];          // fixed columns, or
    const int* dims[TS_MAXB];    // per-tile columns = dims[tile] * mul[b] (if non-NULL)
    int mul[TS_MAXB];
    int64_t brows[TS_MAXB];      // rows stored in block b (rows beyond read as zero; 0 = all)
    const int* coff[TS_MAXB];    // per-tile first column = coff[tile] * coffmul[b] (if non-NULL)
    int coffmul[TS_MAXB];
    const int* imap[TS_MAXB];    // block b of tile t lives at index imap[b][t] of its array (if
                                 // non-NULL; e.g. a preconditioner site shared by several tiles)
    int64_t rows;                // logical rows of the tall matrix
};
// G = A^* B (double-double accumulation when dd != 0; zdd output) or double
struct GramArgs {
    const int* list; int ntiles;
    BlockList A, B;
    int camax, cbmax;            // max columns (for grid sizing)
    void* out; int64_t strideOut; int ldOut;   // zdd* or zd*
    void* part;                  // workspace for partial sums
    int64_t part_stride;         // per (tile, chunk)
    int chunk_rows;
    int nchunks;
    int dd;
    int hermitian_upper_only;
    int out_dd;                  // dd == 0: write the sums as double-double (low parts zero)
};
void launch_gram(GramArgs& a, hipStream_t s);
size_t gram_part_bytes(int64_t rows, int camax, int cbmax, int ntiles, int dd, int chunk_rows);

// Y = alpha A G + beta Y  (A a block list, G small per tile: ca x cb, ldG)
struct GemmTSArgs {
    const int* list; int ntiles;
    BlockList A;
    const zd* G; int64_t strideG; int ldG;
    const int* cbdims; int cbmul; int cb;     // output columns (per tile or fixed)
    zd* Y; int64_t strideY; int64_t ldY;
    int64_t rows;
    double alpha;         // 1 or -1
    double beta;          // 0 or 1
    int camax, cbmax;
};
void launch_gemm_ts(const GemmTSArgs& a, hipStream_t s);

// column squared norms of a block list, per tile: out[tile*ldo + j]
struct NormArgs {
    const int* list; int ntiles;
    BlockList A;
    int camax;
    double* out; int ldo;
    double* part; int nchunks; int chunk_rows;
};
void launch_colnorm2(NormArgs& a, hipStream_t s);

// elementwise helpers
void launch_copy_cols(const int* list, int ntiles, const zd* src, int64_t sstride, int64_t lds,
                      zd* dst, int64_t dstride, int64_t ldd, int64_t rows, int cols, hipStream_t s);
void launch_scale_cols(const int* list, int ntiles, zd* A, int64_t stride, int64_t lda, int64_t rows,
                       int cols, const double* d, int ldd, int invert, hipStream_t s);
// W = Y - conj(z) X[:n] padded: used for C(z)^* Y = C^* Y - conj(z) S^* Y and
// C(z) X = C X - z S X.  mode 0: Y[:n] -= zc * X[:n]; rows beyond n untouched.
// R = Y - X diag(xi^2)
void launch_tile_dot0(const int* list, int ntiles, const zd* X, int64_t xs, const zd* Y, int64_t ys, int64_t n,
                      zd* out, hipStream_t s);
void launch_job_gamma(int njobs, const int* job_tile, const int* kdim, const zd* G, int64_t sG, int ldG, const zd* H,
                      int64_t sH, int ldH, const zd* z, zd* out, hipStream_t s);
void launch_resid_xi(const int* list, int ntiles, zd* Y, int64_t ystride, int64_t ldy, const zd* X,
                     int64_t xstride, int64_t ldx, const double* xi, int ldxi, int64_t rows, int cols,
                     hipStream_t s);
// fill columns flagged in mask[tile] with seeded random CN(0,1) entries
void launch_randfill(const int* list, int ntiles, zd* A, int64_t stride, int64_t lda, int64_t rows,
                     int cols, const uint32_t* mask, uint64_t seed, hipStream_t s);
void launch_zero(zd* A, int64_t count, hipStream_t s);

// ---- operator applies (k_apply.hip) ----------------------------------------
// Dense: Y[:, blk] = A X[:, blk] for column blocks of width w belonging to
// tiles in list; A m x K column-major.  Split-K partials + reduction with the
// shift epilogue  Y -= zsign * z_tile * S X  (S = [I_n; 0] or S^* = [I_n 0]).
struct DenseApplyArgs {
    const zd* A; int64_t lda; int64_t m, K;
    const int* list; int ntiles;
    const zd* X; int64_t xstride; int64_t ldx;
    zd* Y; int64_t ystride; int64_t ldy;
    int w;                       // columns per tile block
    const zd* z; int conjz;      // shift per tile (NULL: no shift)
    int64_t nshift;              // rows of the identity part (n)
    zd* part; int splitk;
};
void launch_dense_apply(DenseApplyArgs& a, hipStream_t s);
size_t dense_apply_part_bytes(int64_t m, int maxcols, int splitk);

// CSR: Y[:, blk] = A X[:, blk] (+ shift epilogue), A m x K in CSR
struct CsrApplyArgs {
    const int64_t* rowptr; const int32_t* colind; const zd* vals; int64_t m;
    const int* list; int ntiles;
    const zd* X; int64_t xstride; int64_t ldx;
    zd* Y; int64_t ystride; int64_t ldy;
    int w;
    const zd* z; int conjz; int64_t nshift;
};
void launch_csr_apply(const CsrApplyArgs& a, hipStream_t s);

// batched complex GEMM C = alpha op(A) B + beta C on the matrix cores
struct ZgemmArgs {
    const int* list;                 // batch -> tile (NULL: identity)
    int64_t M, N, K;
    const zd* A; int64_t lda, strideA; int opA;   // opA: 0 = A, 1 = A^*
    const zd* B; int64_t ldb, strideB;
    zd* C; int64_t ldc, strideC;
    double alpha, beta;
    int upper;                       // compute only tiles touching the upper triangle
    int tri;                         // 1: A upper triangular, 2: A lower triangular (skip zero blocks)
    int splitk;                      // > 1: K split over workgroups, partials in ws
    zd* ws;                          // splitk * nbatch * M * N partial products
    // column-map mode (gtile != NULL): batch entry b multiplies A[list[b]] by
    // the column blocks of the gcnt[b] tiles gtile[goff[b] ...] (cw columns
    // each, B + tile * strideB, C + tile * strideC), so tiles that share an A
    // are one wide product; N is the largest gcnt[b] * cw
    const int* gtile; const int* goff; const int* gcnt; int cw;
};
void launch_zgemm(const ZgemmArgs& a, int nbatch, hipStream_t s, int fact = 0);

// dense base preconditioner (k_precond.hip)
#define PRE_NB 32
#define PRE_OB 128
void launch_form_normal(const int* list, int nt, const zd* CtC, const zd* C, int64_t ldc, const zd* CH,
                        int64_t n, const zd* zdag, const double* shift, zd* N, int64_t strideN, hipStream_t s);
void launch_chol_step(const int* list, int nt, zd* A, int64_t strideA, int64_t n, int64_t k0, int kb, zd* Dinv,
                      int64_t strideD, zd* Finv, int64_t strideF, double floor_piv, int* notpd, hipStream_t s);
void launch_zero_tiles(const int* list, int nt, zd* A, int64_t stride, int64_t count, hipStream_t s);

// ---- sparse base preconditioner (k_sparse.hip) ------------------------------
// Pattern of P (C - z I) P^T (diagonal always present, columns sorted) with P
// the colour ordering; rows of colour c are [cptr[c], cptr[c+1]).
struct SparsePattern {
    int64_t n = 0, nnz = 0;
    int ncolors = 0;
    const int64_t* cptr = nullptr;                  // host array, ncolors + 1
    const int64_t* rp = nullptr; const int32_t* ci = nullptr;
    // contributions of each entry e of N = C(z)^* C(z): pairs (ca[q], cb[q]),
    // q in [ccp[e], ccp[e + 1]), naming entries of C - z I (see k_sparse.hip)
    const int64_t* ccp = nullptr; const int64_t* ca = nullptr; const int64_t* cb = nullptr;
    const int64_t* diag = nullptr;                  // row -> its diagonal entry
    const int64_t* rpT = nullptr; const int32_t* ciT = nullptr; const int64_t* mapT = nullptr;  // transpose
    const int* perm = nullptr;                      // permuted row -> original row
};
// incomplete Cholesky factors of N(z_site) + alpha_site I for the listed
// sites (notpd[site] set on a non-positive pivot)
void launch_icn(const int* list, int ns, const SparsePattern& sp, const zd* vC, const zd* zsite, const double* alpha,
                zd* lu, int* notpd, hipStream_t s);
// inertia tests of N(z_s) - mu_s I for a narrow-band N (bandwidth b <= 63):
// notpd[s] set when the band Cholesky meets a pivot <= floor_rel
void launch_band_inertia(const int* list, int nt, const zd* zsite, const double* mu, const int64_t* cptr,
                         const int64_t* ca, const int64_t* cb, const zd* vC, int64_t n, int b, zd* W,
                         int64_t wstride, double floor_rel, int* notpd, hipStream_t s);
// Y = F^{-1} X (trans 0) or F^{-*} X (trans 1), K = F^* F the incomplete
// Cholesky factorization of each item's site
void launch_ic_solve(const int* list, int ni, const int* site, const SparsePattern& sp, const zd* lu, int trans,
                     const zd* X, int64_t xs, int64_t ldx, zd* Y, int64_t ys, int64_t ldy, int w, zd* T, int64_t ts,
                     hipStream_t s);
