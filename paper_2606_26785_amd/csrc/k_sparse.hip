// Sparse base preconditioner for CSR C (square): an incomplete LU
// factorisation without fill, F = L U ~ P (C - z_dag I) P^T, of the matrix
// reordered by a greedy colouring of its adjacency graph (rows of one colour
// share no edge), so that K = (F P)^* (F P) ~ N(z_dag) is the base
// preconditioner of eq. (twolevel) (the paper uses an incomplete Cholesky
// factor of N(z_dag), Sec. 4; here the incomplete LU of C - z_dag I).  Rows of
// one colour depend only on rows of earlier colours in L and of later colours
// in U, so the factorisation and every triangular solve run one launch per
// colour, each over all rows of the colour and all right-hand sides.
#include "zdev.h"
#include "kernels.h"

#define NT 256

// lu[site][e] = C entry (src[e] >= 0) minus z on the diagonal
__global__ void k_ilu_form(const int* list, const int64_t* rp, const int32_t* ci, const int64_t* src, const zd* vC,
                           const zd* zsite, int64_t nrows, int64_t nnz, zd* lu)
{
    const int s = list[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= nnz) return;
    zd v = src[e] >= 0 ? vC[src[e]] : zmake(0.0, 0.0);
    lu[(size_t)s * nnz + e] = v;
    (void)rp; (void)ci; (void)zsite; (void)nrows;
}
__global__ void k_ilu_shift(const int* list, const int64_t* diag, const zd* zsite, int64_t nrows, int64_t nnz, zd* lu)
{
    const int s = list[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= nrows) return;
    zd* p = lu + (size_t)s * nnz + diag[i];
    *p = zsub(*p, zsite[s]);
}

// rows [r0, r1) (one colour) of each listed site: ILU(0) in the IKJ order.
// For each k < i in row i: l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for
// the j > k of row i that row k also holds.  A pivot below 1e-12 times the
// row's 2-norm is replaced by that size with the pivot's phase and counted.
__global__ void k_ilu_color(const int* list, const int64_t* rp, const int32_t* ci, const int64_t* diag, int64_t r0,
                            int64_t r1, int64_t nnz, zd* lu, int* nfloor)
{
    const int s = list[blockIdx.y];
    const int64_t i = r0 + (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= r1) return;
    zd* a = lu + (size_t)s * nnz;
    const int64_t b = rp[i], e = rp[i + 1];
    double rn = 0.0;
    for (int64_t p = b; p < e; ++p) rn += zabs2(a[p]);
    rn = sqrt(rn);
    for (int64_t p = b; p < e; ++p) {
        const int32_t k = ci[p];
        if (k >= i) break;
        const zd ukk = a[diag[k]];
        const double d2 = zabs2(ukk);
        const zd l = d2 > 0.0 ? zscale(zcmul(ukk, a[p]), 1.0 / d2) : zmake(0.0, 0.0);   // a_ik / u_kk
        a[p] = l;
        // u_kj for the columns j > k of row i, merged with row k (both sorted)
        int64_t q = diag[k] + 1;
        const int64_t qe = rp[k + 1];
        for (int64_t t = p + 1; t < e && q < qe; ++t) {
            const int32_t j = ci[t];
            while (q < qe && ci[q] < j) ++q;
            if (q < qe && ci[q] == j) a[t] = zsub(a[t], zmul(l, a[q]));
        }
    }
    zd* d = a + diag[i];
    const double floor_v = 1e-12 * rn;
    const double ad = sqrt(zabs2(*d));
    if (!(ad >= floor_v) || ad == 0.0) {
        *d = ad > 0.0 ? zscale(*d, floor_v / ad) : zmake(floor_v > 0.0 ? floor_v : 1e-300, 0.0);
        atomicAdd(nfloor, 1);
    }
}

// One colour of a triangular solve, in place on X (n x w per item, ld ldx):
// x_i = (x_i - sum over the part's off-diagonal entries val_ij x_j) / d_i.
// part 0: strict lower entries of (rp, ci), unit diagonal (L);
// part 1: strict upper entries, diagonal at diag[i] (U);
// with a transposed pattern (rpT, ciT, mapT: entry of the transpose -> entry
// of lu) and conj = 1 the same parts give L^* (part 1 of the transpose, unit)
// and U^* (part 0 of the transpose, conjugated diagonal).
struct SpSolveArgs {
    const int* list;        // items (tiles or sites)
    const int* site;        // per item: its site (NULL: the item is the site)
    const int64_t* rp; const int32_t* ci; const int64_t* map;   // map: NULL for lu's own pattern
    const int64_t* diag;    // per row: diagonal entry of lu
    const zd* lu; int64_t nnz;
    zd* X; int64_t xs; int64_t ldx; int w;
    int part;               // 0 lower, 1 upper
    int unit;               // 1: unit diagonal
    int conj;               // 1: conjugate the values
    int64_t r0, r1;         // rows of this colour
};
// one thread per (row of the colour, group of up to TRSV_CW columns): the
// row's entries are loaded once and used for every column of the group
#define TRSV_CW 8
__global__ void k_sptrsv_color(SpSolveArgs a)
{
    const int item = a.list[blockIdx.y];
    const int s = a.site ? a.site[item] : item;
    const int64_t cnt = a.r1 - a.r0;
    const int64_t nrb = (cnt + NT - 1) / NT;
    const int64_t rb = blockIdx.x % nrb;
    const int c0 = (int)(blockIdx.x / nrb) * TRSV_CW;
    const int64_t g = rb * NT + threadIdx.x;
    if (g >= cnt) return;
    const int nc = min(TRSV_CW, a.w - c0);
    const int64_t i = a.r0 + g;
    const zd* v = a.lu + (size_t)s * a.nnz;
    zd* x = a.X + (size_t)item * a.xs + (size_t)c0 * a.ldx;
    zd acc[TRSV_CW];
#pragma unroll
    for (int k = 0; k < TRSV_CW; ++k) acc[k] = (k < nc) ? x[i + (size_t)k * a.ldx] : zmake(0.0, 0.0);
    for (int64_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
        const int32_t j = a.ci[p];
        if (a.part == 0 ? j >= i : j <= i) continue;
        zd val = v[a.map ? a.map[p] : p];
        if (a.conj) val = zconj(val);
#pragma unroll
        for (int k = 0; k < TRSV_CW; ++k)
            if (k < nc) acc[k] = zsub(acc[k], zmul(val, x[j + (size_t)k * a.ldx]));
    }
    zd dinv = zmake(1.0, 0.0);
    if (!a.unit) {
        zd d = v[a.diag[i]];
        if (a.conj) d = zconj(d);
        dinv = zscale(zconj(d), 1.0 / zabs2(d));
    }
#pragma unroll
    for (int k = 0; k < TRSV_CW; ++k)
        if (k < nc) x[i + (size_t)k * a.ldx] = a.unit ? acc[k] : zmul(dinv, acc[k]);
}

// Y[:, c] = X[perm, c] (gather, mode 0) or Y[perm, c] = X[:, c] (scatter, mode 1)
__global__ void k_permute(const int* list, const int* perm, int64_t n, int w, const zd* X, int64_t xs, int64_t ldx,
                          zd* Y, int64_t ys, int64_t ldy, int mode)
{
    const int item = list[blockIdx.y];
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n * w) return;
    const int64_t i = g % n;
    const int c = (int)(g / n);
    const zd* xc = X + (size_t)item * xs + (size_t)c * ldx;
    zd* yc = Y + (size_t)item * ys + (size_t)c * ldy;
    if (mode == 0) yc[i] = xc[perm[i]];
    else yc[perm[i]] = xc[i];
}

// ---------------------------------------------------------------------------
void launch_ilu(const int* list, int ns, const SparsePattern& sp, const zd* vC, const zd* zsite, zd* lu, int* nfloor,
                hipStream_t s)
{
    if (ns <= 0) return;
    dim3 g1((unsigned)((sp.nnz + NT - 1) / NT), ns);
    hipLaunchKernelGGL(k_ilu_form, g1, dim3(NT), 0, s, list, sp.rp, sp.ci, sp.src, vC, zsite, sp.n, sp.nnz, lu);
    dim3 g2((unsigned)((sp.n + NT - 1) / NT), ns);
    hipLaunchKernelGGL(k_ilu_shift, g2, dim3(NT), 0, s, list, sp.diag, zsite, sp.n, sp.nnz, lu);
    for (int c = 0; c < sp.ncolors; ++c) {
        const int64_t r0 = sp.cptr[c], r1 = sp.cptr[c + 1];
        if (r1 <= r0) continue;
        dim3 g((unsigned)((r1 - r0 + NT - 1) / NT), ns);
        hipLaunchKernelGGL(k_ilu_color, g, dim3(NT), 0, s, list, sp.rp, sp.ci, sp.diag, r0, r1, sp.nnz, lu, nfloor);
    }
}

static void solve_pass(const int* list, int ni, const int* site, const SparsePattern& sp, const zd* lu, zd* X,
                       int64_t xs, int64_t ldx, int w, bool transposed, int part, int unit, bool forward,
                       hipStream_t s)
{
    SpSolveArgs a;
    a.list = list;
    a.site = site;
    a.rp = transposed ? sp.rpT : sp.rp;
    a.ci = transposed ? sp.ciT : sp.ci;
    a.map = transposed ? sp.mapT : nullptr;
    a.diag = sp.diag;
    a.lu = lu;
    a.nnz = sp.nnz;
    a.X = X;
    a.xs = xs;
    a.ldx = ldx;
    a.w = w;
    a.part = part;
    a.unit = unit;
    a.conj = transposed ? 1 : 0;
    for (int q = 0; q < sp.ncolors; ++q) {
        const int c = forward ? q : sp.ncolors - 1 - q;
        a.r0 = sp.cptr[c];
        a.r1 = sp.cptr[c + 1];
        if (a.r1 <= a.r0) continue;
        const int64_t nrb = (a.r1 - a.r0 + NT - 1) / NT;
        dim3 g((unsigned)(nrb * ((w + TRSV_CW - 1) / TRSV_CW)), ni);
        hipLaunchKernelGGL(k_sptrsv_color, g, dim3(NT), 0, s, a);
    }
}

// Y = (F P)^{-1} X = P^T U^{-1} L^{-1} X (trans 0) or Y = (F P)^{-*} X =
// L^{-*} U^{-*} P X (trans 1), for n x w blocks of the listed items; T is an
// n x w work block per item (stride ts)
void launch_ilu_solve(const int* list, int ni, const int* site, const SparsePattern& sp, const zd* lu, int trans,
                      const zd* X, int64_t xs, int64_t ldx, zd* Y, int64_t ys, int64_t ldy, int w, zd* T, int64_t ts,
                      hipStream_t s)
{
    if (ni <= 0) return;
    const int64_t n = sp.n;
    dim3 gp((unsigned)((n * w + NT - 1) / NT), ni);
    if (trans == 0) {
        // T = X; L forward (unit); U backward; Y = P^T T
        launch_copy_cols(list, ni, X, xs, ldx, T, ts, n, n, w, s);
        solve_pass(list, ni, site, sp, lu, T, ts, n, w, false, 0, 1, true, s);
        solve_pass(list, ni, site, sp, lu, T, ts, n, w, false, 1, 0, false, s);
        hipLaunchKernelGGL(k_permute, gp, dim3(NT), 0, s, list, sp.perm, n, w, T, ts, n, Y, ys, ldy, 1);
    } else {
        // T = P X; U^* forward (lower part of the transpose); L^* backward (unit)
        hipLaunchKernelGGL(k_permute, gp, dim3(NT), 0, s, list, sp.perm, n, w, X, xs, ldx, T, ts, n, 0);
        solve_pass(list, ni, site, sp, lu, T, ts, n, w, true, 0, 0, true, s);
        solve_pass(list, ni, site, sp, lu, T, ts, n, w, true, 1, 1, false, s);
        launch_copy_cols(list, ni, T, ts, n, Y, ys, ldy, n, w, s);
    }
}
