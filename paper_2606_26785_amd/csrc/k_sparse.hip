// Sparse base preconditioner for CSR C (Sec. 3, the base K of eq.
// (twolevel); Sec. 4 uses an incomplete Cholesky factorization of N(z_dag)):
// K = L D L^* ~ N(z_dag) + alpha I, the incomplete Cholesky factorization
// without fill of the Hermitian positive definite N(z_dag) + alpha I on the
// sparsity pattern of N = C^* C, in the order of a greedy colouring of that
// pattern's graph (rows of one colour share no entry).  alpha is a global
// diagonal shift, raised when a pivot is not positive.  With F = D^{1/2}
// L^* P (P the colour permutation), K = F^* F, F^{-1} = P^T L^{-*} D^{-1/2}
// and F^{-*} = D^{-1/2} L^{-1} P.
//
// Rows of one colour depend only on rows of earlier colours in L and of
// later colours in L^*, so the factorization and every triangular solve run
// one launch per colour, each over all rows of the colour and all
// right-hand sides.  The factorization runs the IKJ elimination on the full
// (Hermitian) pattern and keeps its unit lower factor L and the real parts
// of its pivots D.
#include "zdev.h"
#include "kernels.h"

#define NT 256

// lu[site][e] = N(z)_e = sum over the entry's contributions (a, b) of
// conj(c_a(z)) c_b(z), with c(z) the entry of C - z I that a code names:
// code >= 0: C value code >> 1, minus z when code & 1 (a diagonal entry);
// code < 0: a diagonal entry C does not store (value -z)
__device__ inline zd icn_val(const zd* vC, int64_t code, zd z)
{
    if (code < 0) return zmake(-z.x, -z.y);
    zd v = vC[code >> 1];
    if (code & 1) v = zsub(v, z);
    return v;
}
__global__ void k_icn_form(const int* list, const int64_t* cptr, const int64_t* ca, const int64_t* cb, const zd* vC,
                           const zd* zsite, int64_t nnz, zd* lu)
{
    const int s = list[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= nnz) return;
    const zd z = zsite[s];
    zd acc = zmake(0.0, 0.0);
    for (int64_t q = cptr[e]; q < cptr[e + 1]; ++q) zcfma(acc, icn_val(vC, ca[q], z), icn_val(vC, cb[q], z));
    lu[(size_t)s * nnz + e] = acc;
}
__global__ void k_icn_shift(const int* list, const int64_t* diag, const double* alpha, int64_t nrows, int64_t nnz,
                            zd* lu)
{
    const int s = list[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= nrows) return;
    zd* p = lu + (size_t)s * nnz + diag[i];
    p->x += alpha[s];
}

// rows [r0, r1) (one colour) of each listed site: IKJ elimination without
// fill.  For each k < i in row i: l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj
// for the j > k of row i that row k also holds.  A pivot whose real part is
// not above 1e-14 times the row's 2-norm marks the site (notpd) and is
// replaced by that size so the elimination stays finite.
__global__ void k_ic_color(const int* list, const int64_t* rp, const int32_t* ci, const int64_t* diag, int64_t r0,
                           int64_t r1, int64_t nnz, zd* lu, int* notpd)
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
        int64_t q = diag[k] + 1;
        const int64_t qe = rp[k + 1];
        for (int64_t t = p + 1; t < e && q < qe; ++t) {
            const int32_t j = ci[t];
            while (q < qe && ci[q] < j) ++q;
            if (q < qe && ci[q] == j) a[t] = zsub(a[t], zmul(l, a[q]));
        }
    }
    zd* d = a + diag[i];
    const double floor_v = 1e-14 * rn;
    if (!(d->x > floor_v)) {
        *d = zmake(floor_v > 0.0 ? floor_v : 1e-300, 0.0);
        notpd[s] = 1;
    }
}

// One colour of a triangular solve with the unit factor, in place on X
// (n x w per item, ld ldx): x_i -= sum over the part's off-diagonal entries
// val_ij x_j.  Non-transposed pattern, part 0: L (forward).  Transposed
// pattern (rpT, ciT, mapT: entry of the transpose -> entry of lu) with
// conj = 1, part 1: L^* (backward).
struct SpSolveArgs {
    const int* list;        // items (tiles or sites)
    const int* site;        // per item: its site (NULL: the item is the site)
    const int64_t* rp; const int32_t* ci; const int64_t* map;   // map: NULL for lu's own pattern
    const zd* lu; int64_t nnz;
    zd* X; int64_t xs; int64_t ldx; int w;
    int part;               // 0 lower, 1 upper
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
    // every column's load unguarded, so that they are in flight together:
    // the columns past nc repeat column c0, and their results are dropped
    size_t cof[TRSV_CW];
#pragma unroll
    for (int k = 0; k < TRSV_CW; ++k) cof[k] = (size_t)(k < nc ? k : 0) * a.ldx;
    zd acc[TRSV_CW];
#pragma unroll
    for (int k = 0; k < TRSV_CW; ++k) acc[k] = x[i + cof[k]];
    for (int64_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
        const int32_t j = a.ci[p];
        if (a.part == 0 ? j >= i : j <= i) continue;
        zd val = v[a.map ? a.map[p] : p];
        if (a.conj) val = zconj(val);
#pragma unroll
        for (int k = 0; k < TRSV_CW; ++k) acc[k] = zsub(acc[k], zmul(val, x[j + cof[k]]));
    }
#pragma unroll
    for (int k = 0; k < TRSV_CW; ++k)
        if (k < nc) x[i + (size_t)k * a.ldx] = acc[k];
}

// X[i, c] *= Re(u_ii)^{-1/2} (the D^{-1/2} of the factor)
__global__ void k_scale_dhalf(const int* list, const int* site, const int64_t* diag, const zd* lu, int64_t nnz,
                              int64_t n, int w, zd* X, int64_t xs, int64_t ldx)
{
    const int item = list[blockIdx.y];
    const int s = site ? site[item] : item;
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n * w) return;
    const int64_t i = g % n;
    const int c = (int)(g / n);
    const double d = lu[(size_t)s * nnz + diag[i]].x;
    zd* x = X + (size_t)item * xs + (size_t)c * ldx + i;
    *x = zscale(*x, 1.0 / sqrt(d));
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
void launch_icn(const int* list, int ns, const SparsePattern& sp, const zd* vC, const zd* zsite, const double* alpha,
                zd* lu, int* notpd, hipStream_t s)
{
    if (ns <= 0) return;
    dim3 g1((unsigned)((sp.nnz + NT - 1) / NT), ns);
    hipLaunchKernelGGL(k_icn_form, g1, dim3(NT), 0, s, list, sp.ccp, sp.ca, sp.cb, vC, zsite, sp.nnz, lu);
    dim3 g2((unsigned)((sp.n + NT - 1) / NT), ns);
    hipLaunchKernelGGL(k_icn_shift, g2, dim3(NT), 0, s, list, sp.diag, alpha, sp.n, sp.nnz, lu);
    for (int c = 0; c < sp.ncolors; ++c) {
        const int64_t r0 = sp.cptr[c], r1 = sp.cptr[c + 1];
        if (r1 <= r0) continue;
        dim3 g((unsigned)((r1 - r0 + NT - 1) / NT), ns);
        hipLaunchKernelGGL(k_ic_color, g, dim3(NT), 0, s, list, sp.rp, sp.ci, sp.diag, r0, r1, sp.nnz, lu, notpd);
    }
}

static void solve_pass(const int* list, int ni, const int* site, const SparsePattern& sp, const zd* lu, zd* X,
                       int64_t xs, int64_t ldx, int w, bool transposed, hipStream_t s)
{
    SpSolveArgs a;
    a.list = list;
    a.site = site;
    a.rp = transposed ? sp.rpT : sp.rp;
    a.ci = transposed ? sp.ciT : sp.ci;
    a.map = transposed ? sp.mapT : nullptr;
    a.lu = lu;
    a.nnz = sp.nnz;
    a.X = X;
    a.xs = xs;
    a.ldx = ldx;
    a.w = w;
    a.part = transposed ? 1 : 0;
    a.conj = transposed ? 1 : 0;
    for (int q = 0; q < sp.ncolors; ++q) {
        const int c = transposed ? sp.ncolors - 1 - q : q;
        a.r0 = sp.cptr[c];
        a.r1 = sp.cptr[c + 1];
        if (a.r1 <= a.r0) continue;
        const int64_t nrb = (a.r1 - a.r0 + NT - 1) / NT;
        dim3 g((unsigned)(nrb * ((w + TRSV_CW - 1) / TRSV_CW)), ni);
        hipLaunchKernelGGL(k_sptrsv_color, g, dim3(NT), 0, s, a);
    }
}

// Y = F^{-1} X = P^T L^{-*} D^{-1/2} X (trans 0) or Y = F^{-*} X =
// D^{-1/2} L^{-1} P X (trans 1), for n x w blocks of the listed items; T is
// an n x w work block per item (stride ts)
void launch_ic_solve(const int* list, int ni, const int* site, const SparsePattern& sp, const zd* lu, int trans,
                     const zd* X, int64_t xs, int64_t ldx, zd* Y, int64_t ys, int64_t ldy, int w, zd* T, int64_t ts,
                     hipStream_t s)
{
    if (ni <= 0) return;
    const int64_t n = sp.n;
    dim3 gp((unsigned)((n * w + NT - 1) / NT), ni);
    if (trans == 0) {
        launch_copy_cols(list, ni, X, xs, ldx, T, ts, n, n, w, s);
        hipLaunchKernelGGL(k_scale_dhalf, gp, dim3(NT), 0, s, list, site, sp.diag, lu, sp.nnz, n, w, T, ts, n);
        solve_pass(list, ni, site, sp, lu, T, ts, n, w, true, s);
        hipLaunchKernelGGL(k_permute, gp, dim3(NT), 0, s, list, sp.perm, n, w, T, ts, n, Y, ys, ldy, 1);
    } else {
        hipLaunchKernelGGL(k_permute, gp, dim3(NT), 0, s, list, sp.perm, n, w, X, xs, ldx, T, ts, n, 0);
        solve_pass(list, ni, site, sp, lu, T, ts, n, w, false, s);
        hipLaunchKernelGGL(k_scale_dhalf, gp, dim3(NT), 0, s, list, site, sp.diag, lu, sp.nnz, n, w, T, ts, n);
        launch_copy_cols(list, ni, T, ts, n, Y, ys, ldy, n, w, s);
    }
}

// ---------------------------------------------------------------------------
// Inertia test for a CSR C whose N = C^* C has a narrow band (bandwidth
// b <= 63 in the natural order): the exact Cholesky factorization of the
// band of N(z) - mu I, one workgroup (one wave) per test.  Band storage, row
// j: entries (j, j + d), d = 0..b, at W[j (b + 1) + d], formed from the
// contribution lists of the band (as k_icn_form does for the incomplete
// factor); then for j = 0, 1, ...: thread d forms
// s_d = A(j, j+d) - sum_{k = j-b}^{j-1} conj(R(k, j)) R(k, j+d), the pivot
// s_0 must be positive (else notpd), and R(j, j+d) = s_d / sqrt(s_0).
// Every pivot positive means N(z) - mu I is positive definite.
__global__ void __launch_bounds__(64) k_band_inertia(const int* list, const zd* zsite, const double* mu,
                                                     const int64_t* cptr, const int64_t* ca, const int64_t* cb,
                                                     const zd* vC, int64_t n, int b, zd* W, int64_t wstride,
                                                     double floor_rel, int* notpd)
{
    const int s = list[blockIdx.x];
    const int tid = threadIdx.x;
    const zd z = zsite[s];
    const int bw = b + 1;
    zd* R = W + (size_t)s * wstride;
    // form the band of N(z) - mu I
    for (int64_t e = tid; e < n * bw; e += 64) {
        zd acc = zmake(0.0, 0.0);
        for (int64_t q = cptr[e]; q < cptr[e + 1]; ++q) zcfma(acc, icn_val(vC, ca[q], z), icn_val(vC, cb[q], z));
        if (e % bw == 0) acc.x -= mu[s];
        R[e] = acc;
    }
    __syncthreads();
    __shared__ double piv;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int64_t j = 0; j < n; ++j) {
        const int d = tid;
        zd sacc = zmake(0.0, 0.0);
        const bool live = d <= b && j + d < n;
        if (live) {
            sacc = R[j * bw + d];
            const int64_t k0 = j - b > 0 ? j - b : 0;
            for (int64_t k = k0; k < j; ++k) {
                const int o = (int)(j - k);            // R(k, j) at offset j - k of row k
                if (o + d > b) continue;               // R(k, j + d) outside the band
                sacc = zsub(sacc, zcmul(R[k * bw + o], R[k * bw + o + d]));
            }
        }
        if (d == 0) {
            const double fl = floor_rel;
            double p = sacc.x;
            if (!(p > fl)) {
                bad = 1;
                p = fl > 0.0 ? fl : 1e-300;
            }
            piv = sqrt(p);
        }
        __syncthreads();
        if (live) R[j * bw + d] = (d == 0) ? zmake(piv, 0.0) : zscale(sacc, 1.0 / piv);
        __syncthreads();
    }
    if (tid == 0 && bad) notpd[s] = 1;
}

void launch_band_inertia(const int* list, int nt, const zd* zsite, const double* mu, const int64_t* cptr,
                         const int64_t* ca, const int64_t* cb, const zd* vC, int64_t n, int b, zd* W,
                         int64_t wstride, double floor_rel, int* notpd, hipStream_t s)
{
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_band_inertia, dim3(nt), dim3(64), 0, s, list, zsite, mu, cptr, ca, cb, vC, n, b, W, wstride,
                       floor_rel, notpd);
}
