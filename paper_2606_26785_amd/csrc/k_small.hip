// Small dense kernels: one workgroup per problem, matrices resident in LDS.
//
//  * k_ritz      Ritz singular pairs and residual norms from a recycled
//                subspace, for a batch of grid points (recySing, Alg. 1, in
//                its one-step Rayleigh-Ritz-SVD form, plus the fast residual
//                of eq. (fastresidual) and the acceptance test (tolC)).
//  * k_chol_dd   R factor of a tall matrix from its Gram matrix in
//                double-double (mixed-precision Cholesky QR).
//  * k_rr_hl     Rayleigh-Ritz-SVD and Hetmaniuk-Lehoucq basis selection of
//                one LOBPCG-SVD iteration (supplement, Alg. SM1.1).
//  * k_svqb      orthonormalising transform of a block (SVQB).
//  * k_rotations block unitary rotations restoring the QL form of the
//                recycled basis (Sec. 2.2.2, eq. (blkGS)).
#include <mutex>

#include "zdev.h"
#include "kernels.h"

#define NT 256

static int g_max_lds = 64 * 1024;

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of A (m x n, LDS, column-major, lda) with
// the right rotations accumulated into G (n x n, LDS, ldg), n even.
// Parallel cyclic ordering: in each of the n-1 steps of a sweep the n/2
// column pairs of a round-robin tournament are rotated at once.  A pair is
// rotated when |A_p^* A_q| > m eps ||A_p|| ||A_q||; the phase of A_p^* A_q is
// moved onto column q and the smaller-angle 2x2 Jacobi rotation annihilates
// it.  Stops after a sweep without rotations.  On return sv[j] = ||A_j||.
__device__ int wg_jacobi(zd* A, int lda, int m, int n, zd* G, int ldg, double* sv,
                         int max_sweeps, int* sh_flag)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < n * n; idx += nt) {
        int i = idx % n, j = idx / n;
        G[i + j * ldg] = zmake(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const int np = n / 2;
    int tpp = 64;
    while (tpp > 1 && tpp * np > nt) tpp >>= 1;
    const int g = tid / tpp, lane = tid % tpp;
    const double tol = (double)m * 2.220446049250313e-16;
    int sweep, done = 0;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) *sh_flag = 0;
        __syncthreads();
        for (int s = 0; s < n - 1; ++s) {
            if (g < np) {
                int p, q;
                if (g == 0) { p = s; q = n - 1; }
                else { p = (s + g) % (n - 1); q = (s - g + n - 1) % (n - 1); }
                double a = 0, b = 0, cr = 0, ci = 0;
                for (int i = lane; i < m; i += tpp) {
                    zd x = A[i + p * lda], y = A[i + q * lda];
                    a += zabs2(x);
                    b += zabs2(y);
                    cr += x.x * y.x + x.y * y.y;
                    ci += x.x * y.y - x.y * y.x;
                }
                a = group_sum(a, tpp);
                b = group_sum(b, tpp);
                cr = group_sum(cr, tpp);
                ci = group_sum(ci, tpp);
                double ca = hypot(cr, ci);
                if (ca > 0.0 && ca > tol * sqrt(a) * sqrt(b)) {
                    if (lane == 0) *sh_flag = 1;
                    zd ph = zmake(cr / ca, -ci / ca);
                    double zeta = (b - a) / (2.0 * ca);
                    double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                    double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                    for (int i = lane; i < m; i += tpp) {
                        zd x = A[i + p * lda], y = zmul(A[i + q * lda], ph);
                        A[i + p * lda] = zmake(cs * x.x - sn * y.x, cs * x.y - sn * y.y);
                        A[i + q * lda] = zmake(sn * x.x + cs * y.x, sn * x.y + cs * y.y);
                    }
                    for (int i = lane; i < n; i += tpp) {
                        zd x = G[i + p * ldg], y = zmul(G[i + q * ldg], ph);
                        G[i + p * ldg] = zmake(cs * x.x - sn * y.x, cs * x.y - sn * y.y);
                        G[i + q * ldg] = zmake(sn * x.x + cs * y.x, sn * x.y + cs * y.y);
                    }
                }
            }
            __syncthreads();
        }
        int f = *sh_flag;
        __syncthreads();
        if (f == 0) { done = 1; break; }
    }
    for (int j = tid; j < n; j += nt) {
        double s = 0;
        for (int i = 0; i < m; ++i) s += zabs2(A[i + j * lda]);
        sv[j] = sqrt(s);
    }
    __syncthreads();
    return done ? sweep + 1 : -1;
}

// ascending ranks of sv[0..n) (ties broken by index): perm[rank] = j
__device__ void wg_sort_perm(const double* sv, int n, int* perm)
{
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int rk = 0;
        double v = sv[j];
        for (int i = 0; i < n; ++i) {
            double w = sv[i];
            rk += (w < v) || (w == v && i < j);
        }
        perm[rk] = j;
    }
    __syncthreads();
}

// In-place Householder QR of A (m x n, m >= n, LDS).  R is left in the upper
// triangle; reflector j is H_j = I - 2 v v^* with unit v, v[0] = vhead[j],
// v[1..] stored below the diagonal of column j.  red: >= 8 doubles scratch.
__device__ void wg_house_qr(zd* A, int lda, int m, int n, zd* vhead, double* red)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int j = 0; j < n; ++j) {
        double s = 0;
        for (int i = j + tid; i < m; i += nt) s += zabs2(A[i + j * lda]);
        s = block_sum(s, red);
        zd x0 = A[j + j * lda];
        double nrm = sqrt(s), ax0 = sqrt(zabs2(x0));
        zd alpha = (ax0 > 0.0) ? zscale(x0, -nrm / ax0) : zmake(-nrm, 0.0);
        zd v0 = zsub(x0, alpha);
        double vn2 = s - zabs2(x0) + zabs2(v0);
        __syncthreads();
        if (nrm == 0.0 || vn2 <= 0.0) {
            if (tid == 0) { vhead[j] = zmake(0.0, 0.0); A[j + j * lda] = zmake(0.0, 0.0); }
            for (int i = j + 1 + tid; i < m; i += nt) A[i + j * lda] = zmake(0.0, 0.0);
            __syncthreads();
            continue;
        }
        double inv = 1.0 / sqrt(vn2);
        for (int i = j + 1 + tid; i < m; i += nt) A[i + j * lda] = zscale(A[i + j * lda], inv);
        if (tid == 0) vhead[j] = zscale(v0, inv);
        __syncthreads();
        int nc = n - j - 1;
        if (nc > 0) {
            int tpp = 64;
            while (tpp > 1 && tpp * nc > nt) tpp >>= 1;
            int grp = tid / tpp, lane = tid % tpp, ngrp = nt / tpp;
            zd vh = vhead[j];
            for (int c = j + 1 + grp; c < n; c += ngrp) {
                double dr = 0, di = 0;
                for (int i = j + lane; i < m; i += tpp) {
                    zd v = (i == j) ? vh : A[i + j * lda];
                    zd a = A[i + c * lda];
                    dr += v.x * a.x + v.y * a.y;
                    di += v.x * a.y - v.y * a.x;
                }
                dr = group_sum(dr, tpp);
                di = group_sum(di, tpp);
                zd d2 = zmake(2.0 * dr, 2.0 * di);
                for (int i = j + lane; i < m; i += tpp) {
                    zd v = (i == j) ? vh : A[i + j * lda];
                    A[i + c * lda] = zsub(A[i + c * lda], zmul(v, d2));
                }
            }
        }
        __syncthreads();
        if (tid == 0) A[j + j * lda] = alpha;
        __syncthreads();
    }
}

// Q (m x nq, LDS, ldq) = H_0 H_1 ... H_{n-1} [I_nq; 0] from wg_house_qr output.
__device__ void wg_house_q(const zd* A, int lda, int m, int n, const zd* vhead, zd* Q, int ldq, int nq)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < m * nq; idx += nt) {
        int i = idx % m, c = idx / m;
        Q[i + c * ldq] = zmake(i == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    int tpp = 64;
    while (tpp > 1 && tpp * nq > nt) tpp >>= 1;
    int grp = tid / tpp, lane = tid % tpp, ngrp = nt / tpp;
    for (int j = n - 1; j >= 0; --j) {
        zd vh = vhead[j];
        for (int c = grp; c < nq; c += ngrp) {
            double dr = 0, di = 0;
            for (int i = j + lane; i < m; i += tpp) {
                zd v = (i == j) ? vh : A[i + j * lda];
                zd a = Q[i + c * ldq];
                dr += v.x * a.x + v.y * a.y;
                di += v.x * a.y - v.y * a.x;
            }
            dr = group_sum(dr, tpp);
            di = group_sum(di, tpp);
            zd d2 = zmake(2.0 * dr, 2.0 * di);
            for (int i = j + lane; i < m; i += tpp) {
                zd v = (i == j) ? vh : A[i + j * lda];
                Q[i + c * ldq] = zsub(Q[i + c * ldq], zmul(v, d2));
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_ritz: one workgroup per (tile, point) job.
//
// The recycled store of a tile holds R_A, the R factor of [W1 W2] (2k x 2k),
// and R_res, the R factor of the residual blocks (nres k x nres k).  Since
// M(z) V = W1 - z W2 = Q_A (R_A[:, :k] - z R_A[:, k:]), the Ritz singular
// values and right vectors of M(z) on span V are those of the 2k x k matrix
// B(z) = R_A[:, :k] - z R_A[:, k:] (the Rayleigh-Ritz-SVD of Sec. 2.2.1, done
// with a z-independent QR).  B(z) is QR-reduced to k x k, then SVD'd by
// one-sided Jacobi.  The residual W = T(z) V g - xi^2 V g (eq.
// (fastresidual)) is [W3 W4 W5 W6 (V)] u, so ||W|| = ||R_res u|| with
//   nres = 4 (S^*S = I_n, W6 = V):  u = [g; -z g; -conj(z) g; (|z|^2 - xi^2) g]
//   nres = 5 (general S):           u = [g; -z g; -conj(z) g; |z|^2 g; -xi^2 g].
// Outputs per job: xi[0..nv), residual norms res[0..nv), the first ng right
// vectors (k x ng, column-major), and an acceptance flag:
//   mode 0 (tolC):  accept iff res[0] <= max(eta xi_0 nrm, nrm^2 eps)
//   mode 1 (tolTz): accept iff res[j] <= eta * nrm for all j < nv
__global__ void __launch_bounds__(NT) k_ritz(RitzArgs a)
{
    extern __shared__ double smem_d[];
    zd* sm = (zd*)smem_d;
    __shared__ double red[8];
    __shared__ zd vhead[64];
    __shared__ double sv[64];
    __shared__ int perm[64];
    __shared__ int sh_flag;
    __shared__ double sres[64];

    const int job = blockIdx.x;
    if (job >= a.njobs) return;
    const int tile = a.job_tile[job];
    const int k = a.kdim[tile];
    const zd z = a.z[job];
    const int tid = threadIdx.x;
    if (k <= 0) {
        if (tid == 0) { a.accept[job] = 0; }
        return;
    }
    const int m2 = 2 * k;
    const zd* RA = a.RA + (size_t)tile * a.strideRA;
    zd* B = sm;                       // 2k x k, ld = m2
    // B(z) = R_A[:, :k] - z R_A[:, k:2k]
    for (int idx = tid; idx < m2 * k; idx += blockDim.x) {
        int i = idx % m2, j = idx / m2;
        zd r1 = RA[i + (size_t)j * a.ldRA];
        zd r2 = RA[i + (size_t)(k + j) * a.ldRA];
        B[i + j * m2] = zsub(r1, zmul(z, r2));
    }
    __syncthreads();
    wg_house_qr(B, m2, m2, k, vhead, red);
    // compact R (k x k upper, stride 2k) to stride k in place through
    // registers; then T = sm[0 .. k^2), G = sm[k^2 .. 2k^2)
    zd regs[16];
    {
#pragma unroll
        for (int cnt = 0; cnt < 16; ++cnt) {
            int idx = tid + cnt * NT;
            int i = idx % k, j = idx / k;
            regs[cnt] = (idx < k * k && i <= j) ? B[i + j * m2] : zmake(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int cnt = 0; cnt < 16; ++cnt) {
            int idx = tid + cnt * NT;
            if (idx < k * k) sm[idx] = regs[cnt];
        }
        __syncthreads();
    }
    zd* T = sm;
    zd* G = sm + k * k;
    int sweeps = wg_jacobi(T, k, k, k, G, k, sv, a.max_sweeps, &sh_flag);
    wg_sort_perm(sv, k, perm);
    const int nv = min(a.nv, k);
    const int ng = min(a.ng, k);
    // right vectors out
    zd* Gout = a.Gout + (size_t)job * a.strideG;
    for (int idx = tid; idx < k * ng; idx += blockDim.x) {
        int i = idx % k, c = idx / k;
        Gout[i + (size_t)c * a.ldG] = G[i + perm[c] * k];
    }
    // residual norms
    const zd* Rr = a.Rres + (size_t)tile * a.strideRres;
    const int nres = a.nres;
    const int rows = nres * k;
    const double az2 = zabs2(z);
    const zd mz = zmake(-z.x, -z.y), mzc = zmake(-z.x, z.y);
    for (int v = 0; v < nv; ++v) {
        const int col = perm[v];
        const double xi = sv[col];
        double acc = 0.0;
        for (int i = tid; i < rows; i += blockDim.x) {
            zd s = zmake(0.0, 0.0);
            // R_res upper triangular: row i, columns c >= i (global column index c = blk*k + j)
            for (int c = i; c < rows; ++c) {
                int blk = c / k, j = c - blk * k;
                zd g = G[j + col * k];
                zd coef;
                if (blk == 0) coef = g;
                else if (blk == 1) coef = zmul(mz, g);
                else if (blk == 2) coef = zmul(mzc, g);
                else if (blk == 3) coef = (nres == 4) ? zscale(g, az2 - xi * xi) : zscale(g, az2);
                else coef = zscale(g, -xi * xi);
                zfma(s, Rr[i + (size_t)c * a.ldRres], coef);
            }
            acc += zabs2(s);
        }
        acc = block_sum(acc, red);
        if (tid == 0) sres[v] = sqrt(acc);
        __syncthreads();
    }
    if (tid < nv) {
        a.xi[(size_t)job * a.ldxi + tid] = sv[perm[tid]];
        a.res[(size_t)job * a.ldxi + tid] = sres[tid];
    }
    if (tid == 0) {
        const double nrm = a.nrm[job];
        int acc = 1;
        if (a.mode == 0) {
            double xi0 = sv[perm[0]];
            // a residual w of the Hermitian N(z) puts some sigma_j^2 within w of
            // xi0^2, so |sigma_j - xi0| <= w / xi0: the floor alone decides only
            // where that bound is within floor_tol
            const bool lin = sres[0] <= a.eta * xi0 * nrm;
            const bool flo = sres[0] <= a.floor_c * nrm * nrm * 2.220446049250313e-16 &&
                             (a.floor_tol <= 0.0 || sres[0] <= a.floor_tol * xi0);
            acc = lin || flo || (xi0 <= a.eta_abs * a.normC);
        } else {
            for (int v = 0; v < nv; ++v) acc &= (sres[v] <= a.eta * nrm);
        }
        if (sweeps < 0) acc = 0;
        a.accept[job] = (uint8_t)acc;
    }
}

// ---------------------------------------------------------------------------
// k_chol_dd: R (c x c, upper, double) with R^* R = G, G given as a complex
// double-double Gram matrix (upper triangle used, overwritten).  Pivots below
// c * 1e-30 * max diag(G) are treated as zero and their rows of R are zero
// (semidefinite Cholesky).  One workgroup per matrix.
__global__ void __launch_bounds__(NT) k_chol_dd(CholArgs a)
{
    __shared__ ddv rowr[2 * 320];
    __shared__ ddv piv_s;
    __shared__ int zero_s;
    __shared__ double red[8];
    const int b = blockIdx.x;
    const int tile = a.list ? a.list[b] : b;
    const int c = a.cdim ? a.cdim[tile] * a.cmul : a.c;
    zdd* G = a.G + (size_t)tile * a.strideG;
    zd* R = a.R + (size_t)tile * a.strideR;
    const int ldg = a.ldG, ldr = a.ldR;
    const int tid = threadIdx.x;
    if (c <= 0) {
        if (tid == 0 && a.nzero) a.nzero[tile] = 0;
        return;
    }
    double dmax = 0;
    for (int i = tid; i < c; i += blockDim.x) dmax = fmax(dmax, G[i + (size_t)i * ldg].x.hi);
    dmax = block_max(dmax, red);
    const double thr = (double)c * 1e-30 * dmax;
    int nzero = 0;
    for (int j = 0; j < c; ++j) {
        if (tid == 0) {
            ddv d = G[j + (size_t)j * ldg].x;
            if (!(d.hi > thr)) { zero_s = 1; piv_s = dd_make(0.0); }
            else { zero_s = 0; piv_s = dd_sqrt(d); }
        }
        __syncthreads();
        const int zr = zero_s;
        const ddv piv = piv_s;
        nzero += zr;
        for (int kk = j + tid; kk < c; kk += blockDim.x) {
            zdd v;
            if (zr) v = zdd_zero();
            else if (kk == j) { v.x = piv; v.y = dd_make(0.0); }
            else { zdd g = G[j + (size_t)kk * ldg]; v.x = dd_div(g.x, piv); v.y = dd_div(g.y, piv); }
            rowr[2 * kk] = v.x;
            rowr[2 * kk + 1] = v.y;
            R[j + (size_t)kk * ldr] = zmake(v.x.hi + v.x.lo, v.y.hi + v.y.lo);
        }
        for (int i = tid; i < j; i += blockDim.x) R[j + (size_t)i * ldr] = zmake(0.0, 0.0);
        __syncthreads();
        if (!zr) {
            // trailing update G[kk][ll] -= conj(R[j][kk]) R[j][ll], j < kk <= ll
            for (int kk = j + 1 + tid; kk < c; kk += blockDim.x) {
                zdd rk; rk.x = rowr[2 * kk]; rk.y = rowr[2 * kk + 1];
                for (int ll = kk; ll < c; ++ll) {
                    zdd rl; rl.x = rowr[2 * ll]; rl.y = rowr[2 * ll + 1];
                    G[kk + (size_t)ll * ldg] = zdd_sub(G[kk + (size_t)ll * ldg], zdd_cmul(rk, rl));
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && a.nzero) a.nzero[tile] = nzero;
}

// ---------------------------------------------------------------------------
// k_rr_hl: per tile, from the R factor (c x c, c = 2r or 3r) of C(z) S with
// orthonormal S: SVD R = J Xi G^* by one-sided Jacobi, Ritz values xi
// ascending, G_X = G[:, :r], and the Hetmaniuk-Lehoucq choice of the new
// search direction block G_P: an orthonormal basis of the part of
// span{[I_r; 0], G_X} orthogonal to G_X, namely G_c Q with G_c = G[:, r:] and
// Q from the thin QR of (G_c[:r, :])^*.
__global__ void __launch_bounds__(NT) k_rr_hl(RRArgs a)
{
    extern __shared__ double smem_d[];
    zd* sm = (zd*)smem_d;
    __shared__ double sv[64];
    __shared__ int perm[64];
    __shared__ int sh_flag;
    __shared__ zd vhead[64];
    __shared__ double red[8];
    const int b = blockIdx.x;
    const int tile = a.list[b];
    const int c = a.cdim[tile];
    const int r = a.r;
    const int tid = threadIdx.x;
    const zd* Rin = a.R + (size_t)tile * a.strideR;
    zd* T = sm;            // c x c
    zd* G = T + c * c;     // c x c
    zd* Y = G + c * c;     // (c - r) x r
    zd* Q = Y + (c - r) * r;
    for (int idx = tid; idx < c * c; idx += blockDim.x) {
        int i = idx % c, j = idx / c;
        T[i + j * c] = (i <= j) ? Rin[i + (size_t)j * a.ldR] : zmake(0.0, 0.0);
    }
    __syncthreads();
    int sweeps = wg_jacobi(T, c, c, c, G, c, sv, a.max_sweeps, &sh_flag);
    wg_sort_perm(sv, c, perm);
    zd* GX = a.GX + (size_t)tile * a.strideGX;
    zd* GP = a.GP + (size_t)tile * a.strideGX;
    for (int idx = tid; idx < c * r; idx += blockDim.x) {
        int i = idx % c, j = idx / c;
        GX[i + (size_t)j * a.ldGX] = G[i + perm[j] * c];
    }
    if (tid < r) a.xi[(size_t)tile * a.ldxi + tid] = sv[perm[tid]];
    if (tid == 0 && a.status) a.status[tile] = sweeps;
    const int nc = c - r;
    if (nc < r) {
        // no complement to choose from (first step of the iteration)
        for (int idx = tid; idx < c * r; idx += blockDim.x) {
            int i = idx % c, j = idx / c;
            GP[i + (size_t)j * a.ldGX] = zmake(0.0, 0.0);
        }
        return;
    }
    // Y = (G_c[:r, :])^*  ((c - r) x r): Y[i][j] = conj(G[j, perm[r + i]])
    for (int idx = tid; idx < nc * r; idx += blockDim.x) {
        int i = idx % nc, j = idx / nc;
        Y[i + j * nc] = zconj(G[j + perm[r + i] * c]);
    }
    __syncthreads();
    wg_house_qr(Y, nc, nc, r, vhead, red);
    wg_house_q(Y, nc, nc, r, vhead, Q, nc, r);
    // G_P = G_c Q  (c x r)
    for (int idx = tid; idx < c * r; idx += blockDim.x) {
        int i = idx % c, j = idx / c;
        zd s = zmake(0.0, 0.0);
        for (int l = 0; l < nc; ++l) zfma(s, G[i + perm[r + l] * c], Q[l + j * nc]);
        GP[i + (size_t)j * a.ldGX] = s;
    }
}

// ---------------------------------------------------------------------------
// k_svqb: per tile, from the R factor (r x r) of a block W D^{-1} (columns
// scaled to unit norm, d[] the scales): SVD R = J S U^*, and the transform
// T = D^{-1} U S^{-1} that makes W T orthonormal.  Directions with
// s_j < drop * s_max are flagged in mask (bit j) and their columns of T set
// to zero so the caller can refill them.
__global__ void __launch_bounds__(NT) k_svqb(SvqbArgs a)
{
    extern __shared__ double smem_d[];
    zd* sm = (zd*)smem_d;
    __shared__ double sv[64];
    __shared__ int perm[64];
    __shared__ int sh_flag;
    const int b = blockIdx.x;
    const int tile = a.list[b];
    const int r = a.r;
    const int tid = threadIdx.x;
    const zd* Rin = a.R + (size_t)tile * a.strideR;
    zd* T = sm;
    zd* G = T + r * r;
    for (int idx = tid; idx < r * r; idx += blockDim.x) {
        int i = idx % r, j = idx / r;
        T[i + j * r] = (i <= j) ? Rin[i + (size_t)j * a.ldR] : zmake(0.0, 0.0);
    }
    __syncthreads();
    wg_jacobi(T, r, r, r, G, r, sv, a.max_sweeps, &sh_flag);
    double smax = 0;
    for (int j = 0; j < r; ++j) smax = fmax(smax, sv[j]);
    zd* Tout = a.T + (size_t)tile * a.strideT;
    for (int idx = tid; idx < r * r; idx += blockDim.x) {
        int i = idx % r, j = idx / r;
        double s = sv[j];
        zd v = (s > a.drop * smax && s > 0.0) ? zscale(G[i + j * r], 1.0 / s) : zmake(0.0, 0.0);
        Tout[i + (size_t)j * a.ldT] = v;
    }
    if (tid == 0) {
        uint32_t mask = 0;
        for (int j = 0; j < r; ++j)
            if (!(sv[j] > a.drop * smax && sv[j] > 0.0)) mask |= (1u << j);
        a.mask[tile] = mask;
    }
}

// ---------------------------------------------------------------------------
// k_rotations: per tile, the block unitary transformations of Sec. 2.2.2.
// Input: U (q r x r), the block Gram-Schmidt coefficients U_{j,p+1} of the
// new block against the kept blocks j = 1..q, and Upp (r x r), its own
// coefficient.  For j = 1..q: QR of Y_j = [Upp; U_j] (2r x r) gives a unitary
// Q_loc with Q_loc^* Y_j = [R_loc; 0]; Upp <- R_loc; the pair of block
// columns (new, j) of the accumulated transform Qt ((q+1) r square, block
// order: kept blocks 1..q, then the new block) is multiplied by Q_loc.
__global__ void __launch_bounds__(NT) k_rotations(RotArgs a)
{
    extern __shared__ double smem_d[];
    zd* sm = (zd*)smem_d;
    __shared__ zd vhead[64];
    __shared__ double red[8];
    const int b = blockIdx.x;
    const int tile = a.list[b];
    const int q = a.qdim[tile];
    const int r = a.r;
    const int kk = (q + 1) * r;
    const int tid = threadIdx.x;
    zd* Qt = sm;                       // kk x kk
    zd* Y = Qt + kk * kk;              // 2r x r
    zd* Ql = Y + 2 * r * r;            // 2r x 2r
    zd* Tmp = Ql + 4 * r * r;          // kk x 2r
    zd* Upp = Tmp + kk * 2 * r;        // r x r
    const zd* U = a.U + (size_t)tile * a.strideU;
    const zd* Uin = a.Upp + (size_t)tile * a.strideUpp;
    for (int idx = tid; idx < kk * kk; idx += blockDim.x) {
        int i = idx % kk, j = idx / kk;
        Qt[i + j * kk] = zmake(i == j ? 1.0 : 0.0, 0.0);
    }
    for (int idx = tid; idx < r * r; idx += blockDim.x) {
        int i = idx % r, j = idx / r;
        Upp[i + j * r] = Uin[i + (size_t)j * a.ldUpp];
    }
    __syncthreads();
    for (int jj = 0; jj < q; ++jj) {
        for (int idx = tid; idx < 2 * r * r; idx += blockDim.x) {
            int i = idx % (2 * r), j = idx / (2 * r);
            Y[i + j * 2 * r] = (i < r) ? Upp[i + j * r] : U[(jj * r + i - r) + (size_t)j * a.ldU];
        }
        __syncthreads();
        wg_house_qr(Y, 2 * r, 2 * r, r, vhead, red);
        wg_house_q(Y, 2 * r, 2 * r, r, vhead, Ql, 2 * r, 2 * r);
        for (int idx = tid; idx < r * r; idx += blockDim.x) {
            int i = idx % r, j = idx / r;
            Upp[i + j * r] = (i <= j) ? Y[i + j * 2 * r] : zmake(0.0, 0.0);
        }
        // Qt[:, cols] <- Qt[:, cols] Ql with cols = [new block, block jj]
        for (int idx = tid; idx < kk * 2 * r; idx += blockDim.x) {
            int i = idx % kk, j = idx / kk;
            zd s = zmake(0.0, 0.0);
            for (int l = 0; l < 2 * r; ++l) {
                int col = (l < r) ? (q * r + l) : (jj * r + l - r);
                zfma(s, Qt[i + col * kk], Ql[l + j * 2 * r]);
            }
            Tmp[i + j * kk] = s;
        }
        __syncthreads();
        for (int idx = tid; idx < kk * 2 * r; idx += blockDim.x) {
            int i = idx % kk, j = idx / kk;
            int col = (j < r) ? (q * r + j) : (jj * r + j - r);
            Qt[i + col * kk] = Tmp[i + j * kk];
        }
        __syncthreads();
    }
    zd* Qo = a.Qt + (size_t)tile * a.strideQt;
    for (int idx = tid; idx < kk * kk; idx += blockDim.x) {
        int i = idx % kk, j = idx / kk;
        Qo[i + (size_t)j * a.ldQt] = Qt[i + j * kk];
    }
}

// ---------------------------------------------------------------------------
// host launchers
static size_t ritz_smem(int kmax) { return (size_t)(2 * kmax * kmax) * sizeof(zd); }

void launch_ritz(const RitzArgs& a, int kmax, hipStream_t s)
{
    if (a.njobs <= 0) return;
    size_t sm = ritz_smem(kmax);
    hipLaunchKernelGGL(k_ritz, dim3(a.njobs), dim3(NT), sm, s, a);
}
// Problems of dimension <= 32 run on a single wavefront: their sweeps are
// barrier-bound, and a one-wave workgroup makes every barrier nearly free.
void launch_chol_dd(const CholArgs& a, int nb, hipStream_t s)
{
    if (nb <= 0) return;
    int th = (a.c <= 32) ? 64 : NT;   // a.c: the (maximum) dimension
    hipLaunchKernelGGL(k_chol_dd, dim3(nb), dim3(th), 0, s, a);
}
void launch_rr_hl(const RRArgs& a, int nb, int cmax, hipStream_t s)
{
    if (nb <= 0) return;
    size_t sm = (size_t)(2 * cmax * cmax + 2 * cmax * a.r) * sizeof(zd);
    hipLaunchKernelGGL(k_rr_hl, dim3(nb), dim3(cmax <= 32 ? 64 : NT), sm, s, a);
}
void launch_svqb(const SvqbArgs& a, int nb, hipStream_t s)
{
    if (nb <= 0) return;
    size_t sm = (size_t)(2 * a.r * a.r) * sizeof(zd);
    hipLaunchKernelGGL(k_svqb, dim3(nb), dim3(a.r <= 32 ? 64 : NT), sm, s, a);
}
void launch_rotations(const RotArgs& a, int nb, int qmax, hipStream_t s)
{
    if (nb <= 0) return;
    int kk = (qmax + 1) * a.r, r = a.r;
    size_t sm = (size_t)(kk * kk + 2 * r * r + 4 * r * r + kk * 2 * r + r * r) * sizeof(zd);
    hipLaunchKernelGGL(k_rotations, dim3(nb), dim3(NT), sm, s, a);
}

int small_kernels_max_lds() { return g_max_lds; }

void small_kernels_init()
{
    // Ask for the device's full LDS per workgroup for the LDS-resident
    // kernels, once per process (handles may be created from several
    // threads); if the runtime refuses, keep the default limit and clear the
    // error so that it does not surface at a later call.
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, mx = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && mx > 0)
            g_max_lds = mx;
        const void* ks[] = {(const void*)k_ritz, (const void*)k_rr_hl, (const void*)k_svqb, (const void*)k_rotations};
        for (const void* k : ks) {
            if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, g_max_lds - 4096) != hipSuccess)
                (void)hipGetLastError();
        }
        (void)hipGetLastError();
    });
}
