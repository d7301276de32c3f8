// Kernels of the factorizations of N(z) - mu I, N(z) = (C - z S)^* (C - z S):
// the dense base preconditioner K = F^* F ~ N(z_dag) (Sec. 3, eq. (twolevel)
// and the reconstruction rule of Sec. 3.3), F the upper Cholesky factor of
// N(z_dag) + delta I, and the inertia tests (N(z) - mu I positive definite).
// The blocked Cholesky around them (engine_precond.hip) runs its trailing
// updates and the columns of F^{-1} on the matrix cores (k_zgemm_fact), so
// that K^{-1} W = F^{-1} (F^{-*} W) is two matrix-core products.
#include "zdev.h"
#include "kernels.h"

#define NT 256

// N = C^*C - conj(z) S^*C - z C^*S + (|z|^2 + shift) I for each matrix in list
__global__ void k_form_normal(const int* list, const zd* CtC, const zd* C, int64_t ldc, const zd* CH, int64_t n,
                              const zd* zdag, const double* shift, zd* N, int64_t strideN)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= n * n) return;
    int64_t i = e % n, j = e / n;
    zd z = zdag[tile];
    zd v = CtC[i + j * n];
    zd c = C[i + j * ldc];      // S^* C: first n rows of C
    zd ch = CH[i + j * n];      // C^* S: first n columns of C^*
    v = zsub(v, zmul(zconj(z), c));
    v = zsub(v, zmul(z, ch));
    if (i == j) v.x += zabs2(z) + shift[tile];
    N[(size_t)tile * strideN + i + j * n] = v;
}

void launch_form_normal(const int* list, int nt, const zd* CtC, const zd* C, int64_t ldc, const zd* CH,
                        int64_t n, const zd* zdag, const double* shift, zd* N, int64_t strideN, hipStream_t s)
{
    if (nt <= 0) return;
    dim3 g((unsigned)((n * n + NT - 1) / NT), nt);
    hipLaunchKernelGGL(k_form_normal, g, dim3(NT), 0, s, list, CtC, C, ldc, CH, n, zdag, shift, N, strideN);
}

// One step of the blocked Cholesky, fused: every workgroup of the grid
// (chunk, matrix) factors the diagonal block A_kk (kb <= 32, upper triangle
// read) redundantly in LDS and forms X = R_kk^{-1}; chunk 0 writes X into
// Dinv and into the diagonal block of Finv (when non-null) and raises notpd
// on a non-positive pivot; chunk c >= 1 turns the PANEL_CHUNK columns
// k1 + (c - 1) PANEL_CHUNK ... of the block row (one per thread) into the
// row panel of the factor, A[k, cols] <- R_kk^{-*} A[k, cols] by forward
// substitution.  Replaces a single-workgroup diagonal kernel plus a
// separate panel product per step.
#define PANEL_CHUNK 256
__global__ void __launch_bounds__(NT) k_chol_step(const int* list, zd* A, int64_t strideA, int64_t n, int64_t k0,
                                                  int kb, zd* Dinv, int64_t strideD, zd* Finv, int64_t strideF,
                                                  double floor_piv, int* notpd)
{
    __shared__ zd R[32][33];
    __shared__ zd X[32][33];
    __shared__ int bad;
    const int tile = list[blockIdx.y];
    const int chunk = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t k1 = k0 + kb;
    const int64_t cbeg = k1 + (int64_t)(chunk - 1) * PANEL_CHUNK;
    if (chunk > 0 && cbeg >= n) return;
    zd* Ab = A + (size_t)tile * strideA;
    if (tid == 0) bad = 0;
    // entries outside the kb x kb block hold the identity, so that the
    // register back substitution below runs over all 32 rows unguarded
    for (int e = tid; e < 32 * 32; e += NT) {
        const int i = e & 31, j = e >> 5;
        if (i < kb && j < kb) R[i][j] = (i <= j) ? Ab[k0 + i + (k0 + j) * n] : zmake(0.0, 0.0);
        else R[i][j] = zmake(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // right-looking factorization with one barrier per pivot: in phase j the
    // trailing rows a > j are updated from the unscaled row j
    // (R[a][c] -= conj(R[j][a]) R[j][c] / d_j), and row j - 1, which nothing
    // reads any more, is scaled by 1 / sqrt(d_{j-1})
    // each thread owns up to three entries (a2 <= c) of the upper triangle
    int ua[3], uc[3];
    const int ntri = kb * (kb + 1) / 2;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int u = tid + NT * q, a2 = 0;
        ua[q] = -1;
        uc[q] = 0;
        if (u < ntri) {
            while (u >= kb - a2) {
                u -= kb - a2;
                ++a2;
            }
            ua[q] = a2;
            uc[q] = a2 + u;
        }
    }
    double pprev = 1.0;
    for (int j = 0; j <= kb; ++j) {
        double pj = 1.0, ipj2 = 1.0;
        if (j < kb) {
            double d = R[j][j].x;
            if (!(d > 0.0) && tid == 0) bad = 1;
            if (!(d > floor_piv)) d = floor_piv;
            pj = sqrt(d);
            ipj2 = 1.0 / d;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int a2 = ua[q], c = uc[q];
            if (a2 < 0) continue;
            if (j < kb && a2 > j) R[a2][c] = zsub(R[a2][c], zscale(zcmul(R[j][a2], R[j][c]), ipj2));
            if (j > 0 && a2 == j - 1) R[a2][c] = (c == a2) ? zmake(pprev, 0.0) : zscale(R[a2][c], 1.0 / pprev);
        }
        pprev = pj;
        __syncthreads();
    }
    if (chunk == 0) {
        if (tid == 0 && bad) notpd[tile] = 1;
        zd* Db = Dinv ? Dinv + (size_t)tile * strideD + k0 : nullptr;
        zd* Fb = Finv ? Finv + (size_t)tile * strideF + k0 + k0 * n : nullptr;
        if (!Db && !Fb) return;
        // X = R^{-1} (upper) by back substitution, column c held in the
        // registers of thread c; rows below c come out zero, since x[l] = 0
        // for l > c throughout
        if (tid < kb) {
            const int c = tid;
            zd x[32];
#pragma unroll
            for (int i = 31; i >= 0; --i) {
                zd sacc = zmake(i == c ? 1.0 : 0.0, 0.0);
#pragma unroll
                for (int l = i + 1; l < 32; ++l) sacc = zsub(sacc, zmul(R[i][l], x[l]));
                x[i] = zscale(sacc, 1.0 / R[i][i].x);
            }
#pragma unroll
            for (int i = 0; i < 32; ++i)
                if (i < kb) X[i][c] = x[i];
        }
        __syncthreads();
        // (R_kk is not written back: the other workgroups of this launch
        // read the unfactored block, and later steps need only X and the
        // row panels)
        for (int e = tid; e < kb * kb; e += NT) {
            int i = e % kb, j = e / kb;
            if (Db) Db[i + (int64_t)j * n] = X[i][j];
            if (Fb) Fb[i + (int64_t)j * n] = X[i][j];
        }
        return;
    }
    // R_kk^* Y = A[k, c] for the columns c of this chunk: one column per
    // thread, held in registers, forward substitution with R read from LDS
    const int64_t c = cbeg + tid;
    if (c >= n) return;
    zd* col = Ab + k0 + c * n;
    zd y[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) y[i] = (i < kb) ? col[i] : zmake(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        if (i < kb) {
            zd sacc = y[i];
#pragma unroll
            for (int l = 0; l < i; ++l) sacc = zsub(sacc, zcmul(R[l][i], y[l]));
            y[i] = zscale(sacc, 1.0 / R[i][i].x);
        }
    }
#pragma unroll
    for (int i = 0; i < 32; ++i)
        if (i < kb) col[i] = y[i];
}

void launch_chol_step(const int* list, int nt, zd* A, int64_t strideA, int64_t n, int64_t k0, int kb, zd* Dinv,
                      int64_t strideD, zd* Finv, int64_t strideF, double floor_piv, int* notpd, hipStream_t s)
{
    if (nt <= 0) return;
    const int64_t rest = n - (k0 + kb);
    const unsigned chunks = 1 + (unsigned)((rest + PANEL_CHUNK - 1) / PANEL_CHUNK);
    hipLaunchKernelGGL(k_chol_step, dim3(chunks, nt), dim3(NT), 0, s, list, A, strideA, n, k0, kb, Dinv, strideD,
                       Finv, strideF, floor_piv, notpd);
}

__global__ void k_zero_tiles(const int* list, zd* A, int64_t stride, int64_t count)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e < count) A[(size_t)tile * stride + e] = zmake(0.0, 0.0);
}

void launch_zero_tiles(const int* list, int nt, zd* A, int64_t stride, int64_t count, hipStream_t s)
{
    if (nt <= 0 || count <= 0) return;
    dim3 g((unsigned)((count + NT - 1) / NT), nt);
    hipLaunchKernelGGL(k_zero_tiles, g, dim3(NT), 0, s, list, A, stride, count);
}
