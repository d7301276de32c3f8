// Tall-skinny batched kernels: Gram matrices (double or double-double
// accumulation), products with small matrices, column norms and the
// elementwise epilogues of LOBPCG-SVD.  All are HBM-bandwidth kernels; one
// launch covers every active tile.
#include "zdev.h"
#include "kernels.h"

#define NT 256

// array index of block b for tile t
__device__ __host__ inline int bl_t(const BlockList& L, int b, int t)
{
    return L.imap[b] ? L.imap[b][t] : t;
}
// column count of block b for tile t
__device__ __host__ inline int bl_cols(const BlockList& L, int b, int t)
{
    return L.dims[b] ? L.dims[b][bl_t(L, b, t)] * L.mul[b] : L.ncols[b];
}
// column c of tile t: pointer to its first element and the rows stored
// (NULL beyond the tile's columns)
__device__ inline const zd* bl_col(const BlockList& L, int t, int c, int64_t& rows)
{
    for (int b = 0; b < L.nb; ++b) {
        const int nc = bl_cols(L, b, t);
        if (c < nc) {
            rows = L.brows[b] ? L.brows[b] : L.rows;
            const int tb = bl_t(L, b, t);
            const int c0 = L.coff[b] ? L.coff[b][tb] * L.coffmul[b] : 0;
            return L.ptr[b] + (size_t)tb * L.stride[b] + (size_t)(c + c0) * L.ld[b];
        }
        c -= nc;
    }
    rows = 0;
    return nullptr;
}
__device__ inline int bl_total(const BlockList& L, int t)
{
    int s = 0;
    for (int b = 0; b < L.nb; ++b) s += bl_cols(L, b, t);
    return s;
}

// v where keep holds, +0 otherwise, by a bit mask. The Gram staging below loads
// from a clamped in-bounds address unconditionally and masks the value: a
// conditional load must complete before the code after it, which keeps the
// next loads from being issued early, and a select on the loaded value can
// be turned into a load through a selected private-memory address
__device__ __forceinline__ zd zkeep(zd v, bool keep)
{
    const unsigned long long m = keep ? ~0ull : 0ull;
    return zmake(__longlong_as_double(__double_as_longlong(v.x) & m),
                 __longlong_as_double(__double_as_longlong(v.y) & m));
}

// ---------------------------------------------------------------------------
// Gram: part[(tile, chunk)] = A[rows of chunk]^* B[rows of chunk] for one
// CA x CB output tile per workgroup (grid: chunks x out-tiles x tiles), CA and
// CB the column counts rounded up to 8, 16 or 32, so that narrow blocks do
// not compute padding.  Each thread owns Q outputs; when the tile has fewer
// outputs than threads, G groups of threads split the staged rows and their
// sums are added at the end.
template <int DD, int CA, int CB>
__global__ void __launch_bounds__(NT) k_gram_part(GramArgs a, int ntj)
{
    constexpr int O = CA * CB;
    constexpr int Q = O >= NT ? O / NT : 1;
    constexpr int G = O >= NT ? 1 : NT / O;
    constexpr int SR = 32;                       // rows per staging step
    __shared__ zd As[SR][CA + 1];
    __shared__ zd Bs[SR][CB + 1];
    const int chunk = blockIdx.x;
    const int ot = blockIdx.y;
    const int ti = ot / ntj, tj = ot % ntj;
    const int tix = blockIdx.z;
    const int tile = a.list[tix];
    const int ca = bl_total(a.A, tile), cb = bl_total(a.B, tile);
    if (ti * CA >= ca || tj * CB >= cb) return;
    if (a.hermitian_upper_only && tj * CB + CB - 1 < ti * CA) return;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)chunk * a.chunk_rows;
    int64_t r1 = r0 + a.chunk_rows;
    if (r1 > a.A.rows) r1 = a.A.rows;
    // the columns this thread stages, resolved once into registers (held in
    // LDS, the pointers would lose their address space and every staging
    // load would become a flat load that LDS waits also wait for); a column
    // past the operand's last points at its first column with no rows, so
    // that the staging loads below always have a valid address
    constexpr int QA = (SR * CA + NT - 1) / NT, QB = (SR * CB + NT - 1) / NT;
    const zd* pa[QA];
    const zd* pb[QB];
    int64_t na[QA], nb_[QB];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        const int g = ti * CA + ((tid + NT * q) / SR) % CA;
        int64_t nr = 0;
        pa[q] = bl_col(a.A, tile, g < ca ? g : 0, nr);
        na[q] = (g < ca) ? nr : 0;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const int g = tj * CB + ((tid + NT * q) / SR) % CB;
        int64_t nr = 0;
        pb[q] = bl_col(a.B, tile, g < cb ? g : 0, nr);
        nb_[q] = (g < cb) ? nr : 0;
    }
    int oi[Q], oj[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int o = (G == 1) ? tid + NT * q : tid % O;
        oi[q] = o % CA;
        oj[q] = o / CA;
    }
    const int grp = (G == 1) ? 0 : tid / O;
    zacc acc[Q];
    zd accd[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) { zacc_init(acc[q]); accd[q] = zmake(0.0, 0.0); }
    for (int64_t rb = r0; rb < r1; rb += SR) {
        // stage SR rows of the CA + CB columns (consecutive threads take
        // consecutive rows of one column)
        zd va[QA], vb[QB];
        bool ka[QA], kb[QB];
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            const int64_t i = rb + e % SR;
            ka[q] = e < SR * CA && i < r1 && i < na[q];
            va[q] = pa[q][ka[q] ? i : 0];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            const int64_t i = rb + e % SR;
            kb[q] = e < SR * CB && i < r1 && i < nb_[q];
            vb[q] = pb[q][kb[q] ? i : 0];
        }
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            if (e < SR * CA) As[e % SR][e / SR] = zkeep(va[q], ka[q]);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            if (e < SR * CB) Bs[e % SR][e / SR] = zkeep(vb[q], kb[q]);
        }
        __syncthreads();
        const int nr = (int)((r1 - rb) < SR ? (r1 - rb) : SR);
        for (int rr = grp; rr < nr; rr += G) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const zd x = As[rr][oi[q]], y = Bs[rr][oj[q]];
                if (DD) zacc_cfma(acc[q], x, y);
                else zcfma(accd[q], x, y);
            }
        }
        __syncthreads();
    }
    const size_t base = ((size_t)tix * a.nchunks + chunk) * a.part_stride;
    if (G == 1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int gi = ti * CA + oi[q], gj = tj * CB + oj[q];
            if (gi < ca && gj < cb) {
                const size_t off = base + gi + (size_t)gj * a.camax;
                if (DD) ((zdd*)a.part)[off] = zacc_value(acc[q]);
                else ((zd*)a.part)[off] = accd[q];
            }
        }
        return;
    }
    // G > 1: add the groups' sums (double-double for DD)
    __shared__ zdd red[(O < NT) ? NT : 1];
    red[tid] = DD ? zacc_value(acc[0]) : zdd{dd_make(accd[0].x), dd_make(accd[0].y)};
    __syncthreads();
    if (grp == 0) {
        zdd sum = red[tid];
        for (int h = 1; h < G; ++h) sum = zdd_add(sum, red[tid + h * O]);
        const int gi = ti * CA + oi[0], gj = tj * CB + oj[0];
        if (gi < ca && gj < cb) {
            const size_t off = base + gi + (size_t)gj * a.camax;
            if (DD) ((zdd*)a.part)[off] = sum;
            else ((zd*)a.part)[off] = zmake(sum.x.hi + sum.x.lo, sum.y.hi + sum.y.lo);
        }
    }
}

template <int DD>
__global__ void __launch_bounds__(NT) k_gram_reduce(GramArgs a)
{
    const int tix = blockIdx.y;
    const int tile = a.list[tix];
    const int ca = bl_total(a.A, tile), cb = bl_total(a.B, tile);
    int e = blockIdx.x * NT + threadIdx.x;
    if (e >= ca * cb) return;
    int gi = e % ca, gj = e / ca;
    if (a.hermitian_upper_only && (gj / 32) < (gi / 32)) return;
    const size_t base = (size_t)tix * a.nchunks * a.part_stride + gi + (size_t)gj * a.camax;
    if (DD) {
        zdd s = zdd_zero();
        for (int c = 0; c < a.nchunks; ++c) {
            int64_t r0 = (int64_t)c * a.chunk_rows;
            if (r0 >= a.A.rows) break;
            s = zdd_add(s, ((const zdd*)a.part)[base + (size_t)c * a.part_stride]);
        }
        ((zdd*)a.out)[(size_t)tile * a.strideOut + gi + (size_t)gj * a.ldOut] = s;
    } else {
        zd s = zmake(0.0, 0.0);
        for (int c = 0; c < a.nchunks; ++c) {
            int64_t r0 = (int64_t)c * a.chunk_rows;
            if (r0 >= a.A.rows) break;
            s = zadd(s, ((const zd*)a.part)[base + (size_t)c * a.part_stride]);
        }
        if (a.out_dd) {
            zdd v;
            v.x = dd_make(s.x);
            v.y = dd_make(s.y);
            ((zdd*)a.out)[(size_t)tile * a.strideOut + gi + (size_t)gj * a.ldOut] = v;
        } else {
            ((zd*)a.out)[(size_t)tile * a.strideOut + gi + (size_t)gj * a.ldOut] = s;
        }
    }
}

size_t gram_part_bytes(int64_t rows, int camax, int cbmax, int ntiles, int dd, int chunk_rows)
{
    int64_t nch = (rows + chunk_rows - 1) / chunk_rows;
    return (size_t)ntiles * nch * camax * cbmax * (dd ? sizeof(zdd) : sizeof(zd));
}

void launch_gram(GramArgs& a, hipStream_t s)
{
    if (a.ntiles <= 0) return;
    a.nchunks = (int)((a.A.rows + a.chunk_rows - 1) / a.chunk_rows);
    a.part_stride = (int64_t)a.camax * a.cbmax;
    const int ta = a.camax <= 8 ? 8 : (a.camax <= 16 ? 16 : 32);
    const int tb = a.cbmax <= 8 ? 8 : (a.cbmax <= 16 ? 16 : 32);
    const int nti = (a.camax + ta - 1) / ta, ntj = (a.cbmax + tb - 1) / tb;
    dim3 g1(a.nchunks, nti * ntj, a.ntiles);
    dim3 g2((a.camax * a.cbmax + NT - 1) / NT, a.ntiles);
#define GRAM_PART(DDV, X, Y) hipLaunchKernelGGL((k_gram_part<DDV, X, Y>), g1, dim3(NT), 0, s, a, ntj)
#define GRAM_ROW(DDV, X)                        \
    do {                                        \
        if (tb == 8) GRAM_PART(DDV, X, 8);      \
        else if (tb == 16) GRAM_PART(DDV, X, 16); \
        else GRAM_PART(DDV, X, 32);             \
    } while (0)
    if (a.dd) {
        if (ta == 8) GRAM_ROW(1, 8);
        else if (ta == 16) GRAM_ROW(1, 16);
        else GRAM_ROW(1, 32);
        hipLaunchKernelGGL(k_gram_reduce<1>, g2, dim3(NT), 0, s, a);
    } else {
        if (ta == 8) GRAM_ROW(0, 8);
        else if (ta == 16) GRAM_ROW(0, 16);
        else GRAM_ROW(0, 32);
        hipLaunchKernelGGL(k_gram_reduce<0>, g2, dim3(NT), 0, s, a);
    }
#undef GRAM_ROW
#undef GRAM_PART
}

// ---------------------------------------------------------------------------
// Y[:, chunk] = A G[:, chunk] (+ Y if beta == 1): one row per thread,
// 16 output columns per workgroup column (grid: rowblocks x colchunks x tiles)
#define TSC 16
__global__ void __launch_bounds__(NT) k_gemm_ts(GemmTSArgs a)
{
    extern __shared__ double smem_d[];
    zd* Gs = (zd*)smem_d;   // camax x TSC
    const int tix = blockIdx.z;
    const int tile = a.list[tix];
    const int ca = bl_total(a.A, tile);
    const int cb = a.cbdims ? a.cbdims[tile] * a.cbmul : a.cb;
    const int c0 = blockIdx.y * TSC;
    if (c0 >= cb) return;
    const int nc = min(TSC, cb - c0);
    const zd* G = a.G + (size_t)tile * a.strideG;
    for (int e = threadIdx.x; e < ca * TSC; e += NT) {
        int i = e % ca, j = e / ca;
        Gs[i + j * ca] = (j < nc) ? G[i + (size_t)(c0 + j) * a.ldG] : zmake(0.0, 0.0);
    }
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (row >= a.rows) return;
    zd acc[TSC];
#pragma unroll
    for (int j = 0; j < TSC; ++j) acc[j] = zmake(0.0, 0.0);
    int cglob = 0;
    for (int b = 0; b < a.A.nb; ++b) {
        int ncb = bl_cols(a.A, b, tile);
        int64_t br = a.A.brows[b] ? a.A.brows[b] : a.A.rows;
        if (row < br) {
            const int tb = bl_t(a.A, b, tile);
            int cof = a.A.coff[b] ? a.A.coff[b][tb] * a.A.coffmul[b] : 0;
            const zd* p = a.A.ptr[b] + (size_t)tb * a.A.stride[b] + (size_t)cof * a.A.ld[b] + row;
            const int64_t ld = a.A.ld[b];
            int c = 0;
            // four columns' loads in flight at once; per output column the
            // products are still added in column order
            for (; c + 4 <= ncb; c += 4) {
                const zd x0 = p[(size_t)c * ld], x1 = p[(size_t)(c + 1) * ld];
                const zd x2 = p[(size_t)(c + 2) * ld], x3 = p[(size_t)(c + 3) * ld];
                const zd* gr = Gs + (cglob + c);
#pragma unroll
                for (int j = 0; j < TSC; ++j) {
                    zfma(acc[j], x0, gr[j * ca]);
                    zfma(acc[j], x1, gr[j * ca + 1]);
                    zfma(acc[j], x2, gr[j * ca + 2]);
                    zfma(acc[j], x3, gr[j * ca + 3]);
                }
            }
            for (; c < ncb; ++c) {
                const zd x = p[(size_t)c * ld];
                const zd* gr = Gs + (cglob + c);
#pragma unroll
                for (int j = 0; j < TSC; ++j) zfma(acc[j], x, gr[j * ca]);
            }
        }
        cglob += ncb;
    }
    zd* Y = a.Y + (size_t)tile * a.strideY + row;
    // the old values are all read before the first store (column c0 stands
    // in for the columns past nc)
    zd yo[TSC];
    if (a.beta != 0.0) {
#pragma unroll
        for (int j = 0; j < TSC; ++j) yo[j] = Y[(size_t)(c0 + (j < nc ? j : 0)) * a.ldY];
    }
#pragma unroll
    for (int j = 0; j < TSC; ++j) {
        if (j < nc) {
            zd v = zscale(acc[j], a.alpha);
            if (a.beta != 0.0) v = zadd(v, yo[j]);
            Y[(size_t)(c0 + j) * a.ldY] = v;
        }
    }
}

void launch_gemm_ts(const GemmTSArgs& a, hipStream_t s)
{
    if (a.ntiles <= 0 || a.rows <= 0) return;
    dim3 g((unsigned)((a.rows + NT - 1) / NT), (a.cbmax + TSC - 1) / TSC, a.ntiles);
    size_t sm = (size_t)a.camax * TSC * sizeof(zd);
    hipLaunchKernelGGL(k_gemm_ts, g, dim3(NT), sm, s, a);
}

// ---------------------------------------------------------------------------
// column squared norms: partials per chunk, then reduce
__global__ void __launch_bounds__(NT) k_colnorm_part(NormArgs a)
{
    const int chunk = blockIdx.x;
    const int tix = blockIdx.y;
    const int tile = a.list[tix];
    const int ca = bl_total(a.A, tile);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = (int64_t)chunk * a.chunk_rows;
    int64_t r1 = r0 + a.chunk_rows;
    if (r1 > a.A.rows) r1 = a.A.rows;
    for (int c = w; c < ca; c += NT / 64) {
        double s = 0;
        int64_t nr = 0;
        const zd* col = bl_col(a.A, tile, c, nr);
        const int64_t re = r1 < nr ? r1 : nr;
        int64_t i = r0 + lane;
        // four loads in flight at once; the sum keeps the row order
        for (; i + 192 < re; i += 256) {
            const zd v0 = col[i], v1 = col[i + 64], v2 = col[i + 128], v3 = col[i + 192];
            s += zabs2(v0);
            s += zabs2(v1);
            s += zabs2(v2);
            s += zabs2(v3);
        }
        for (; i < re; i += 64) s += zabs2(col[i]);
        s = wave_sum(s);
        if (lane == 0) a.part[((size_t)tix * a.nchunks + chunk) * a.camax + c] = s;
    }
}
__global__ void k_colnorm_reduce(NormArgs a)
{
    const int tix = blockIdx.x;
    const int tile = a.list[tix];
    const int ca = bl_total(a.A, tile);
    for (int c = threadIdx.x; c < ca; c += blockDim.x) {
        double s = 0;
        for (int ch = 0; ch < a.nchunks; ++ch) s += a.part[((size_t)tix * a.nchunks + ch) * a.camax + c];
        a.out[(size_t)tile * a.ldo + c] = s;
    }
}
void launch_colnorm2(NormArgs& a, hipStream_t s)
{
    if (a.ntiles <= 0) return;
    a.nchunks = (int)((a.A.rows + a.chunk_rows - 1) / a.chunk_rows);
    hipLaunchKernelGGL(k_colnorm_part, dim3(a.nchunks, a.ntiles), dim3(NT), 0, s, a);
    hipLaunchKernelGGL(k_colnorm_reduce, dim3(a.ntiles), dim3(64), 0, s, a);
}

// ---------------------------------------------------------------------------
// elementwise
__global__ void k_copy_cols(const int* list, const zd* src, int64_t sstride, int64_t lds, zd* dst,
                            int64_t dstride, int64_t ldd, int64_t rows, int cols)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t i = e % rows, j = e / rows;
    dst[(size_t)tile * dstride + i + j * ldd] = src[(size_t)tile * sstride + i + j * lds];
}
void launch_copy_cols(const int* list, int ntiles, const zd* src, int64_t sstride, int64_t lds, zd* dst,
                      int64_t dstride, int64_t ldd, int64_t rows, int cols, hipStream_t s)
{
    if (ntiles <= 0 || rows * cols == 0) return;
    dim3 g((unsigned)((rows * cols + NT - 1) / NT), ntiles);
    hipLaunchKernelGGL(k_copy_cols, g, dim3(NT), 0, s, list, src, sstride, lds, dst, dstride, ldd, rows, cols);
}

__global__ void k_scale_cols(const int* list, zd* A, int64_t stride, int64_t lda, int64_t rows, int cols,
                             const double* d, int ldd, int invert)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t i = e % rows, j = e / rows;
    double v = d[(size_t)tile * ldd + j];
    double f = (invert == 2) ? (v > 0.0 ? 1.0 / sqrt(v) : 0.0) : invert ? (v > 0.0 ? 1.0 / v : 0.0) : v;
    zd* p = A + (size_t)tile * stride + i + j * lda;
    *p = zscale(*p, f);
}
void launch_scale_cols(const int* list, int ntiles, zd* A, int64_t stride, int64_t lda, int64_t rows, int cols,
                       const double* d, int ldd, int invert, hipStream_t s)
{
    if (ntiles <= 0 || rows * cols == 0) return;
    dim3 g((unsigned)((rows * cols + NT - 1) / NT), ntiles);
    hipLaunchKernelGGL(k_scale_cols, g, dim3(NT), 0, s, list, A, stride, lda, rows, cols, d, ldd, invert);
}

__global__ void k_resid_xi(const int* list, zd* Y, int64_t ystride, int64_t ldy, const zd* X, int64_t xstride,
                           int64_t ldx, const double* xi, int ldxi, int64_t rows, int cols)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t i = e % rows, j = e / rows;
    double x2 = xi[(size_t)tile * ldxi + j];
    x2 *= x2;
    zd* y = Y + (size_t)tile * ystride + i + j * ldy;
    zd x = X[(size_t)tile * xstride + i + j * ldx];
    *y = zmake(y->x - x2 * x.x, y->y - x2 * x.y);
}
void launch_resid_xi(const int* list, int ntiles, zd* Y, int64_t ystride, int64_t ldy, const zd* X, int64_t xstride,
                     int64_t ldx, const double* xi, int ldxi, int64_t rows, int cols, hipStream_t s)
{
    if (ntiles <= 0 || rows * cols == 0) return;
    dim3 g((unsigned)((rows * cols + NT - 1) / NT), ntiles);
    hipLaunchKernelGGL(k_resid_xi, g, dim3(NT), 0, s, list, Y, ystride, ldy, X, xstride, ldx, xi, ldxi, rows, cols);
}

__global__ void k_randfill(const int* list, zd* A, int64_t stride, int64_t lda, int64_t rows, int cols,
                           const uint32_t* mask, uint64_t seed)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t i = e % rows, j = e / rows;
    if (mask && !((mask[tile] >> j) & 1u)) return;
    uint64_t key = seed ^ ((uint64_t)tile << 48) ^ ((uint64_t)j << 40) ^ (uint64_t)i;
    // Box-Muller on two uniforms
    double u1 = u01(key * 2 + 1), u2 = u01(key * 2 + 2);
    double rad = sqrt(-2.0 * log(u1)) * 0.7071067811865476;
    A[(size_t)tile * stride + i + j * lda] = zmake(rad * cos(6.283185307179586 * u2), rad * sin(6.283185307179586 * u2));
}
void launch_randfill(const int* list, int ntiles, zd* A, int64_t stride, int64_t lda, int64_t rows, int cols,
                     const uint32_t* mask, uint64_t seed, hipStream_t s)
{
    if (ntiles <= 0 || rows * cols == 0) return;
    dim3 g((unsigned)((rows * cols + NT - 1) / NT), ntiles);
    hipLaunchKernelGGL(k_randfill, g, dim3(NT), 0, s, list, A, stride, lda, rows, cols, mask, seed);
}

__global__ void k_zero(zd* A, int64_t count)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) A[e] = zmake(0.0, 0.0);
}
void launch_zero(zd* A, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, s, A, count);
}

// gamma[t] = x^* y[0:n] for the first columns x of X and y of Y of each tile
// (with y = C(z) x this is (S x)^* C(z) x, the first-order coefficient of
// ||C(z') x|| in z' - z)
__global__ void __launch_bounds__(256) k_tile_dot0(const int* list, const zd* X, int64_t xs, const zd* Y, int64_t ys,
                                                   int64_t n, zd* out)
{
    __shared__ double red[4];
    const int t = list[blockIdx.x];
    const zd* x = X + (size_t)t * xs;
    const zd* y = Y + (size_t)t * ys;
    double re = 0.0, im = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        zd a = x[i], b = y[i];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    re = block_sum(re, red);
    im = block_sum(im, red);
    if (threadIdx.x == 0) out[t] = zmake(re, im);
}

void launch_tile_dot0(const int* list, int ntiles, const zd* X, int64_t xs, const zd* Y, int64_t ys, int64_t n,
                      zd* out, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_tile_dot0, dim3(ntiles), dim3(256), 0, s, list, X, xs, Y, ys, n, out);
}

// gamma_j = g^* H g - z_j for every Ritz job j, g the job's first Ritz
// coefficient vector (unit, k entries) and H = V^* S^* C V of its tile
// (k x k), so gamma_j = (S x)^* C(z_j) x for the Ritz vector x = V g
__global__ void __launch_bounds__(64) k_job_gamma(int njobs, const int* job_tile, const int* kdim, const zd* G,
                                                  int64_t sG, int ldG, const zd* H, int64_t sH, int ldH,
                                                  const zd* z, zd* out)
{
    __shared__ double red[1];
    const int j = blockIdx.x;
    if (j >= njobs) return;
    const int t = job_tile[j];
    const int k = kdim[t];
    const zd* g = G + (size_t)j * sG;
    const zd* Hb = H + (size_t)t * sH;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < k; i += 64) {
        zd s = zmake(0.0, 0.0);
        for (int c = 0; c < k; ++c) zfma(s, Hb[i + (size_t)c * ldH], g[c]);
        zd gi = g[i];
        re += gi.x * s.x + gi.y * s.y;
        im += gi.x * s.y - gi.y * s.x;
    }
    re = block_sum(re, red);
    im = block_sum(im, red);
    if (threadIdx.x == 0) out[j] = (k > 0) ? zmake(re - z[j].x, im - z[j].y) : zmake(0.0, 0.0);
}

void launch_job_gamma(int njobs, const int* job_tile, const int* kdim, const zd* G, int64_t sG, int ldG, const zd* H,
                      int64_t sH, int ldH, const zd* z, zd* out, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_job_gamma, dim3(njobs), dim3(64), 0, s, njobs, job_tile, kdim, G, sG, ldG, H, sH, ldH, z,
                       out);
}
