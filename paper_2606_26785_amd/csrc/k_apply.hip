// Operator applies C X and C^* Y for the column blocks of many tiles at once.
//
// Dense C: complex GEMM on the FP64 matrix cores.  The complex product is
// split into four real products accumulated into two 16 x 16 accumulators
// (re += Ar Xr - Ai Xi, im += Ar Xi + Ai Xr) with v_mfma_f64_16x16x4f64.
// Tiles of A (64 x 32) and X (32 x 32) are staged through LDS.  K is split
// over workgroups so that narrow right-hand sides still fill all 256 CUs; a
// second pass sums the partials and applies the shift epilogue
//   Y[:n] -= z X[:n]          (C(z) X = C X - z S X, S = [I_n; 0]), or
//   Y     -= conj(z) X[:n]    (C(z)^* Y = C^* Y - conj(z) S^* Y).
// Sparse C: CSR, one thread per (row, tile), looping over the w columns.
#include "zdev.h"
#include "kernels.h"

typedef double dvec4 __attribute__((ext_vector_type(4)));

#define BM 64
#define BN 32
#define BK 32
#define NT 256

__global__ void __launch_bounds__(NT) k_dense_gemm(DenseApplyArgs a, int64_t kchunk)
{
    __shared__ zd As[BK][BM + 1];
    __shared__ zd Xs[BK][BN + 1];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t i0 = (int64_t)blockIdx.x * BM;
    const int j0 = blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    int64_t kend = kbeg + kchunk;
    if (kend > a.K) kend = a.K;
    const int N = a.ntiles * a.w;

    // this thread's X column for staging loads: column jl = tid % BN, rows tid / BN + 8 q
    const int jl = tid % BN;
    const int gc = j0 + jl;
    const zd* xcol = nullptr;
    if (gc < N) {
        int t = gc / a.w, j = gc - t * a.w;
        xcol = a.X + (size_t)a.list[t] * a.xstride + (size_t)j * a.ldx;
    }
    dvec4 acc_re[2], acc_im[2];
    for (int c = 0; c < 2; ++c) {
        acc_re[c] = (dvec4){0.0, 0.0, 0.0, 0.0};
        acc_im[c] = (dvec4){0.0, 0.0, 0.0, 0.0};
    }
    const int mrow = lane & 15;     // row within a 16-row block (A operand) / column (B operand)
    const int kq = lane >> 4;       // k index within the 4-wide step
    // software pipeline: the next K tile is loaded into registers while the
    // matrix cores work on the current one from LDS
    constexpr int AQ = BM * BK / NT, XQ = BK * BN / NT;
    zd ra[AQ], rx[XQ];
    auto gload = [&](int64_t kt) {
        const int64_t gi = i0 + tid % BM;
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int64_t gk = kt + tid / BM + (NT / BM) * q;
            ra[q] = (gi < a.m && gk < kend) ? a.A[gi + gk * a.lda] : zmake(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < XQ; ++q) {
            const int64_t gk = kt + tid / BN + (NT / BN) * q;
            rx[q] = (xcol && gk < kend) ? xcol[gk] : zmake(0.0, 0.0);
        }
    };
    if (kbeg < kend) gload(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) As[tid / BM + (NT / BM) * q][tid % BM] = ra[q];
#pragma unroll
        for (int q = 0; q < XQ; ++q) Xs[tid / BN + (NT / BN) * q][jl] = rx[q];
        __syncthreads();
        if (k0 + BK < kend) gload(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            zd av = As[ks + kq][wave * 16 + mrow];
            double ar = av.x, ai = av.y, nai = -av.y;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                zd xv = Xs[ks + kq][cb * 16 + mrow];
                acc_re[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xv.x, acc_re[cb], 0, 0, 0);
                acc_re[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, xv.y, acc_re[cb], 0, 0, 0);
                acc_im[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xv.y, acc_im[cb], 0, 0, 0);
                acc_im[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, xv.x, acc_im[cb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D layout of v_mfma_f64_16x16x4f64: lane l, element v -> row (l / 16) + 4 v, column l % 16
    zd* part = a.part + (size_t)blockIdx.z * (size_t)a.m * N;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        int col = j0 + cb * 16 + (lane & 15);
        if (col >= N) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int64_t row = i0 + wave * 16 + (lane >> 4) + 4 * v;
            if (row < a.m) part[row + (size_t)col * a.m] = zmake(acc_re[cb][v], acc_im[cb][v]);
        }
    }
}

__global__ void __launch_bounds__(NT) k_dense_reduce(DenseApplyArgs a)
{
    const int N = a.ntiles * a.w;
    int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= a.m * N) return;
    int64_t row = e % a.m;
    int col = (int)(e / a.m);
    zd s = zmake(0.0, 0.0);
    for (int z = 0; z < a.splitk; ++z) s = zadd(s, a.part[(size_t)z * a.m * N + e]);
    int t = col / a.w, j = col - t * a.w;
    int tile = a.list[t];
    if (a.z && row < a.nshift) {
        zd zz = a.z[tile];
        if (a.conjz) zz.y = -zz.y;
        zd x = a.X[(size_t)tile * a.xstride + row + (size_t)j * a.ldx];
        s = zsub(s, zmul(zz, x));
    }
    a.Y[(size_t)tile * a.ystride + row + (size_t)j * a.ldy] = s;
}

size_t dense_apply_part_bytes(int64_t m, int maxcols, int splitk)
{
    return (size_t)m * maxcols * splitk * sizeof(zd);
}

void launch_dense_apply(DenseApplyArgs& a, hipStream_t s)
{
    if (a.ntiles <= 0) return;
    const int N = a.ntiles * a.w;
    int64_t mb = (a.m + BM - 1) / BM;
    int nbk = (N + BN - 1) / BN;
    // enough workgroups to fill the chip: aim for ~2048
    int64_t base = mb * nbk;
    int sk = (int)((2048 + base - 1) / base);
    int64_t maxsk = (a.K + BK * 4 - 1) / (BK * 4);
    if (sk > maxsk) sk = (int)maxsk;
    if (sk > a.splitk) sk = a.splitk;   // a.splitk carries the workspace capacity
    if (sk < 1) sk = 1;
    int64_t kchunk = (a.K + sk - 1) / sk;
    kchunk = (kchunk + BK - 1) / BK * BK;
    sk = (int)((a.K + kchunk - 1) / kchunk);
    a.splitk = sk;
    hipLaunchKernelGGL(k_dense_gemm, dim3((unsigned)mb, nbk, sk), dim3(NT), 0, s, a, kchunk);
    int64_t tot = a.m * N;
    hipLaunchKernelGGL(k_dense_reduce, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, s, a);
}

// ---------------------------------------------------------------------------
// CSR SpMM: one thread per (row, group of CSR_CW right-hand-side columns),
// the columns of all listed tiles flattened (tile-major, w per tile).  The
// row's values and column indices are loaded once per group and used for
// every column of it; neighbouring threads take neighbouring rows, so the
// loads of X (same stencil offset) and the stores of Y are coalesced.
#define CSR_CW 8
__global__ void __launch_bounds__(NT) k_csr_apply(CsrApplyArgs a)
{
    const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (row >= a.m) return;
    const int q0 = blockIdx.y * CSR_CW;
    const int qtot = a.ntiles * a.w;
    const int nq = min(CSR_CW, qtot - q0);
    const zd* xc[CSR_CW];
    zd* yc[CSR_CW];
    zd zz[CSR_CW];
    zd acc[CSR_CW];
#pragma unroll
    for (int k = 0; k < CSR_CW; ++k) {
        const int q = q0 + (k < nq ? k : 0);
        const int tile = a.list[q / a.w], j = q % a.w;
        xc[k] = a.X + (size_t)tile * a.xstride + (size_t)j * a.ldx;
        yc[k] = a.Y + (size_t)tile * a.ystride + (size_t)j * a.ldy;
        zz[k] = zmake(0.0, 0.0);
        if (a.z) { zz[k] = a.z[tile]; if (a.conjz) zz[k].y = -zz[k].y; }
        acc[k] = zmake(0.0, 0.0);
    }
    const int64_t b = a.rowptr[row], e = a.rowptr[row + 1];
    for (int64_t p = b; p < e; ++p) {
        const zd v = a.vals[p];
        const int32_t c = a.colind[p];
#pragma unroll
        for (int k = 0; k < CSR_CW; ++k)
            if (k < nq) zfma(acc[k], v, xc[k][c]);
    }
#pragma unroll
    for (int k = 0; k < CSR_CW; ++k) {
        if (k < nq) {
            zd s = acc[k];
            if (a.z && row < a.nshift) s = zsub(s, zmul(zz[k], xc[k][row]));
            yc[k][row] = s;
        }
    }
}

void launch_csr_apply(const CsrApplyArgs& a, hipStream_t s)
{
    if (a.ntiles <= 0 || a.w <= 0) return;
    const int qtot = a.ntiles * a.w;
    dim3 g((unsigned)((a.m + NT - 1) / NT), (unsigned)((qtot + CSR_CW - 1) / CSR_CW));
    hipLaunchKernelGGL(k_csr_apply, g, dim3(NT), 0, s, a);
}

// ---------------------------------------------------------------------------
// Batched complex GEMM on the FP64 matrix cores:
//   C_b[0:M, 0:N] = alpha op(A_b) B_b + beta C_b,  op(A) = A or A^*,
// one matrix triple per entry of the batch list (pointer + list[i] * stride).
// With upper != 0 only 64 x 32 tiles that touch the upper triangle of C are
// computed (Hermitian rank-k updates).  The K loop of a workgroup finishes
// before its epilogue writes, so C may alias B when M <= 64 (in-place
// left-multiplication of a panel by a small matrix).
// Four waves, each 16 rows x 32 columns of the 64 x 32 tile (2 MFMA
// blocks); TBK is the K step staged through LDS.
// v where keep holds, +0 otherwise, by a bit mask: a select on the value
// would let the compiler turn the staging into a load through a selected
// private-memory address
__device__ __forceinline__ zd zkeep(zd v, bool keep)
{
    const unsigned long long m = keep ? ~0ull : 0ull;
    return zmake(__longlong_as_double(__double_as_longlong(v.x) & m),
                 __longlong_as_double(__double_as_longlong(v.y) & m));
}

template <int TBK>
__device__ __forceinline__ void k_zgemm_body(const ZgemmArgs& a)
{
    constexpr int TBN = BN;
    constexpr int RB = 1;   // 16-row blocks per wave
    __shared__ zd As[TBK][BM + 1];
    __shared__ zd Bs[TBK][TBN + 1];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr0 = wave * 16;   // wave's first row in the tile
    const int wc0 = 0;           // wave's first column
    const int64_t i0 = (int64_t)blockIdx.x * BM;
    const int64_t j0 = (int64_t)blockIdx.y * TBN;
    const int nb = gridDim.z / a.splitk;
    const int bidx = blockIdx.z % nb, split = blockIdx.z / nb;
    const int tile = a.list ? a.list[bidx] : bidx;
    if (a.upper && i0 > j0 + TBN - 1) return;
    const int64_t Nb = a.gtile ? (int64_t)a.gcnt[bidx] * a.cw : a.N;
    if (j0 >= Nb) return;
    const int* gt = a.gtile ? a.gtile + a.goff[bidx] : nullptr;
    const int64_t kc = (a.K + a.splitk - 1) / a.splitk;
    int64_t kbeg = (int64_t)split * kc;
    int64_t kend = (kbeg + kc < a.K) ? kbeg + kc : a.K;
    // triangular A: rows i0..i0+63 have nonzeros only in k >= i0 (upper) or
    // k < i0 + 64 (lower); the staging masks below keep the rest at zero
    if (a.tri == 1 && kbeg < i0) kbeg = (i0 / TBK) * TBK > kbeg ? (i0 / TBK) * TBK : kbeg;
    if (a.tri == 2 && kend > i0 + BM) kend = i0 + BM;
    const zd* A = a.A + (size_t)tile * a.strideA;
    const zd* B = a.B + (size_t)(gt ? 0 : tile) * a.strideB;
    zd* C = a.C + (size_t)(gt ? 0 : tile) * a.strideC;
    // B staging: thread tid loads rows k0 + tid % TBK of columns
    // j0 + tid / TBK + (NT / TBK) q, q = 0 .. TBN*TBK/NT - 1; their base
    // pointers (column-map mode: through the tile map) are fixed for the
    // whole K loop
    constexpr int BQ = TBN * TBK / NT;
    const zd* bcol[BQ];
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
        int64_t gj = j0 + tid / TBK + (NT / TBK) * q;
        bcol[q] = B;
        if (gj < Nb) bcol[q] = gt ? B + (size_t)gt[gj / a.cw] * a.strideB + (gj % a.cw) * a.ldb : B + gj * a.ldb;
    }
    dvec4 acc_re[RB][2], acc_im[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            acc_re[rb][c] = (dvec4){0.0, 0.0, 0.0, 0.0};
            acc_im[rb][c] = (dvec4){0.0, 0.0, 0.0, 0.0};
        }
    const int mrow = lane & 15, kq = lane >> 4;
    // software pipeline: the next K tile is loaded into registers while the
    // matrix cores work on the current one from LDS
    constexpr int AQ = BM * TBK / NT;
    // every load is issued unconditionally (an element outside the operand
    // reads the operand's first element instead) and masked when staged
    // into LDS: a conditional load would have to complete before the
    // matrix-core work of the current tile, which defeats the prefetch
    zd ra[AQ], rb_[BQ];
    auto a_ok = [&](int q, int64_t kt) {
        if (a.opA == 0) return i0 + tid % BM < a.M && kt + tid / BM + (NT / BM) * q < kend;
        return i0 + tid / TBK + (NT / TBK) * q < a.M && kt + tid % TBK < kend;
    };
    auto b_ok = [&](int q, int64_t kt) { return j0 + tid / TBK + (NT / TBK) * q < Nb && kt + tid % TBK < kend; };
    auto gload = [&](int64_t kt) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int64_t idx = (a.opA == 0) ? (i0 + tid % BM) + (kt + tid / BM + (NT / BM) * q) * a.lda
                                             : (kt + tid % TBK) + (i0 + tid / TBK + (NT / TBK) * q) * a.lda;
            ra[q] = A[a_ok(q, kt) ? idx : 0];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) rb_[q] = bcol[q][b_ok(q, kt) ? kt + tid % TBK : 0];
    };
    if (kbeg < kend) gload(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += TBK) {
        if (a.opA == 0) {
#pragma unroll
            for (int q = 0; q < AQ; ++q) As[tid / BM + (NT / BM) * q][tid % BM] = zkeep(ra[q], a_ok(q, k0));
        } else {
#pragma unroll
            for (int q = 0; q < AQ; ++q)
                As[tid % TBK][tid / TBK + (NT / TBK) * q] = zkeep(zconj(ra[q]), a_ok(q, k0));
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) Bs[tid % TBK][tid / TBK + (NT / TBK) * q] = zkeep(rb_[q], b_ok(q, k0));
        __syncthreads();
        if (k0 + TBK < kend) gload(k0 + TBK);
#pragma unroll
        for (int ks = 0; ks < TBK; ks += 4) {
            double ar[RB], ai[RB], nai[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const zd av = As[ks + kq][wr0 + rb * 16 + mrow];
                ar[rb] = av.x;
                ai[rb] = av.y;
                nai[rb] = -av.y;
            }
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const zd xv = Bs[ks + kq][wc0 + cb * 16 + mrow];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc_re[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[rb], xv.x, acc_re[rb][cb], 0, 0, 0);
                    acc_re[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[rb], xv.y, acc_re[rb][cb], 0, 0, 0);
                    acc_im[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[rb], xv.y, acc_im[rb][cb], 0, 0, 0);
                    acc_im[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[rb], xv.x, acc_im[rb][cb], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        int64_t col = j0 + wc0 + cb * 16 + (lane & 15);
        if (col >= Nb) continue;
        zd* ccol = gt ? C + (size_t)gt[col / a.cw] * a.strideC + (col % a.cw) * a.ldc : C + col * a.ldc;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t row = i0 + wr0 + rb * 16 + (lane >> 4) + 4 * v;
                if (row >= a.M) continue;
                if (a.splitk > 1) {
                    a.ws[((size_t)split * nb + bidx) * a.M * a.N + row + (size_t)col * a.M] =
                        zmake(acc_re[rb][cb][v], acc_im[rb][cb][v]);
                    continue;
                }
                zd val = zmake(a.alpha * acc_re[rb][cb][v], a.alpha * acc_im[rb][cb][v]);
                zd* cp = ccol + row;
                if (a.beta != 0.0) val = zadd(val, *cp);
                *cp = val;
            }
    }
}

// k_zgemm: preconditioner applies and small products; k_zgemm_fact_wide and
// k_zgemm_fact: products inside factorizations at least 64 columns wide and
// narrower ones, under their own names so that profiles separate them.  The
// factorization products take 64 x 32 tiles with a K step of 16: on the
// Hermitian trailing updates of order 400 to 3,900 (rank 128) these ran at
// 1.15 to 1.7 times the rate of 64 x 64 tiles and ahead of K steps of 8, 32
// and 64
__global__ void __launch_bounds__(NT) k_zgemm(ZgemmArgs a) { k_zgemm_body<BK>(a); }
__global__ void __launch_bounds__(NT) k_zgemm_fact(ZgemmArgs a) { k_zgemm_body<16>(a); }
__global__ void __launch_bounds__(NT) k_zgemm_fact_wide(ZgemmArgs a) { k_zgemm_body<16>(a); }

// sum of the split-K partials into C (alpha, beta as in k_zgemm)
__global__ void __launch_bounds__(NT) k_zgemm_reduce(ZgemmArgs a, int nb)
{
    const int bidx = blockIdx.y;
    const int tile = a.list ? a.list[bidx] : bidx;
    int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= a.M * a.N) return;
    int64_t row = e % a.M, col = e / a.M;
    zd* cp;
    if (a.gtile) {
        if (col >= (int64_t)a.gcnt[bidx] * a.cw) return;
        const int ct = a.gtile[a.goff[bidx] + col / a.cw];
        cp = a.C + (size_t)ct * a.strideC + row + (col % a.cw) * a.ldc;
    } else {
        cp = a.C + (size_t)tile * a.strideC + row + col * a.ldc;
    }
    zd s = zmake(0.0, 0.0);
    for (int sp = 0; sp < a.splitk; ++sp) s = zadd(s, a.ws[((size_t)sp * nb + bidx) * a.M * a.N + e]);
    zd val = zscale(s, a.alpha);
    if (a.beta != 0.0) val = zadd(val, *cp);
    *cp = val;
}

void launch_zgemm(const ZgemmArgs& a, int nbatch, hipStream_t s, int fact)
{
    if (nbatch <= 0 || a.M <= 0 || a.N <= 0) return;
    const int sk = a.splitk > 1 ? a.splitk : 1;
    // factorization products at least 64 columns wide under their own name
    const bool wide = (fact == 2) && !a.gtile && a.N >= 64;
    dim3 g((unsigned)((a.M + BM - 1) / BM), (unsigned)((a.N + BN - 1) / BN), nbatch * sk);
    if (wide) hipLaunchKernelGGL(k_zgemm_fact_wide, g, dim3(NT), 0, s, a);
    else if (fact) hipLaunchKernelGGL(k_zgemm_fact, g, dim3(NT), 0, s, a);
    else hipLaunchKernelGGL(k_zgemm, g, dim3(NT), 0, s, a);
    if (sk > 1) {
        dim3 g2((unsigned)((a.M * a.N + NT - 1) / NT), nbatch);
        hipLaunchKernelGGL(k_zgemm_reduce, g2, dim3(NT), 0, s, a, nbatch);
    }
}
