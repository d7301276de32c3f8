// Host-side engine: operator setup, batched building blocks, LOBPCG-SVD,
// the recycled-subspace update and the grid-front scheduler (Alg. 5 per tile).
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

static const double EPSM = 2.220446049250313e-16;

// ---------------------------------------------------------------------------
BlockList bl_empty(int64_t rows)
{
    BlockList L;
    memset(&L, 0, sizeof(L));
    L.rows = rows;
    return L;
}
void bl_map(BlockList& L, const int* imap) { L.imap[L.nb - 1] = imap; }
void bl_add(BlockList& L, const zd* ptr, int64_t stride, int64_t ld, int ncols, const int* dims, int mul,
            int64_t brows, const int* coff, int coffmul)
{
    int b = L.nb++;
    L.ptr[b] = ptr;
    L.stride[b] = stride;
    L.ld[b] = ld;
    L.ncols[b] = ncols;
    L.dims[b] = dims;
    L.mul[b] = mul;
    L.brows[b] = brows;
    L.coff[b] = coff;
    L.coffmul[b] = coffmul;
}

__global__ void k_gather(const int* list, const int* srcidx, const zd* src, int64_t sstride, zd* dst,
                         int64_t dstride, int64_t count)
{
    const int t = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    dst[(size_t)t * dstride + e] = src[(size_t)srcidx[t] * sstride + e];
}
void launch_gather(const int* list, int nt, const int* srcidx, const zd* src, int64_t sstride, zd* dst,
                   int64_t dstride, int64_t count, hipStream_t s)
{
    if (nt <= 0 || count <= 0) return;
    dim3 g((unsigned)((count + 255) / 256), nt);
    hipLaunchKernelGGL(k_gather, g, dim3(256), 0, s, list, srcidx, src, sstride, dst, dstride, count);
}

// conjugate transpose: B (n x m, ld n) = A^* (A m x n, ld lda)
__global__ void k_conj_transpose(const zd* A, int64_t lda, int64_t m, int64_t n, zd* B)
{
    __shared__ zd t[32][33];
    int64_t bi = (int64_t)blockIdx.x * 32, bj = (int64_t)blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        int64_t i = bi + threadIdx.x, j = bj + k;
        if (i < m && j < n) t[k][threadIdx.x] = A[i + j * lda];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        int64_t j = bj + threadIdx.x, i = bi + k;
        if (i < m && j < n) B[j + i * n] = zconj(t[threadIdx.x][k]);
    }
}

// sqrt-and-invert helper for column scaling: d holds squared norms
__global__ void k_scale_cols_rsqrt(const int* list, zd* A, int64_t stride, int64_t lda, int64_t rows, int cols,
                                   const double* d, int ldd)
{
    const int tile = list[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t i = e % rows, j = e / rows;
    double v = d[(size_t)tile * ldd + j];
    double f = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    zd* p = A + (size_t)tile * stride + i + j * lda;
    *p = zscale(*p, f);
}

// ---------------------------------------------------------------------------
int KProf::begin(hipStream_t s, int c, double fl, double by)
{
    if (!on || (c >= 5 && c <= 7 && level < 2)) return -1;
    if (2 * used + 2 > ev.size()) {
        size_t old = ev.size();
        ev.resize(std::max<size_t>(64, 2 * old));
        for (size_t i = old; i < ev.size(); ++i) HIPCHK(hipEventCreate(&ev[i]));
    }
    if (cls.size() <= used) { cls.resize(used + 1); flops.resize(used + 1); bytes.resize(used + 1); }
    cls[used] = c;
    flops[used] = fl;
    bytes[used] = by;
    HIPCHK(hipEventRecord(ev[2 * used], s));
    return (int)used++;
}
void KProf::end(hipStream_t s, int idx)
{
    if (idx < 0) return;
    HIPCHK(hipEventRecord(ev[2 * idx + 1], s));
}
void KProf::collect(ps_stats& st)
{
    for (int c = 0; c < PS_NCLASS; ++c) { st.k_launches[c] = 0; st.k_ms[c] = 0; st.k_flops[c] = 0; st.k_bytes[c] = 0; }
    for (size_t i = 0; i < used; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventSynchronize(ev[2 * i + 1]));
        HIPCHK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
        int c = cls[i];
        st.k_launches[c] += 1;
        st.k_ms[c] += ms;
        st.k_flops[c] += flops[i];
        st.k_bytes[c] += bytes[i];
    }
    used = 0;
}
KProf::~KProf()
{
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
void Engine::h2d(void* dst, const void* src, size_t bytes)
{
    if (bytes == 0) return;
    const size_t cap = (size_t)8 << 20;
    if (!ring.p) ring.alloc(cap);
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (need > cap) {
        // larger than the ring: a synchronous copy from the caller's memory
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return;
    }
    if (ring_pos + need > cap) {
        // every earlier slice must have been read before it is overwritten
        HIPCHK(hipStreamSynchronize(st));
        ring_pos = 0;
    }
    memcpy(ring.p + ring_pos, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, ring.p + ring_pos, bytes, hipMemcpyHostToDevice, st));
    ring_pos += need;
}

void Engine::upload_list(const std::vector<int>& L, DBuf<int>& dst)
{
    if (dst.n < std::max<size_t>(L.size(), 1)) {
        // reallocation frees the old buffer: earlier work on the stream may still read it
        HIPCHK(hipStreamSynchronize(st));
        dst.alloc(std::max<size_t>(L.size(), 1));
    }
    if (!L.empty()) h2d(dst.p, L.data(), L.size() * sizeof(int));
}

void Engine::gram(const int* dlist, int nt, const BlockList& A, const BlockList& Bl, int camax, int cbmax,
                  void* out, int64_t strideOut, int ldOut, bool dd, bool upper, bool out_dd)
{
    if (nt <= 0) return;
    GramArgs g;
    memset(&g, 0, sizeof(g));
    g.list = dlist;
    g.ntiles = nt;
    g.A = A;
    g.B = Bl;
    g.camax = camax;
    g.cbmax = cbmax;
    g.out = out;
    g.strideOut = strideOut;
    g.ldOut = ldOut;
    g.part = gram_ws.p;
    g.dd = dd ? 1 : 0;
    g.hermitian_upper_only = upper ? 1 : 0;
    g.out_dd = (!dd && out_dd) ? 1 : 0;
    size_t esz = dd ? sizeof(zdd) : sizeof(zd);
    // rows per chunk: enough chunks to fill the GPU, within the workspace
    int64_t rows = A.rows;
    int nout = ((camax + 31) / 32) * ((cbmax + 31) / 32);
    int64_t want = std::max<int64_t>(1, 512 / std::max(1, nt * nout));
    want = std::min<int64_t>(want, std::max<int64_t>(1, rows / 256));
    int64_t cap = (int64_t)(gram_ws_bytes / ((size_t)nt * camax * cbmax * esz));
    if (cap < 1) throw DeviceError("gram workspace too small");
    int64_t nch = std::min<int64_t>(std::max<int64_t>(want, 1), cap);
    int64_t cr = (rows + nch - 1) / nch;
    cr = std::max<int64_t>(32, (cr + 31) / 32 * 32);
    while ((rows + cr - 1) / cr > cap) cr += 32;
    g.chunk_rows = (int)cr;
    int pi = prof.begin(st, 6, 8.0 * (double)rows * camax * cbmax * nt * (dd ? 4.0 : 1.0),
                        16.0 * (double)rows * (camax + cbmax) * nt);
    launch_gram(g, st);
    prof.end(st, pi);
}

void Engine::gemm_ts(const int* dlist, int nt, const BlockList& A, int camax, const zd* G, int64_t strideG, int ldG,
                     const int* cbdims, int cbmul, int cb, zd* Y, int64_t strideY, int64_t ldY, int64_t rows,
                     double alpha, double beta)
{
    if (nt <= 0) return;
    GemmTSArgs g;
    memset(&g, 0, sizeof(g));
    g.list = dlist;
    g.ntiles = nt;
    g.A = A;
    g.G = G;
    g.strideG = strideG;
    g.ldG = ldG;
    g.cbdims = cbdims;
    g.cbmul = cbmul;
    g.cb = cb;
    g.Y = Y;
    g.strideY = strideY;
    g.ldY = ldY;
    g.rows = rows;
    g.alpha = alpha;
    g.beta = beta;
    g.camax = camax;
    g.cbmax = cbdims ? K * cbmul : cb;
    if (cbdims) g.cbmax = std::max(g.cbmax, cb);
    int pi = prof.begin(st, 6, 8.0 * (double)rows * camax * g.cbmax * nt,
                        16.0 * (double)rows * (camax + g.cbmax * (beta != 0.0 ? 2 : 1)) * nt);
    launch_gemm_ts(g, st);
    prof.end(st, pi);
}

void Engine::colnorm2(const int* dlist, int nt, const BlockList& A, int camax, double* out, int ldo)
{
    if (nt <= 0) return;
    NormArgs a;
    memset(&a, 0, sizeof(a));
    a.list = dlist;
    a.ntiles = nt;
    a.A = A;
    a.camax = camax;
    a.out = out;
    a.ldo = ldo;
    a.part = norm_ws.p;
    int64_t nch = std::max<int64_t>(1, std::min<int64_t>(256 / std::max(1, nt) + 1,
                                                         (int64_t)(norm_ws.n / ((size_t)nt * camax))));
    int64_t cr = (A.rows + nch - 1) / nch;
    cr = std::max<int64_t>(64, cr);
    while ((A.rows + cr - 1) / cr * (int64_t)nt * camax > (int64_t)norm_ws.n) cr *= 2;
    a.chunk_rows = (int)cr;
    int pi = prof.begin(st, 6, 8.0 * (double)A.rows * camax * nt, 16.0 * (double)A.rows * camax * nt);
    launch_colnorm2(a, st);
    prof.end(st, pi);
}

// R (c x c upper) of the tall matrix A from a double-double Gram matrix and
// a double-double Cholesky (mixed-precision Cholesky QR): R^* R = A^* A to
// double-double accuracy, so R equals the R factor of a backward-stable QR
// of A up to rounding of R itself.
void Engine::r_factor(const int* dlist, int nt, const BlockList& A, int cmax, const int* cdims, int cmul,
                      int cfixed, zd* R, int64_t strideR, int ldR, int* nzero, zdd* gbuf, bool dd_gram)
{
    if (nt <= 0) return;
    zdd* gb = gbuf ? gbuf : gdd.p;
    gram(dlist, nt, A, A, cmax, cmax, gb, (int64_t)cmax * cmax, cmax, dd_gram, true, true);
    CholArgs c;
    memset(&c, 0, sizeof(c));
    c.list = dlist;
    c.cdim = cdims;
    c.cmul = cmul;
    c.c = cfixed > 0 ? cfixed : cmax;   // with cdims: the maximum, used to size the launch
    c.G = gb;
    c.strideG = (int64_t)cmax * cmax;
    c.ldG = cmax;
    c.R = R;
    c.strideR = strideR;
    c.ldR = ldR;
    c.nzero = nzero;
    int pi = prof.begin(st, 5, 0.0, 0.0);
    launch_chol_dd(c, nt, st);
    prof.end(st, pi);
}

// Orthonormalise the cols-column block W of each tile in L (in place), and
// make it orthogonal to `against` if given: repeated block projection
// followed by SVQB on the column-scaled block; directions that vanish are
// refilled with seeded random vectors and orthonormalised again.
void Engine::orthonormalize(const std::vector<int>& L, const int* dlist, zd* W, int64_t wstride, int64_t ldw,
                            int64_t rows, int cols, const BlockList* against, int against_max, uint64_t seed)
{
    const int nt = (int)L.size();
    if (nt == 0) return;
    BlockList Wl = bl_empty(rows);
    bl_add(Wl, W, wstride, ldw, cols, nullptr, 0);
    // the last pass orthonormalises what the previous one refilled and
    // refills nothing: a direction it still drops stays zero, which the
    // callers detect (zero pivot of the next R factor) and repair
    const int npass = 7;
    for (int pass = 0; pass < npass; ++pass) {
        if (against) {
            for (int rep = 0; rep < 2; ++rep) {
                gram(dlist, nt, *against, Wl, against_max, cols, Csm.p, (int64_t)K * 3 * r, against_max, false,
                     false);
                gemm_ts(dlist, nt, *against, against_max, Csm.p, (int64_t)K * 3 * r, against_max, nullptr, 0, cols,
                        W, wstride, ldw, rows, -1.0, 1.0);
            }
        }
        colnorm2(dlist, nt, Wl, cols, nrm2.p, 3 * r);
        {
            dim3 g((unsigned)((rows * cols + 255) / 256), nt);
            hipLaunchKernelGGL(k_scale_cols_rsqrt, g, dim3(256), 0, st, dlist, W, wstride, ldw, rows, cols, nrm2.p,
                               3 * r);
        }
        // the Gram matrix of the unit-norm columns in double: directions
        // below the drop level 1e-6 are refilled, and the at least two
        // passes below bring the rest to orthonormality as Cholesky QR
        // twice does
        r_factor(dlist, nt, Wl, cols, nullptr, 0, cols, Rsm.p, (int64_t)9 * r * r, 3 * r, nullptr, nullptr, false);
        SvqbArgs sa;
        memset(&sa, 0, sizeof(sa));
        sa.list = dlist;
        sa.r = cols;
        sa.max_sweeps = 40;
        sa.drop = 1e-6;   // directions this small lose orthogonality ~ eps / 1e-6: refill them
        sa.R = Rsm.p;
        sa.strideR = (int64_t)9 * r * r;
        sa.ldR = 3 * r;
        sa.T = Tsm.p;
        sa.strideT = (int64_t)9 * r * r;
        sa.ldT = 3 * r;
        sa.mask = mask.p;
        int pi = prof.begin(st, 5, 0.0, 0.0);
        launch_svqb(sa, nt, st);
        prof.end(st, pi);
        gemm_ts(dlist, nt, Wl, cols, Tsm.p, (int64_t)9 * r * r, 3 * r, nullptr, 0, cols, Tn1.p, (int64_t)m * 3 * r,
                m, rows, 1.0, 0.0);
        launch_copy_cols(dlist, nt, Tn1.p, (int64_t)m * 3 * r, m, W, wstride, ldw, rows, cols, st);
        if (pass == npass - 1) break;
        launch_randfill(dlist, nt, W, wstride, ldw, rows, cols, mask.p, seed + 7919ull * pass, st);
        if (pass == 0) continue;
        // check whether any direction was refilled in this pass
        h_small.alloc(T + 1);
        HIPCHK(hipMemcpyAsync(h_small.p, mask.p, sizeof(uint32_t) * T, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const uint32_t* hm = (const uint32_t*)h_small.p;
        bool any = false;
        for (int t : L) any |= (hm[t] != 0);
        if (!any) break;
    }
}

// ---------------------------------------------------------------------------
void Engine::apply(bool herm, const int* dlist, int nt, const zd* X, int64_t xstride, int64_t ldx, zd* Y,
                   int64_t ystride, int64_t ldy, int w, const zd* dz, zd* ws, size_t ws_n)
{
    if (!ws) { ws = apply_ws.p; ws_n = apply_ws.n; }
    if (nt <= 0) return;
    stats.mv_M += (int64_t)nt * w;
    if (op.kind == PS_DENSE) {
        DenseApplyArgs a;
        memset(&a, 0, sizeof(a));
        if (!herm) { a.A = op.A.p; a.lda = op.m; a.m = op.m; a.K = op.n; }
        else { a.A = op.AH.p; a.lda = op.n; a.m = op.n; a.K = op.m; }
        a.list = dlist;
        a.ntiles = nt;
        a.X = X;
        a.xstride = xstride;
        a.ldx = ldx;
        a.Y = Y;
        a.ystride = ystride;
        a.ldy = ldy;
        a.w = w;
        a.z = dz;
        a.conjz = herm ? 1 : 0;
        a.nshift = op.n;
        a.part = ws;
        int64_t N = (int64_t)nt * w;
        if (ws_n < (size_t)a.m * N) throw DeviceError("operator-apply workspace too small");
        a.splitk = (int)std::max<int64_t>(1, (int64_t)(ws_n / ((size_t)a.m * N)));
        int pi = prof.begin(st, 0, 8.0 * a.m * a.K * N, 16.0 * ((double)a.m * a.K + (double)a.K * N + (double)a.m * N));
        launch_dense_apply(a, st);
        prof.end(st, pi);
    } else {
        CsrApplyArgs a;
        memset(&a, 0, sizeof(a));
        if (!herm) { a.rowptr = op.rp.p; a.colind = op.ci.p; a.vals = op.v.p; a.m = op.m; }
        else { a.rowptr = op.rpH.p; a.colind = op.ciH.p; a.vals = op.vH.p; a.m = op.n; }
        a.list = dlist;
        a.ntiles = nt;
        a.X = X;
        a.xstride = xstride;
        a.ldx = ldx;
        a.Y = Y;
        a.ystride = ystride;
        a.ldy = ldy;
        a.w = w;
        a.z = dz;
        a.conjz = herm ? 1 : 0;
        a.nshift = op.n;
        int64_t N = (int64_t)nt * w;
        double rows_in = herm ? (double)op.m : (double)op.n;
        int pi = prof.begin(st, 0, 8.0 * op.nnz * N,
                            20.0 * op.nnz + 8.0 * a.m + 16.0 * N * (rows_in + (double)a.m));
        launch_csr_apply(a, st);
        prof.end(st, pi);
    }
}

// ---------------------------------------------------------------------------
void Engine::create(const ps_matrix_desc* d, const ps_params* p, hipStream_t s)
{
    st = s;
    P = *p;
    op.kind = d->kind;
    op.m = d->m;
    op.n = d->n;
    small_kernels_init();
    {
        // LDS of the per-workgroup kernels: Ritz (2 k^2 complex) and the
        // rotations ((k^2 + 7 r^2 + 2 r k) complex), plus static arrays
        size_t need = std::max<size_t>((size_t)2 * P.k_max * P.k_max,
                                       (size_t)P.k_max * P.k_max + 7 * P.r * P.r + 2 * P.r * P.k_max) * sizeof(zd);
        if (need + 4096 > (size_t)small_kernels_max_lds())
            throw InvalidArg("k_max too large for this device's LDS per workgroup");
        // recyProj runs the same kernel on the projection store (kbar_max)
        const int pc = P.precond < 0 ? (d->kind == PS_DENSE ? 1 : (d->m == d->n ? 2 : 0)) : P.precond;
        if (pc == 2 && (size_t)2 * P.kbar_max * P.kbar_max * sizeof(zd) + 4096 > (size_t)small_kernels_max_lds())
            throw InvalidArg("kbar_max too large for this device's LDS per workgroup");
    }
    if (d->kind == PS_DENSE) {
        size_t cnt = (size_t)d->m * d->n;
        op.A.alloc(cnt);
        op.AH.alloc(cnt);
        hipMemcpyKind kind = d->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIPCHK(hipMemcpy2DAsync(op.A.p, sizeof(zd) * d->m, d->dense, sizeof(zd) * d->ld, sizeof(zd) * d->m, d->n,
                                kind, st));
        dim3 g((unsigned)((d->m + 31) / 32), (unsigned)((d->n + 31) / 32));
        hipLaunchKernelGGL(k_conj_transpose, g, dim3(32, 8), 0, st, op.A.p, (int64_t)d->m, d->m, d->n, op.AH.p);
        HIPCHK(hipGetLastError());
    } else {
        // CSR of C and of C^* (the transpose is built once on the host)
        int64_t mm = d->m, nn = d->n, nnz = d->nnz;
        std::vector<int64_t> rp(mm + 1);
        std::vector<int32_t> ci(nnz);
        std::vector<zd> v(nnz);
        hipMemcpyKind kind = d->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
        HIPCHK(hipMemcpy(rp.data(), d->rowptr, sizeof(int64_t) * (mm + 1), kind));
        HIPCHK(hipMemcpy(ci.data(), d->colind, sizeof(int32_t) * nnz, kind));
        HIPCHK(hipMemcpy(v.data(), d->vals, sizeof(zd) * nnz, kind));
        if (rp[0] != 0 || rp[mm] != nnz) throw InvalidArg("CSR rowptr inconsistent with nnz");
        for (int64_t i = 0; i < mm; ++i) {
            if (rp[i + 1] < rp[i]) throw InvalidArg("CSR rowptr not monotone");
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
                if (ci[q] < 0 || ci[q] >= nn) throw InvalidArg("CSR column index out of range");
                if (q > rp[i] && ci[q] <= ci[q - 1]) throw InvalidArg("CSR columns not sorted/unique");
                if (!std::isfinite(v[q].x) || !std::isfinite(v[q].y)) throw InvalidArg("non-finite entry");
            }
        }
        std::vector<int64_t> rpH(nn + 1, 0);
        for (int64_t q = 0; q < nnz; ++q) rpH[ci[q] + 1]++;
        for (int64_t j = 0; j < nn; ++j) rpH[j + 1] += rpH[j];
        std::vector<int32_t> ciH(nnz);
        std::vector<zd> vH(nnz);
        std::vector<int64_t> pos(rpH.begin(), rpH.end() - 1);
        for (int64_t i = 0; i < mm; ++i)
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
                int64_t o = pos[ci[q]]++;
                ciH[o] = (int32_t)i;
                vH[o] = zconj(v[q]);
            }
        op.nnz = nnz;
        op.rp.alloc(mm + 1); op.ci.alloc(nnz); op.v.alloc(nnz);
        op.rpH.alloc(nn + 1); op.ciH.alloc(nnz); op.vH.alloc(nnz);
        HIPCHK(hipMemcpy(op.rp.p, rp.data(), sizeof(int64_t) * (mm + 1), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(op.ci.p, ci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(op.v.p, v.data(), sizeof(zd) * nnz, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(op.rpH.p, rpH.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(op.ciH.p, ciH.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(op.vH.p, vH.data(), sizeof(zd) * nnz, hipMemcpyHostToDevice));
    }
    n = op.n;
    m = op.m;
    r = P.r;
    K = P.k_max;
    if (P.precond < 0) P.precond = (op.kind == PS_DENSE) ? 1 : 2;
    use_prec = P.precond > 0;
    two_level = P.precond == 2;
    if (use_prec && op.kind != PS_DENSE) build_sparse_pattern();
    size_for(1);
    estimate_norm();
    if (use_prec && op.kind == PS_DENSE) {
        // C^* C once, for N(z) = C^*C - conj(z) S^*C - z C^*S + |z|^2 I
        CtC.alloc((size_t)n * n);
        zgemm(nullptr, 1, n, n, m, op.A.p, m, 0, 1, op.A.p, m, 0, CtC.p, n, 0, 1.0, 0.0);
        HIPCHK(hipStreamSynchronize(st));
    }
}

// ||C||_2 by power iteration on C^* C (60 steps, on the device), scaled by 1.01.
void Engine::estimate_norm()
{
    std::vector<int> L0 = {0};
    upload_list(L0, d_list);
    launch_randfill(d_list.p, 1, S.p, 0, n, n, 1, nullptr, 0x5eedull, st);
    double lam = 0.0;
    for (int it = 0; it < 60; ++it) {
        apply(false, d_list.p, 1, S.p, 0, n, CS.p, 0, m, 1, nullptr);
        apply(true, d_list.p, 1, CS.p, 0, m, S.p, 0, n, 1, nullptr);
        BlockList Ls = bl_empty(n);
        bl_add(Ls, S.p, 0, n, 1, nullptr, 0);
        colnorm2(d_list.p, 1, Ls, 1, nrm2.p, 3 * r);
        h_xi.alloc(8);
        HIPCHK(hipMemcpyAsync(h_xi.p, nrm2.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double s2 = h_xi[0];
        lam = sqrt(s2);  // ||C^* C x|| with ||x|| = 1
        if (!(s2 > 0)) { lam = 0; break; }
        dim3 g((unsigned)((n + 255) / 256), 1);
        hipLaunchKernelGGL(k_scale_cols_rsqrt, g, dim3(256), 0, st, d_list.p, S.p, (int64_t)0, (int64_t)n, (int64_t)n,
                           1, nrm2.p, 3 * r);
    }
    stats.mv_M = 0;
    op.normC = 1.01 * sqrt(lam);
}

void Engine::size_for(int tiles)
{
    T = tiles;
    const size_t t = (size_t)tiles;
    const size_t nk = (size_t)n * K, mk = (size_t)m * K;
    sV.alloc(t * nk); sW1.alloc(t * mk); sW3.alloc(t * nk); sW4.alloc(t * nk);
    uV.alloc(t * nk); uW1.alloc(t * mk); uW3.alloc(t * nk); uW4.alloc(t * nk);
    sRA.alloc(t * 4 * K * K);
    sH.alloc(t * K * K);
    d_gamt.alloc(t);
    h_gamt.alloc(t + 8);
    sRres.alloc(t * 16 * K * K);
    const int cmax = std::max(4 * K, 3 * r);
    gdd.alloc(t * cmax * cmax);
    d_k.alloc(t); d_q.alloc(t); d_l.alloc(t);
    S.alloc(t * n * 3 * r); Sn.alloc(t * n * 3 * r);
    CS.alloc(t * m * 3 * r); CSn.alloc(t * m * 3 * r);
    Wres.alloc(t * n * r); Xw.alloc(t * n * r);
    Tn1.alloc(t * m * 3 * r); Tn2.alloc(t * n * r); Tn3.alloc(t * n * r);
    Rsm.alloc(t * 9 * r * r); GX.alloc(t * 9 * r * r); GP.alloc(t * 9 * r * r);
    Csm.alloc(t * K * 3 * r); Tsm.alloc(t * 9 * r * r);
    Qt.alloc(t * K * K); Upp.alloc(t * r * r); Ucoef.alloc(t * K * r); X0c.alloc(t * K * r);
    xi.alloc(t * 3 * r); nrm2.alloc(t * 3 * r); xi_out.alloc(t * 3 * r);
    mask.alloc(t); cdim.alloc(3 * t); d_list.alloc(t);
    d_cdimt.alloc(t); d_pcols.alloc(t);
    lob_it.assign(t, 0);
    lob_sigma.assign(t, 0.0);
    lob_xi.assign(t, 0.0);
    esc_at.assign(t, 0);
    site_exact.assign(t, 0);
    lob_prev.assign(t, 0.0);
    stag.assign(t, 0);
    cert_next.assign(t, 0);
    cert_fail.assign(t, 0);
    nop.assign(t, 0);
    lob_bad.assign(t, 0);
    h_zt.assign(t, zmake(0.0, 0.0)); d_list2.alloc(t); d_jobsrc.alloc(t);
    d_z.alloc(t);
    const size_t J = t * B;
    j_tile.alloc(J); j_z.alloc(J); j_G.alloc(J * K * r);
    j_nrm.alloc(J); j_xi.alloc(J); j_res.alloc(J); j_acc.alloc(J); j_gam.alloc(J); h_gamj.alloc(J + 8);
    gram_ws_bytes = std::max<size_t>((size_t)256 << 20, t * (size_t)cmax * cmax * sizeof(zdd) * 2);
    gram_ws.alloc(gram_ws_bytes);
    const size_t maxw = (size_t)std::max(r, P.rbar);
    // projection-store refresh: 32 sites x KB columns (two-level only)
    const size_t kbw = (P.precond == 2) ? (size_t)32 * std::max(P.kbar_max, 1) : 0;
    if (op.kind == PS_DENSE)
        apply_ws.alloc((size_t)std::max(m, n) * std::max<size_t>(std::max<size_t>(t * maxw, 64), kbw) * 4);
    norm_ws.alloc(std::max<size_t>(1 << 20, t * 3 * r * 256));
    {
        std::vector<int> cv(3 * t);
        for (size_t i = 0; i < t; ++i) { cv[i] = r; cv[t + i] = 2 * r; cv[2 * t + i] = 3 * r; }
        HIPCHK(hipMemcpy(cdim.p, cv.data(), sizeof(int) * 3 * t, hipMemcpyHostToDevice));
    }
    NBLD = 0;
    NS = 0;
    if (use_prec && op.kind == PS_DENSE) {
        const size_t nn = (size_t)n * n;
        // staging for up to 32 simultaneous constructions; the site pool holds
        // one slot per tile plus the staging count (so a free slot always
        // exists), within 128 GB
        // sites and staging share site_mem_gb: NBLD staging pairs (N(z) and
        // the factor) and NS slots of F^{-1}
        const size_t tot = std::max<size_t>(4, ((size_t)P.site_mem_gb << 30) / (nn * sizeof(zd)));
        NBLD = (int)std::min<size_t>(32, std::max<size_t>(1, tot / 6));
        const size_t cap = std::max<size_t>(2, tot - 2 * (size_t)NBLD);
        NS = (int)std::min<size_t>(t + NBLD, cap);
        // with the two-level preconditioner a site serves a whole region
        if (two_level) NS = std::min(NS, 160);
        PN.alloc(NBLD * nn); Fb.alloc(NBLD * nn); Finv.alloc((size_t)NS * nn);
        Dinv.alloc(NBLD * n * PRE_NB); T1p.alloc(NBLD * n * PRE_NB); T2p.alloc(NBLD * n * PRE_OB); pvec.alloc(NBLD * 2 * n); d_zdag.alloc(NBLD);
        d_shift.alloc(NBLD); d_notpd.alloc(NBLD);
        zgemm_ws.alloc(std::max<size_t>((size_t)32 << 20, t * (size_t)n * r * 16));
    } else if (use_prec) {
        // incomplete Cholesky sites: values, power-iteration vectors, solve work;
        // the projection stores (8 n x kbar blocks per site) bound the count
        NBLD = 8;
        const double per = 16.0 * ((double)op.spat.nnz + 3.0 * n + m + (two_level ? 9.0 : 1.0) * n * P.kbar_max);
        NS = (int)std::max(2.0, std::min((double)t + NBLD, std::min(64.0, P.site_mem_gb * 1e9 / 5.0 / per)));
        Slu.alloc((size_t)NS * op.spat.nnz);
        Svec.alloc((size_t)NS * (3 * n + m));
        pS.alloc((size_t)NS * n * std::max(P.kbar_max, 1));
        d_slotz.alloc(NS);
        d_icbad.alloc(NS);
        d_alpha.alloc(NS);
        slot_alpha.assign(NS, 0.0);
        Tq.alloc(t * n * r);
        d_listC.alloc(std::max<size_t>(t, NS));
        std::vector<zd> z0((size_t)NS, zmake(0.0, 0.0));
        HIPCHK(hipMemcpy(d_slotz.p, z0.data(), sizeof(zd) * NS, hipMemcpyHostToDevice));
    }
    nrm2.alloc(std::max<size_t>(std::max<size_t>(t, NBLD), (size_t)NS + 1) * 3 * r);
    if (use_prec) {
        Tp.alloc(t * std::max(m, n) * r);
        d_tslot.alloc(std::max<size_t>(t, (size_t)NS + 1));
    }
    if (two_level) {
        KB = P.kbar_max;
        const size_t ns = (size_t)NS, snk = (size_t)n * KB, smk = (size_t)m * KB;
        pV.alloc(ns * snk); pE.alloc(ns * snk); pW3.alloc(ns * snk); pW4.alloc(ns * snk);
        pW5.alloc(ns * snk); pW6.alloc(ns * snk); pW1.alloc(ns * smk); pT.alloc(ns * smk);
        pRA.alloc(ns * 4 * KB * KB); pRres.alloc(ns * 25 * KB * KB); pgdd.alloc((ns + 1) * 25 * KB * KB);
        d_pk.alloc(ns + 1); d_nzp.alloc(ns + 1);
        pk.assign(ns, 0);
        tE.alloc(t * n * r); tX0.alloc(t * n * r); tCoef.alloc(t * r * r);
        Tp.alloc(t * std::max(m, n) * r); pG.alloc(t * KB * r);
        tLam.alloc(t * r); pj_xi.alloc(t * r); pj_res.alloc(t * r); pj_nrm.alloc(t); pj_acc.alloc(t);
        pj_slot.alloc(t); pj_z.alloc(t); d_listA.alloc(t); d_listB.alloc(std::max(t, ns));
        d_tslot.alloc(std::max(t, ns + 1));
        phase.assign(t, 0);
        use2l.assign(t, 0);
        lob_sv.assign(t * r, 0.0);
        tlam_h.assign(t * r, 0.0);
        upload_pk();
    } else {
        phase.assign(t, 0);
        use2l.assign(t, 0);
        lob_sv.assign(t * r, 0.0);
        d_listA.alloc(t); d_listB.alloc(t);
    }
    slot_lamn.assign(NS, 1.0);
    slot_dreg.assign(NS, 0.0);
    slot_z.assign(NS, zmake(0.0, 0.0));
    slot_gam.assign(NS, 0.0);
    slot_ref.assign(NS, 0);
    slot_last.assign(NS, 0);
    slot_valid.assign(NS, 0);
    slot_priv.assign(NS, 0);
    tile_slot.assign(t, -1);
    d_listI.alloc(t);
    usek.assign(t, 1);
    h_acc.alloc(J); h_xi.alloc(std::max<size_t>(J, t * 3 * r));
    h_nrm2.alloc(std::max<size_t>(std::max<size_t>(t, NBLD), (size_t)NS + 1) * 3 * r);
    h_small.alloc(std::max<size_t>(t, NBLD) * 4 + 8); h_C.alloc(t * K * r + 8); h_list.alloc(t + 1); h_z.alloc(t + J);
}

// ---------------------------------------------------------------------------
// R_A = R([W1 W2]) and R_res = R([W3 W4 W5 W6]) of the singular store, with
// W2 = [V; 0], W5 = W1[:n] and W6 = V because S = [I_n; 0].
void Engine::refresh_store(const std::vector<int>& L)
{
    if (L.empty()) return;
    upload_list(L, d_list2);
    const int nt = (int)L.size();
    BlockList La = bl_empty(m);
    bl_add(La, sW1.p, (int64_t)m * K, m, 0, d_k.p, 1);
    bl_add(La, sV.p, (int64_t)n * K, n, 0, d_k.p, 1, n);
    r_factor(d_list2.p, nt, La, 2 * K, d_k.p, 2, 0, sRA.p, (int64_t)4 * K * K, 2 * K);
    BlockList Lr = bl_empty(n);
    bl_add(Lr, sW3.p, (int64_t)n * K, n, 0, d_k.p, 1);
    bl_add(Lr, sW4.p, (int64_t)n * K, n, 0, d_k.p, 1);
    bl_add(Lr, sW1.p, (int64_t)m * K, m, 0, d_k.p, 1);
    bl_add(Lr, sV.p, (int64_t)n * K, n, 0, d_k.p, 1);
    r_factor(d_list2.p, nt, Lr, 4 * K, d_k.p, 4, 0, sRres.p, (int64_t)16 * K * K, 4 * K);
    // H = V^* (S^* W1) = V^* W1[0:n]
    BlockList Lv = bl_empty(n);
    bl_add(Lv, sV.p, (int64_t)n * K, n, 0, d_k.p, 1);
    BlockList Lw = bl_empty(n);
    bl_add(Lw, sW1.p, (int64_t)m * K, m, 0, d_k.p, 1);
    gram(d_list2.p, nt, Lv, Lw, K, K, sH.p, (int64_t)K * K, K, false, false);
}

