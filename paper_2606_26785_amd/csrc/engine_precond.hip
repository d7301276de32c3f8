// Dense base preconditioner of the two-level scheme (Sec. 3): construction at
// z_dag and application K^{-1} W = F^{-1} F^{-*} W.
#include "engine.h"

#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstring>

void Engine::zgemm(const int* dl, int nt, int64_t M, int64_t N, int64_t Kd, const zd* A, int64_t lda, int64_t sA,
                   int opA, const zd* Bm, int64_t ldb, int64_t sB, zd* Cm, int64_t ldc, int64_t sC, double alpha,
                   double beta, int upper, int tri, const int* gmap, int cw, int64_t cols_total)
{
    if (nt <= 0 || M <= 0 || N <= 0) return;
    ZgemmArgs a;
    memset(&a, 0, sizeof(a));
    a.list = dl;
    a.M = M;
    a.N = N;
    a.K = Kd;
    a.A = A;
    a.lda = lda;
    a.strideA = sA;
    a.opA = opA;
    a.B = Bm;
    a.ldb = ldb;
    a.strideB = sB;
    a.C = Cm;
    a.ldc = ldc;
    a.strideC = sC;
    a.alpha = alpha;
    a.beta = beta;
    a.upper = upper;
    a.tri = tri;
    if (gmap) {
        a.goff = gmap;
        a.gcnt = gmap + nt;
        a.gtile = gmap + 2 * nt;
        a.cw = cw;
    }
    // split K when the output is too small to fill the GPU (narrow right-hand sides)
    {
        int64_t wgs = ((M + 63) / 64) * ((N + 31) / 32) * nt;
        int sk = 1;
        if (!upper && wgs < 1024 && Kd >= 256) {
            sk = (int)std::min<int64_t>((2048 + wgs - 1) / wgs, Kd / 128);
            int64_t cap = (int64_t)(zgemm_ws.n / std::max<int64_t>(1, M * N * nt));
            sk = (int)std::max<int64_t>(1, std::min<int64_t>(sk, cap));
        }
        a.splitk = sk;
        a.ws = zgemm_ws.p;
    }
    // algorithmic work: in column-map mode N is the widest group, the
    // columns actually multiplied are cols_total over all groups
    const double ncols = (gmap && cols_total >= 0) ? (double)cols_total : (double)N * nt;
    double fl = 8.0 * (double)M * ncols * Kd * ((upper || tri) ? 0.5 : 1.0);
    double by = 16.0 * ((double)nt * M * Kd * (tri ? 0.5 : 1.0) + (double)Kd * ncols +
                        (double)M * ncols * (beta != 0.0 ? 2.0 : 1.0));
    // inside factorizations: class 3 for the wide-product kernel (products
    // at least 64 columns wide), 8 for the narrower ones
    const int cls = (zgemm_cls == 3 && (gmap || N < 64)) ? 8 : zgemm_cls;
    int pi = prof.begin(st, cls, fl, by);
    launch_zgemm(a, nt, st, zgemm_cls == 3 ? 2 : 0);
    prof.end(st, pi);
}

void Engine::fact_gemm(const int* dl, int nb, int64_t M, int64_t N, int64_t Kd, const zd* A, int64_t lda, int64_t sA,
                       int opA, const zd* Bm, int64_t ldb, int64_t sB, zd* Cm, int64_t ldc, int64_t sC, double alpha,
                       double beta, int upper, int tri)
{
    if (!P.fact_blas) {
        zgemm(dl, nb, M, N, Kd, A, lda, sA, opA, Bm, ldb, sB, Cm, ldc, sC, alpha, beta, upper, tri);
        return;
    }
    if (nb <= 0 || M <= 0 || N <= 0) return;
    if (!blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) throw DeviceError("rocblas_create_handle failed");
        blas = h;
    }
    rocblas_handle h = (rocblas_handle)blas;
    if (rocblas_set_stream(h, st) != rocblas_status_success) throw DeviceError("rocblas_set_stream failed");
    const double fl = 8.0 * (double)M * N * Kd * nb * ((upper || tri) ? 0.5 : 1.0);
    const double by = 16.0 * nb * ((double)M * Kd * (tri ? 0.5 : 1.0) + (double)Kd * N +
                                   (double)M * N * (beta != 0.0 ? 2.0 : 1.0));
    const int pi = prof.begin(st, zgemm_cls, fl, by);
    rocblas_status rs;
    if (upper && Kd > 0) {
        // C = alpha A^* A + beta C on the upper triangle (A == B, A stored Kd x M)
        if (opA != 1 || A != Bm || M != N) throw DeviceError("fact_gemm: Hermitian update needs C = A^* A");
        rs = rocblas_zherk_strided_batched(h, rocblas_fill_upper, rocblas_operation_conjugate_transpose, (rocblas_int)M,
                                           (rocblas_int)Kd, &alpha, (const rocblas_double_complex*)A, (rocblas_int)lda,
                                           (rocblas_stride)sA, &beta, (rocblas_double_complex*)Cm, (rocblas_int)ldc,
                                           (rocblas_stride)sC, (rocblas_int)nb);
    } else {
        // a triangular A (tri) is stored with zeros outside its triangle
        const rocblas_double_complex al = {alpha, 0.0}, be = {beta, 0.0};
        rs = rocblas_zgemm_strided_batched(h, opA ? rocblas_operation_conjugate_transpose : rocblas_operation_none,
                                           rocblas_operation_none, (rocblas_int)M, (rocblas_int)N, (rocblas_int)Kd,
                                           &al, (const rocblas_double_complex*)A, (rocblas_int)lda, (rocblas_stride)sA,
                                           (const rocblas_double_complex*)Bm, (rocblas_int)ldb, (rocblas_stride)sB, &be,
                                           (rocblas_double_complex*)Cm, (rocblas_int)ldc, (rocblas_stride)sC,
                                           (rocblas_int)nb);
    }
    prof.end(st, pi);
    if (rs != rocblas_status_success) throw DeviceError("rocBLAS product failed");
    (void)dl;
}

Engine::~Engine()
{
    if (blas) (void)rocblas_destroy_handle((rocblas_handle)blas);
}

void Engine::reset_slots()
{
    std::fill(slot_valid.begin(), slot_valid.end(), 0);
    std::fill(slot_ref.begin(), slot_ref.end(), 0);
    std::fill(slot_last.begin(), slot_last.end(), 0);
    std::fill(slot_priv.begin(), slot_priv.end(), 0);
    std::fill(tile_slot.begin(), tile_slot.end(), -1);
    slot_clock = 0;
}

// The rebuild rule of eq. (tauRecycle) for the base preconditioner alone:
// with gamma = ||F^{-1}||_2, g = gamma |z - z_dag| bounds the drift of the
// preconditioned spectrum, which stays within [(1 - g)^2, (1 + g)^2]; a site
// serves z while g < 1 and ((1 + g) / (1 - g))^2 <= tau_max.
int Engine::find_slot(zd z) const
{
    int best = -1;
    double bg = 0.0;
    for (int s = 0; s < NS; ++s) {
        if (!slot_valid[s] || slot_priv[s]) continue;
        const double d = sqrt(zabs2(zsub(z, slot_z[s])));
        const double g = (d == 0.0) ? 0.0 : slot_gam[s] * d;   // a site always serves its own point
        if (!(g < 1.0)) continue;
        double q = (1.0 + g) / (1.0 - g);
        if (q * q > P.tau_max) continue;
        if (best < 0 || g < bg) { best = s; bg = g; }
    }
    return best;
}

// K^{-1} W = F^{-1} (F^{-*} W) for the tiles in L (each through its site):
// tiles that share a site form one wide product, so each F^{-1} is streamed
// once per 32 right-hand sides rather than once per tile.
void Engine::precond_apply(const std::vector<int>& L, const zd* W, int64_t ws, zd* Y, int64_t ys)
{
    if (L.empty()) return;
    if (op.kind != PS_DENSE) {
        // K^{-1} W = F^{-1} F^{-*} W with each tile's incomplete Cholesky site
        finv_apply(L, 1, W, ws, n, Tn2.p, (int64_t)n * r, n);
        finv_apply(L, 0, Tn2.p, (int64_t)n * r, n, Y, ys, n);
        return;
    }
    std::vector<int> order(L);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tile_slot[x] < tile_slot[y]; });
    std::vector<int> gs, goff, gcnt;
    for (size_t i = 0; i < order.size(); ++i) {
        int s = tile_slot[order[i]];
        if (gs.empty() || gs.back() != s) { gs.push_back(s); goff.push_back((int)i); gcnt.push_back(0); }
        gcnt.back()++;
    }
    const int ng = (int)gs.size();
    const int nt = (int)order.size();
    h_gmap.alloc((size_t)4 * ng + nt + 8);
    d_gmap.alloc((size_t)4 * ng + nt + 8);
    int* h = h_gmap.p;
    int maxc = 0;
    for (int g = 0; g < ng; ++g) {
        h[g] = gs[g];                 // A index of group g (the slot)
        h[ng + g] = goff[g];
        h[2 * ng + g] = gcnt[g];
        maxc = std::max(maxc, gcnt[g]);
    }
    for (int i = 0; i < nt; ++i) h[3 * ng + i] = order[i];
    h2d(d_gmap.p, h, sizeof(int) * (3 * ng + nt));
    const int64_t nn = n * n;
    stats.sv_F += (int64_t)2 * nt * r;
    const int* gm = d_gmap.p + ng;
    // T = F^{-*} W (F^{-*} lower triangular: A = Finv read conjugate-transposed)
    zgemm(d_gmap.p, ng, n, (int64_t)maxc * r, n, Finv.p, n, nn, 1, W, n, ws, Tn2.p, n, (int64_t)n * r, 1.0, 0.0, 0,
          2, gm, r, (int64_t)nt * r);
    // Y = F^{-1} T
    zgemm(d_gmap.p, ng, n, (int64_t)maxc * r, n, Finv.p, n, nn, 0, Tn2.p, n, (int64_t)n * r, Y, n, ys, 1.0, 0.0, 0,
          1, gm, r, (int64_t)nt * r);
}

// Build one site per entry of `sites` (z_dag): N(z_dag) + delta I, its upper
// Cholesky factor F by a right-looking blocked Cholesky (block PRE_NB,
// trailing updates and the columns of F^{-1} on the matrix cores), F^{-1}
// formed alongside, then gamma = ||F^{-1}||_2 by power iteration on
// F^{-1} F^{-*}.  Up to NBLD sites are built at once in the staging blocks
// and copied into free slots (least recently used first).
std::vector<int> Engine::build_precond(const std::vector<zd>& sites, const std::vector<double>* mu,
                                       std::vector<char>* pd, bool priv, bool cert_only)
{
    std::vector<int> out;
    if (pd) pd->assign(sites.size(), 0);
    if (op.kind != PS_DENSE) {
        // sparse sites: incomplete Cholesky of N(z_dag) + alpha I.  Inertia
        // tests need an exact factorization: a band Cholesky when N has a
        // narrow band, otherwise the test is reported as not positive
        // definite, so no certificate is taken from it
        if (cert_only) {
            out.assign(sites.size(), -1);
            if (pd && mu && band_b >= 0) band_inertia(sites, *mu, *pd);
            return out;
        }
        std::vector<zd> zs_ok;
        std::vector<int> sl_ok;
        for (size_t i = 0; i < sites.size(); ++i) {
            int s = -1;
            for (int q = 0; q < NS && s < 0; ++q) if (!slot_valid[q]) s = q;
            if (s < 0)
                for (int q = 0; q < NS; ++q) {
                    if (slot_ref[q] > 0) continue;
                    if (s < 0 || slot_last[q] < slot_last[s]) s = q;
                }
            out.push_back(s);
            if (s < 0) continue;
            slot_valid[s] = 1;           // taken for this batch
            slot_ref[s]++;
            zs_ok.push_back(sites[i]);
            sl_ok.push_back(s);
        }
        build_sparse_sites(zs_ok, sl_ok);
        for (size_t i = 0; i < sl_ok.size(); ++i) {
            const int s = sl_ok[i];
            slot_ref[s]--;
            slot_priv[s] = priv ? 1 : 0;
            slot_z[s] = zs_ok[i];
            slot_last[s] = ++slot_clock;
            if (two_level) pk[s] = 0;
            stats.rebuilds++;
            if (priv) stats.builds_private++;
            else stats.builds_shared++;
            if (pd) (*pd)[i] = 1;
        }
        if (two_level) upload_pk();
        return out;
    }
    struct ClsGuard {
        int& c;
        ClsGuard(int& x) : c(x) { c = 3; }
        ~ClsGuard() { c = 1; }
    } cls_guard(zgemm_cls);
    const int64_t nn = n * n;
    for (size_t b0 = 0; b0 < sites.size(); b0 += (size_t)NBLD) {
        const int nb = (int)std::min<size_t>((size_t)NBLD, sites.size() - b0);
        std::vector<int> pos(nb);
        for (int i = 0; i < nb; ++i) pos[i] = i;
        upload_list(pos, d_list2);
        const int* dl = d_list2.p;
        h_z.alloc((size_t)nb + 8);
        double zmax = 0;
        for (int i = 0; i < nb; ++i) {
            h_z[i] = sites[b0 + i];
            zmax = std::max(zmax, sqrt(zabs2(sites[b0 + i])));
        }
        h2d(d_zdag.p, h_z.p, sizeof(zd) * nb);
        const double scale = (op.normC + zmax) * (op.normC + zmax);
        const double delta = 1e-13 * scale;
        h_shift.alloc((size_t)nb + 8);
        for (int i = 0; i < nb; ++i) {
            double mv = mu ? (*mu)[b0 + i] : 0.0;
            h_shift[i] = (mv == 0.0) ? delta : -mv;
        }
        h2d(d_shift.p, h_shift.p, sizeof(double) * nb);
        HIPCHK(hipMemsetAsync(d_notpd.p, 0, sizeof(int) * nb, st));
        int pf = prof.begin(st, 4, 8.0 * (double)nn * nb, 16.0 * 4.0 * (double)nn * nb);
        launch_form_normal(dl, nb, CtC.p, op.A.p, m, op.AH.p, n, d_zdag.p, d_shift.p, PN.p, nn, st);
        prof.end(st, pf);
        if (!cert_only) launch_zero_tiles(dl, nb, Fb.p, nn, nn, st);
        // two-level blocked Cholesky: outer blocks of PRE_OB columns updated
        // right-looking (one rank-PRE_OB trailing product per outer block,
        // so the trailing matrix is streamed n / PRE_OB times), inner blocks
        // of PRE_NB rows updated left-looking within the outer block row
        for (int64_t K0 = 0; K0 < n; K0 += PRE_OB) {
            const int64_t K1 = std::min<int64_t>(n, K0 + PRE_OB);
            for (int64_t k0 = K0; k0 < K1; k0 += PRE_NB) {
                const int kb = (int)std::min<int64_t>(PRE_NB, K1 - k0);
                if (k0 > K0) {
                    // A[k, k0:] -= R[K0:k0, k]^* R[K0:k0, k0:]
                    fact_gemm(dl, nb, kb, n - k0, k0 - K0, PN.p + K0 + k0 * n, n, nn, 1, PN.p + K0 + k0 * n, n, nn,
                          PN.p + k0 + k0 * n, n, nn, -1.0, 1.0);
                }
                // diagonal block and row panel R[k, k1:] = R_kk^{-*} A[k, k1:] in one launch
                const int pc = prof.begin(st, 4, 8.0 * nb * ((double)kb * kb * kb / 3.0 + (double)kb * kb * (n - k0 - kb)),
                                          16.0 * nb * (double)kb * (n - k0) * 2.0);
                launch_chol_step(dl, nb, PN.p, nn, n, k0, kb, cert_only ? nullptr : Dinv.p, (int64_t)n * PRE_NB,
                                 cert_only ? nullptr : Fb.p, nn, 1e-2 * delta, d_notpd.p, st);
                prof.end(st, pc);
                if (!cert_only && k0 > K0) {
                    // F^{-1}[K0:k0, k] = -F^{-1}[K0:k0, K0:k0] R[K0:k0, k] R_kk^{-1}
                    fact_gemm(dl, nb, k0 - K0, kb, k0 - K0, Fb.p + K0 + K0 * n, n, nn, 0, PN.p + K0 + k0 * n, n, nn,
                          T1p.p, n, (int64_t)n * PRE_NB, 1.0, 0.0);
                    fact_gemm(dl, nb, k0 - K0, kb, kb, T1p.p, n, (int64_t)n * PRE_NB, 0, Dinv.p + k0, n,
                          (int64_t)n * PRE_NB, Fb.p + K0 + k0 * n, n, nn, -1.0, 0.0);
                }
            }
            if (K1 < n) {
                // trailing Hermitian update (upper part), rank K1 - K0
                fact_gemm(dl, nb, n - K1, n - K1, K1 - K0, PN.p + K0 + K1 * n, n, nn, 1, PN.p + K0 + K1 * n, n, nn,
                      PN.p + K1 + K1 * n, n, nn, -1.0, 1.0, 1);
            }
            if (!cert_only && K0 > 0) {
                // F^{-1}[0:K0, K] = -F^{-1}[0:K0, 0:K0] (R[0:K0, K] F^{-1}[K, K])
                fact_gemm(dl, nb, K0, K1 - K0, K1 - K0, PN.p + K0 * n, n, nn, 0, Fb.p + K0 + K0 * n, n, nn, T2p.p, n,
                      (int64_t)n * PRE_OB, 1.0, 0.0);
                fact_gemm(dl, nb, K0, K1 - K0, K0, Fb.p, n, nn, 0, T2p.p, n, (int64_t)n * PRE_OB, Fb.p + K0 * n, n, nn,
                      -1.0, 0.0, 0, 1);
            }
        }
        HIPCHK(hipGetLastError());
        if (cert_only) {
            h_notpd.alloc((size_t)nb + 8);
            HIPCHK(hipMemcpyAsync(h_notpd.p, d_notpd.p, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int i = 0; i < nb; ++i) {
                if (pd) (*pd)[b0 + i] = h_notpd[i] == 0;
                out.push_back(-1);
            }
            continue;
        }
        // gamma^2 = lambda_max(F^{-1} F^{-*}) by power iteration
        const int64_t sp = 2 * n;
        launch_randfill(dl, nb, pvec.p, sp, n, n, 1, nullptr, 0x7a11ull, st);
        std::vector<double> g2(nb, 0.0);
        for (int it = 0; it < 12; ++it) {
            zgemm(dl, nb, n, 1, n, Fb.p, n, nn, 1, pvec.p, n, sp, pvec.p + n, n, sp, 1.0, 0.0, 0, 2);
            zgemm(dl, nb, n, 1, n, Fb.p, n, nn, 0, pvec.p + n, n, sp, pvec.p, n, sp, 1.0, 0.0, 0, 1);
            BlockList Lp = bl_empty(n);
            bl_add(Lp, pvec.p, sp, n, 1, nullptr, 0);
            colnorm2(dl, nb, Lp, 1, nrm2.p, 3 * r);
            if (it == 11) {
                HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * nb * 3 * r, hipMemcpyDeviceToHost, st));
                h_notpd.alloc((size_t)nb + 8);
                HIPCHK(hipMemcpyAsync(h_notpd.p, d_notpd.p, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i < nb; ++i) g2[i] = sqrt(h_nrm2[(size_t)i * 3 * r]);
                if (pd)
                    for (int i = 0; i < nb; ++i) (*pd)[b0 + i] = h_notpd[i] == 0;
            }
            launch_scale_cols(dl, nb, pvec.p, sp, n, n, 1, nrm2.p, 3 * r, 2, st);
        }
        for (int i = 0; i < nb; ++i) {
            // slot: an unused one, else the least recently used unreferenced one
            int s = -1;
            for (int q = 0; q < NS && s < 0; ++q) if (!slot_valid[q]) s = q;
            if (s < 0) {
                for (int q = 0; q < NS; ++q) {
                    if (slot_ref[q] > 0) continue;
                    if (s < 0 || slot_last[q] < slot_last[s]) s = q;
                }
            }
            out.push_back(s);
            if (s < 0) continue;
            HIPCHK(hipMemcpyAsync(Finv.p + (size_t)s * nn, Fb.p + (size_t)i * nn, sizeof(zd) * nn,
                                  hipMemcpyDeviceToDevice, st));
            slot_valid[s] = 1;
            slot_priv[s] = priv ? 1 : 0;
            if (two_level) {
                pk[s] = 0;            // a new site starts with an empty projection store
                slot_lamn[s] = 1.0;
            }
            slot_z[s] = sites[b0 + i];
            slot_gam[s] = sqrt(std::max(g2[i], 0.0));
            slot_last[s] = ++slot_clock;
            stats.rebuilds++;
            if (priv) stats.builds_private++;
            else stats.builds_shared++;
        }
        HIPCHK(hipStreamSynchronize(st));
    }
    if (two_level && !cert_only) upload_pk();
    return out;
}
