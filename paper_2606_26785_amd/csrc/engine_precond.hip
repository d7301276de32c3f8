// Dense base preconditioner of the two-level scheme (Sec. 3): construction at
// z_dag and application K^{-1} W = F^{-1} F^{-*} W.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

void Engine::zgemm(const int* dl, int nt, int64_t M, int64_t N, int64_t Kd, const zd* A, int64_t lda, int64_t sA,
                   int opA, const zd* Bm, int64_t ldb, int64_t sB, zd* Cm, int64_t ldc, int64_t sC, double alpha,
                   double beta, int upper, int tri)
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
    double fl = 8.0 * (double)M * N * Kd * nt * ((upper || tri) ? 0.5 : 1.0);
    double by = 16.0 * nt * ((double)M * Kd * (tri ? 0.5 : 1.0) + (double)Kd * N +
                             (double)M * N * (beta != 0.0 ? 2.0 : 1.0));
    int pi = prof.begin(st, 1, fl, by);
    launch_zgemm(a, nt, st);
    prof.end(st, pi);
}

// K^{-1} W for the tiles in dl: Y = F^{-1} (F^{-*} W), W and Y n x r per tile
void Engine::precond_apply(const int* dl, int nt, const zd* W, int64_t ws, zd* Y, int64_t ys)
{
    if (nt <= 0) return;
    const int64_t nn = n * n;
    stats.sv_F += (int64_t)2 * nt * r;
    zgemm(dl, nt, n, r, n, FinvH.p, n, nn, 0, W, n, ws, Tn2.p, n, (int64_t)n * r, 1.0, 0.0, 0, 2);
    zgemm(dl, nt, n, r, n, Finv.p, n, nn, 0, Tn2.p, n, (int64_t)n * r, Y, n, ys, 1.0, 0.0, 0, 1);
}

// Build K = F^* F with F^* F = N(z_dag) + delta I for every tile in L, at the
// z_dag already stored in zdag[] (right-looking blocked Cholesky, block
// PRE_NB, trailing updates and the columns of F^{-1} on the matrix cores),
// then gamma = ||F^{-1}||_2 by power iteration on F^{-1} F^{-*}.
void Engine::build_precond(const std::vector<int>& L)
{
    if (L.empty()) return;
    const int nt = (int)L.size();
    upload_list(L, d_list2);
    const int* dl = d_list2.p;
    const int64_t nn = n * n;
    h_z.alloc((size_t)T + 8);
    for (int t = 0; t < T; ++t) h_z[t] = zdag[t];
    HIPCHK(hipMemcpyAsync(d_zdag.p, h_z.p, sizeof(zd) * T, hipMemcpyHostToDevice, st));
    double zmax = 0;
    for (int t : L) zmax = std::max(zmax, sqrt(zabs2(zdag[t])));
    const double scale = (op.normC + zmax) * (op.normC + zmax);
    const double delta = 1e-13 * scale;
    launch_form_normal(dl, nt, CtC.p, op.A.p, m, op.AH.p, n, d_zdag.p, delta, PN.p, nn, st);
    launch_zero_tiles(dl, nt, Finv.p, nn, nn, st);
    for (int64_t k0 = 0; k0 < n; k0 += PRE_NB) {
        const int kb = (int)std::min<int64_t>(PRE_NB, n - k0);
        launch_chol_diag(dl, nt, PN.p, nn, n, k0, kb, Dinv.p, (int64_t)n * PRE_NB, Finv.p, nn, 1e-2 * delta, st);
        const int64_t k1 = k0 + kb, rest = n - k1;
        if (rest > 0) {
            // row panel: R[k, k1:] = R_kk^{-*} A[k, k1:]
            zgemm(dl, nt, kb, rest, kb, Dinv.p + k0, n, (int64_t)n * PRE_NB, 1, PN.p + k0 + k1 * n, n, nn,
                  PN.p + k0 + k1 * n, n, nn, 1.0, 0.0);
            // trailing Hermitian update (upper part)
            zgemm(dl, nt, rest, rest, kb, PN.p + k0 + k1 * n, n, nn, 1, PN.p + k0 + k1 * n, n, nn,
                  PN.p + k1 + k1 * n, n, nn, -1.0, 1.0, 1);
        }
        if (k0 > 0) {
            // F^{-1}[0:k0, k-block] = -F^{-1}[0:k0, 0:k0] R[0:k0, k-block] R_kk^{-1}
            zgemm(dl, nt, k0, kb, k0, Finv.p, n, nn, 0, PN.p + k0 * n, n, nn, T1p.p, n, (int64_t)n * PRE_NB, 1.0,
                  0.0);
            zgemm(dl, nt, k0, kb, kb, T1p.p, n, (int64_t)n * PRE_NB, 0, Dinv.p + k0, n, (int64_t)n * PRE_NB,
                  Finv.p + k0 * n, n, nn, -1.0, 0.0);
        }
    }
    launch_conj_transpose_b(dl, nt, Finv.p, nn, n, FinvH.p, st);
    HIPCHK(hipGetLastError());
    // gamma^2 = lambda_max(F^{-1} F^{-*}) by power iteration
    const int64_t sp = 2 * n;
    launch_randfill(dl, nt, pvec.p, sp, n, n, 1, nullptr, 0x7a11ull, st);
    std::vector<double> g2(T, 0.0);
    for (int it = 0; it < 30; ++it) {
        zgemm(dl, nt, n, 1, n, FinvH.p, n, nn, 0, pvec.p, n, sp, pvec.p + n, n, sp, 1.0, 0.0);
        zgemm(dl, nt, n, 1, n, Finv.p, n, nn, 0, pvec.p + n, n, sp, pvec.p, n, sp, 1.0, 0.0);
        BlockList Lp = bl_empty(n);
        bl_add(Lp, pvec.p, sp, n, 1, nullptr, 0);
        colnorm2(dl, nt, Lp, 1, nrm2.p, 3 * r);
        if (it == 29 || it % 10 == 9) {
            HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * T * 3 * r, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int t : L) g2[t] = sqrt(h_nrm2[(size_t)t * 3 * r]);
        }
        dim3 g((unsigned)((n + 255) / 256), nt);
        // normalise
        launch_scale_cols(dl, nt, pvec.p, sp, n, n, 1, nrm2.p, 3 * r, 2, st);
    }
    for (int t : L) {
        gam[t] = sqrt(std::max(g2[t], 0.0));
        has_prec[t] = 1;
    }
    stats.rebuilds += nt;
}
