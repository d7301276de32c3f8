// LOBPCG-SVD (supplement, Alg. SM1.1) on C(z) = C - z S for many tiles at
// once, written as a per-tile state machine so that the scheduler can keep
// the batch full: tiles enter (lob_start) and leave (lob_step returns them)
// independently.  Block size r, r_v = 1, preconditioner K = F^*F (tiles with
// usek) or K = I.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

static const double EPSM_L = 2.220446049250313e-16;

// First Rayleigh-Ritz-SVD step: X0 (S[:, 0:r]) orthonormalised, R of C(z) X0,
// SVD R = J Xi G^*, X1 = X0 G, C X1 = (C X0) G, residual W = C^*(C X1) - X1 Xi^2.
void Engine::lob_start(const std::vector<int>& L, uint64_t seed)
{
    if (L.empty()) return;
    const int nt = (int)L.size();
    upload_list(L, d_list);
    const int64_t sS = (int64_t)n * 3 * r, sC = (int64_t)m * 3 * r;
    const int r3 = 3 * r;
    orthonormalize(L, d_list.p, S.p, sS, n, n, r, nullptr, 0, seed);
    op_apply(false, L, S.p, sS, n, CS.p, sC, m, r);
    BlockList Lcx = bl_empty(m);
    bl_add(Lcx, CS.p, sC, m, r, nullptr, 0);
    r_factor(d_list.p, nt, Lcx, r, nullptr, 0, r, Rsm.p, (int64_t)9 * r * r, r3);
    RRArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.list = d_list.p;
    ra.cdim = cdim.p;              // preset row: r for every tile
    ra.r = r;
    ra.max_sweeps = 40;
    ra.R = Rsm.p;
    ra.strideR = (int64_t)9 * r * r;
    ra.ldR = r3;
    ra.GX = GX.p;
    ra.GP = GP.p;
    ra.strideGX = (int64_t)9 * r * r;
    ra.ldGX = r3;
    ra.xi = xi.p;
    ra.ldxi = r3;
    int pi0 = prof.begin(st, 5, 0.0, 0.0);
    launch_rr_hl(ra, nt, r, st);
    prof.end(st, pi0);
    BlockList Ls = bl_empty(n);
    bl_add(Ls, S.p, sS, n, r, nullptr, 0);
    gemm_ts(d_list.p, nt, Ls, r, GX.p, (int64_t)9 * r * r, r3, nullptr, 0, r, Sn.p, sS, n, n, 1.0, 0.0);
    gemm_ts(d_list.p, nt, Lcx, r, GX.p, (int64_t)9 * r * r, r3, nullptr, 0, r, CSn.p, sC, m, m, 1.0, 0.0);
    launch_copy_cols(d_list.p, nt, Sn.p, sS, n, S.p, sS, n, n, r, st);
    launch_copy_cols(d_list.p, nt, CSn.p, sC, m, CS.p, sC, m, m, r, st);
    op_apply(true, L, CS.p, sC, m, Wres.p, (int64_t)n * r, n, r);
    launch_resid_xi(d_list.p, nt, Wres.p, (int64_t)n * r, n, S.p, sS, n, xi.p, r3, n, r, st);
    for (int t : L) lob_it[t] = 0;
}

std::vector<double> Engine::explicit_rq(const std::vector<int>& L)
{
    std::vector<double> out(L.size(), 0.0);
    if (L.empty()) return out;
    const int64_t sS = (int64_t)n * 3 * r, sC = (int64_t)m * 3 * r;
    const int r3 = 3 * r;
    upload_list(L, d_list2);
    const int nt = (int)L.size();
    op_apply(false, L, S.p, sS, n, CS.p, sC, m, r);
    BlockList Lx = bl_empty(n);
    bl_add(Lx, S.p, sS, n, 1, nullptr, 0);
    BlockList Lcx = bl_empty(m);
    bl_add(Lcx, CS.p, sC, m, 1, nullptr, 0);
    colnorm2(d_list2.p, nt, Lx, 1, nrm2.p, r3);
    colnorm2(d_list2.p, nt, Lcx, 1, nrm2.p + 1, r3);
    HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * T * r3, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < L.size(); ++i) {
        const int t = L[i];
        const double xn2 = h_nrm2[(size_t)t * r3], cn2 = h_nrm2[(size_t)t * r3 + 1];
        out[i] = (xn2 > 0.0) ? sqrt(std::max(cn2, 0.0) / xn2) : INFINITY;
    }
    return out;
}

// One iteration for every tile in L:
//   W <- K^{-1} W; W orthonormal and orthogonal to [X P]; S = [X W P];
//   R of C(z) S (mixed-precision Cholesky QR); SVD of R; Hetmaniuk-Lehoucq
//   X, P; implicit C X, C P; W = C^*(C X) - X Xi^2; the test of eq. (tolSVD)
//   on the first Ritz pair, confirmed with an explicitly recomputed C X.
void Engine::lob_step(const std::vector<int>& L, uint64_t seed, std::vector<int>& done, std::vector<int>& okv)
{
    done.clear();
    okv.clear();
    if (L.empty()) return;
    const int nt = (int)L.size();
    const int64_t sS = (int64_t)n * 3 * r, sC = (int64_t)m * 3 * r;
    const int r3 = 3 * r;
    upload_list(L, d_list);
    // per-tile widths: S has 2r columns on a tile's first iteration, 3r after
    {
        h_small.alloc(2 * T + 8);
        int* hc = (int*)h_small.p;
        for (int t = 0; t < T; ++t) {
            bool hasP = lob_it[t] > 0 && !nop[t];
            hc[t] = hasP ? 3 * r : 2 * r;
            hc[T + t] = hasP ? r : 0;
        }
        h2d(d_cdimt.p, hc, sizeof(int) * T);
        h2d(d_pcols.p, hc + T, sizeof(int) * T);
    }
    // W <- K^{-1} W into S[:, r:2r]: K = F^* F of the tile's site, plus the
    // coarse term Ebar Lambda_bar^{-1} Ebar^* W of eq. (twolevel) when the
    // tile has projection vectors; projection-phase tiles run with K = I
    if (use_prec) {
        std::vector<int> Lk, Li, L2;
        for (int t : L) {
            const bool pre = usek[t] && !(two_level && phase[t]);
            (pre ? Lk : Li).push_back(t);
            if (pre && two_level && use2l[t]) L2.push_back(t);
            if (two_level && phase[t]) stats.proj_iters++;
        }
        stats.precond_iters += (int64_t)Lk.size();
        upload_list(Li, d_listI);
        precond_apply(Lk, Wres.p, (int64_t)n * r, S.p + (size_t)n * r, sS);
        twolevel_add(L2, Wres.p, (int64_t)n * r, S.p + (size_t)n * r, sS);
        launch_copy_cols(d_listI.p, (int)Li.size(), Wres.p, (int64_t)n * r, n, S.p + (size_t)n * r, sS, n, n, r,
                         st);
    } else {
        launch_copy_cols(d_list.p, nt, Wres.p, (int64_t)n * r, n, S.p + (size_t)n * r, sS, n, n, r, st);
    }
    stats.lobpcg_iters += nt;
    BlockList Lxp = bl_empty(n);
    bl_add(Lxp, S.p, sS, n, r, nullptr, 0);
    bl_add(Lxp, S.p + (size_t)2 * n * r, sS, n, 0, d_pcols.p, 1);
    orthonormalize(L, d_list.p, S.p + (size_t)n * r, sS, n, n, r, &Lxp, 2 * r, seed);
    op_apply(false, L, S.p + (size_t)n * r, sS, n, CS.p + (size_t)m * r, sC, m, r);
    BlockList Lcs = bl_empty(m);
    bl_add(Lcs, CS.p, sC, m, 0, d_cdimt.p, 1);
    // R of C(z) S: a Gram matrix in double perturbs an eigenvalue xi^2 by
    // about eps ||C(z) S||^2, i.e. xi by eps (||C|| + |z|)^2 / (2 xi); for a
    // tile whose previous smallest Ritz value is at least 1e-4 (||C|| + |z|)
    // that is below 1e-12 (||C|| + |z|), four orders under the tolerance, and
    // the double Gram is used; otherwise (and on a refinement's first
    // iteration) the Gram is accumulated in double-double
    {
        std::vector<int> Ldd, Lpl;
        for (int t : L) {
            const double nz = op.normC + sqrt(zabs2(h_zt[t]));
            const bool proj = two_level && phase[t];     // Mbar(z): another scale, keep double-double
            if (!proj && lob_it[t] >= 1 && lob_xi[t] >= 1e-4 * nz) Lpl.push_back(t);
            else Ldd.push_back(t);
        }
        if (Lpl.empty()) {
            r_factor(d_list.p, nt, Lcs, r3, d_cdimt.p, 1, 0, Rsm.p, (int64_t)9 * r * r, r3);
        } else {
            upload_list(Lpl, d_listPL);
            r_factor(d_listPL.p, (int)Lpl.size(), Lcs, r3, d_cdimt.p, 1, 0, Rsm.p, (int64_t)9 * r * r, r3, nullptr,
                     nullptr, false);
            if (!Ldd.empty()) {
                upload_list(Ldd, d_listDD);
                r_factor(d_listDD.p, (int)Ldd.size(), Lcs, r3, d_cdimt.p, 1, 0, Rsm.p, (int64_t)9 * r * r, r3);
            }
        }
    }
    for (int t : L) nop[t] = 0;
    RRArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.list = d_list.p;
    ra.cdim = d_cdimt.p;
    ra.r = r;
    ra.max_sweeps = 40;
    ra.R = Rsm.p;
    ra.strideR = (int64_t)9 * r * r;
    ra.ldR = r3;
    ra.GX = GX.p;
    ra.GP = GP.p;
    ra.strideGX = (int64_t)9 * r * r;
    ra.ldGX = r3;
    ra.xi = xi.p;
    ra.ldxi = r3;
    int pi0 = prof.begin(st, 5, 0.0, 0.0);
    launch_rr_hl(ra, nt, r3, st);
    prof.end(st, pi0);
    BlockList Ls = bl_empty(n);
    bl_add(Ls, S.p, sS, n, 0, d_cdimt.p, 1);
    gemm_ts(d_list.p, nt, Ls, r3, GX.p, (int64_t)9 * r * r, r3, nullptr, 0, r, Sn.p, sS, n, n, 1.0, 0.0);
    gemm_ts(d_list.p, nt, Ls, r3, GP.p, (int64_t)9 * r * r, r3, nullptr, 0, r, Sn.p + (size_t)n * r, sS, n, n, 1.0,
            0.0);
    gemm_ts(d_list.p, nt, Lcs, r3, GX.p, (int64_t)9 * r * r, r3, nullptr, 0, r, CSn.p, sC, m, m, 1.0, 0.0);
    gemm_ts(d_list.p, nt, Lcs, r3, GP.p, (int64_t)9 * r * r, r3, nullptr, 0, r, CSn.p + (size_t)m * r, sC, m, m, 1.0,
            0.0);
    launch_copy_cols(d_list.p, nt, Sn.p, sS, n, S.p, sS, n, n, r, st);
    launch_copy_cols(d_list.p, nt, Sn.p + (size_t)n * r, sS, n, S.p + (size_t)2 * n * r, sS, n, n, r, st);
    launch_copy_cols(d_list.p, nt, CSn.p, sC, m, CS.p, sC, m, m, r, st);
    launch_copy_cols(d_list.p, nt, CSn.p + (size_t)m * r, sC, m, CS.p + (size_t)2 * m * r, sC, m, m, r, st);
    for (int t : L) lob_it[t]++;
    auto residual = [&](const std::vector<int>& Lh, const int* dl) {
        op_apply(true, Lh, CS.p, sC, m, Wres.p, (int64_t)n * r, n, r);
        launch_resid_xi(dl, (int)Lh.size(), Wres.p, (int64_t)n * r, n, S.p, sS, n, xi.p, r3, n, r, st);
    };
    residual(L, d_list.p);
    BlockList Lw = bl_empty(n);
    bl_add(Lw, Wres.p, (int64_t)n * r, n, r, nullptr, 0);
    BlockList Lx = bl_empty(n);
    bl_add(Lx, S.p, sS, n, r, nullptr, 0);
    BlockList Lcx = bl_empty(m);
    bl_add(Lcx, CS.p, sC, m, r, nullptr, 0);
    // per tile, at stride 3r: residual norms^2 (columns 0..r), ||x_j||^2 (r..2r)
    colnorm2(d_list.p, nt, Lw, r, nrm2.p, r3);
    colnorm2(d_list.p, nt, Lx, r, nrm2.p + r, r3);
    HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * T * r3, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_xi.p, xi.p, sizeof(double) * T * r3, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double nC = op.normC;
    // The Rayleigh-Ritz-SVD takes S as orthonormal.  If S lost rank (a
    // direction of W or P that collapsed), the singular values of R are not
    // Ritz values of C(z): the right vector of a spurious zero selects the
    // collapsed direction, and the new X then has a column far from unit
    // norm.  Such a step is a breakdown: the block X is orthonormalised
    // again, C(z) X recomputed, and the next iteration runs without P.  (A
    // zero pivot in the R factor alone is no breakdown: near the spectrum
    // C(z) has singular values far below the rounding of its Gram matrix.)
    auto xdev = [&](int t, int off) {
        double d = 0.0;
        for (int j = 0; j < r; ++j) d = std::max(d, fabs(h_nrm2[(size_t)t * r3 + off + j] - 1.0));
        return d;
    };
    std::vector<int> bad;
    for (int t : L) {
        lob_bad[t] = !(xdev(t, r) <= 1e-6) ? 1 : 0;
        if (lob_bad[t]) bad.push_back(t);
    }
    // floor of eq. (tolSVD): the residual C(z)^*(C(z) x) - xi^2 x is itself
    // computed with an error of order sqrt(n) eps ||C(z)||^2, so a floor of
    // exactly eps ||C(z)||^2 can be out of reach; the constant scales with it.
    // A residual w of the Hermitian N(z) = C(z)^* C(z) at the unit vector x
    // places an eigenvalue sigma_j^2 within w of xi^2, hence |sigma_j - xi|
    // <= w / xi: the floor branch is taken only where that bound is within
    // tol_abs ||C||.
    const double floor_c = std::max(16.0, 4.0 * sqrt((double)n));
    auto passes = [&](int t, double x0) {
        double nz = nC + sqrt(zabs2(h_zt[t]));
        double w0 = sqrt(std::max(0.0, h_nrm2[(size_t)t * r3]));
        bool lin = w0 <= P.eta_svd * nz * x0;
        bool flo = w0 <= floor_c * nz * nz * EPSM_L && w0 <= P.tol_abs * nC * x0;
        return lin || flo || x0 <= P.eta_abs * nC;
    };
    // projection phase (LOBPCG-SVD on Mbar(z) with r_v = r): every Ritz pair
    // meets the relaxed test of eq. (tolTz), ||W_j|| <= eta_proj ||Tbar(z)||
    auto passes_proj = [&](int t) {
        const double nT = tbar_norm(tile_slot[t], h_zt[t]);
        for (int j = 0; j < r; ++j)
            if (!(sqrt(std::max(0.0, h_nrm2[(size_t)t * r3 + j])) <= P.eta_proj * nT)) return false;
        return true;
    };
    std::vector<int> cand;
    std::vector<char> fin(T, 0);
    for (int t : L) {
        lob_xi[t] = h_xi[(size_t)t * r3];
        for (int j = 0; j < r; ++j) lob_sv[(size_t)t * r + j] = h_xi[(size_t)t * r3 + j];
    }
    for (int t : L) {
        if (two_level && phase[t]) {
            if (!lob_bad[t] && passes_proj(t)) fin[t] = 1;
            continue;
        }
        if (!lob_bad[t] && passes(t, h_xi[(size_t)t * r3])) cand.push_back(t);
    }
    if (!cand.empty()) {
        // explicit recomputation of C(z) X before accepting (the implicit
        // updates of C X drift); the value returned for the point is the
        // Rayleigh quotient ||C(z) x_1|| / ||x_1|| of the recomputed product,
        // an upper bound of sigma_min up to the rounding of one apply
        upload_list(cand, d_list2);
        op_apply(false, cand, S.p, sS, n, CS.p, sC, m, r);
        residual(cand, d_list2.p);
        colnorm2(d_list2.p, (int)cand.size(), Lw, r, nrm2.p, r3);
        colnorm2(d_list2.p, (int)cand.size(), Lcx, r, nrm2.p + r, r3);
        colnorm2(d_list2.p, (int)cand.size(), Lx, r, nrm2.p + 2 * r, r3);
        HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * T * r3, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int t : cand) {
            const double xn2 = h_nrm2[(size_t)t * r3 + 2 * r];
            const double cn2 = h_nrm2[(size_t)t * r3 + r];
            if (!(fabs(xn2 - 1.0) <= 1e-6)) { lob_bad[t] = 1; bad.push_back(t); continue; }
            const double xe = sqrt(std::max(cn2, 0.0) / xn2);
            if (passes(t, xe)) {
                fin[t] = 1;
                lob_sigma[t] = xe;
            }
        }
    }
    if (!bad.empty()) {
        stats.repairs += (int64_t)bad.size();
        upload_list(bad, d_list2);
        orthonormalize(bad, d_list2.p, S.p, sS, n, n, r, nullptr, 0, seed ^ 0x5bd1e995ull);
        op_apply(false, bad, S.p, sS, n, CS.p, sC, m, r);
        residual(bad, d_list2.p);
        for (int t : bad) nop[t] = 1;
    }
    const int proj_cap = std::min(P.max_iters, 100);
    for (int t : L) {
        if (two_level && phase[t]) {
            if (fin[t] || lob_it[t] >= proj_cap) {
                done.push_back(t);
                okv.push_back(fin[t] ? 3 : 4);
            }
            continue;
        }
        if (fin[t] || lob_it[t] >= P.max_iters) {
            if (!fin[t]) lob_sigma[t] = h_xi[(size_t)t * r3];
            done.push_back(t);
            okv.push_back(fin[t] ? 1 : 0);
        }
    }
}
