// Sparse base preconditioner sites (square CSR C): the colour ordering and
// patterns of the incomplete LU factorisation (host, once per handle), and
// the construction of sites: F = ILU(0) of P (C - z_dag I) P^T, gamma =
// ||(F P)^{-1}||_2 and lambda_n^dagger = lambda_max of the pencil
// (N(z_dag), K) by power iteration (the quantities of the rebuild rule, eq.
// (tauRecycle)).
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

void Engine::build_sparse_pattern()
{
    const int64_t nn = n;
    std::vector<int64_t> rp(m + 1);
    std::vector<int32_t> ci(op.nnz);
    HIPCHK(hipMemcpy(rp.data(), op.rp.p, sizeof(int64_t) * (m + 1), hipMemcpyDeviceToHost));
    if (op.nnz) HIPCHK(hipMemcpy(ci.data(), op.ci.p, sizeof(int32_t) * op.nnz, hipMemcpyDeviceToHost));
    // symmetrised adjacency without the diagonal (duplicates are harmless)
    std::vector<int64_t> deg(nn + 1, 0);
    for (int64_t i = 0; i < nn; ++i)
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int64_t j = ci[q];
            if (j == i) continue;
            deg[i + 1]++;
            deg[j + 1]++;
        }
    for (int64_t i = 0; i < nn; ++i) deg[i + 1] += deg[i];
    std::vector<int32_t> adj(deg[nn]);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t i = 0; i < nn; ++i)
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int64_t j = ci[q];
            if (j == i) continue;
            adj[fill[i]++] = (int32_t)j;
            adj[fill[j]++] = (int32_t)i;
        }
    // greedy colouring in natural order: the smallest colour no coloured
    // neighbour has
    std::vector<int> color(nn, -1), stamp(64 + nn, -1);
    int ncol = 0;
    for (int64_t i = 0; i < nn; ++i) {
        for (int64_t q = deg[i]; q < deg[i + 1]; ++q) {
            const int c = color[adj[q]];
            if (c >= 0) stamp[c] = (int)i;
        }
        int c = 0;
        while (stamp[c] == (int)i) ++c;
        color[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    // colour-major permutation (stable inside a colour)
    std::vector<int64_t> cptr(ncol + 1, 0);
    for (int64_t i = 0; i < nn; ++i) cptr[color[i] + 1]++;
    for (int c = 0; c < ncol; ++c) cptr[c + 1] += cptr[c];
    std::vector<int> perm(nn), iperm(nn);
    {
        std::vector<int64_t> pos(cptr.begin(), cptr.end() - 1);
        for (int64_t i = 0; i < nn; ++i) {
            const int64_t p = pos[color[i]]++;
            perm[p] = (int)i;
            iperm[i] = (int)p;
        }
    }
    // permuted pattern with the diagonal, columns sorted
    std::vector<int64_t> rp2(nn + 1, 0), src2, diag2(nn);
    std::vector<int32_t> ci2;
    src2.reserve(op.nnz + nn);
    ci2.reserve(op.nnz + nn);
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t p = 0; p < nn; ++p) {
        const int64_t i = perm[p];
        row.clear();
        bool hasd = false;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            row.push_back({iperm[ci[q]], q});
            hasd |= (ci[q] == i);
        }
        if (!hasd) row.push_back({(int32_t)p, -1});
        std::sort(row.begin(), row.end());
        for (auto& e : row) {
            if (e.first == p) diag2[p] = (int64_t)ci2.size();
            ci2.push_back(e.first);
            src2.push_back(e.second);
        }
        rp2[p + 1] = (int64_t)ci2.size();
    }
    const int64_t nz = (int64_t)ci2.size();
    // transpose pattern: entry e' = (j, i) of the transpose maps to entry (i, j)
    std::vector<int64_t> rpT(nn + 1, 0), mapT(nz);
    std::vector<int32_t> ciT(nz);
    for (int64_t e = 0; e < nz; ++e) rpT[ci2[e] + 1]++;
    for (int64_t i = 0; i < nn; ++i) rpT[i + 1] += rpT[i];
    {
        std::vector<int64_t> pos(rpT.begin(), rpT.end() - 1);
        for (int64_t i = 0; i < nn; ++i)
            for (int64_t e = rp2[i]; e < rp2[i + 1]; ++e) {
                const int64_t o = pos[ci2[e]]++;
                ciT[o] = (int32_t)i;
                mapT[o] = e;
            }
    }
    op.sp_rp.alloc(nn + 1); op.sp_ci.alloc(nz); op.sp_src.alloc(nz); op.sp_diag.alloc(nn);
    op.sp_rpT.alloc(nn + 1); op.sp_ciT.alloc(nz); op.sp_mapT.alloc(nz); op.sp_perm.alloc(nn);
    HIPCHK(hipMemcpy(op.sp_rp.p, rp2.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_ci.p, ci2.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_src.p, src2.data(), sizeof(int64_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_diag.p, diag2.data(), sizeof(int64_t) * nn, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_rpT.p, rpT.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_ciT.p, ciT.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_mapT.p, mapT.data(), sizeof(int64_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_perm.p, perm.data(), sizeof(int) * nn, hipMemcpyHostToDevice));
    op.sp_cptr = cptr;
    SparsePattern& sp = op.spat;
    sp.n = nn;
    sp.nnz = nz;
    sp.ncolors = ncol;
    sp.cptr = op.sp_cptr.data();
    sp.rp = op.sp_rp.p; sp.ci = op.sp_ci.p; sp.src = op.sp_src.p; sp.diag = op.sp_diag.p;
    sp.rpT = op.sp_rpT.p; sp.ciT = op.sp_ciT.p; sp.mapT = op.sp_mapT.p; sp.perm = op.sp_perm.p;
}

// Factor the sites (slots[i] at sites[i]) and estimate gamma and
// lambda_n^dagger by 12 power steps each.
std::vector<int> Engine::build_sparse_sites(const std::vector<zd>& sites, const std::vector<int>& slots)
{
    std::vector<int> ok;
    if (sites.empty()) return ok;
    const int ns = (int)slots.size();
    const SparsePattern& sp = op.spat;
    std::vector<zd> hz((size_t)NS, zmake(0.0, 0.0));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(hz.data(), d_slotz.p, sizeof(zd) * NS, hipMemcpyDeviceToHost));
    for (int i = 0; i < ns; ++i) hz[slots[i]] = sites[i];
    h2d(d_slotz.p, hz.data(), sizeof(zd) * NS);
    upload_list(slots, d_listB);
    const int* dl = d_listB.p;
    HIPCHK(hipMemsetAsync(d_nfloor.p, 0, sizeof(int), st));
    launch_ilu(dl, ns, sp, op.v.p, d_slotz.p, Slu.p, d_nfloor.p, st);
    // power iterations on (F P)^{-1} (F P)^{-*} (gamma^2) and on
    // Tbar(z_dag) = (F P)^{-*} N(z_dag) (F P)^{-1} (lambda_n^dagger)
    const int64_t sv = 4 * n, sw = (int64_t)n * KB;
    const int r3 = 3 * r;
    std::vector<double> g2(ns, 0.0), ln(ns, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
        launch_randfill(dl, ns, Svec.p, sv, n, n, 1, nullptr, 0x5ca1ull + pass, st);
        for (int it = 0; it < 12; ++it) {
            if (pass == 0) {
                launch_ilu_solve(dl, ns, nullptr, sp, Slu.p, 1, Svec.p, sv, n, Svec.p + n, sv, n, 1, pS.p, sw, st);
                launch_ilu_solve(dl, ns, nullptr, sp, Slu.p, 0, Svec.p + n, sv, n, Svec.p, sv, n, 1, pS.p, sw, st);
            } else {
                launch_ilu_solve(dl, ns, nullptr, sp, Slu.p, 0, Svec.p, sv, n, Svec.p + n, sv, n, 1, pS.p, sw, st);
                apply(false, dl, ns, Svec.p + n, sv, n, Svec.p + 2 * n, sv, n, 1, d_slotz.p);
                apply(true, dl, ns, Svec.p + 2 * n, sv, n, Svec.p + 3 * n, sv, n, 1, d_slotz.p);
                launch_ilu_solve(dl, ns, nullptr, sp, Slu.p, 1, Svec.p + 3 * n, sv, n, Svec.p, sv, n, 1, pS.p, sw, st);
            }
            BlockList Lp = bl_empty(n);
            bl_add(Lp, Svec.p, sv, n, 1, nullptr, 0);
            colnorm2(dl, ns, Lp, 1, nrm2.p, r3);
            if (it == 11) {
                HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * (size_t)(NS + 1) * r3, hipMemcpyDeviceToHost,
                                      st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i < ns; ++i) {
                    const double v = sqrt(std::max(h_nrm2[(size_t)slots[i] * r3], 0.0));
                    (pass == 0 ? g2 : ln)[i] = v;
                }
            }
            launch_scale_cols(dl, ns, Svec.p, sv, n, n, 1, nrm2.p, r3, 2, st);
        }
    }
    int nf = 0;
    HIPCHK(hipMemcpy(&nf, d_nfloor.p, sizeof(int), hipMemcpyDeviceToHost));
    ilu_floors += nf;
    for (int i = 0; i < ns; ++i) {
        const int s = slots[i];
        slot_gam[s] = sqrt(std::max(g2[i], 0.0));
        slot_lamn[s] = std::max(ln[i], 1e-300);
        slot_dreg[s] = 0.0;
        ok.push_back(s);
    }
    return ok;
}
