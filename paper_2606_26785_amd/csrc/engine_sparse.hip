// Sparse base preconditioner sites (CSR C, m >= n): the pattern of N = C^* C,
// its colour ordering and the contribution lists that form N(z) from the
// values of C (host, once per handle), and the construction of sites: the
// incomplete Cholesky factorization of N(z_dag) + alpha I (Sec. 3 and 4; the
// shift alpha raised until every pivot is positive), gamma = ||F^{-1}||_2
// and lambda_n^dagger = lambda_max of the pencil (N(z_dag), K) by power
// iteration (the quantities of the rebuild rule, eq. (tauRecycle)).
#include "engine.h"

#include <algorithm>
#include <climits>
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
    // entries of each row of C - z I as (column, code): code = 2 q + [diagonal]
    // for the CSR entry q, -1 for a diagonal entry C does not store
    auto row_entries = [&](int64_t i, std::vector<std::pair<int32_t, int64_t>>& E) {
        E.clear();
        bool hasd = false;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const bool d = (ci[q] == i);
            hasd |= d;
            E.push_back({ci[q], 2 * q + (d ? 1 : 0)});
        }
        if (i < nn && !hasd) E.push_back({(int32_t)i, -1});
    };
    // pattern of N: (j, k) for every pair of entries in one row of C, plus
    // the diagonal
    std::vector<std::vector<int32_t>> adj(nn);
    std::vector<std::pair<int32_t, int64_t>> E;
    for (int64_t i = 0; i < m; ++i) {
        row_entries(i, E);
        for (auto& a : E)
            for (auto& b : E) adj[a.first].push_back(b.first);
    }
    for (int64_t j = 0; j < nn; ++j) {
        adj[j].push_back((int32_t)j);
        std::sort(adj[j].begin(), adj[j].end());
        adj[j].erase(std::unique(adj[j].begin(), adj[j].end()), adj[j].end());
    }
    // greedy colouring of N's graph in natural order: the smallest colour no
    // coloured neighbour has
    std::vector<int> color(nn, -1), stamp(nn + 64, -1);
    int ncol = 0;
    for (int64_t j = 0; j < nn; ++j) {
        for (int32_t k : adj[j]) {
            const int c = color[k];
            if (c >= 0) stamp[c] = (int)j;
        }
        int c = 0;
        while (stamp[c] == (int)j) ++c;
        color[j] = c;
        ncol = std::max(ncol, c + 1);
    }
    // colour-major permutation (stable inside a colour)
    std::vector<int64_t> cptr(ncol + 1, 0);
    for (int64_t j = 0; j < nn; ++j) cptr[color[j] + 1]++;
    for (int c = 0; c < ncol; ++c) cptr[c + 1] += cptr[c];
    std::vector<int> perm(nn), iperm(nn);
    {
        std::vector<int64_t> pos(cptr.begin(), cptr.end() - 1);
        for (int64_t j = 0; j < nn; ++j) {
            const int64_t p = pos[color[j]]++;
            perm[p] = (int)j;
            iperm[j] = (int)p;
        }
    }
    // permuted pattern, columns sorted, diagonal positions
    std::vector<int64_t> rp2(nn + 1, 0), diag2(nn);
    for (int64_t p = 0; p < nn; ++p) rp2[p + 1] = rp2[p] + (int64_t)adj[perm[p]].size();
    const int64_t nz = rp2[nn];
    std::vector<int32_t> ci2(nz);
    for (int64_t p = 0; p < nn; ++p) {
        int64_t o = rp2[p];
        for (int32_t k : adj[perm[p]]) ci2[o++] = iperm[k];
        std::sort(ci2.begin() + rp2[p], ci2.begin() + rp2[p + 1]);
        for (int64_t e = rp2[p]; e < rp2[p + 1]; ++e)
            if (ci2[e] == p) diag2[p] = e;
    }
    std::vector<std::vector<int32_t>>().swap(adj);
    auto find_entry = [&](int64_t p, int32_t q) -> int64_t {
        auto b = ci2.begin() + rp2[p], e = ci2.begin() + rp2[p + 1];
        auto it = std::lower_bound(b, e, q);
        return (int64_t)(it - ci2.begin());
    };
    // contribution lists: N_{jk} += conj(c_a) c_b for entries a (column j)
    // and b (column k) of one row of C - z I
    std::vector<int64_t> ccp(nz + 1, 0);
    for (int64_t i = 0; i < m; ++i) {
        row_entries(i, E);
        for (auto& a : E)
            for (auto& b : E) ccp[find_entry(iperm[a.first], iperm[b.first]) + 1]++;
    }
    for (int64_t e = 0; e < nz; ++e) ccp[e + 1] += ccp[e];
    std::vector<int64_t> ca(ccp[nz]), cb(ccp[nz]);
    {
        std::vector<int64_t> fill(ccp.begin(), ccp.end() - 1);
        for (int64_t i = 0; i < m; ++i) {
            row_entries(i, E);
            for (auto& a : E)
                for (auto& b : E) {
                    const int64_t o = fill[find_entry(iperm[a.first], iperm[b.first])]++;
                    ca[o] = a.second;
                    cb[o] = b.second;
                }
        }
    }
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
    const int64_t nc = ccp[nz];
    op.sp_rp.alloc(nn + 1); op.sp_ci.alloc(nz); op.sp_diag.alloc(nn);
    op.sp_rpT.alloc(nn + 1); op.sp_ciT.alloc(nz); op.sp_mapT.alloc(nz); op.sp_perm.alloc(nn);
    op.sp_ccp.alloc(nz + 1); op.sp_ca.alloc(std::max<int64_t>(nc, 1)); op.sp_cb.alloc(std::max<int64_t>(nc, 1));
    HIPCHK(hipMemcpy(op.sp_rp.p, rp2.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_ci.p, ci2.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_diag.p, diag2.data(), sizeof(int64_t) * nn, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_rpT.p, rpT.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_ciT.p, ciT.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_mapT.p, mapT.data(), sizeof(int64_t) * nz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_perm.p, perm.data(), sizeof(int) * nn, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(op.sp_ccp.p, ccp.data(), sizeof(int64_t) * (nz + 1), hipMemcpyHostToDevice));
    if (nc) {
        HIPCHK(hipMemcpy(op.sp_ca.p, ca.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(op.sp_cb.p, cb.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice));
    }
    // narrow band of N in the natural order: exact inertia tests by a band
    // Cholesky (the entries (j, j + d), d <= b, from the same row pairs)
    {
        int64_t b = 0;
        for (int64_t i = 0; i < m; ++i) {
            row_entries(i, E);
            int32_t lo = INT32_MAX, hi = -1;
            for (auto& a : E) { lo = std::min(lo, a.first); hi = std::max(hi, a.first); }
            if (hi >= 0) b = std::max<int64_t>(b, hi - lo);
        }
        band_b = (b <= 63) ? (int)b : -1;
        if (band_b >= 0) {
            const int64_t bw = band_b + 1, ne = nn * bw;
            std::vector<int64_t> bcp(ne + 1, 0);
            for (int64_t i = 0; i < m; ++i) {
                row_entries(i, E);
                for (auto& a : E)
                    for (auto& c : E)
                        if (c.first >= a.first) bcp[(int64_t)a.first * bw + (c.first - a.first) + 1]++;
            }
            for (int64_t e = 0; e < ne; ++e) bcp[e + 1] += bcp[e];
            std::vector<int64_t> ba(std::max<int64_t>(bcp[ne], 1)), bb(std::max<int64_t>(bcp[ne], 1));
            std::vector<int64_t> fill(bcp.begin(), bcp.end() - 1);
            for (int64_t i = 0; i < m; ++i) {
                row_entries(i, E);
                for (auto& a : E)
                    for (auto& c : E)
                        if (c.first >= a.first) {
                            const int64_t o = fill[(int64_t)a.first * bw + (c.first - a.first)]++;
                            ba[o] = a.second;
                            bb[o] = c.second;
                        }
            }
            bn_cp.alloc(ne + 1); bn_ca.alloc(ba.size()); bn_cb.alloc(bb.size());
            HIPCHK(hipMemcpy(bn_cp.p, bcp.data(), sizeof(int64_t) * (ne + 1), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(bn_ca.p, ba.data(), sizeof(int64_t) * ba.size(), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(bn_cb.p, bb.data(), sizeof(int64_t) * bb.size(), hipMemcpyHostToDevice));
        }
    }
    op.sp_cptr = cptr;
    SparsePattern& sp = op.spat;
    sp.n = nn;
    sp.nnz = nz;
    sp.ncolors = ncol;
    sp.cptr = op.sp_cptr.data();
    sp.rp = op.sp_rp.p; sp.ci = op.sp_ci.p; sp.diag = op.sp_diag.p;
    sp.rpT = op.sp_rpT.p; sp.ciT = op.sp_ciT.p; sp.mapT = op.sp_mapT.p; sp.perm = op.sp_perm.p;
    sp.ccp = op.sp_ccp.p; sp.ca = op.sp_ca.p; sp.cb = op.sp_cb.p;
}

// Factor the sites (slots[i] at sites[i]) and estimate gamma and
// lambda_n^dagger by 12 power steps each.  The shift starts at
// alpha = (reg_base (||C|| + |z_dag|))^2 (at least 1e-8 (||C|| + |z_dag|)^2)
// and is multiplied by 4 for a site whose factorization met a non-positive
// pivot, up to 16 times.
std::vector<int> Engine::build_sparse_sites(const std::vector<zd>& sites, const std::vector<int>& slots)
{
    std::vector<int> ok;
    if (sites.empty()) return ok;
    const int ns = (int)slots.size();
    const SparsePattern& sp = op.spat;
    std::vector<zd> hz((size_t)NS, zmake(0.0, 0.0));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(hz.data(), d_slotz.p, sizeof(zd) * NS, hipMemcpyDeviceToHost));
    for (int i = 0; i < ns; ++i) {
        hz[slots[i]] = sites[i];
        const double sc = op.normC + sqrt(zabs2(sites[i]));
        slot_alpha[slots[i]] = std::max(P.reg_base * P.reg_base, 1e-8) * sc * sc;
    }
    h2d(d_slotz.p, hz.data(), sizeof(zd) * NS);
    std::vector<int> todo(slots);
    std::vector<int> bad((size_t)NS, 0);
    for (int attempt = 0; !todo.empty(); ++attempt) {
        if (attempt > 16) throw DeviceError("incomplete Cholesky: no positive factorization after raising the shift");
        h2d(d_alpha.p, slot_alpha.data(), sizeof(double) * NS);
        std::vector<int> zero((size_t)NS, 0);
        h2d(d_icbad.p, zero.data(), sizeof(int) * NS);
        upload_list(todo, d_listB);
        launch_icn(d_listB.p, (int)todo.size(), sp, op.v.p, d_slotz.p, d_alpha.p, Slu.p, d_icbad.p, st);
        HIPCHK(hipMemcpyAsync(bad.data(), d_icbad.p, sizeof(int) * NS, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<int> again;
        for (int s : todo)
            if (bad[s]) {
                slot_alpha[s] *= 4.0;
                again.push_back(s);
                stats.ic_retries++;
            }
        todo.swap(again);
    }
    upload_list(slots, d_listB);
    const int* dl = d_listB.p;
    // power iterations on F^{-1} F^{-*} (gamma^2) and on
    // Tbar(z_dag) = F^{-*} N(z_dag) F^{-1} (lambda_n^dagger)
    // per slot: x (n), F^{-1} x (n), C(z) F^{-1} x (m), C(z)^* C(z) F^{-1} x (n)
    const int64_t sv = 3 * n + m, sw = (int64_t)n * KB;
    const int r3 = 3 * r;
    std::vector<double> g2(ns, 0.0), ln(ns, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
        launch_randfill(dl, ns, Svec.p, sv, n, n, 1, nullptr, 0x5ca1ull + pass, st);
        for (int it = 0; it < 12; ++it) {
            if (pass == 0) {
                launch_ic_solve(dl, ns, nullptr, sp, Slu.p, 1, Svec.p, sv, n, Svec.p + n, sv, n, 1, pS.p, sw, st);
                launch_ic_solve(dl, ns, nullptr, sp, Slu.p, 0, Svec.p + n, sv, n, Svec.p, sv, n, 1, pS.p, sw, st);
            } else {
                launch_ic_solve(dl, ns, nullptr, sp, Slu.p, 0, Svec.p, sv, n, Svec.p + n, sv, n, 1, pS.p, sw, st);
                apply(false, dl, ns, Svec.p + n, sv, n, Svec.p + 2 * n, sv, m, 1, d_slotz.p);
                apply(true, dl, ns, Svec.p + 2 * n, sv, m, Svec.p + 2 * n + m, sv, n, 1, d_slotz.p);
                launch_ic_solve(dl, ns, nullptr, sp, Slu.p, 1, Svec.p + 2 * n + m, sv, n, Svec.p, sv, n, 1, pS.p,
                                sw, st);
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
    for (int i = 0; i < ns; ++i) {
        const int s = slots[i];
        slot_gam[s] = sqrt(std::max(g2[i], 0.0));
        slot_lamn[s] = std::max(ln[i], 1e-300);
        slot_dreg[s] = 0.0;
        ok.push_back(s);
    }
    return ok;
}

// Inertia tests N(z_i) - mu_i I > 0 for a narrow-band CSR C (band_b >= 0),
// up to 32 at a time: pd[i] = 1 when every pivot of the band Cholesky is
// positive.
void Engine::band_inertia(const std::vector<zd>& zs, const std::vector<double>& mus, std::vector<char>& pd)
{
    pd.assign(zs.size(), 0);
    if (band_b < 0 || zs.empty()) return;
    const int64_t bw = band_b + 1;
    const int cap = 32;
    if (bn_W.n < (size_t)cap * n * bw) {
        HIPCHK(hipStreamSynchronize(st));
        bn_W.alloc((size_t)cap * n * bw);
        bn_z.alloc(cap); bn_mu.alloc(cap); bn_bad.alloc(cap); bn_list.alloc(cap);
        std::vector<int> id(cap);
        for (int i = 0; i < cap; ++i) id[i] = i;
        HIPCHK(hipMemcpy(bn_list.p, id.data(), sizeof(int) * cap, hipMemcpyHostToDevice));
    }
    for (size_t b0 = 0; b0 < zs.size(); b0 += cap) {
        const int nb = (int)std::min<size_t>(cap, zs.size() - b0);
        std::vector<zd> hz(zs.begin() + b0, zs.begin() + b0 + nb);
        std::vector<double> hm(mus.begin() + b0, mus.begin() + b0 + nb);
        std::vector<int> zero(nb, 0), bad(nb, 0);
        h2d(bn_z.p, hz.data(), sizeof(zd) * nb);
        h2d(bn_mu.p, hm.data(), sizeof(double) * nb);
        h2d(bn_bad.p, zero.data(), sizeof(int) * nb);
        launch_band_inertia(bn_list.p, nb, bn_z.p, bn_mu.p, bn_cp.p, bn_ca.p, bn_cb.p, op.v.p, n, band_b, bn_W.p,
                            n * bw, 0.0, bn_bad.p, st);
        HIPCHK(hipMemcpyAsync(bad.data(), bn_bad.p, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int i = 0; i < nb; ++i) pd[b0 + i] = bad[i] ? 0 : 1;
    }
}
