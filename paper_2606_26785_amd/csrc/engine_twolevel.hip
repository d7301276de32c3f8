// The two-level preconditioner of Sec. 3 with its recycled projection
// subspace: K_Ebar^{-1} W = F^{-1} F^{-*} W + Ebar Lambda_bar^{-1} Ebar^* W
// (eq. (twolevel) with Z = Ebar, for which Z^* N(z) Z = Lambda_bar), the
// projection store of each preconditioner site, recyProj (Alg. 4) and the
// projection-store update (Alg. 2 with r_breve leading columns).
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

// ---------------------------------------------------------------------------
// small kernels

// A[i, j] /= lam[tile * ldl + i] for the r x r coefficient block of each tile
// (rows whose lambda is not positive are zeroed)
__global__ void k_scale_rows(const int* list, zd* A, int64_t stride, int lda, int rows, int cols, const double* lam,
                             int ldl)
{
    const int tile = list[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    const int i = e % rows, j = e / rows;
    const double l = lam[(size_t)tile * ldl + i];
    zd* p = A + (size_t)tile * stride + i + (size_t)j * lda;
    *p = (l > 0.0) ? zscale(*p, 1.0 / l) : zmake(0.0, 0.0);
}

// Rinv = R^{-1} for the upper-triangular c x c R of each listed slot (c =
// dims[slot] <= 64); columns c..cmax of Rinv are zero.  One thread per
// column, back substitution on an LDS copy of R.
__global__ void k_trinv(const int* list, const int* dims, const zd* R, int64_t sR, int ldR, zd* Ri, int64_t sRi,
                        int ldRi, int cmax)
{
    __shared__ zd Rs[64 * 64];
    const int s = list[blockIdx.x];
    const int c = min(dims[s], 64);
    const zd* Rp = R + (size_t)s * sR;
    for (int e = threadIdx.x; e < c * c; e += blockDim.x) {
        const int i = e % c, j = e / c;
        Rs[i + j * c] = (i <= j) ? Rp[i + (size_t)j * ldR] : zmake(0.0, 0.0);
    }
    __syncthreads();
    zd* Op = Ri + (size_t)s * sRi;
    const int j = threadIdx.x;
    if (j >= cmax) return;
    if (j >= c) {
        for (int i = 0; i < cmax; ++i) Op[i + (size_t)j * ldRi] = zmake(0.0, 0.0);
        return;
    }
    // x = R^{-1} e_j: x_i = 0 for i > j; x_j = 1 / R_jj; x_i = -(sum_{k>i} R_ik x_k) / R_ii
    zd x[64];
    for (int i = 0; i < 64; ++i) x[i] = zmake(0.0, 0.0);
    for (int i = j; i >= 0; --i) {
        zd acc = zmake(i == j ? 1.0 : 0.0, 0.0);
        for (int k = i + 1; k <= j; ++k) acc = zsub(acc, zmul(Rs[i + k * c], x[k]));
        const zd d = Rs[i + i * c];
        const double dd = zabs2(d);
        x[i] = (dd > 0.0) ? zscale(zmul(acc, zconj(d)), 1.0 / dd) : zmake(0.0, 0.0);
    }
    for (int i = 0; i < cmax; ++i) Op[i + (size_t)j * ldRi] = (i <= j) ? x[i] : zmake(0.0, 0.0);
}

// ---------------------------------------------------------------------------
void Engine::upload_pk()
{
    std::vector<int> v(pk.begin(), pk.end());
    v.push_back(0);   // index NS: the empty store
    h2d(d_pk.p, v.data(), sizeof(int) * v.size());
}

void Engine::proj_reset(int slot)
{
    if (!two_level || slot < 0) return;
    pk[slot] = 0;
    upload_pk();
}

bool Engine::site_at(int t) const
{
    const int s = tile_slot[t];
    return s >= 0 && slot_z[s].x == h_zt[t].x && slot_z[s].y == h_zt[t].y;
}

std::vector<int> Engine::build_regularized(const std::vector<zd>& sites)
{
    std::vector<double> mu(sites.size());
    for (size_t i = 0; i < sites.size(); ++i) {
        const double d = P.reg_base * (op.normC + sqrt(zabs2(sites[i])));
        mu[i] = -std::max(d * d, 1e-300);    // a negative shift mu adds |mu| I
    }
    std::vector<int> got = build_precond(sites, &mu);
    for (size_t i = 0; i < sites.size(); ++i)
        if (got[i] >= 0) {
            slot_dreg[got[i]] = -mu[i];
            // K = N(z_dag) + d I: the pencil (N(z_dag), K) has eigenvalues
            // s^2 / (s^2 + d) < 1, so lambda_n^dagger <= 1
            slot_lamn[got[i]] = 1.0;
        }
    return got;
}

void Engine::rebuild_here(const std::vector<int>& tl, std::vector<uint8_t>& fl)
{
    if (tl.empty()) return;
    std::vector<zd> sites;
    for (int t : tl) sites.push_back(h_zt[t]);
    std::vector<int> got = build_regularized(sites);
    for (size_t i = 0; i < tl.size(); ++i) {
        const int t = tl[i];
        if (got[i] < 0) {
            // no free slot: keep the current site and its projection vectors
            use2l[t] = phase[t] ? 0 : use2l[t];
            phase[t] = 0;
            continue;
        }
        if (tile_slot[t] >= 0) slot_ref[tile_slot[t]]--;
        tile_slot[t] = got[i];
        slot_ref[got[i]]++;
        slot_last[got[i]] = ++slot_clock;
        usek[t] = 1;
        use2l[t] = 0;
        phase[t] = 1;
        stats.proj_refined++;
        fl[tiles[t].order[tiles[t].cursor]] |= PS_FLAG_REBUILD;
    }
}

double Engine::tbar_norm(int slot, zd z) const
{
    const double g = slot_gam[slot] * sqrt(zabs2(zsub(z, slot_z[slot])));
    const double a = sqrt(std::max(slot_lamn[slot], 0.0)) + g;
    return a * a;
}

// The upper part of eq. (tauRecycle): the Weyl bound of the largest pencil
// eigenvalue, (sqrt(lambda_n^dagger) + gamma |z - z_dag|)^2 <= tau_max.  The
// lower part (lambda_bar_rbar >= tau_min) is tested once the projection
// vectors at z are known.  Among the admissible sites the closest (smallest
// gamma |z - z_dag|) is taken.
int Engine::find_slot2(zd z) const
{
    int best = -1;
    double bg = 0.0;
    for (int s = 0; s < NS; ++s) {
        if (!slot_valid[s] || slot_priv[s]) continue;
        const double g = slot_gam[s] * sqrt(zabs2(zsub(z, slot_z[s])));
        const double a = sqrt(std::max(slot_lamn[s], 0.0)) + g;
        if (a * a > P.tau_max) continue;
        if (best < 0 || g < bg) { best = s; bg = g; }
    }
    return best;
}

// Y = F^{-1} X (trans 0) or F^{-*} X (trans 1) with each tile's site; tiles
// that share a site form one wide product
void Engine::finv_apply(const std::vector<int>& L, int trans, const zd* X, int64_t xs, int64_t ldx, zd* Y,
                        int64_t ys, int64_t ldy)
{
    if (L.empty()) return;
    if (op.kind != PS_DENSE) {
        // (F P)^{-1} X or (F P)^{-*} X by colour-scheduled triangular solves
        std::vector<int> ts(T, 0);
        for (int t : L) {
            if (tile_slot[t] < 0) throw DeviceError("finv_apply: tile without a preconditioner site");
            ts[t] = tile_slot[t];
        }
        h2d(d_tslot.p, ts.data(), sizeof(int) * T);
        upload_list(L, d_listC);
        stats.sv_F += (int64_t)L.size() * r;
        const int pi = prof.begin(st, 1, 0.0, 16.0 * 2.0 * op.spat.nnz * L.size());
        launch_ic_solve(d_listC.p, (int)L.size(), d_tslot.p, op.spat, Slu.p, trans, X, xs, ldx, Y, ys, ldy, r, Tq.p,
                         (int64_t)n * r, st);
        prof.end(st, pi);
        return;
    }
    std::vector<int> order(L);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tile_slot[x] < tile_slot[y]; });
    std::vector<int> gs, goff, gcnt;
    for (size_t i = 0; i < order.size(); ++i) {
        const int s = tile_slot[order[i]];
        if (s < 0) throw DeviceError("finv_apply: tile without a preconditioner site");
        if (gs.empty() || gs.back() != s) { gs.push_back(s); goff.push_back((int)i); gcnt.push_back(0); }
        gcnt.back()++;
    }
    const int ng = (int)gs.size(), nt = (int)order.size();
    std::vector<int> h(3 * ng + nt);
    int maxc = 0;
    for (int g = 0; g < ng; ++g) {
        h[g] = gs[g];
        h[ng + g] = goff[g];
        h[2 * ng + g] = gcnt[g];
        maxc = std::max(maxc, gcnt[g]);
    }
    for (int i = 0; i < nt; ++i) h[3 * ng + i] = order[i];
    if (d_gmap.n < h.size()) {
        HIPCHK(hipStreamSynchronize(st));
        d_gmap.alloc(h.size() + 64);
    }
    h2d(d_gmap.p, h.data(), sizeof(int) * h.size());
    stats.sv_F += (int64_t)nt * r;
    const int64_t nn = n * n;
    // Finv is upper triangular; F^{-*} is read as its conjugate transpose (lower)
    zgemm(d_gmap.p, ng, n, (int64_t)maxc * r, n, Finv.p, n, nn, trans ? 1 : 0, X, ldx, xs, Y, ldy, ys, 1.0, 0.0, 0,
          trans ? 2 : 1, d_gmap.p + ng, r, (int64_t)nt * r);
}

void Engine::op_apply(bool herm, const std::vector<int>& L, const zd* X, int64_t xs, int64_t ldx, zd* Y, int64_t ys,
                      int64_t ldy, int w)
{
    std::vector<int> L0, L1;
    for (int t : L) (two_level && phase[t] ? L1 : L0).push_back(t);
    if (!L0.empty()) {
        upload_list(L0, d_listA);
        apply(herm, d_listA.p, (int)L0.size(), X, xs, ldx, Y, ys, ldy, w, d_z.p);
    }
    if (L1.empty()) return;
    if (w != r) throw DeviceError("op_apply: projection tiles need w = r");
    upload_list(L1, d_listB);
    const int64_t sT = (int64_t)std::max(m, n) * r;
    if (!herm) {
        // Mbar(z) X = C(z) (F^{-1} X)
        finv_apply(L1, 0, X, xs, ldx, Tp.p, sT, n);
        apply(false, d_listB.p, (int)L1.size(), Tp.p, sT, n, Y, ys, ldy, w, d_z.p);
    } else {
        // Mbar(z)^* Y = F^{-*} (C(z)^* Y)
        apply(true, d_listB.p, (int)L1.size(), X, xs, ldx, Tp.p, sT, n, w, d_z.p);
        finv_apply(L1, 1, Tp.p, sT, n, Y, ys, ldy);
    }
}

// Y += Ebar Lambda_bar^{-1} (Ebar^* W) for the tiles of L (K_Ebar^{-1} W
// after Y = F^{-1} F^{-*} W)
void Engine::twolevel_add(const std::vector<int>& L, const zd* W, int64_t ws, zd* Y, int64_t ys)
{
    if (L.empty()) return;
    upload_list(L, d_listA);
    const int nt = (int)L.size();
    BlockList Le = bl_empty(n);
    bl_add(Le, tE.p, (int64_t)n * r, n, r, nullptr, 0);
    BlockList Lw = bl_empty(n);
    bl_add(Lw, W, ws, n, r, nullptr, 0);
    gram(d_listA.p, nt, Le, Lw, r, r, tCoef.p, (int64_t)r * r, r, false, false);
    {
        dim3 g((unsigned)((r * r + 255) / 256), nt);
        hipLaunchKernelGGL(k_scale_rows, g, dim3(256), 0, st, d_listA.p, tCoef.p, (int64_t)r * r, r, r, r, tLam.p,
                           r);
    }
    gemm_ts(d_listA.p, nt, Le, r, tCoef.p, (int64_t)r * r, r, nullptr, 0, r, Y, ys, n, n, 1.0, 1.0);
}

// ---------------------------------------------------------------------------
// Projection store of a site.  With Ebar_V = F^{-1} Vbar (pE), W1 = C Ebar_V,
// Mbar(z) Vbar = W1 - z S Ebar_V, so R_A = R([W1, S Ebar_V]) gives the
// Rayleigh-Ritz-SVD of Mbar(z) on span Vbar for any z as in recySing, and
// Tbar(z) Vbar g = [W3 W4 W5 W6] (g; -z g; -conj(z) g; |z|^2 g) with
// W3 = F^{-*} C^* W1, W4 = F^{-*} C^* S Ebar_V, W5 = F^{-*} S^* W1 and
// W6 = F^{-*} S^* S Ebar_V, so the residual norm of a Ritz pair is
// ||R_res u|| with R_res = R([W3 W4 W5 W6 Vbar]) (nres = 5).
void Engine::proj_refresh(const std::vector<int>& slots)
{
    if (slots.empty()) return;
    const int64_t nn = n * n, snk = (int64_t)n * KB, smk = (int64_t)m * KB;
    for (size_t c0 = 0; c0 < slots.size(); c0 += 32) {
        std::vector<int> Ls(slots.begin() + c0, slots.begin() + std::min(slots.size(), c0 + 32));
        const int ns = (int)Ls.size();
        upload_list(Ls, d_listB);
        const int* dl = d_listB.p;
        // Y = F^{-1} X (trans 0) or F^{-*} X (trans 1) for n x KB slot blocks
        auto fsol = [&](int trans, const zd* X, int64_t xs, int64_t ldx, zd* Y) {
            if (op.kind == PS_DENSE)
                zgemm(dl, ns, n, KB, n, Finv.p, n, nn, trans, X, ldx, xs, Y, n, snk, 1.0, 0.0, 0, trans ? 2 : 1);
            else
                launch_ic_solve(dl, ns, nullptr, op.spat, Slu.p, trans, X, xs, ldx, Y, snk, n, KB, pS.p, snk, st);
        };
        // pE = F^{-1} Vbar
        fsol(0, pV.p, snk, n, pE.p);
        // pT = [pE; 0] (m rows), W1 = C pE
        if (m > n) launch_zero_tiles(dl, ns, pT.p, smk, smk, st);
        launch_copy_cols(dl, ns, pE.p, snk, n, pT.p, smk, m, n, KB, st);
        apply(false, dl, ns, pE.p, snk, n, pW1.p, smk, m, KB, nullptr);
        // W3 = F^{-*} (C^* W1), W4 = F^{-*} (C^* [pE; 0]) (via pW5 as scratch)
        apply(true, dl, ns, pW1.p, smk, m, pW5.p, snk, n, KB, nullptr);
        fsol(1, pW5.p, snk, n, pW3.p);
        apply(true, dl, ns, pT.p, smk, m, pW5.p, snk, n, KB, nullptr);
        fsol(1, pW5.p, snk, n, pW4.p);
        // W5 = F^{-*} W1[0:n], W6 = F^{-*} pE
        fsol(1, pW1.p, smk, m, pW5.p);
        fsol(1, pE.p, snk, n, pW6.p);
        BlockList La = bl_empty(m);
        bl_add(La, pW1.p, smk, m, 0, d_pk.p, 1);
        bl_add(La, pE.p, snk, n, 0, d_pk.p, 1, n);
        r_factor(dl, ns, La, 2 * KB, d_pk.p, 2, 0, pRA.p, (int64_t)4 * KB * KB, 2 * KB, nullptr, pgdd.p);
        BlockList Lr = bl_empty(n);
        bl_add(Lr, pW3.p, snk, n, 0, d_pk.p, 1);
        bl_add(Lr, pW4.p, snk, n, 0, d_pk.p, 1);
        bl_add(Lr, pW5.p, snk, n, 0, d_pk.p, 1);
        bl_add(Lr, pW6.p, snk, n, 0, d_pk.p, 1);
        bl_add(Lr, pV.p, snk, n, 0, d_pk.p, 1);
        r_factor(dl, ns, Lr, 5 * KB, d_pk.p, 5, 0, pRres.p, (int64_t)25 * KB * KB, 5 * KB, nullptr, pgdd.p);
    }
}

// updateRecy (Alg. 2) on site projection stores.  slots[i] receives the block
// Xbar = S[:, 0:r] of tiles[i] (orthonormal); the omega test of eq.
// (omegaCond) uses its rbrev[i] leading columns (Frobenius norm).  The store
// keeps the newest block first: V = [V^1 V^2 ...] with V^1 from the latest
// refinement, so dropping trailing blocks drops the oldest subspaces.  With
// C1 = V^* X, rho_j^2 = ||X_{:r}||_F^2 - ||C1 of the blocks kept||^2.
void Engine::proj_update(const std::vector<int>& slots, const std::vector<int>& tiles_in, const std::vector<int>& rbrev)
{
    if (slots.empty()) return;
    const int q = (int)slots.size();
    const int64_t snk = (int64_t)n * KB, smk = (int64_t)m * KB, sS = (int64_t)n * 3 * r;
    const int pmax = std::max(1, KB / r);
    // per tile: its slot (for the imap of the store blocks)
    {
        std::vector<int> ts(T, NS);
        for (int i = 0; i < q; ++i) ts[tiles_in[i]] = slots[i];
        h2d(d_tslot.p, ts.data(), sizeof(int) * T);
    }
    upload_list(tiles_in, d_listA);
    // C1 = Vbar^* X (KB x r per tile)
    BlockList Lv = bl_empty(n);
    bl_add(Lv, pV.p, snk, n, 0, d_pk.p, 1);
    bl_map(Lv, d_tslot.p);
    BlockList Lx = bl_empty(n);
    bl_add(Lx, S.p, sS, n, r, nullptr, 0);
    gram(d_listA.p, q, Lv, Lx, KB, r, pG.p, (int64_t)KB * r, KB, false, false);
    std::vector<zd> c1((size_t)q * KB * r);
    for (int i = 0; i < q; ++i)
        HIPCHK(hipMemcpyAsync(c1.data() + (size_t)i * KB * r, pG.p + (size_t)tiles_in[i] * KB * r,
                              sizeof(zd) * KB * r, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> Lu, keep_blocks(NS + 1, 0), srct(NS + 1, 0);
    for (int i = 0; i < q; ++i) {
        const int s = slots[i], t = tiles_in[i];
        const int p = pk[s] / r;
        const int rb = std::max(1, std::min(r, rbrev[i]));
        const zd* C = c1.data() + (size_t)i * KB * r;
        auto blk2 = [&](int b) {
            double a = 0;
            for (int c = 0; c < rb; ++c)
                for (int j = b * r; j < (b + 1) * r; ++j) a += zabs2(C[j + (size_t)c * KB]);
            return a;
        };
        double tot = 0;
        for (int b = 0; b < p; ++b) tot += blk2(b);
        const double rho0 = sqrt(std::max(0.0, (double)rb - tot));
        if (p > 0 && rho0 <= 1e-14 * sqrt((double)rb)) continue;   // X already in the recycled subspace
        int l = 0;
        if (p > 0) {
            // drop the j oldest blocks while rho_j <= omega rho_0
            int j;
            for (j = 1; j <= p; ++j) {
                double kept = 0;
                for (int b = 0; b < p - j; ++b) kept += blk2(b);
                const double rhoj = sqrt(std::max(0.0, (double)rb - kept));
                if (rhoj > P.omega * rho0) break;
            }
            if (j > p) j = p;
            l = j - 1;
            if (p - l + 1 > pmax) l = p - pmax + 1;
            if (l < 0) l = 0;
        }
        keep_blocks[s] = p - l;
        srct[s] = t;
        Lu.push_back(s);
        (void)t;
    }
    if (Lu.empty()) return;
    const int nu = (int)Lu.size();
    upload_list(Lu, d_listB);
    h2d(d_tslot.p, srct.data(), sizeof(int) * (NS + 1));   // per slot: source tile (reused as a map)
    // pT = [X | V blocks kept] (newest first), column by column (pT has ld m)
    for (int c = 0; c < r; ++c)
        launch_gather(d_listB.p, nu, d_tslot.p, S.p + (size_t)c * n, sS, pT.p + (size_t)c * m, smk, n, st);
    launch_copy_cols(d_listB.p, nu, pV.p, snk, n, pT.p + (size_t)m * r, smk, m, n, KB - r, st);
    for (int s : Lu) pk[s] = (keep_blocks[s] + 1) * r;
    upload_pk();
    // CholQR twice with an explicit triangular inverse, so that the leading
    // columns keep their span (the new block stays first); a block that adds
    // no direction (zero pivot) drops the old blocks of its store
    DBuf<int>& nz = d_nzp;      // per-slot zero-pivot counts
    for (int pass = 0; pass < 2; ++pass) {
        zd* src = pass == 0 ? pT.p : pV.p;
        const int64_t ssrc = pass == 0 ? smk : snk, ldsrc = pass == 0 ? m : n;
        zd* dst = pass == 0 ? pV.p : pT.p;
        const int64_t sdst = pass == 0 ? snk : smk, lddst = pass == 0 ? n : m;
        BlockList Lb = bl_empty(n);
        bl_add(Lb, src, ssrc, ldsrc, 0, d_pk.p, 1);
        r_factor(d_listB.p, nu, Lb, KB, d_pk.p, 1, 0, pRres.p, (int64_t)25 * KB * KB, KB, nz.p, pgdd.p);
        std::vector<int> hz(NS + 1, 0);
        HIPCHK(hipMemcpyAsync(hz.data(), nz.p, sizeof(int) * (NS + 1), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool redo = false;
        for (int s : Lu)
            if (hz[s] > 0 && pk[s] > r) { pk[s] = r; redo = true; }
        if (redo) {
            upload_pk();
            r_factor(d_listB.p, nu, Lb, KB, d_pk.p, 1, 0, pRres.p, (int64_t)25 * KB * KB, KB, nullptr, pgdd.p);
        }
        hipLaunchKernelGGL(k_trinv, dim3(nu), dim3(64), 0, st, d_listB.p, d_pk.p, pRres.p, (int64_t)25 * KB * KB, KB,
                           pRA.p, (int64_t)4 * KB * KB, KB, KB);
        BlockList Ls = bl_empty(n);
        bl_add(Ls, src, ssrc, ldsrc, 0, d_pk.p, 1);
        gemm_ts(d_listB.p, nu, Ls, KB, pRA.p, (int64_t)4 * KB * KB, KB, nullptr, 0, KB, dst, sdst, lddst, n, 1.0, 0.0);
    }
    // the second pass wrote pT: copy back into Vbar
    launch_copy_cols(d_listB.p, nu, pT.p, smk, m, pV.p, snk, n, n, KB, st);
    proj_refresh(Lu);
}

// recyProj (Alg. 4) for the tiles of L, each at its site tile_slot[t]:
// Rayleigh-Ritz-SVD of Mbar(z) on span Vbar from the cached R factors
// (k_ritz, nres = 5), Ritz vectors Xcheck = Vbar G, projection vectors
// Echeck = F^{-1} Vbar G = pE G and the test of eq. (tolTz) on all r
// residuals with ||Tbar(z)|| estimated by the Weyl bound.  Accepted tiles
// get Ebar = Echeck and Lambda_bar = Theta^2; the others start their
// projection LOBPCG from Xcheck (written to S[:, 0:r]) unless the store is
// empty.
void Engine::recy_proj(const std::vector<int>& L, std::vector<char>& acc)
{
    acc.assign(L.size(), 0);
    if (L.empty()) return;
    std::vector<int> js(T, NS);
    std::vector<zd> jz(T, zmake(0.0, 0.0));
    std::vector<double> jn(T, 1.0);
    bool any = false;
    for (int t : L) {
        const int s = tile_slot[t];
        if (s < 0 || pk[s] <= 0) continue;
        js[t] = s;
        jz[t] = h_zt[t];
        jn[t] = tbar_norm(s, h_zt[t]);
        any = true;
    }
    if (!any) return;
    h2d(pj_slot.p, js.data(), sizeof(int) * T);
    h2d(pj_z.p, jz.data(), sizeof(zd) * T);
    h2d(pj_nrm.p, jn.data(), sizeof(double) * T);
    RitzArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.njobs = T;
    ra.job_tile = pj_slot.p;
    ra.kdim = d_pk.p;
    ra.z = pj_z.p;
    ra.nrm = pj_nrm.p;
    ra.RA = pRA.p;
    ra.strideRA = (int64_t)4 * KB * KB;
    ra.ldRA = 2 * KB;
    ra.Rres = pRres.p;
    ra.strideRres = (int64_t)25 * KB * KB;
    ra.ldRres = 5 * KB;
    ra.nres = 5;
    ra.nv = r;
    ra.ng = r;
    ra.max_sweeps = 40;
    ra.mode = 1;
    ra.eta = P.eta_proj;
    ra.floor_c = 0.0;
    ra.eta_abs = 0.0;
    ra.normC = op.normC;
    ra.xi = pj_xi.p;
    ra.res = pj_res.p;
    ra.ldxi = r;
    ra.Gout = pG.p;
    ra.strideG = (int64_t)KB * r;
    ra.ldG = KB;
    ra.accept = pj_acc.p;
    int pi = prof.begin(st, 2, 250.0 * KB * KB * KB * (double)L.size(), 16.0 * 50.0 * KB * KB * (double)L.size());
    launch_ritz(ra, KB, st);
    prof.end(st, pi);
    std::vector<uint8_t> ha(T);
    std::vector<double> hx((size_t)T * r);
    HIPCHK(hipMemcpyAsync(ha.data(), pj_acc.p, T, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hx.data(), pj_xi.p, sizeof(double) * T * r, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> La, Lr;
    for (size_t i = 0; i < L.size(); ++i) {
        const int t = L[i];
        if (js[t] == NS) continue;
        if (ha[t]) {
            acc[i] = 1;
            La.push_back(t);
            for (int j = 0; j < r; ++j) tlam_h[(size_t)t * r + j] = hx[(size_t)t * r + j] * hx[(size_t)t * r + j];
        } else {
            Lr.push_back(t);
        }
    }
    h2d(d_tslot.p, js.data(), sizeof(int) * T);
    BlockList Le = bl_empty(n);
    bl_add(Le, pE.p, (int64_t)n * KB, n, 0, d_pk.p, 1);
    bl_map(Le, d_tslot.p);
    BlockList Lv = bl_empty(n);
    bl_add(Lv, pV.p, (int64_t)n * KB, n, 0, d_pk.p, 1);
    bl_map(Lv, d_tslot.p);
    if (!La.empty()) {
        upload_list(La, d_listA);
        gemm_ts(d_listA.p, (int)La.size(), Le, KB, pG.p, (int64_t)KB * r, KB, nullptr, 0, r, tE.p, (int64_t)n * r, n,
                n, 1.0, 0.0);
        h2d(tLam.p, tlam_h.data(), sizeof(double) * T * r);
        stats.proj_accepted += (int64_t)La.size();
    }
    if (!Lr.empty()) {
        upload_list(Lr, d_listB);
        gemm_ts(d_listB.p, (int)Lr.size(), Lv, KB, pG.p, (int64_t)KB * r, KB, nullptr, 0, r, S.p,
                (int64_t)n * 3 * r, n, n, 1.0, 0.0);
    }
}
