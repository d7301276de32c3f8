// updateRecy (Alg. 2) for the singular store and the grid-front scheduler.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

void Engine::upload_k()
{
    h_small.alloc(T + 8);
    int* hp = (int*)h_small.p;
    for (int t = 0; t < T; ++t) hp[t] = tiles[t].k;
    h2d(d_k.p, hp, sizeof(int) * T);
}

// updateRecy with r_breve = 1 (Alg. 2, Sec. 2.2.2) for every tile in L; the
// new singular block X (orthonormal, n x r) is S[:, 0:r] of the tile.
//  1. projection errors rho_j = ||(I - V_j V_j^*) x_1|| of x_1 = X[:, 0] onto
//     the trailing blocks V_j = [V^{j+1} .. V^p]; l = first j with
//     rho_j / rho_0 > omega, minus one (eq. (omegaCond)), capped so that at
//     most k_max / r blocks remain; rho_0 ~ 0 means X is already recycled.
//     Because V is orthonormal, rho_j^2 = rho_0^2 + ||V_{<j}^* x_1||^2, which
//     avoids cancellation.
//  2. block Gram-Schmidt of X against the kept blocks V_l: coefficients U,
//     new orthonormal block Q with X = V_l U + Q Upp (eq. (blkGS)).
//  3. the new operator blocks C Q, C^* C Q, C^* S Q (3r column-applies).
//  4. block unitary rotations restoring the QL form, applied to V and to the
//     W blocks in one product with the accumulated transform.
//  5. refresh of the cached R factors.
void Engine::update_store(const std::vector<int>& Lin)
{
    if (Lin.empty()) return;
    const int64_t sS = (int64_t)n * 3 * r, sX = (int64_t)n * r;
    const int64_t snk = (int64_t)n * K, smk = (int64_t)m * K;
    std::vector<int> L = Lin;
    upload_list(L, d_list2);
    int nt = (int)L.size();
    // Xw <- X
    launch_copy_cols(d_list2.p, nt, S.p, sS, n, Xw.p, sX, n, n, r, st);
    BlockList Lv = bl_empty(n);
    bl_add(Lv, sV.p, snk, n, 0, d_k.p, 1);
    BlockList Lx = bl_empty(n);
    bl_add(Lx, S.p, sS, n, r, nullptr, 0);
    BlockList Lxw = bl_empty(n);
    bl_add(Lxw, Xw.p, sX, n, r, nullptr, 0);
    // 1. C1 = V^* X, Xw = X - V C1, C2 = V^* Xw, Xw -= V C2
    gram(d_list2.p, nt, Lv, Lx, K, r, Csm.p, (int64_t)K * 3 * r, K, false, false);
    gemm_ts(d_list2.p, nt, Lv, K, Csm.p, (int64_t)K * 3 * r, K, nullptr, 0, r, Xw.p, sX, n, n, -1.0, 1.0);
    gram(d_list2.p, nt, Lv, Lxw, K, r, Ucoef.p, (int64_t)K * r, K, false, false);
    gemm_ts(d_list2.p, nt, Lv, K, Ucoef.p, (int64_t)K * r, K, nullptr, 0, r, Xw.p, sX, n, n, -1.0, 1.0);
    colnorm2(d_list2.p, nt, Lxw, r, nrm2.p, 3 * r);
    h_C.alloc((size_t)T * K * 2 + 8);
    zd* hc1 = h_C.p;
    zd* hc2 = h_C.p + (size_t)T * K;
    for (int t : L) {
        HIPCHK(hipMemcpyAsync(hc1 + (size_t)t * K, Csm.p + (size_t)t * K * 3 * r, sizeof(zd) * K,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hc2 + (size_t)t * K, Ucoef.p + (size_t)t * K * r, sizeof(zd) * K,
                              hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(h_nrm2.p, nrm2.p, sizeof(double) * T * 3 * r, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int pmax = std::max(1, K / r);
    std::vector<int> Lu;
    std::vector<int> lsel(T, 0), qsel(T, 0);
    for (int t : L) {
        const int p = tiles[t].k / r;
        const double rho0 = sqrt(std::max(0.0, h_nrm2[(size_t)t * 3 * r]));
        if (p > 0 && rho0 <= 1e-14) continue;  // x_1 already in the recycled subspace
        int l = 0;
        if (p > 0) {
            int j = 1;
            double acc = rho0 * rho0;
            for (j = 1; j <= p; ++j) {
                // add the coefficients of block j-1 (dropped when the trailing set starts at block j)
                for (int i = (j - 1) * r; i < j * r; ++i) {
                    zd c = zadd(hc1[(size_t)t * K + i], hc2[(size_t)t * K + i]);
                    acc += zabs2(c);
                }
                if (sqrt(acc) / rho0 > P.omega) break;
            }
            if (j > p) j = p;
            l = j - 1;
            if (p - l + 1 > pmax) l = p - pmax + 1;
            if (l < 0) l = 0;
        }
        lsel[t] = l;
        qsel[t] = p - l;
        Lu.push_back(t);
    }
    if (Lu.empty()) return;
    L = Lu;
    nt = (int)L.size();
    upload_list(L, d_list2);
    {
        h_small.alloc(2 * T + 8);
        int* hl = (int*)h_small.p;
        for (int t = 0; t < T; ++t) { hl[t] = lsel[t]; hl[T + t] = qsel[t]; }
        h2d(d_l.p, hl, sizeof(int) * T);
        h2d(d_q.p, hl + T, sizeof(int) * T);
    }
    // 2. block Gram-Schmidt against the kept blocks V_l = V[:, l r : p r]
    BlockList Lvl = bl_empty(n);
    bl_add(Lvl, sV.p, snk, n, 0, d_q.p, r, 0, d_l.p, r);
    launch_copy_cols(d_list2.p, nt, S.p, sS, n, Xw.p, sX, n, n, r, st);
    gram(d_list2.p, nt, Lvl, Lx, K, r, Ucoef.p, (int64_t)K * r, K, false, false);
    gemm_ts(d_list2.p, nt, Lvl, K, Ucoef.p, (int64_t)K * r, K, nullptr, 0, r, Xw.p, sX, n, n, -1.0, 1.0);
    orthonormalize(L, d_list2.p, Xw.p, sX, n, n, r, &Lvl, K, P.seed ^ 0xabcdefull ^ (uint64_t)stats.refined);
    gram(d_list2.p, nt, Lxw, Lx, r, r, Upp.p, (int64_t)r * r, r, false, false);
    RotArgs ro;
    memset(&ro, 0, sizeof(ro));
    ro.list = d_list2.p;
    ro.qdim = d_q.p;
    ro.r = r;
    ro.U = Ucoef.p;
    ro.strideU = (int64_t)K * r;
    ro.ldU = K;
    ro.Upp = Upp.p;
    ro.strideUpp = (int64_t)r * r;
    ro.ldUpp = r;
    ro.Qt = Qt.p;
    ro.strideQt = (int64_t)K * K;
    ro.ldQt = K;
    int pi = prof.begin(st, 5, 0.0, 0.0);
    launch_rotations(ro, nt, pmax - 1, st);
    prof.end(st, pi);
    stats.store_updates += nt;
    // 3. operator blocks of the new basis block (before rotation)
    const int64_t sT1 = (int64_t)m * 3 * r;
    const int64_t mv0 = stats.mv_M;
    launch_zero(Tn1.p, (int64_t)T * sT1, st);
    launch_copy_cols(d_list2.p, nt, Xw.p, sX, n, Tn1.p + (size_t)m * r, sT1, m, n, r, st);
    apply(false, d_list2.p, nt, Xw.p, sX, n, Tn1.p, sT1, m, r, nullptr);                 // C Q
    apply(true, d_list2.p, nt, Tn1.p, sT1, m, Tn2.p, sX, n, r, nullptr);                 // C^* C Q
    apply(true, d_list2.p, nt, Tn1.p + (size_t)m * r, sT1, m, Tn3.p, sX, n, r, nullptr); // C^* S Q
    stats.mv_update += stats.mv_M - mv0;
    // 4. new k, then [kept | new] Qt for V and each W block
    for (int t : L) tiles[t].k = (qsel[t] + 1) * r;
    upload_k();
    auto rot = [&](zd* src, int64_t srcstride, int64_t srcld, const zd* nb, int64_t nbstride, int64_t nbld,
                   int64_t rows, zd* dst) {
        BlockList A = bl_empty(rows);
        bl_add(A, src, srcstride, srcld, 0, d_q.p, r, 0, d_l.p, r);
        bl_add(A, nb, nbstride, nbld, r, nullptr, 0);
        gemm_ts(d_list2.p, nt, A, K, Qt.p, (int64_t)K * K, K, d_k.p, 1, 0, dst, srcstride, srcld, rows, 1.0, 0.0);
        launch_copy_cols(d_list2.p, nt, dst, srcstride, srcld, src, srcstride, srcld, rows, K, st);
    };
    rot(sV.p, snk, n, Xw.p, sX, n, n, uV.p);
    rot(sW1.p, smk, m, Tn1.p, sT1, m, m, uW1.p);
    rot(sW3.p, snk, n, Tn2.p, sX, n, n, uW3.p);
    rot(sW4.p, snk, n, Tn3.p, sX, n, n, uW4.p);
    // 5. cached R factors
    refresh_store(L);
}

// ---------------------------------------------------------------------------
// Grid-front scheduler.  The grid is cut into tiles; each tile is traversed
// in batch-zigzag order (Sec. 2.3: bands of height b, columns visited in
// alternating directions, a snake inside each column batch) and runs the
// sequential algorithm with its own recycled store, so that every point is
// tested against the store as updated by all refinements before it in its
// tile.  Tiles are scheduled by continuous batching: an idle tile tests its
// next b points against its store (one batched launch for all idle tiles),
// accepts the leading run of points that pass and starts LOBPCG-SVD on the
// first rejected one; every scheduler step advances all running refinements
// by one iteration, and a tile whose refinement ends updates its store and
// becomes idle again.
// Hilbert curve on a 2^k x 2^k square: position d along the curve -> cell
// (x, y), built level by level (each level places the quadrant from two
// bits of d and reflects / transposes the coordinates so far, so that the
// sub-curves join end to end)
static void hilbert_cell(int side, int64_t d, int& x, int& y)
{
    x = y = 0;
    for (int s = 1; s < side; s *= 2) {
        const int qx = (int)(1 & (d / 2));
        const int qy = (int)(1 & (d ^ qx));
        if (qy == 0) {
            if (qx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            std::swap(x, y);
        }
        x += s * qx;
        y += s * qy;
        d /= 4;
    }
}

// interleaved bits of (x, y): the Morton (Z-order) key
static uint64_t morton_key(uint32_t x, uint32_t y)
{
    uint64_t k = 0;
    for (int bit = 0; bit < 32; ++bit) {
        k |= (uint64_t)((x >> bit) & 1u) << (2 * bit);
        k |= (uint64_t)((y >> bit) & 1u) << (2 * bit + 1);
    }
    return k;
}

// Points of the rectangle [x0, x1) x [y0, y1) in the chosen traversal:
// 0 batch zigzag (bands of height b, columns visited in alternating
// directions, a vertical snake inside each band), 1 Hilbert curve (the
// curve on the enclosing power-of-two square, cells outside the rectangle
// skipped), 2 Morton order.
static void rect_order(int nx, int x0, int x1, int y0, int y1, int b, int traversal, std::vector<int64_t>& out)
{
    const int w = x1 - x0, h = y1 - y0;
    if (traversal == 1) {
        int side = 1;
        while (side < std::max(w, h)) side *= 2;
        for (int64_t d = 0; d < (int64_t)side * side; ++d) {
            int x, y;
            hilbert_cell(side, d, x, y);
            if (x < w && y < h) out.push_back((int64_t)(y0 + y) * nx + (x0 + x));
        }
        return;
    }
    if (traversal == 2) {
        std::vector<std::pair<uint64_t, int64_t>> pts;
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) pts.push_back({morton_key((uint32_t)x, (uint32_t)y), (int64_t)(y0 + y) * nx + x0 + x});
        std::sort(pts.begin(), pts.end());
        for (auto& q : pts) out.push_back(q.second);
        return;
    }
    int band = 0;
    for (int yb = y0; yb < y1; yb += b, ++band) {
        const int ye = std::min(y1, yb + b);
        const bool ltr = (band % 2 == 0);
        for (int ci = 0; ci < w; ++ci) {
            const int x = ltr ? (x0 + ci) : (x1 - 1 - ci);
            const bool up = (ci % 2 == 0);
            for (int yi = 0; yi < ye - yb; ++yi) {
                const int y = up ? (yb + yi) : (ye - 1 - yi);
                out.push_back((int64_t)y * nx + x);
            }
        }
    }
}

void tile_orders(int nx, int ny, int tx, int ty, int b, int traversal, std::vector<Tile>& tiles)
{
    tiles.clear();
    for (int jy = 0; jy < ty; ++jy) {
        int y0 = (int)((int64_t)ny * jy / ty), y1 = (int)((int64_t)ny * (jy + 1) / ty);
        for (int jx = 0; jx < tx; ++jx) {
            int x0 = (int)((int64_t)nx * jx / tx), x1 = (int)((int64_t)nx * (jx + 1) / tx);
            Tile t;
            std::vector<int64_t> o;
            rect_order(nx, x0, x1, y0, y1, b, traversal, o);
            for (int64_t p : o) t.order.push_back((int)p);
            if (!t.order.empty()) tiles.push_back(std::move(t));
        }
    }
}

ps_status Engine::eval(const ps_gridh* g, const double* eps, int n_eps, double* sigma, uint8_t* member,
                       uint8_t* flags, ps_stats* st_out)
{
    auto t_start = std::chrono::steady_clock::now();
    memset(&stats, 0, sizeof(stats));
    prof.on = P.profile != 0;
    prof.level = P.profile;
    prof.used = 0;
    const int nx = g->nx, ny = g->ny;
    const int64_t npts = (int64_t)nx * ny;
    zs.resize(npts);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double x = (nx > 1) ? g->re_lo + (g->re_hi - g->re_lo) * i / (nx - 1) : g->re_lo;
            double y = (ny > 1) ? g->im_lo + (g->im_hi - g->im_lo) * j / (ny - 1) : g->im_lo;
            zs[(size_t)j * nx + i] = zmake(x, y);
        }
    const int b = std::max(1, P.batch);
    B = b;
    // Default partition: tiles of about tile_points points each, as many as
    // the per-tile device state allows within tile_mem_gb (stores, LOBPCG
    // blocks and work arrays, ~16 (8 n K + 14 n r) bytes per tile).  Every
    // tile is one point in flight; many tiles keep the batched products wide.
    int tx = P.tiles_x, ty = P.tiles_y;
    if (tx <= 0 || ty <= 0) {
        const double per_tile = 16.0 * (8.0 * (double)std::max(m, n) * K + 14.0 * (double)std::max(m, n) * r);
        const double cap_t = std::max(1.0, (double)P.tile_mem_gb * 1e9 / per_tile);
        double want = std::max(1.0, std::min((double)npts / std::max(1, P.tile_points), cap_t));
        if (tx <= 0 && ty <= 0) {
            tx = (int)std::max(1L, std::lround(sqrt(want * nx / (double)ny)));
            ty = (int)std::max(1L, std::lround(want / tx));
        } else if (tx <= 0) {
            tx = (int)std::max(1L, std::lround(want / ty));
        } else {
            ty = (int)std::max(1L, std::lround(want / tx));
        }
    }
    ty = std::min(ty, ny);
    tx = std::min(tx, nx);
    tile_orders(nx, ny, tx, ty, b, P.traversal, tiles);
    size_for((int)tiles.size());
    for (auto& t : tiles) { t.cursor = 0; t.k = 0; }
    reset_slots();
    upload_k();
    std::vector<uint8_t> fl(npts, 0);
    std::vector<double> sig(npts, 0.0);
    const double nC = op.normC;
    bool any_uncert = false;
    const int64_t sS = (int64_t)n * 3 * r;
    std::vector<double> h_xi_keep;
    double t_ritz = 0, t_lob = 0, t_upd = 0;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b2) {
        return std::chrono::duration<double, std::milli>(b2 - a).count();
    };
    // tile states: 0 idle (next point needs its Ritz test), 1 in LOBPCG, 2 done
    std::vector<int> state(T, 0);
    uint64_t step_seed = P.seed ^ 0x9e3779b97f4a7c15ull;
    int64_t loops = 0;
    auto t_last_print = std::chrono::steady_clock::now();
    const double EPSM_E = 2.220446049250313e-16;
    const double tau_c = P.tol_abs * nC;          // certification half-width
    bool redo_pass = false;                       // Lipschitz re-refinement: no store updates
    pgam.assign(npts, zmake(0.0, 0.0));
    pgok.assign(npts, 0);
    std::vector<uint8_t> pdone(npts, 0);
    // Upper bound of sigma_min at grid point pt from its finished neighbours q:
    // for the unit vector x behind sigma(q), ||C(z) x||^2 = sigma(q)^2 -
    // 2 Re(conj(z - z_q) gamma_q) + |z - z_q|^2 ||S x||^2 with gamma_q =
    // (S x)^* C(z_q) x and ||S x|| <= 1; neighbours without gamma give the
    // 1-Lipschitz bound sigma(q) + |z - z_q|.
    auto nb_bound = [&](int64_t pt) -> double {
        const int i = (int)(pt % nx), j = (int)(pt / nx);
        double b = INFINITY;
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                if (!di && !dj) continue;
                const int ii = i + di, jj = j + dj;
                if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
                const int64_t q = (int64_t)jj * nx + ii;
                if (!pdone[q]) continue;
                const zd d = zsub(zs[pt], zs[q]);
                double v;
                if (pgok[q]) {
                    v = sig[q] * sig[q] - 2.0 * (d.x * pgam[q].x + d.y * pgam[q].y) + zabs2(d);
                    v = sqrt(std::max(v, 0.0));
                } else {
                    v = sig[q] + sqrt(zabs2(d));
                }
                b = std::min(b, v);
            }
        return b;
    };
    std::vector<int> pending;                     // tiles waiting for an inertia test
    std::vector<char> cluster(T, 0);              // the tile's last refinement ended by the inertia test
    std::vector<char> cert_pend(T, 0), cert_ok(T, 0);
    std::vector<double> cert_mu(T, 0.0), cert_xi(T, 0.0);
    std::vector<int64_t> cert_since(T, 0);
    // a refinement (re)starts on tile t: reset the LOBPCG bookkeeping
    auto begin_refinement = [&](int t) {
        state[t] = 1;
        cert_pend[t] = 0;
        cert_ok[t] = 0;
        esc_at[t] = P.esc_iters;
        site_exact[t] = 0;
        stag[t] = 0;
        cert_next[t] = 0;
        cert_fail[t] = 0;
        lob_prev[t] = INFINITY;
    };
    auto run_tiles = [&]() {
    pending.clear();
    std::fill(cert_pend.begin(), cert_pend.end(), 0);
    std::fill(cert_ok.begin(), cert_ok.end(), 0);
    std::fill(cluster.begin(), cluster.end(), 0);
    for (int t = 0; t < T; ++t) state[t] = tiles[t].done() ? 2 : 0;
    std::fill(esc_at.begin(), esc_at.end(), P.esc_iters);
    std::fill(site_exact.begin(), site_exact.end(), 0);
    while (true) {
        ++loops;
        // ---- A. idle tiles: Ritz test on their next window of points
        std::vector<int> idle;
        for (int t = 0; t < T; ++t) if (state[t] == 0) idle.push_back(t);
        std::vector<int> R, Rsrc;   // tiles that start a refinement, job of their Ritz vectors (-1: none)
        auto t0 = now();
        if (!idle.empty()) {
            stats.rounds++;
            if (P.recycle && !redo_pass) {
                std::vector<int> jt, jp;
                for (int t : idle) {
                    if (tiles[t].k == 0) continue;
                    size_t e = std::min(tiles[t].order.size(), tiles[t].cursor + (size_t)B);
                    for (size_t c = tiles[t].cursor; c < e; ++c) { jt.push_back(t); jp.push_back(tiles[t].order[c]); }
                }
                const int nj = (int)jt.size();
                if (nj > 0) {
                    h_small.alloc((size_t)nj * 2 + 8);
                    h_z.alloc((size_t)nj + T + 8);
                    int* hjt = (int*)h_small.p;
                    double* hn = (double*)(h_small.p + nj);
                    for (int j = 0; j < nj; ++j) {
                        hjt[j] = jt[j];
                        h_z[j] = zs[jp[j]];
                        hn[j] = nC + sqrt(zabs2(zs[jp[j]]));
                    }
                    h2d(j_tile.p, hjt, sizeof(int) * nj);
                    h2d(j_z.p, h_z.p, sizeof(zd) * nj);
                    h2d(j_nrm.p, hn, sizeof(double) * nj);
                    RitzArgs ra;
                    memset(&ra, 0, sizeof(ra));
                    ra.njobs = nj;
                    ra.job_tile = j_tile.p;
                    ra.kdim = d_k.p;
                    ra.z = j_z.p;
                    ra.nrm = j_nrm.p;
                    ra.RA = sRA.p;
                    ra.strideRA = (int64_t)4 * K * K;
                    ra.ldRA = 2 * K;
                    ra.Rres = sRres.p;
                    ra.strideRres = (int64_t)16 * K * K;
                    ra.ldRres = 4 * K;
                    ra.nres = 4;
                    ra.nv = 1;
                    ra.ng = r;
                    ra.max_sweeps = 40;
                    ra.mode = 0;
                    ra.eta = P.eta;
                    ra.floor_c = std::max(16.0, 4.0 * sqrt((double)n));
                    ra.floor_tol = P.tol_abs * nC;
                    ra.eta_abs = P.eta_abs;
                    ra.normC = nC;
                    ra.xi = j_xi.p;
                    ra.res = j_res.p;
                    ra.ldxi = 1;
                    ra.Gout = j_G.p;
                    ra.strideG = (int64_t)K * r;
                    ra.ldG = K;
                    ra.accept = j_acc.p;
                    stats.ritz_jobs += nj;
                    int pi = prof.begin(st, 2, 250.0 * K * K * K * (double)nj, 16.0 * 20.0 * K * K * (double)nj);
                    launch_ritz(ra, K, st);
                    prof.end(st, pi);
                    HIPCHK(hipGetLastError());
                    launch_job_gamma(nj, j_tile.p, d_k.p, j_G.p, (int64_t)K * r, K, sH.p, (int64_t)K * K, K, j_z.p,
                                     j_gam.p, st);
                    HIPCHK(hipMemcpyAsync(h_acc.p, j_acc.p, nj, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipMemcpyAsync(h_xi.p, j_xi.p, sizeof(double) * nj, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipMemcpyAsync(h_gamj.p, j_gam.p, sizeof(zd) * nj, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                }
                h_xi_keep.assign(h_xi.p, h_xi.p + nj);
                int j = 0;
                for (int t : idle) {
                    if (tiles[t].k == 0) { R.push_back(t); Rsrc.push_back(-1); continue; }
                    size_t e = std::min(tiles[t].order.size(), tiles[t].cursor + (size_t)B);
                    size_t w = e - tiles[t].cursor;
                    bool rejected = false;
                    for (size_t c = 0; c < w; ++c, ++j) {
                        if (rejected) continue;
                        const int pt = tiles[t].order[tiles[t].cursor];
                        const bool guard = h_acc[j] && h_xi[j] > nb_bound(pt) * (1.0 + 1e-9) + 1e-12 * nC;
                        if (h_acc[j] && !guard) {
                            sig[pt] = h_xi[j];
                            pgam[pt] = h_gamj[j];
                            pgok[pt] = 1;
                            pdone[pt] = 1;
                            fl[pt] |= PS_FLAG_ACCEPTED;
                            stats.accepted++;
                            tiles[t].cursor++;
                        } else {
                            // failed eq. (tolC), or passed it with a value above
                            // what a finished neighbour's vector attains here (a
                            // Ritz value of a larger singular value: start from
                            // a random block instead of the recycled vectors)
                            rejected = true;
                            R.push_back(t);
                            Rsrc.push_back(guard ? -1 : j);
                            if (guard) stats.guard_rejects++;
                        }
                    }
                    if (!rejected && tiles[t].done()) state[t] = 2;
                }
                // tiles whose last refinement was ended by the inertia test are
                // in a cluster regime, where the recycled Ritz value is often
                // already within tau although its residual fails eq. (tolC):
                // test it directly before starting LOBPCG
                if (use_prec && tau_c > 0.0 && P.esc_iters > 0 && P.cert_recycled) {
                    std::vector<int> ci;
                    for (size_t i = 0; i < R.size(); ++i) {
                        const int t = R[i], jb = Rsrc[i];
                        if (jb < 0 || !cluster[t]) continue;
                        const zd z = zs[tiles[t].order[tiles[t].cursor]];
                        const double xi = h_xi_keep[jb];
                        const double nz = nC + sqrt(zabs2(z));
                        const double slack = 8.0 * (double)n * EPSM_E * nz * nz;
                        if (xi > 64.0 * tau_c && 2.0 * xi * tau_c - tau_c * tau_c > 4.0 * slack) ci.push_back((int)i);
                    }
                    if (!ci.empty()) {
                        std::vector<zd> cs;
                        std::vector<double> cm;
                        for (int i : ci) {
                            const int t = R[i];
                            const zd z = zs[tiles[t].order[tiles[t].cursor]];
                            const double xi = h_xi_keep[Rsrc[i]];
                            const double nz = nC + sqrt(zabs2(z));
                            cs.push_back(z);
                            cm.push_back((xi - tau_c) * (xi - tau_c) + 8.0 * (double)n * EPSM_E * nz * nz);
                        }
                        // the inertia tests waiting for running refinements join this batch
                        std::vector<int> pj;
                        for (int t : pending)
                            if (cert_pend[t] && state[t] == 1) {
                                pj.push_back(t);
                                cs.push_back(h_zt[t]);
                                cm.push_back(cert_mu[t]);
                            }
                        pending.clear();
                        auto tc0 = now();
                        std::vector<char> pd;
                        build_precond(cs, &cm, &pd, true, true);
                        stats.cert_tests += (int64_t)cs.size();
                        stats.t_precond_ms += ms(tc0, now());
                        for (size_t q = 0; q < pj.size(); ++q) {
                            const int t = pj[q];
                            cert_pend[t] = 0;
                            if (pd[ci.size() + q]) cert_ok[t] = 1;
                            else { cert_fail[t]++; cert_next[t] = lob_it[t] + 10; }
                        }
                        std::vector<char> drop(R.size(), 0);
                        for (size_t q = 0; q < ci.size(); ++q) {
                            // a failed test ends the cluster regime of the tile
                            // until one of its refinements is certified again
                            if (!pd[q]) { cluster[R[ci[q]]] = 0; continue; }
                            const int i = ci[q], t = R[i], jb = Rsrc[i];
                            const int pt = tiles[t].order[tiles[t].cursor];
                            sig[pt] = h_xi_keep[jb];
                            pgam[pt] = h_gamj[jb];
                            pgok[pt] = 1;
                            pdone[pt] = 1;
                            fl[pt] |= PS_FLAG_ACCEPTED | PS_FLAG_CERTIFIED;
                            stats.accepted++;
                            stats.certified++;
                            tiles[t].cursor++;
                            drop[i] = 1;
                            state[t] = tiles[t].done() ? 2 : 0;
                        }
                        std::vector<int> R2, S2;
                        for (size_t i = 0; i < R.size(); ++i)
                            if (!drop[i]) { R2.push_back(R[i]); S2.push_back(Rsrc[i]); }
                        R.swap(R2);
                        Rsrc.swap(S2);
                    }
                }
            } else {
                for (int t : idle) { R.push_back(t); Rsrc.push_back(-1); }
            }
        }
        auto t1 = now();
        t_ritz += ms(t0, t1);
        // ---- B. start LOBPCG on the newly rejected points
        if (!R.empty()) {
            std::vector<int> Rr, Rv;
            h_small.alloc(T + 8);
            int* hsrc = (int*)h_small.p;
            for (size_t i = 0; i < R.size(); ++i) {
                if (Rsrc[i] < 0) Rr.push_back(R[i]);
                else { Rv.push_back(R[i]); hsrc[R[i]] = Rsrc[i]; }
            }
            if (!Rv.empty()) {
                h2d(d_jobsrc.p, hsrc, sizeof(int) * T);
                upload_list(Rv, d_list);
                launch_gather(d_list.p, (int)Rv.size(), d_jobsrc.p, j_G.p, (int64_t)K * r, X0c.p, (int64_t)K * r,
                              (int64_t)K * r, st);
                BlockList Lv = bl_empty(n);
                bl_add(Lv, sV.p, (int64_t)n * K, n, 0, d_k.p, 1);
                gemm_ts(d_list.p, (int)Rv.size(), Lv, K, X0c.p, (int64_t)K * r, K, nullptr, 0, r, S.p, sS, n, n,
                        1.0, 0.0);
            }
            if (!Rr.empty()) {
                upload_list(Rr, d_list);
                step_seed = step_seed * 6364136223846793005ull + 1442695040888963407ull;
                launch_randfill(d_list.p, (int)Rr.size(), S.p, sS, n, n, r, nullptr, step_seed, st);
            }
            // base preconditioner.  Near-singular points (recycled Ritz value
            // below rho_small ||M(z)||) have a well separated smallest
            // singular value and run with K = I.  Every other refinement takes
            // the site that satisfies the rebuild rule of eq. (tauRecycle) at z
            // (base part only: without the coarse two-level correction nothing
            // lifts the small end of the pencil spectrum, bounded below by
            // (1 - gamma |z - z_dag|)^2, so the rule bounds the condition
            // number ((1 + g)/(1 - g))^2 <= tau_max); when no site does, a new
            // one is built at z.  Sites are shared by all tiles.
            if (use_prec) {
                std::vector<int> pend;
                std::vector<double> est(T, 0.0);
                for (size_t i = 0; i < R.size(); ++i) {
                    const int t = R[i];
                    zd z = zs[tiles[t].order[tiles[t].cursor]];
                    usek[t] = 1;
                    tile_slot[t] = -1;
                    if (Rsrc[i] >= 0) est[t] = h_xi_keep[Rsrc[i]];
                    if (Rsrc[i] >= 0 && h_xi_keep[Rsrc[i]] <= P.rho_small * (nC + sqrt(zabs2(z)))) {
                        usek[t] = 0;
                        continue;
                    }
                    pend.push_back(t);
                }
                auto tp0 = now();
                while (!pend.empty()) {
                    std::vector<int> rest;
                    for (int t : pend) {
                        const zd zt = zs[tiles[t].order[tiles[t].cursor]];
                        int s = two_level ? find_slot2(zt) : find_slot(zt);
                        if (s >= 0) {
                            tile_slot[t] = s;
                            slot_ref[s]++;
                            slot_last[s] = ++slot_clock;
                        } else {
                            rest.push_back(t);
                        }
                    }
                    if (rest.empty()) break;
                    // new sites: the first waiting point, and every later one
                    // not within a quarter of a chosen site's recycled Ritz
                    // value (an upper bound of sigma_min there, so such a point
                    // is likely served by that site; find_slot decides)
                    std::vector<zd> sites;
                    std::vector<double> sest;
                    for (int t : rest) {
                        if ((int)sites.size() >= NBLD) break;
                        zd z = zs[tiles[t].order[tiles[t].cursor]];
                        bool near = false;
                        for (size_t q = 0; q < sites.size() && !near; ++q)
                            near = sest[q] > 0.0 && sqrt(zabs2(zsub(z, sites[q]))) <= 0.25 * sest[q];
                        if (near) continue;
                        sites.push_back(z);
                        sest.push_back(est[t]);
                        fl[tiles[t].order[tiles[t].cursor]] |= PS_FLAG_REBUILD;
                    }
                    std::vector<int> got = two_level ? build_regularized(sites) : build_precond(sites);
                    bool failed = sites.empty();
                    for (int s : got) failed |= (s < 0);
                    if (failed) {
                        // pool exhausted (every slot referenced): nearest site
                        // regardless of the rule, else K = I
                        for (int t : rest) {
                            zd z = zs[tiles[t].order[tiles[t].cursor]];
                            int best = -1;
                            for (int s = 0; s < NS; ++s)
                                if (slot_valid[s] && (best < 0 || zabs2(zsub(z, slot_z[s])) < zabs2(zsub(z, slot_z[best]))))
                                    best = s;
                            if (best >= 0) { tile_slot[t] = best; slot_ref[best]++; }
                            else usek[t] = 0;
                        }
                        break;
                    }
                    pend.swap(rest);
                }
                stats.t_precond_ms += ms(tp0, now());
            }
            h_z.alloc((size_t)T + 8);
            for (int t : R) h_zt[t] = zs[tiles[t].order[tiles[t].cursor]];
            for (int t = 0; t < T; ++t) h_z[t] = h_zt[t];
            h2d(d_z.p, h_z.p, sizeof(zd) * T);
            // Alg. 5 with the two-level preconditioner: recyProj at the
            // tile's site gives Ebar and Lambda_bar when eq. (tolTz) holds;
            // otherwise the projection LOBPCG on Mbar(z) runs first (phase
            // 1), and the singular start block waits in tX0
            if (two_level) {
                std::vector<int> Lp;
                for (int t : R) {
                    phase[t] = 0;
                    use2l[t] = 0;
                    if (usek[t] && tile_slot[t] >= 0) Lp.push_back(t);
                }
                if (!Lp.empty()) {
                    auto tq0 = now();
                    upload_list(Lp, d_listI);
                    launch_copy_cols(d_listI.p, (int)Lp.size(), S.p, sS, n, tX0.p, (int64_t)n * r, n, n, r, st);
                    std::vector<char> acc;
                    recy_proj(Lp, acc);
                    std::vector<int> rebuild;
                    for (size_t i = 0; i < Lp.size(); ++i) {
                        const int t = Lp[i];
                        if (acc[i]) {
                            // lower part of eq. (tauRecycle)
                            if (tlam_h[(size_t)t * r + r - 1] < P.tau_min && !site_at(t)) rebuild.push_back(t);
                            else use2l[t] = 1;
                        } else {
                            phase[t] = 1;
                            stats.proj_refined++;
                        }
                    }
                    rebuild_here(rebuild, fl);
                    stats.t_precond_ms += ms(tq0, now());
                }
            }
            step_seed = step_seed * 6364136223846793005ull + 1442695040888963407ull;
            lob_start(R, step_seed);
            for (int t : R) begin_refinement(t);
        }
        // ---- C. one LOBPCG iteration for every running tile
        std::vector<int> run;
        for (int t = 0; t < T; ++t) if (state[t] == 1) run.push_back(t);
        if (run.empty()) {
            bool all = true;
            for (int t = 0; t < T; ++t) all &= (state[t] == 2);
            if (all) break;
            continue;
        }
        auto t2 = now();
        std::vector<int> fin, okv;
        step_seed = step_seed * 6364136223846793005ull + 1442695040888963407ull;
        lob_step(run, step_seed, fin, okv);
        // ---- C'. slow refinements.  In a cluster of small singular values
        // the smallest Ritz value xi converges long before the residual of
        // eq. (tolSVD) does.  When xi has stalled (two steps that lower it by
        // less than tau / 10), and every esc_iters iterations, a refinement
        // whose xi is large enough for the test to resolve gets the inertia
        // test at its own point: N(z) - mu0 I with mu0 = (xi - tau)^2 + slack
        // positive definite (every Cholesky pivot positive) certifies
        // sigma_min >= xi - tau by Sylvester's law of inertia, and xi is
        // accepted.  After two failed tests it gets a shifted preconditioner
        // (N(z) - mu I)^{-1}, mu = (xi - 64 tau)^2, else (xi - 4096 tau)^2,
        // whichever is positive definite: a shift just below the bottom of
        // the cluster separates it.  Refinements with smaller xi (the test
        // cannot resolve them) get an exact site N(z) + delta I at their own
        // point instead.  slack bounds the rounding of forming N(z) and of the
        // Cholesky factorization.
        if (use_prec && P.esc_iters > 0 && (op.kind == PS_DENSE || band_b >= 0)) {
            std::vector<char> isfin(T, 0);
            for (int t : fin) isfin[t] = 1;
            std::vector<zd> fsites;
            std::vector<double> fmus;
            std::vector<int> fown, fkind;
            for (int t : run) {
                if (isfin[t]) continue;
                if (two_level && phase[t]) continue;
                if (cert_pend[t]) continue;
                const zd z = h_zt[t];
                const double xi = lob_xi[t];
                if (lob_prev[t] - xi <= 0.1 * tau_c) stag[t]++;
                else stag[t] = 0;
                lob_prev[t] = xi;
                const double nz = nC + sqrt(zabs2(z));
                const double slack = 8.0 * (double)n * EPSM_E * nz * nz;
                const bool resolvable =
                    tau_c > 0.0 && xi > 64.0 * tau_c && 2.0 * xi * tau_c - tau_c * tau_c > 4.0 * slack;
                const bool period = lob_it[t] >= esc_at[t];
                if (period) esc_at[t] = lob_it[t] + P.esc_iters;
                if (resolvable) {
                    if ((stag[t] >= 2 && lob_it[t] >= cert_next[t]) || period) {
                        cert_pend[t] = 1;
                        cert_mu[t] = (xi - tau_c) * (xi - tau_c) + slack;
                        cert_xi[t] = xi;
                        cert_since[t] = loops;
                        pending.push_back(t);
                    }
                    if (period && cert_fail[t] >= 2 && !site_exact[t] && op.kind == PS_DENSE) {
                        fsites.push_back(z); fmus.push_back((xi - 64.0 * tau_c) * (xi - 64.0 * tau_c));
                        fown.push_back(t); fkind.push_back(1);
                        if (xi > 4096.0 * tau_c) {
                            fsites.push_back(z); fmus.push_back((xi - 4096.0 * tau_c) * (xi - 4096.0 * tau_c));
                            fown.push_back(t); fkind.push_back(3);
                        }
                    }
                } else if (period && !site_exact[t] && op.kind == PS_DENSE) {
                    fsites.push_back(z); fmus.push_back(0.0); fown.push_back(t); fkind.push_back(2);
                }
            }
            auto te0 = now();
            std::vector<char> certified(T, 0);
            for (int t : run)
                if (cert_ok[t]) {
                    cert_ok[t] = 0;
                    if (!isfin[t] && !lob_bad[t]) certified[t] = 1;
                }
            // inertia tests wait (while their refinements keep iterating) until
            // a full batch is pending, the oldest has waited 10 steps, or
            // nothing else is running
            {
                std::vector<int> still;
                for (int t : pending)
                    if (cert_pend[t] && state[t] == 1 && !isfin[t]) still.push_back(t);
                    else cert_pend[t] = 0;
                pending.swap(still);
                int nrun = 0;
                for (int t : run) nrun += !isfin[t];
                bool flush = (int)pending.size() >= NBLD || (int)pending.size() >= nrun;
                for (int t : pending) flush |= loops - cert_since[t] >= 10;
                if (flush && !pending.empty()) {
                    std::vector<zd> cs;
                    std::vector<double> cm;
                    for (int t : pending) { cs.push_back(h_zt[t]); cm.push_back(cert_mu[t]); }
                    std::vector<char> pd;
                    build_precond(cs, &cm, &pd, true, true);
                    stats.cert_tests += (int64_t)cs.size();
                    for (size_t i = 0; i < pending.size(); ++i) {
                        const int t = pending[i];
                        cert_pend[t] = 0;
                        if (pd[i] && !lob_bad[t]) certified[t] = 1;
                        else { cert_fail[t]++; cert_next[t] = lob_it[t] + 10; }
                    }
                    pending.clear();
                }
            }
            if (!fsites.empty()) {
                // the shifts are tried closest first: kind 1 (with the exact
                // sites of kind 2) in one batch, kind 3 only for the tiles
                // whose kind-1 factorization was indefinite, and a tile whose
                // shifted sites are all indefinite has an eigenvalue of N(z)
                // far below xi^2 (xi is not yet sigma_min): it gets the site
                // N(z) + delta I at z (kind 4: unlike kind 2 it leaves later
                // shifts possible, for when xi has come down to the bottom of
                // a cluster)
                std::vector<int> got(fsites.size(), -1);
                std::vector<char> pd(fsites.size(), 0);
                std::vector<int> idx3(T, -1);
                auto build_stage = [&](const std::vector<int>& idx) {
                    if (idx.empty()) return;
                    std::vector<zd> ss;
                    std::vector<double> mm;
                    for (int i : idx) { ss.push_back(fsites[i]); mm.push_back(fmus[i]); }
                    std::vector<char> pp;
                    std::vector<int> gg = build_precond(ss, &mm, &pp, true);
                    for (size_t k = 0; k < idx.size(); ++k) { got[idx[k]] = gg[k]; pd[idx[k]] = pp[k]; }
                    // indefinite shifted sites are of no use: free their slots
                    for (int i : idx)
                        if (got[i] >= 0 && !pd[i] && (fkind[i] == 1 || fkind[i] == 3)) {
                            slot_valid[got[i]] = 0;
                            got[i] = -1;
                        }
                };
                {
                    std::vector<int> st1;
                    for (size_t i = 0; i < fsites.size(); ++i) {
                        if (fkind[i] == 3) idx3[fown[i]] = (int)i;
                        else st1.push_back((int)i);
                    }
                    build_stage(st1);
                    std::vector<int> st3;
                    for (size_t i = 0; i < fsites.size(); ++i)
                        if (fkind[i] == 1 && got[i] < 0 && idx3[fown[i]] >= 0 && !certified[fown[i]])
                            st3.push_back(idx3[fown[i]]);
                    build_stage(st3);
                }
                {
                    std::vector<char> has_pd(T, 0), asked(T, 0);
                    for (size_t i = 0; i < fsites.size(); ++i) {
                        if (fkind[i] != 1 && fkind[i] != 3) continue;
                        asked[fown[i]] = 1;
                        if (got[i] >= 0 && pd[i]) has_pd[fown[i]] = 1;
                    }
                    std::vector<zd> xs;
                    std::vector<double> xm;
                    std::vector<int> xo;
                    for (int t = 0; t < T; ++t)
                        if (asked[t] && !has_pd[t] && !certified[t]) {
                            xs.push_back(h_zt[t]);
                            xm.push_back(0.0);
                            xo.push_back(t);
                        }
                    if (!xs.empty()) {
                        std::vector<char> pd2;
                        std::vector<int> got2 = build_precond(xs, &xm, &pd2, true);
                        for (size_t i = 0; i < xs.size(); ++i) {
                            fsites.push_back(xs[i]); fmus.push_back(0.0); fown.push_back(xo[i]); fkind.push_back(4);
                            got.push_back(got2[i]);
                            pd.push_back(pd2[i]);
                        }
                    }
                }
                std::vector<int> pick(T, -1);
                // preference: the closest shift (kind 1), then kind 3, then the exact sites
                auto rank = [](int kd) { return kd == 1 ? 0 : (kd == 3 ? 1 : (kd == 2 ? 2 : 3)); };
                for (size_t i = 0; i < fsites.size(); ++i) {
                    const int t = fown[i];
                    const bool usable = got[i] >= 0 && (fkind[i] == 2 || fkind[i] == 4 || pd[i]) && !certified[t];
                    if (usable && (pick[t] < 0 || rank(fkind[i]) < rank(fkind[pick[t]]))) pick[t] = (int)i;
                }
                for (size_t i = 0; i < fsites.size(); ++i) {
                    const int t = fown[i], sl = got[i];
                    if (sl < 0) continue;
                    if (pick[t] == (int)i) {
                        if (tile_slot[t] >= 0) slot_ref[tile_slot[t]]--;
                        tile_slot[t] = sl;
                        slot_ref[sl]++;
                        usek[t] = 1;
                        if (fkind[i] == 1 || fkind[i] == 2) site_exact[t] = 1;
                        use2l[t] = 0;   // the projection vectors belong to the previous site
                    } else {
                        slot_valid[sl] = 0;
                    }
                }
            }
            // a certified tile returns the explicit Rayleigh quotient
            // ||C(z) x_1|| of its current vector; the certificate holds for
            // it when that value is within 0.2 tau above the value tested
            // (the interval [xi_c - tau, rq] then has width <= 1.2 tau)
            {
                std::vector<int> cl;
                for (int t = 0; t < T; ++t) if (certified[t]) cl.push_back(t);
                std::vector<double> rq = explicit_rq(cl);
                for (size_t i = 0; i < cl.size(); ++i) {
                    const int t = cl[i];
                    if (rq[i] <= cert_xi[t] + 0.2 * tau_c) {
                        fin.push_back(t);
                        okv.push_back(2);
                        lob_sigma[t] = rq[i];
                        stats.certified++;
                    } else {
                        cert_fail[t]++;
                        cert_next[t] = lob_it[t] + 10;
                    }
                }
            }
            stats.t_precond_ms += ms(te0, now());
        }
        auto t3 = now();
        t_lob += ms(t1, t3) - 0.0 * ms(t1, t2);
        // ---- D0. finished projection refinements (Alg. 5): Ebar = F^{-1}
        // Xbar, Lambda_bar = Sigma_bar^2, updateRecy on the site's projection
        // store with the r_breve columns whose sigma_bar^2 <= tau_min, the
        // lower part of eq. (tauRecycle) (a new site at z and the projection
        // refinement again when lambda_bar_rbar < tau_min), then the singular
        // LOBPCG from the saved start block with K_Ebar
        if (two_level && !fin.empty()) {
            std::vector<int> pf, fin2, okv2;
            for (size_t i = 0; i < fin.size(); ++i) {
                if (phase[fin[i]]) pf.push_back(fin[i]);
                else { fin2.push_back(fin[i]); okv2.push_back(okv[i]); }
            }
            if (!pf.empty()) {
                auto tq0 = now();
                fin.swap(fin2);
                okv.swap(okv2);
                finv_apply(pf, 0, S.p, sS, n, tE.p, (int64_t)n * r, n);
                for (int t : pf) fl[tiles[t].order[tiles[t].cursor]] |= PS_FLAG_PROJ_REFINED;
                std::vector<int> us, ut, ub, rebuild, go;
                std::vector<char> seen(NS, 0);
                for (int t : pf) {
                    int rb = 0;
                    for (int j = 0; j < r; ++j) {
                        const double l = lob_sv[(size_t)t * r + j] * lob_sv[(size_t)t * r + j];
                        tlam_h[(size_t)t * r + j] = l;
                        if (l <= P.tau_min) rb = j + 1;
                    }
                    // with no pencil eigenvalue below tau_min the paper's
                    // r_breve is 0 and nothing would be stored, so every later
                    // point would repeat this refinement; the block is then
                    // stored with all its columns in the omega test
                    const int sl = tile_slot[t];
                    if (!seen[sl]) {
                        seen[sl] = 1;
                        us.push_back(sl);
                        ut.push_back(t);
                        ub.push_back(rb > 0 ? rb : r);
                    }
                    if (tlam_h[(size_t)t * r + r - 1] < P.tau_min && !site_at(t)) rebuild.push_back(t);
                    else go.push_back(t);
                }
                h2d(tLam.p, tlam_h.data(), sizeof(double) * T * r);
                proj_update(us, ut, ub);
                rebuild_here(rebuild, fl);
                std::vector<int> again;
                for (int t : rebuild) {
                    if (phase[t]) again.push_back(t);
                    else go.push_back(t);
                }
                for (int t : go) {
                    phase[t] = 0;
                    use2l[t] = 1;
                }
                if (!go.empty()) {
                    upload_list(go, d_list2);
                    launch_copy_cols(d_list2.p, (int)go.size(), tX0.p, (int64_t)n * r, n, S.p, sS, n, n, r, st);
                }
                std::vector<int> restart(again);
                restart.insert(restart.end(), go.begin(), go.end());
                step_seed = step_seed * 6364136223846793005ull + 1442695040888963407ull;
                lob_start(restart, step_seed);
                for (int t : restart) begin_refinement(t);
                stats.t_precond_ms += ms(tq0, now());
            }
        }
        // ---- D. finished tiles: record sigma and gamma = x^* C(z) x of the
        // first Ritz vector, update their recycled store
        if (!fin.empty()) {
            upload_list(fin, d_list2);
            launch_tile_dot0(d_list2.p, (int)fin.size(), S.p, sS, CS.p, (int64_t)m * 3 * r, n, d_gamt.p, st);
            HIPCHK(hipMemcpyAsync(h_gamt.p, d_gamt.p, sizeof(zd) * T, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        for (size_t i = 0; i < fin.size(); ++i) {
            int t = fin[i];
            {
                const int pt0 = tiles[t].order[tiles[t].cursor];
                pgam[pt0] = h_gamt[t];
                pgok[pt0] = 1;
                pdone[pt0] = 1;
            }
            if (use_prec && tile_slot[t] >= 0) { slot_ref[tile_slot[t]]--; tile_slot[t] = -1; }
            int pt = tiles[t].order[tiles[t].cursor];
            sig[pt] = lob_sigma[t];
            fl[pt] |= PS_FLAG_REFINED;
            if (okv[i] == 2) fl[pt] |= PS_FLAG_CERTIFIED;
            cluster[t] = (okv[i] == 2) ? 1 : 0;
            if (!okv[i]) fl[pt] |= PS_FLAG_UNCERTIFIED;
            else fl[pt] &= (uint8_t)~PS_FLAG_UNCERTIFIED;
            stats.refined++;
            tiles[t].cursor++;
        }
        if (!fin.empty()) {
            if (P.recycle && !redo_pass) update_store(fin);
            for (int t : fin) state[t] = tiles[t].done() ? 2 : 0;
        }
        t_upd += ms(t3, now());
        if (P.verbose && ms(t_last_print, now()) >= 5000.0) {
            t_last_print = now();
            int64_t done_pts = stats.accepted + stats.refined;
            fprintf(stderr, "[ps] step %lld: points %lld/%lld accepted %lld refined %lld rebuilds %lld iters %lld  %.1f s\n",
                    (long long)loops, (long long)done_pts, (long long)npts, (long long)stats.accepted,
                    (long long)stats.refined, (long long)stats.rebuilds, (long long)stats.lobpcg_iters,
                    ms(t_start, now()) / 1000.0);
            fflush(stderr);
        }
    }
    };
    run_tiles();
    // Neighbour pass: every value computed here is a Ritz value, an upper
    // bound of sigma_min, and each finished neighbour gives an upper bound of
    // sigma_min at z (nb_bound: the norm of C(z) on the neighbour's vector,
    // or the 1-Lipschitz bound), so a point whose value exceeds one of them is
    // certainly too high (a Ritz value of a larger singular value).  Such
    // points are refined again from a random start block, one point per tile,
    // without touching any recycled store; repeated while violations remain
    // (at most 4 passes).
    if (P.lipschitz) {
        for (int pass = 0; pass < 4; ++pass) {
            std::vector<int> viol;
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const int64_t p = (int64_t)j * nx + i;
                    if (sig[p] > nb_bound(p) * (1.0 + 1e-9) + 1e-12 * nC) viol.push_back((int)p);
                }
            if (viol.empty()) break;
            stats.lipschitz_redo += (int64_t)viol.size();
            if (P.verbose) {
                fprintf(stderr, "[ps] Lipschitz pass %d: %zu points refined again\n", pass, viol.size());
                fflush(stderr);
            }
            for (size_t c0 = 0; c0 < viol.size(); c0 += (size_t)T) {
                const size_t c1 = std::min(viol.size(), c0 + (size_t)T);
                for (int t = 0; t < T; ++t) {
                    tiles[t].order.clear();
                    tiles[t].cursor = 0;
                    tiles[t].k = 0;
                }
                for (size_t c = c0; c < c1; ++c) {
                    tiles[c - c0].order.push_back(viol[c]);
                    fl[viol[c]] = PS_FLAG_LIPSCHITZ;
                }
                upload_k();
                redo_pass = true;
                run_tiles();
                redo_pass = false;
            }
        }
    }
    if (prof.on) prof.collect(stats);
    stats.points = npts;
    stats.uncertified = 0;
    for (int64_t p = 0; p < npts; ++p) stats.uncertified += (fl[p] & PS_FLAG_UNCERTIFIED) ? 1 : 0;
    any_uncert = stats.uncertified > 0;
    for (int64_t p = 0; p < npts; ++p) sigma[p] = sig[p];
    if (flags) memcpy(flags, fl.data(), npts);
    if (member)
        for (int e = 0; e < n_eps; ++e)
            for (int64_t p = 0; p < npts; ++p) member[(size_t)e * npts + p] = (uint8_t)(sig[p] < eps[e]);
    stats.t_ritz_ms = t_ritz;
    stats.t_lobpcg_ms = t_lob;
    stats.t_update_ms = t_upd;
    stats.t_total_ms = ms(t_start, now());
    if (st_out) *st_out = stats;
    return any_uncert ? PS_WARN_UNCERTIFIED : PS_OK;
}
