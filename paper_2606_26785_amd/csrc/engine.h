// Host-side engine: device buffers, operators, the grid-front scheduler and
// the batched solver steps.  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdexcept>
#include <string>
#include <vector>
#include "kernels.h"
#include "../../include/ps.h"

struct DeviceError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct InvalidArg : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define HIPCHK(x)                                                                            \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess)                                                                \
            throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_) + " at " +      \
                              __FILE__ + ":" + std::to_string(__LINE__));                    \
    } while (0)

template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t cnt) {
        if (cnt <= n && p) return;
        release();
        if (cnt == 0) cnt = 1;
        HIPCHK(hipMalloc((void**)&p, cnt * sizeof(T)));
        n = cnt;
    }
    void zero(hipStream_t s) { if (p) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), s)); }
    operator T*() const { return p; }
};

template <class T>
struct HBuf {  // pinned host buffer
    T* p = nullptr;
    size_t n = 0;
    HBuf() = default;
    HBuf(const HBuf&) = delete;
    HBuf& operator=(const HBuf&) = delete;
    ~HBuf() { if (p) (void)hipHostFree(p); }
    void alloc(size_t cnt) {
        if (cnt <= n && p) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        if (cnt == 0) cnt = 1;
        HIPCHK(hipHostMalloc((void**)&p, cnt * sizeof(T), hipHostMallocDefault));
        n = cnt;
    }
    T& operator[](size_t i) { return p[i]; }
};

// The matrix C on the device, with applies of C(z) = C - z S and C(z)^*.
struct Operator {
    int kind = PS_DENSE;
    int64_t m = 0, n = 0, nnz = 0;
    DBuf<zd> A, AH;                     // dense C (m x n, ld m) and C^* (n x m, ld n)
    DBuf<int64_t> rp, rpH;              // CSR of C and of C^*
    DBuf<int32_t> ci, ciH;
    DBuf<zd> v, vH;
    double normC = 0.0;                 // ||C||_2 estimate (power iteration, x1.01)
    // colour-ordered pattern of N = C^* C for the incomplete Cholesky base
    // preconditioner (square CSR)
    DBuf<int64_t> sp_rp, sp_diag, sp_rpT, sp_mapT, sp_ccp, sp_ca, sp_cb;
    DBuf<int32_t> sp_ci, sp_ciT;
    DBuf<int> sp_perm;
    std::vector<int64_t> sp_cptr;
    SparsePattern spat;
};

struct ps_gridh {
    double re_lo, re_hi, im_lo, im_hi;
    int32_t nx, ny;
};

struct Tile {
    std::vector<int> order;   // grid point indices in traversal order
    size_t cursor = 0;
    int k = 0;                // recycled singular dimension
    bool done() const { return cursor >= order.size(); }
};

// grid partition into tx x ty tiles and the order of the points inside each
// (traversal: 0 batch zigzag with band height b, 1 Hilbert, 2 Morton)
void tile_orders(int nx, int ny, int tx, int ty, int b, int traversal, std::vector<Tile>& tiles);

// HIP-event timing of kernel classes (enabled by ps_params.profile)
struct KProf {
    std::vector<hipEvent_t> ev;   // pairs (start, stop)
    std::vector<int> cls;
    std::vector<double> flops, bytes;
    size_t used = 0;
    bool on = false;
    int level = 0;    // 1: classes 0-4; 2: every class
    int begin(hipStream_t s, int c, double fl, double by);
    void end(hipStream_t s, int idx);
    void collect(ps_stats& st);
    ~KProf();
};

struct Engine {
    hipStream_t st = nullptr;
    void* blas = nullptr;      // rocBLAS handle on st (dense sites with fact_blas)
    ps_params P{};
    Operator op;

    // ---- per-eval sizing
    int T = 0;         // tile slots
    int r = 8, K = 32; // block size, recycled cap
    int B = 20;        // points per Ritz test window of a tile
    int64_t n = 0, m = 0;

    // singular store (primary + update scratch)
    DBuf<zd> sV, sW1, sW3, sW4, uV, uW1, uW3, uW4;
    DBuf<zd> sRA, sRres;
    DBuf<zd> sH;          // per tile: H = V^* S^* C V (k x k), first-order coefficients of Ritz vectors
    DBuf<zd> j_gam, d_gamt;   // per Ritz job / per tile: gamma = (S x)^* C(z) x of the first Ritz vector
    HBuf<zd> h_gamj, h_gamt;
    std::vector<zd> pgam;     // per grid point: gamma of the vector behind sigma
    std::vector<uint8_t> pgok;
    DBuf<zdd> gdd;        // Gram workspace (per tile, (4K)^2)
    DBuf<int> d_k, d_q, d_l;

    // LOBPCG state (per tile)
    DBuf<zd> S, CS, Sn, CSn, Wres, Xw, Tn1, Tn2, Tn3;
    DBuf<zd> Rsm, GX, GP, Csm, Tsm, Qt, Upp, Ucoef, X0c;
    DBuf<double> xi, nrm2, xi_out;
    DBuf<uint32_t> mask;
    DBuf<int> cdim, d_list, d_list2, d_jobsrc;
    DBuf<zd> d_z;         // per tile current z

    // ritz jobs
    DBuf<int> j_tile;
    DBuf<zd> j_z, j_G;
    DBuf<double> j_nrm, j_xi, j_res;
    DBuf<uint8_t> j_acc;

    // workspaces
    DBuf<char> gram_ws;
    size_t gram_ws_bytes = 0;
    DBuf<zd> apply_ws;
    int apply_splitk = 1;
    DBuf<double> norm_ws;

    // pinned host mirrors
    HBuf<uint8_t> h_acc;
    HBuf<double> h_xi, h_nrm2, h_small;
    HBuf<zd> h_C;
    HBuf<int> h_list;
    HBuf<zd> h_z;

    // dense base preconditioner: a pool of NS sites, each K = F^* F with F the
    // upper Cholesky factor of N(z_dag) + delta I and F^{-1} kept explicitly
    // (Finv, one n x n block per slot).  A refinement references one site
    // (tile_slot); sites are shared by every tile whose point satisfies the
    // rebuild rule for them and are built NBLD at a time in the Fb/PN staging
    // blocks.
    DBuf<zd> CtC, PN, Fb, Finv, Dinv, T1p, T2p, pvec, d_zdag, zgemm_ws;
    int NS = 0, NBLD = 0;
    std::vector<zd> slot_z;
    std::vector<double> slot_gam;
    std::vector<int> slot_ref;
    std::vector<int64_t> slot_last;
    std::vector<char> slot_valid;
    std::vector<char> slot_priv;     // built for one refinement (shifted or escalated): never shared
    int64_t slot_clock = 0;
    DBuf<double> d_shift;
    DBuf<int> d_notpd;
    HBuf<double> h_shift;
    HBuf<int> h_notpd;
    std::vector<int> tile_slot;      // per tile: site of the running refinement (-1: K = I)
    std::vector<char> usek;          // per tile: this refinement uses the base preconditioner
    DBuf<int> d_listI, d_gmap;
    HBuf<int> h_gmap;
    bool use_prec = false;
    void reset_slots();
    // builds one site per entry of `sites` into free slots; slot ids out (-1:
    // no free slot).  mu (optional): per-site shift, the factored matrix is
    // N(z) - mu I (+ delta I when mu = 0); pd (optional) receives whether the
    // Cholesky met only positive pivots; priv: sites are private to one tile.
    // cert_only: factor only (no F^{-1}, no slot), for the inertia test
    std::vector<int> build_precond(const std::vector<zd>& sites, const std::vector<double>* mu = nullptr,
                                   std::vector<char>* pd = nullptr, bool priv = false, bool cert_only = false);
    // slot whose site satisfies the rebuild rule at z with the smallest gamma |z - z_dag|, or -1
    int find_slot(zd z) const;
    void precond_apply(const std::vector<int>& L, const zd* W, int64_t ws, zd* Y, int64_t ys);
    void zgemm(const int* dl, int nt, int64_t M, int64_t N, int64_t Kd, const zd* A, int64_t lda, int64_t sA,
               int opA, const zd* Bm, int64_t ldb, int64_t sB, zd* Cm, int64_t ldc, int64_t sC, double alpha,
               double beta, int upper = 0, int tri = 0, const int* gmap = nullptr, int cw = 0,
               int64_t cols_total = -1);   // column-map mode: columns over all groups (for the flop count)

    // ---- two-level preconditioner (Sec. 3, eq. (twolevel), Alg. 4, Alg. 5)
    // Each preconditioner site (slot) carries a recycled projection subspace
    // Vbar (n x KB, newest block first, so that its leading blocks span the
    // most recent refinements as the QL form of Alg. 2 does) and the cached
    // R factors of Mbar(z) Vbar = (C - z S) F^{-1} Vbar and of the residual
    // blocks, so that recyProj is the same per-point Rayleigh-Ritz-SVD as
    // recySing.  The projection block size equals r.
    bool two_level = false;
    int KB = 0;                                  // projection capacity (kbar_max)
    DBuf<zd> pV, pE, pW1, pW3, pW4, pW5, pW6, pT; // per slot; pE = F^{-1} Vbar
    DBuf<zd> pRA, pRres;                         // per slot: (2 KB)^2, (5 KB)^2
    DBuf<zdd> pgdd;                              // per slot Gram workspace (5 KB)^2
    DBuf<int> d_pk, d_nzp;                       // per slot: current kbar (index NS: empty); zero pivots
    std::vector<int> pk;
    std::vector<double> slot_lamn;               // lambda_bar_n^dagger of the site
    std::vector<double> slot_dreg;               // regularisation shift of the site
    // per tile
    DBuf<zd> tE, tX0, tCoef, Tp, pG;             // Ebar (n x r), saved start block, Ebar^* W, temp, recyProj G
    DBuf<double> tLam, pj_xi, pj_res, pj_nrm;
    DBuf<uint8_t> pj_acc;
    DBuf<int> pj_slot, d_listA, d_listB, d_tslot;
    DBuf<zd> pj_z;
    std::vector<char> phase;                     // 1: projection LOBPCG on Mbar(z) running
    std::vector<char> use2l;                     // singular LOBPCG uses K_Ebar
    std::vector<double> lob_sv;                  // per tile r Ritz values of the last step
    std::vector<double> tlam_h;                  // per tile Lambda_bar (host copy)
    void finv_apply(const std::vector<int>& L, int trans, const zd* X, int64_t xs, int64_t ldx, zd* Y, int64_t ys,
                    int64_t ldy);
    // C(z) X (or C(z)^* X) for singular-phase tiles, Mbar(z) X = C(z) F^{-1} X
    // (or Mbar(z)^* X = F^{-*} C(z)^* X) for projection-phase tiles
    void op_apply(bool herm, const std::vector<int>& L, const zd* X, int64_t xs, int64_t ldx, zd* Y, int64_t ys,
                  int64_t ldy, int w);
    void twolevel_add(const std::vector<int>& L, const zd* W, int64_t ws, zd* Y, int64_t ys);
    double tbar_norm(int slot, zd z) const;      // (sqrt(lambda_n^dagger) + gamma |z - z_dag|)^2
    int find_slot2(zd z) const;                  // the rule of eq. (tauRecycle), upper part
    void proj_reset(int slot);
    void proj_refresh(const std::vector<int>& slots);
    // updateRecy (Alg. 2) on the projection store of `slot` with the block
    // X = S[:, 0:r] of tile t and r_breve leading columns in the omega test
    void proj_update(const std::vector<int>& slots, const std::vector<int>& tiles, const std::vector<int>& rbrev);
    // recyProj (Alg. 4) for the tiles of L at their sites: accepted tiles get
    // Ebar and Lambda_bar; acc[i] = 1 when eq. (tolTz) holds
    void recy_proj(const std::vector<int>& L, std::vector<char>& acc);
    void upload_pk();
    // sparse sites: incomplete Cholesky values per slot, site points, work blocks
    DBuf<zd> Slu, Svec, pS, d_slotz, Tq;
    DBuf<int> d_listC;
    DBuf<int> d_icbad;          // per slot: a pivot of its incomplete Cholesky was not positive
    // inertia tests for a CSR C whose N = C^* C has bandwidth band_b <= 63 in
    // the natural order (-1: no such tests): contribution lists of the band
    // entries (row j, offset d) at j (band_b + 1) + d, per-test band storage
    int band_b = -1;
    DBuf<int64_t> bn_cp, bn_ca, bn_cb;
    DBuf<zd> bn_W, bn_z;
    DBuf<double> bn_mu;
    DBuf<int> bn_bad, bn_list;
    void band_inertia(const std::vector<zd>& zs, const std::vector<double>& mus, std::vector<char>& pd);
    DBuf<double> d_alpha;       // per slot: diagonal shift alpha of N(z_dag) + alpha I
    std::vector<double> slot_alpha;
    void build_sparse_pattern();        // colouring and patterns (host, once per handle)
    std::vector<int> build_sparse_sites(const std::vector<zd>& sites, const std::vector<int>& slots);
    bool site_at(int t) const;                   // the tile's site was built at its current point
    // regularised base sites (precond = 2): N(z_dag) + (reg_base (||C|| + |z_dag|))^2 I
    std::vector<int> build_regularized(const std::vector<zd>& sites);
    // lower part of eq. (tauRecycle) failed: a new site at each tile's point,
    // whose projection refinement then runs (phase 1); fl gets the rebuild flag
    void rebuild_here(const std::vector<int>& tl, std::vector<uint8_t>& fl);

    // plain products inside the blocked Cholesky of the dense sites (list =
    // staging positions 0 .. nb-1): rocBLAS strided-batched ZHERK (upper,
    // A == B) / ZGEMM when fact_blas, else zgemm()
    void fact_gemm(const int* dl, int nb, int64_t M, int64_t N, int64_t Kd, const zd* A, int64_t lda, int64_t sA,
                   int opA, const zd* Bm, int64_t ldb, int64_t sB, zd* Cm, int64_t ldc, int64_t sC, double alpha,
                   double beta, int upper = 0, int tri = 0);
    ~Engine();

    KProf prof;
    int zgemm_cls = 1;        // profiling class of zgemm launches (3 inside factorizations)
    ps_stats stats{};
    std::vector<Tile> tiles;
    std::vector<zd> zs;       // grid points of the current eval

    // ---- setup
    void create(const ps_matrix_desc* d, const ps_params* p, hipStream_t s);
    void estimate_norm();
    void size_for(int tiles);

    // ---- operator applies on tiles (columns w per tile)
    // Y (m rows) = C(z) X (n rows);  herm: Y (n rows) = C(z)^* X (m rows)
    // ws / ws_n: a caller-provided workspace for the dense split-K partials
    // (default: the handle's own apply_ws)
    void apply(bool herm, const int* dlist, int nt, const zd* X, int64_t xstride, int64_t ldx, zd* Y,
               int64_t ystride, int64_t ldy, int w, const zd* dz, zd* ws = nullptr, size_t ws_n = 0);

    // pinned staging ring for host-to-device uploads: every upload copies its
    // bytes into a fresh slice, so an upload never waits for the stream (the
    // stream is drained only when the ring wraps around)
    HBuf<char> ring;
    size_t ring_pos = 0;
    void h2d(void* dst, const void* src, size_t bytes);

    // ---- building blocks
    void upload_list(const std::vector<int>& L, DBuf<int>& dst);
    void gram(const int* dlist, int nt, const BlockList& A, const BlockList& Bl, int camax, int cbmax, void* out,
              int64_t strideOut, int ldOut, bool dd, bool upper, bool out_dd = false);
    void gemm_ts(const int* dlist, int nt, const BlockList& A, int camax, const zd* G, int64_t strideG, int ldG,
                 const int* cbdims, int cbmul, int cb, zd* Y, int64_t strideY, int64_t ldY, int64_t rows,
                 double alpha, double beta);
    void colnorm2(const int* dlist, int nt, const BlockList& A, int camax, double* out, int ldo);
    void orthonormalize(const std::vector<int>& L, const int* dlist, zd* W, int64_t wstride, int64_t ldw,
                        int64_t rows, int cols, const BlockList* against, int against_max, uint64_t seed);
    // nzero (optional, per tile): number of pivots the Cholesky treated as zero
    // dd_gram: Gram matrix accumulated in double-double (mixed-precision
    // Cholesky QR); false: in double, where its rounding is known to be small
    void r_factor(const int* dlist, int nt, const BlockList& A, int cmax, const int* cdims, int cmul, int cfixed,
                  zd* R, int64_t strideR, int ldR, int* nzero = nullptr, zdd* gbuf = nullptr, bool dd_gram = true);
    DBuf<int> d_listDD, d_listPL;   // LOBPCG tiles whose R factor uses the double-double / double Gram

    // ---- algorithm steps
    // LOBPCG-SVD as a per-tile state machine: lob_start runs the first
    // Rayleigh-Ritz-SVD on the start block of the listed tiles, lob_step one
    // iteration for every listed tile (tiles may be at different iterations).
    std::vector<int> lob_it;          // per tile: iteration count (0 = after start)
    std::vector<double> lob_sigma;    // per tile: smallest Ritz value at exit
    std::vector<double> lob_xi;       // per tile: smallest Ritz value after the last step
    std::vector<int> esc_at;          // per tile: iteration of the next escalation
    std::vector<char> site_exact;     // per tile: its preconditioner was built at its own point
    std::vector<double> lob_prev;     // per tile: xi after the previous step
    std::vector<int> stag, cert_next, cert_fail;   // per tile: inertia-test bookkeeping
    std::vector<char> nop;            // per tile: next iteration runs without the P block (after a repair)
    std::vector<char> lob_bad;        // per tile: the last step broke down (S lost rank); repaired
    std::vector<zd> h_zt;             // per tile: current grid point
    DBuf<int> d_cdimt, d_pcols;       // per tile: width of S, width of P
    void lob_start(const std::vector<int>& L, uint64_t seed);
    // ||C(z) x_1|| / ||x_1|| with C(z) X recomputed explicitly, per tile of L
    std::vector<double> explicit_rq(const std::vector<int>& L);
    // returns the tiles that finished (converged, or at max_iters: ok = 0)
    void lob_step(const std::vector<int>& L, uint64_t seed, std::vector<int>& done, std::vector<int>& ok);
    void update_store(const std::vector<int>& L);
    void upload_k();
    void refresh_store(const std::vector<int>& L);
    ps_status eval(const ps_gridh* g, const double* eps, int n_eps, double* sigma, uint8_t* member,
                   uint8_t* flags, ps_stats* st_out);
};

BlockList bl_empty(int64_t rows);
// the last block added to L is indexed through imap (array index imap[tile])
void bl_map(BlockList& L, const int* imap);
void bl_add(BlockList& L, const zd* ptr, int64_t stride, int64_t ld, int ncols, const int* dims, int mul,
            int64_t brows = 0, const int* coff = nullptr, int coffmul = 0);
void launch_gather(const int* list, int nt, const int* srcidx, const zd* src, int64_t sstride, zd* dst,
                   int64_t dstride, int64_t count, hipStream_t s);
