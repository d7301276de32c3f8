// C ABI (include/ps.h): argument checking, handle lifecycle, error mapping.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "engine.h"

struct ps_matrix {
    Engine eng;
    int dev = 0;       // device current at ps_create
};

// Workspace of ps_apply_noalloc: one copy of this array per GPU, resident
// until the process ends.  Host code never uses the array's name as an
// address: scratch_setup() takes each device's own address once, with that
// device current, and the entry point passes that address to its kernels.
// Layout: bytes [0, 256) hold the one-item tile list and z; the dense
// split-K partial products follow.
#define PS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
#define PS_NOALLOC_HEADER 256
static __device__ __align__(256) unsigned char scratch[PS_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[256];      // per device ordinal

static hipError_t scratch_setup(int dev)
{
    if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[dev] = ptr;
    return e;
}

static void* scratch_ptr(int dev)
{
    if (dev < 0 || dev >= 256) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// writes the one-item tile list and z into the scratch header (a kernel, not
// a memset or host copy, so that the call can be captured into a graph)
__global__ void k_noalloc_header(int* list, zd* z, double zr, double zi)
{
    if (threadIdx.x == 0) {
        list[0] = 0;
        z[0] = zmake(zr, zi);
    }
}

static thread_local std::string g_last_error;

static ps_status fail(ps_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

extern "C" {

void ps_default_params(ps_params* p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->r = 8;
    p->k_max = 32;
    p->rbar = 8;
    p->kbar_max = 64;
    p->max_iters = 300;
    p->precond = -1;
    p->tiles_x = 0;
    p->tiles_y = 0;
    p->tile_points = 80;
    p->tile_mem_gb = 48;
    p->site_mem_gb = 128;
    p->batch = 20;
    p->traversal = 0;
    p->recycle = 1;
    p->eta = 1e-6;
    p->eta_svd = 1e-9;
    p->eta_proj = 1e-4;
    p->omega = 1.6;
    p->tau_min = 1e-3;
    p->tau_max = 30.0;
    p->zdag_re = NAN;
    p->zdag_im = NAN;
    p->seed = 20261203ull;
    p->eta_abs = 8e-9;
    p->rho_small = 1e-5;
    p->profile = 0;
    p->verbose = 0;
    p->tol_abs = 8e-9;
    p->esc_iters = 30;
    p->cert_recycled = 0;
    p->lipschitz = 1;
    p->reg_base = 0.02;
    p->fact_blas = 0;
}

const char* ps_strerror(ps_status s)
{
    switch (s) {
    case PS_OK: return "ok";
    case PS_WARN_UNCERTIFIED: return "some points hit the LOBPCG iteration cap";
    case PS_EINVAL: return "invalid argument";
    case PS_ENOMEM: return "out of device memory";
    case PS_EDEVICE: return "HIP device error";
    case PS_EBREAKDOWN: return "numerical breakdown";
    case PS_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

ps_status ps_create(const ps_matrix_desc* d, const ps_params* params, void* hip_stream, ps_matrix** out)
{
    if (!d || !out) return fail(PS_EINVAL, "NULL descriptor or output handle");
    *out = nullptr;
    ps_params p;
    if (params) p = *params; else ps_default_params(&p);
    if (d->m < d->n || d->n < 1) return fail(PS_EINVAL, "need m >= n >= 1");
    if (d->m > ((int64_t)1 << 31) - 1) return fail(PS_EINVAL, "m too large for int32 column indices");
    if (d->kind == PS_DENSE) {
        if (!d->dense || d->ld < d->m) return fail(PS_EINVAL, "dense: NULL data or ld < m");
    } else if (d->kind == PS_CSR) {
        if (!d->rowptr || !d->colind || !d->vals || d->nnz < 0) return fail(PS_EINVAL, "CSR: NULL arrays");
    } else {
        return fail(PS_EINVAL, "unknown matrix kind");
    }
    if (p.r < 2 || p.r > 16 || (p.r & 1)) return fail(PS_EINVAL, "r must be even, 2..16");
    if (p.k_max < p.r || p.k_max % p.r || p.k_max > 64) return fail(PS_EINVAL, "k_max must be a multiple of r, <= 64");
    if (p.rbar < 2 || p.rbar > 16 || (p.rbar & 1)) return fail(PS_EINVAL, "rbar must be even, 2..16");
    if (p.kbar_max < p.rbar || p.kbar_max % p.rbar || p.kbar_max > 64)
        return fail(PS_EINVAL, "kbar_max must be a multiple of rbar, <= 64");
    if (p.max_iters < 1 || p.batch < 1) return fail(PS_EINVAL, "max_iters and batch must be positive");
    if (p.traversal < 0 || p.traversal > 2) return fail(PS_EINVAL, "traversal must be 0, 1 or 2");
    if (p.fact_blas < 0 || p.fact_blas > 1) return fail(PS_EINVAL, "fact_blas must be 0 or 1");
    if (p.tile_points < 1 || p.tile_mem_gb < 1 || p.site_mem_gb < 1)
        return fail(PS_EINVAL, "tile_points, tile_mem_gb and site_mem_gb must be positive");
    if (!(p.eta > 0) || !(p.eta_svd > 0) || !(p.omega >= 1.0) || !(p.eta_abs >= 0) || p.eta_abs > 1e-8 ||
        !(p.tol_abs >= 0) || p.tol_abs > 1e-6 || p.esc_iters < 0)
        return fail(PS_EINVAL, "bad tolerances");
    if (p.precond > 2 || p.precond < -1) return fail(PS_EINVAL, "precond must be -1, 0, 1 or 2");
    const int pc = p.precond < 0 ? (d->kind == PS_DENSE ? 1 : 2) : p.precond;
    if (pc == 2 && p.rbar != p.r)
        return fail(PS_EINVAL, "the two-level preconditioner runs its projection LOBPCG with block rbar = r");
    if (!(p.eta_proj > 0) || !(p.tau_min > 0) || !(p.tau_max > 1.0) || !(p.reg_base >= 0) || p.reg_base > 1.0)
        return fail(PS_EINVAL, "bad projection or rebuild thresholds");
    if (d->kind == PS_DENSE && !d->on_device) {
        for (int64_t j = 0; j < d->n; ++j)
            for (int64_t i = 0; i < 2 * d->m; ++i)
                if (!std::isfinite(d->dense[2 * d->ld * j + i])) return fail(PS_EINVAL, "non-finite entry");
    }
    ps_matrix* h = new (std::nothrow) ps_matrix();
    if (!h) return fail(PS_ENOMEM, "host allocation failed");
    if (hipGetDevice(&h->dev) != hipSuccess || scratch_setup(h->dev) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return fail(PS_EDEVICE, "no usable device (static workspace address)");
    }
    try {
        h->eng.create(d, &p, (hipStream_t)hip_stream);
    } catch (const InvalidArg& e) {
        delete h;
        return fail(PS_EINVAL, e.what());
    } catch (const DeviceError& e) {
        delete h;
        std::string w = e.what();
        return fail(w.find("out of memory") != std::string::npos ? PS_ENOMEM : PS_EDEVICE, w);
    } catch (const std::bad_alloc&) {
        delete h;
        return fail(PS_ENOMEM, "host allocation failed");
    }
    *out = h;
    return PS_OK;
}

ps_status ps_grid(double re_lo, double re_hi, double im_lo, double im_hi, int32_t nx, int32_t ny, ps_gridh** out)
{
    if (!out) return fail(PS_EINVAL, "NULL output handle");
    *out = nullptr;
    if (nx < 1 || ny < 1) return fail(PS_EINVAL, "nx and ny must be >= 1");
    if (!std::isfinite(re_lo) || !std::isfinite(re_hi) || !std::isfinite(im_lo) || !std::isfinite(im_hi))
        return fail(PS_EINVAL, "non-finite region");
    ps_gridh* g = new (std::nothrow) ps_gridh();
    if (!g) return fail(PS_ENOMEM, "host allocation failed");
    g->re_lo = re_lo;
    g->re_hi = re_hi;
    g->im_lo = im_lo;
    g->im_hi = im_hi;
    g->nx = nx;
    g->ny = ny;
    *out = g;
    return PS_OK;
}

ps_status ps_eval(ps_matrix* h, const ps_gridh* g, const double* eps, int32_t n_eps, double* sigma,
                  uint8_t* member, uint8_t* flags, ps_stats* stats)
{
    if (!h || !g || !sigma) return fail(PS_EINVAL, "NULL handle, grid or sigma");
    if (n_eps < 0 || (n_eps > 0 && !eps)) return fail(PS_EINVAL, "bad eps list");
    if (n_eps > 0 && !member) return fail(PS_EINVAL, "member output required when n_eps > 0");
    try {
        return h->eng.eval(g, eps, n_eps, sigma, member, flags, stats);
    } catch (const InvalidArg& e) {
        return fail(PS_EINVAL, e.what());
    } catch (const DeviceError& e) {
        std::string w = e.what();
        return fail(w.find("out of memory") != std::string::npos ? PS_ENOMEM : PS_EDEVICE, w);
    } catch (const std::bad_alloc&) {
        return fail(PS_ENOMEM, "host allocation failed");
    }
}

void ps_grid_destroy(ps_gridh* g) { delete g; }

void ps_destroy(ps_matrix* h)
{
    if (!h) return;
    if (h->eng.st) (void)hipStreamSynchronize(h->eng.st);
    else (void)hipDeviceSynchronize();
    delete h;
}

}  // extern "C"

#include "../../include/ps_debug.h"

extern "C" ps_status ps_debug_apply(ps_matrix* h, int32_t herm, double z_re, double z_im, const double* X,
                                    int32_t w, double* Y)
{
    if (!h || !X || !Y) return fail(PS_EINVAL, "NULL argument");
    if (w < 1 || w > 64) return fail(PS_EINVAL, "w must be 1..64");
    try {
        Engine& E = h->eng;
        int64_t rin = herm ? E.m : E.n, rout = herm ? E.n : E.m;
        DBuf<zd> dX, dY;
        DBuf<int> dl;
        DBuf<zd> dz;
        dX.alloc((size_t)rin * w);
        dY.alloc((size_t)rout * w);
        dl.alloc(1);
        dz.alloc(1);
        int zero = 0;
        zd zz = zmake(z_re, z_im);
        HIPCHK(hipMemcpy(dl.p, &zero, sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dz.p, &zz, sizeof(zd), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dX.p, X, sizeof(zd) * rin * w, hipMemcpyHostToDevice));
        E.apply(herm != 0, dl.p, 1, dX.p, 0, rin, dY.p, 0, rout, w, dz.p);
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(Y, dY.p, sizeof(zd) * rout * w, hipMemcpyDeviceToHost));
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}

extern "C" ps_status ps_apply_noalloc(ps_matrix* h, int32_t herm, double z_re, double z_im, const double* X,
                                      int64_t ldx, int32_t w, double* Y, int64_t ldy)
{
    if (!h || !X || !Y) return fail(PS_EINVAL, "NULL argument");
    if (w < 1 || w > 64) return fail(PS_EINVAL, "w must be 1..64");
    if (!std::isfinite(z_re) || !std::isfinite(z_im)) return fail(PS_EINVAL, "non-finite z");
    Engine& E = h->eng;
    const int64_t rin = herm ? E.m : E.n, rout = herm ? E.n : E.m;
    if (ldx < rin || ldy < rout) return fail(PS_EINVAL, "ldx or ldy below the row count");
    const size_t part_need = (E.op.kind == PS_DENSE) ? (size_t)rout * w * sizeof(zd) : 0;
    if (PS_NOALLOC_HEADER + part_need > PS_NOALLOC_SCRATCH_BYTES)
        return fail(PS_EINVAL, "rows x w exceed the static workspace (32 MiB: rows * w * 16 bytes <= 32 MiB - 256)");
    char* base = (char*)scratch_ptr(h->dev);
    if (!base) return fail(PS_EDEVICE, "static workspace not set up on this device");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(PS_EDEVICE, "hipGetDevice failed");
    if (cur != h->dev && hipSetDevice(h->dev) != hipSuccess) return fail(PS_EDEVICE, "hipSetDevice failed");
    ps_status rc = PS_OK;
    const bool prof_on = E.prof.on;
    try {
        E.prof.on = false;     // no profiling events (they are created on demand)
        int* dl = (int*)base;
        zd* dz = (zd*)(base + 16);
        zd* part = (zd*)(base + PS_NOALLOC_HEADER);
        const size_t part_n = (PS_NOALLOC_SCRATCH_BYTES - PS_NOALLOC_HEADER) / sizeof(zd);
        hipLaunchKernelGGL(k_noalloc_header, dim3(1), dim3(64), 0, E.st, dl, dz, z_re, z_im);
        HIPCHK(hipGetLastError());
        E.apply(herm != 0, dl, 1, (const zd*)X, 0, ldx, (zd*)Y, 0, ldy, w, dz, part, part_n);
        HIPCHK(hipGetLastError());
    } catch (const std::exception& e) {
        rc = fail(PS_EDEVICE, e.what());
    }
    E.prof.on = prof_on;
    if (cur != h->dev) (void)hipSetDevice(cur);
    return rc;
}

extern "C" ps_status ps_debug_order(int32_t nx, int32_t ny, int32_t tx, int32_t ty, int32_t b, int32_t traversal,
                                    int32_t* order, int32_t* tile_start)
{
    if (!order || !tile_start) return fail(PS_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || tx < 1 || ty < 1 || tx > nx || ty > ny || b < 1 || traversal < 0 || traversal > 2)
        return fail(PS_EINVAL, "bad grid, tiling or traversal");
    std::vector<Tile> tiles;
    tile_orders(nx, ny, tx, ty, b, traversal, tiles);
    int64_t pos = 0;
    for (size_t t = 0; t < tiles.size(); ++t) {
        tile_start[t] = (int32_t)pos;
        for (int p : tiles[t].order) order[pos++] = p;
    }
    tile_start[tiles.size()] = (int32_t)pos;
    return PS_OK;
}

extern "C" double ps_debug_norm(const ps_matrix* h) { return h ? h->eng.op.normC : 0.0; }

// Build one dense base-preconditioner site at z and copy F^{-1} (n x n,
// column-major) to the host; returns gamma = ||F^{-1}||_2 estimate.
extern "C" ps_status ps_debug_precond(ps_matrix* h, double z_re, double z_im, double* Finv_out, double* gamma_out)
{
    if (!h || !Finv_out) return fail(PS_EINVAL, "NULL argument");
    try {
        Engine& E = h->eng;
        if (!E.use_prec) return fail(PS_EUNSUPPORTED, "no dense preconditioner on this handle");
        if (E.T < 1 || E.NS < 1) E.size_for(std::max(E.T, 1));
        E.reset_slots();
        std::vector<int> sl = E.build_precond({zmake(z_re, z_im)});
        if (sl.empty() || sl[0] < 0) return fail(PS_ENOMEM, "no preconditioner slot");
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(Finv_out, E.Finv.p + (size_t)sl[0] * E.n * E.n, sizeof(zd) * E.n * E.n,
                         hipMemcpyDeviceToHost));
        if (gamma_out) *gamma_out = E.slot_gam[sl[0]];
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}

// One refinement of the projection subspace at z against a regularised site
// at z_dag, then Y = K_Ebar^{-1} W with the resulting two-level
// preconditioner (eq. (twolevel)); Ebar (n x r) and Lambda_bar (r) out.
extern "C" ps_status ps_debug_twolevel(ps_matrix* h, double zd_re, double zd_im, double z_re, double z_im,
                                       const double* W, double* Y, double* Ebar, double* lam, int32_t* iters)
{
    if (!h || !W || !Y || !Ebar || !lam) return fail(PS_EINVAL, "NULL argument");
    try {
        Engine& E = h->eng;
        if (!E.two_level) return fail(PS_EUNSUPPORTED, "no two-level preconditioner on this handle");
        if (E.T < 1 || E.NS < 1) E.size_for(std::max(E.T, 1));
        E.reset_slots();
        std::vector<int> sl = E.build_regularized({zmake(zd_re, zd_im)});
        if (sl.empty() || sl[0] < 0) return fail(PS_ENOMEM, "no preconditioner slot");
        const int t = 0, r = E.r;
        const int64_t n = E.n, sS = n * 3 * r;
        E.tile_slot[t] = sl[0];
        E.slot_ref[sl[0]]++;
        E.usek[t] = 1;
        E.phase[t] = 1;
        E.use2l[t] = 0;
        E.h_zt[t] = zmake(z_re, z_im);
        std::vector<zd> hz(E.T, zmake(z_re, z_im));
        E.h2d(E.d_z.p, hz.data(), sizeof(zd) * E.T);
        std::vector<int> L = {t};
        E.upload_list(L, E.d_list);
        launch_randfill(E.d_list.p, 1, E.S.p, sS, n, n, r, nullptr, 0x7e57ull, E.st);
        E.lob_start(L, 0x1234ull);
        std::vector<int> done, okv;
        int it = 0;
        for (it = 0; it < 200 && done.empty(); ++it) E.lob_step(L, 0x9876ull + it, done, okv);
        E.finv_apply(L, 0, E.S.p, sS, n, E.tE.p, n * r, n);
        for (int j = 0; j < r; ++j) {
            const double s = E.lob_sv[(size_t)t * r + j];
            E.tlam_h[(size_t)t * r + j] = s * s;
            lam[j] = s * s;
        }
        E.h2d(E.tLam.p, E.tlam_h.data(), sizeof(double) * E.T * r);
        E.phase[t] = 0;
        E.use2l[t] = 1;
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(E.Wres.p, W, sizeof(zd) * n * r, hipMemcpyHostToDevice));
        E.precond_apply(L, E.Wres.p, n * r, E.S.p + (size_t)n * r, sS);
        E.twolevel_add(L, E.Wres.p, n * r, E.S.p + (size_t)n * r, sS);
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(Y, E.S.p + (size_t)n * r, sizeof(zd) * n * r, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(Ebar, E.tE.p, sizeof(zd) * n * r, hipMemcpyDeviceToHost));
        if (iters) *iters = it;
        E.slot_ref[sl[0]]--;
        E.tile_slot[t] = -1;
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}

// The regularisation shift d of the site last built by ps_debug_twolevel
// (K = F^* F = N(z_dag) + d I) and gamma = ||F^{-1}||_2 (estimate).
extern "C" ps_status ps_debug_site(ps_matrix* h, double* dreg, double* gamma)
{
    if (!h || !dreg || !gamma) return fail(PS_EINVAL, "NULL argument");
    Engine& E = h->eng;
    for (int s = 0; s < E.NS; ++s)
        if (E.slot_valid[s]) {
            *dreg = E.slot_dreg[s];
            *gamma = E.slot_gam[s];
            return PS_OK;
        }
    return fail(PS_EINVAL, "no site built");
}

// One sparse base site at z: Y = F^{-1} X (trans 0) or F^{-*} X (trans 1).
extern "C" ps_status ps_debug_sparse_site(ps_matrix* h, double z_re, double z_im, int32_t trans, const double* X,
                                          int32_t w, double* Y, double* alpha)
{
    if (!h || !X || !Y || !alpha) return fail(PS_EINVAL, "NULL argument");
    if (w < 1 || w > 64 || trans < 0 || trans > 1) return fail(PS_EINVAL, "w must be 1..64, trans 0 or 1");
    try {
        Engine& E = h->eng;
        if (E.op.kind == PS_DENSE || !E.use_prec) return fail(PS_EUNSUPPORTED, "no sparse base preconditioner");
        if (E.T < 1 || E.NS < 1) E.size_for(std::max(E.T, 1));
        E.reset_slots();
        std::vector<int> sl = E.build_precond({zmake(z_re, z_im)});
        if (sl.empty() || sl[0] < 0) return fail(PS_ENOMEM, "no preconditioner slot");
        const int64_t n = E.n;
        DBuf<zd> dX, dY, dT;
        DBuf<int> dl, ds;
        dX.alloc((size_t)n * w);
        dY.alloc((size_t)n * w);
        dT.alloc((size_t)n * w);
        dl.alloc(1);
        ds.alloc(1);
        const int zero = 0;
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(dl.p, &zero, sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ds.p, &sl[0], sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dX.p, X, sizeof(zd) * n * w, hipMemcpyHostToDevice));
        launch_ic_solve(dl.p, 1, ds.p, E.op.spat, E.Slu.p, trans, dX.p, 0, n, dY.p, 0, n, w, dT.p, 0, E.st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(Y, dY.p, sizeof(zd) * n * w, hipMemcpyDeviceToHost));
        *alpha = E.slot_alpha[sl[0]];
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}

// One inertia test: is N(z) - mu I positive definite?
extern "C" ps_status ps_debug_inertia(ps_matrix* h, double z_re, double z_im, double mu, int32_t* pd)
{
    if (!h || !pd) return fail(PS_EINVAL, "NULL argument");
    try {
        Engine& E = h->eng;
        if (!E.use_prec) return fail(PS_EUNSUPPORTED, "no preconditioner on this handle");
        if (E.op.kind != PS_DENSE && E.band_b < 0) return fail(PS_EUNSUPPORTED, "N(z) has no narrow band");
        if (E.T < 1 || E.NS < 1) E.size_for(std::max(E.T, 1));
        std::vector<double> mus = {mu};
        std::vector<char> p;
        E.build_precond({zmake(z_re, z_im)}, &mus, &p, true, true);
        HIPCHK(hipStreamSynchronize(E.st));
        *pd = p.empty() ? 0 : p[0];
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}

// The recycled singular store of one tile as the last ps_eval left it.
extern "C" ps_status ps_debug_store(ps_matrix* h, int32_t tile, int32_t* k, double* V, double* W1, double* W3,
                                    double* W4, double* RA, double* Rres)
{
    if (!h || !k || !V || !W1 || !W3 || !W4 || !RA || !Rres) return fail(PS_EINVAL, "NULL argument");
    try {
        Engine& E = h->eng;
        if (tile < 0 || tile >= E.T) return fail(PS_EINVAL, "tile out of range");
        const int K = E.K;
        const int64_t n = E.n, m = E.m;
        *k = E.tiles.size() > (size_t)tile ? E.tiles[tile].k : 0;
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(V, E.sV.p + (size_t)tile * n * K, sizeof(zd) * n * K, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(W1, E.sW1.p + (size_t)tile * m * K, sizeof(zd) * m * K, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(W3, E.sW3.p + (size_t)tile * n * K, sizeof(zd) * n * K, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(W4, E.sW4.p + (size_t)tile * n * K, sizeof(zd) * n * K, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(RA, E.sRA.p + (size_t)tile * 4 * K * K, sizeof(zd) * 4 * K * K, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(Rres, E.sRres.p + (size_t)tile * 16 * K * K, sizeof(zd) * 16 * K * K,
                         hipMemcpyDeviceToHost));
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}

// recySing (the Ritz stage) for one tile's store at z: all k Ritz values
// (ascending), their residual norms ||T(z) V g_j - xi_j^2 V g_j|| and the
// right vectors G (k x k, column-major, ld k_max).
extern "C" ps_status ps_debug_ritz(ps_matrix* h, int32_t tile, double z_re, double z_im, double* xi, double* res,
                                   double* G)
{
    if (!h || !xi || !res || !G) return fail(PS_EINVAL, "NULL argument");
    try {
        Engine& E = h->eng;
        if (tile < 0 || tile >= E.T) return fail(PS_EINVAL, "tile out of range");
        const int K = E.K;
        const int k = E.tiles[tile].k;
        if (k <= 0) return fail(PS_EINVAL, "empty store");
        DBuf<int> jt;
        DBuf<zd> jz, jg;
        DBuf<double> jn, jx, jr;
        DBuf<uint8_t> ja;
        jt.alloc(1); jz.alloc(1); jg.alloc((size_t)K * K); jn.alloc(1); jx.alloc(K); jr.alloc(K); ja.alloc(1);
        const zd z = zmake(z_re, z_im);
        const double nrm = E.op.normC + sqrt(zabs2(z));
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(jt.p, &tile, sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(jz.p, &z, sizeof(zd), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(jn.p, &nrm, sizeof(double), hipMemcpyHostToDevice));
        RitzArgs ra;
        memset(&ra, 0, sizeof(ra));
        ra.njobs = 1;
        ra.job_tile = jt.p;
        ra.kdim = E.d_k.p;
        ra.z = jz.p;
        ra.nrm = jn.p;
        ra.RA = E.sRA.p;
        ra.strideRA = (int64_t)4 * K * K;
        ra.ldRA = 2 * K;
        ra.Rres = E.sRres.p;
        ra.strideRres = (int64_t)16 * K * K;
        ra.ldRres = 4 * K;
        ra.nres = 4;
        ra.nv = k;
        ra.ng = k;
        ra.max_sweeps = 40;
        ra.mode = 0;
        ra.eta = E.P.eta;
        ra.floor_c = 16.0;
        ra.eta_abs = 0.0;
        ra.normC = E.op.normC;
        ra.xi = jx.p;
        ra.res = jr.p;
        ra.ldxi = K;
        ra.Gout = jg.p;
        ra.strideG = (int64_t)K * K;
        ra.ldG = K;
        ra.accept = ja.p;
        launch_ritz(ra, K, E.st);
        HIPCHK(hipStreamSynchronize(E.st));
        HIPCHK(hipMemcpy(xi, jx.p, sizeof(double) * k, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(res, jr.p, sizeof(double) * k, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(G, jg.p, sizeof(zd) * K * k, hipMemcpyDeviceToHost));
        return PS_OK;
    } catch (const std::exception& e) {
        return fail(PS_EDEVICE, e.what());
    }
}
