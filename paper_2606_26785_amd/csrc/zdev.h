// Complex double and double-double helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double2 zd;  // (x, y) = (re, im), 16-byte aligned

__host__ __device__ inline zd zmake(double x, double y) { zd r; r.x = x; r.y = y; return r; }
__host__ __device__ inline zd zadd(zd a, zd b) { return zmake(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zd zsub(zd a, zd b) { return zmake(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zd zmul(zd a, zd b) { return zmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
__host__ __device__ inline zd zcmul(zd a, zd b) { return zmake(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__host__ __device__ inline zd zconj(zd a) { return zmake(a.x, -a.y); }
__host__ __device__ inline zd zscale(zd a, double s) { return zmake(a.x * s, a.y * s); }
__host__ __device__ inline double zabs2(zd a) { return a.x * a.x + a.y * a.y; }
// acc += a * b
__host__ __device__ inline void zfma(zd& acc, zd a, zd b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__host__ __device__ inline void zcfma(zd& acc, zd a, zd b) {
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (unevaluated sums hi + lo) from the error-free
// transformations of Knuth (two-sum) and Dekker (two-product, here with a
// fused multiply-add).
struct ddv { double hi, lo; };

__host__ __device__ inline ddv dd_make(double a) { ddv r; r.hi = a; r.lo = 0.0; return r; }
__host__ __device__ inline void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__host__ __device__ inline void fast_two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    e = b - (s - a);
}
__host__ __device__ inline void two_prod(double a, double b, double& p, double& e) {
    p = a * b;
    e = fma(a, b, -p);
}
__host__ __device__ inline ddv dd_add(ddv a, ddv b) {
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    ddv r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}
__host__ __device__ inline ddv dd_neg(ddv a) { ddv r; r.hi = -a.hi; r.lo = -a.lo; return r; }
__host__ __device__ inline ddv dd_sub(ddv a, ddv b) { return dd_add(a, dd_neg(b)); }
__host__ __device__ inline ddv dd_mul(ddv a, ddv b) {
    double p, e;
    two_prod(a.hi, b.hi, p, e);
    e += a.hi * b.lo + a.lo * b.hi;
    ddv r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
}
// exact product of two doubles as a double-double
__host__ __device__ inline ddv dd_prod(double a, double b) {
    ddv r;
    two_prod(a, b, r.hi, r.lo);
    return r;
}
__host__ __device__ inline ddv dd_div(ddv a, ddv b) {
    double q1 = a.hi / b.hi;
    ddv r = dd_sub(a, dd_mul(dd_make(q1), b));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul(dd_make(q2), b));
    double q3 = r.hi / b.hi;
    double s, e;
    fast_two_sum(q1, q2, s, e);
    ddv out = dd_add(ddv{s, e}, dd_make(q3));
    return out;
}
__host__ __device__ inline ddv dd_sqrt(ddv a) {
    if (a.hi <= 0.0) return dd_make(0.0);
    double x = sqrt(a.hi);
    // one Newton step in double-double: x + (a - x^2) / (2x)
    ddv x2 = dd_prod(x, x);
    ddv d = dd_sub(a, x2);
    double corr = d.hi / (2.0 * x);
    double s, e;
    fast_two_sum(x, corr, s, e);
    ddv r; r.hi = s; r.lo = e;
    return r;
}

// complex double-double
struct zdd { ddv x, y; };
__host__ __device__ inline zdd zdd_zero() { zdd r; r.x = dd_make(0); r.y = dd_make(0); return r; }
__host__ __device__ inline zdd zdd_add(zdd a, zdd b) { zdd r; r.x = dd_add(a.x, b.x); r.y = dd_add(a.y, b.y); return r; }
__host__ __device__ inline zdd zdd_sub(zdd a, zdd b) { zdd r; r.x = dd_sub(a.x, b.x); r.y = dd_sub(a.y, b.y); return r; }
// conj(a) * b with a, b complex double-double
__host__ __device__ inline zdd zdd_cmul(zdd a, zdd b) {
    zdd r;
    r.x = dd_add(dd_mul(a.x, b.x), dd_mul(a.y, b.y));
    r.y = dd_sub(dd_mul(a.x, b.y), dd_mul(a.y, b.x));
    return r;
}
__host__ __device__ inline zdd zdd_scale(zdd a, ddv s) { zdd r; r.x = dd_mul(a.x, s); r.y = dd_mul(a.y, s); return r; }

// Compensated accumulator for conj(a) * b summed over many terms: every
// product is split exactly into a double-double, the running sums are
// double-doubles.
struct zacc {
    double sx, ex, sy, ey;  // re = sx + ex, im = sy + ey
};
__host__ __device__ inline void zacc_init(zacc& a) { a.sx = a.ex = a.sy = a.ey = 0.0; }
__host__ __device__ inline void acc_add_prod(double& s, double& e, double a, double b) {
    double p, pe, t, te;
    two_prod(a, b, p, pe);
    two_sum(s, p, t, te);
    s = t;
    e += pe + te;
}
__host__ __device__ inline void zacc_cfma(zacc& acc, zd a, zd b) {
    // re: a.x b.x + a.y b.y ; im: a.x b.y - a.y b.x
    acc_add_prod(acc.sx, acc.ex, a.x, b.x);
    acc_add_prod(acc.sx, acc.ex, a.y, b.y);
    acc_add_prod(acc.sy, acc.ey, a.x, b.y);
    acc_add_prod(acc.sy, acc.ey, -a.y, b.x);
}
__host__ __device__ inline zdd zacc_value(const zacc& a) {
    zdd r;
    fast_two_sum(a.sx, a.ex, r.x.hi, r.x.lo);
    fast_two_sum(a.sy, a.ey, r.y.hi, r.y.lo);
    return r;
}

// ---------------------------------------------------------------------------
// Wavefront and block reductions (64-wide wavefronts on gfx950).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// sum within aligned groups of `width` lanes (power of two <= 64)
__device__ inline double group_sum(double v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// block-wide sum; `red` must hold at least blockDim.x/64 doubles; all threads get the result
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}
__device__ inline double block_max(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
    return s;
}

// counter-based random numbers (SplitMix64 finaliser), used for start blocks
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline double u01(uint64_t key) {
    return ((mix64(key) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
