// Measured peaks of the GPU this runs on, to set beside the datasheet figures
// that the roofline fractions use: HBM bandwidth (a device-to-device copy
// kernel), FP64 vector FMA rate and FP64 matrix-core rate
// (v_mfma_f64_16x16x4f64).  Build: see build_peaks() in build.py; run with no
// arguments; prints one line per probe.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                         \
        }                                                                                     \
    } while (0)

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef double dvec4 __attribute__((ext_vector_type(4)));

// dst[i] = src[i] over n 16-byte elements, grid-stride
__global__ void __launch_bounds__(256) k_copy(const dvec2* __restrict__ src, dvec2* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// 8 independent FMA chains per thread, iters steps each; one result per thread
__global__ void __launch_bounds__(256) k_fma(double* out, int iters, double a, double b)
{
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = threadIdx.x * 1e-9 + j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = fma(x[j], a, b);
    }
    double s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 independent accumulator blocks per wave, iters steps of 8 MFMAs each
__global__ void __launch_bounds__(256) k_mfma(double* out, int iters, double a)
{
    dvec4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = (dvec4){0.0, 0.0, 0.0, 0.0};
    const double av = a + threadIdx.x * 1e-12, bv = 1.0 - threadIdx.x * 1e-12;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
    }
    double s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    std::printf("device %s, %d compute units\n", prop.name, cus);

    // copy: 2 GiB read + 2 GiB written per launch
    const int64_t n = (int64_t)1 << 27;   // 16-byte elements: 2 GiB
    dvec2 *src = nullptr, *dst = nullptr;
    CHECK(hipMalloc(&src, sizeof(dvec2) * n));
    CHECK(hipMalloc(&dst, sizeof(dvec2) * n));
    CHECK(hipMemset(src, 0, sizeof(dvec2) * n));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const int cblocks = cus * 16;
    for (int r = 0; r < 2; ++r) hipLaunchKernelGGL(k_copy, dim3(cblocks), dim3(256), 0, 0, src, dst, n);
    CHECK(hipEventRecord(e0, 0));
    const int creps = 10;
    for (int r = 0; r < creps; ++r) hipLaunchKernelGGL(k_copy, dim3(cblocks), dim3(256), 0, 0, src, dst, n);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double gbs = 2.0 * sizeof(dvec2) * n * creps / (ms * 1e-3) / 1e9;
    std::printf("hbm copy: %.1f GB/s (read + write, 2 GiB each way per launch)\n", gbs);
    CHECK(hipFree(src));
    CHECK(hipFree(dst));

    // FP64 vector FMA: blocks x 256 threads x 8 chains x iters FMAs
    const int blocks = cus * 8, iters = 1 << 12;
    double* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(double) * blocks * 256));
    hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999999, 1e-7);
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999999, 1e-7);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double vf = 2.0 * blocks * 256.0 * 8.0 * iters / (ms * 1e-3) / 1e12;
    std::printf("fp64 vector fma: %.1f TFLOP/s\n", vf);

    // FP64 matrix cores: blocks x 4 waves x 8 MFMAs x iters, 2 * 16 * 16 * 4 flops each
    const int miters = 1 << 10;
    hipLaunchKernelGGL(k_mfma, dim3(blocks), dim3(256), 0, 0, out, miters, 1e-3);
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(k_mfma, dim3(blocks), dim3(256), 0, 0, out, miters, 1e-3);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double mf = 2048.0 * blocks * 4.0 * 8.0 * miters / (ms * 1e-3) / 1e12;
    std::printf("fp64 mfma 16x16x4: %.1f TFLOP/s\n", mf);
    CHECK(hipGetLastError());
    CHECK(hipFree(out));
    return 0;
}
