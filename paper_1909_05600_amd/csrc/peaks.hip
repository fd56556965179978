// ffm_peaks: measured issue rates of the gfx950 units the FFM kernels are bound by.
//
//   fma32  FP32 FMA (non-packed)            -> TFLOP/s (2 flops per FMA)
//   fma64  FP64 FMA                         -> TFLOP/s
//   mfma32 FP32 matrix core, 16x16x4 blocks -> TFLOP/s (2 flops per multiply-add)
//   sin    v_sin_f32 (revolutions)          -> G evaluations/s
//   pw32   plane-wave transform inner step  -> G (point, direction-pair) updates/s, FP32 phase
//   pw64   the same with an FP64 phase      -> G updates/s
//   copy   float4 device copy               -> GB/s (read + write)
//
// Every kernel runs a fixed grid with no global memory access except copy (bounds-checked), and
// writes one value per thread so the compiler keeps the arithmetic.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e = (x);                                                               \
        if (e != hipSuccess) {                                                            \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));                   \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

constexpr int kIter = 2048;
constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) k_fma32(float *out, float b, float c) {
    float a[8];
    for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-3f + i;
    for (int it = 0; it < kIter; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = fmaf(a[i], b, c);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_fma64(double *out, double b, double c) {
    double a[8];
    for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-3 + i;
    for (int it = 0; it < kIter; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = fma(a[i], b, c);
    double s = 0.0;
    for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Eight independent accumulator tiles per wave, so that the matrix pipe never waits on a result.
typedef float floatx4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kThreads) k_mfma32(float *out, float b) {
    floatx4 acc[8];
    for (int i = 0; i < 8; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float a = threadIdx.x * 1e-3f;
    for (int it = 0; it < kIter; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_sin(float *out) {
    float a[8];
    for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-4f + 0.1f * i;
    for (int it = 0; it < kIter; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_sinf(a[i]);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// The inner step of the plane-wave transform: for 4 direction pairs and a stream of points,
// phase = s . y (3 ops), fract, sin, cos, 4 FMAs of accumulation.
template <bool P64>
__global__ void __launch_bounds__(kThreads) k_pw(float *out, float dx) {
    typedef typename std::conditional<P64, double, float>::type real;
    real sx[4], sy[4], sz[4];
    float acc[4][4];
    for (int j = 0; j < 4; ++j) {
        sx[j] = (real)(0.3 + 0.01 * j + threadIdx.x * 1e-5);
        sy[j] = (real)(-0.2 + 0.02 * j);
        sz[j] = (real)(0.7 - 0.01 * j);
        for (int q = 0; q < 4; ++q) acc[j][q] = 0.f;
    }
    real x = (real)(threadIdx.x * 1e-3), y = (real)0.25, z = (real)-0.125;
    float ur = 1.f, ui = 0.5f;
    for (int it = 0; it < kIter; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float f;
            if (P64) {
                const double ph = fma((double)sx[j], (double)x, fma((double)sy[j], (double)y, (double)sz[j] * z));
                f = (float)__builtin_amdgcn_fract(ph);
            } else {
                const float ph = fmaf((float)sx[j], (float)x, fmaf((float)sy[j], (float)y, (float)sz[j] * (float)z));
                f = __builtin_amdgcn_fractf(ph);
            }
            const float sn = __builtin_amdgcn_sinf(f), cs = __builtin_amdgcn_cosf(f);
            acc[j][0] = fmaf(cs, ur, acc[j][0]);
            acc[j][1] = fmaf(cs, ui, acc[j][1]);
            acc[j][2] = fmaf(sn, ur, acc[j][2]);
            acc[j][3] = fmaf(sn, ui, acc[j][3]);
        }
        x += (real)dx;   // next "point"
    }
    float s = 0.f;
    for (int j = 0; j < 4; ++j)
        for (int q = 0; q < 4; ++q) s += acc[j][q];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_copy(const float4 *a, float4 *b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) b[i] = a[i];
}

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int ncu = prop.multiProcessorCount;
    const int grid = ncu * 32;   // 32 blocks of 256 threads per CU
    const double threads = (double)grid * kThreads;
    float *of;
    double *od;
    CHECK(hipMalloc(&of, sizeof(float) * grid * kThreads));
    CHECK(hipMalloc(&od, sizeof(double) * grid * kThreads));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto timeit = [&](auto launch) {
        launch();
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0));
        for (int r = 0; r < 5; ++r) launch();
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        return ms / 5.0 * 1e-3;
    };
    double t;
    std::printf("device: %s, %d CUs, clock %.0f MHz\n", prop.name, ncu, prop.clockRate / 1e3);
    t = timeit([&] { hipLaunchKernelGGL(k_fma32, dim3(grid), dim3(kThreads), 0, 0, of, 0.999f, 1e-3f); });
    std::printf("fma32  %8.2f TFLOP/s\n", threads * kIter * 8 * 2 / t / 1e12);
    t = timeit([&] { hipLaunchKernelGGL(k_fma64, dim3(grid), dim3(kThreads), 0, 0, od, 0.999, 1e-3); });
    std::printf("fma64  %8.2f TFLOP/s\n", threads * kIter * 8 * 2 / t / 1e12);
    t = timeit([&] { hipLaunchKernelGGL(k_mfma32, dim3(grid / 4), dim3(kThreads), 0, 0, of, 0.999f); });
    // per wave and iteration: 8 products of 16 x 16 x 4 multiply-adds
    std::printf("mfma32 %8.2f TFLOP/s\n", (double)grid / 4 * (kThreads / 64) * kIter * 8 * 16 * 16 * 4 * 2 / t / 1e12);
    t = timeit([&] { hipLaunchKernelGGL(k_sin, dim3(grid), dim3(kThreads), 0, 0, of); });
    const double sin_rate = threads * kIter * 8 / t;
    std::printf("sin    %8.2f G/s  (%.2f lanes/clk/CU)\n", sin_rate / 1e9, sin_rate / (ncu * prop.clockRate * 1e3));
    t = timeit([&] { hipLaunchKernelGGL(k_pw<false>, dim3(grid), dim3(kThreads), 0, 0, of, 1e-6f); });
    double r = threads * kIter * 4 / t;
    std::printf("pw32   %8.2f G pair-updates/s  (%.2f cycles per update per lane)\n", r / 1e9,
                ncu * 64.0 * prop.clockRate * 1e3 / r);
    t = timeit([&] { hipLaunchKernelGGL(k_pw<true>, dim3(grid), dim3(kThreads), 0, 0, of, 1e-6f); });
    r = threads * kIter * 4 / t;
    std::printf("pw64   %8.2f G pair-updates/s  (%.2f cycles per update per lane)\n", r / 1e9,
                ncu * 64.0 * prop.clockRate * 1e3 / r);
    const size_t n = (size_t)1 << 26;   // 64 Mi float4 = 1 GiB each way
    float4 *a, *b;
    CHECK(hipMalloc(&a, n * sizeof(float4)));
    CHECK(hipMalloc(&b, n * sizeof(float4)));
    CHECK(hipMemset(a, 0, n * sizeof(float4)));
    t = timeit([&] { hipLaunchKernelGGL(k_copy, dim3(ncu * 16), dim3(kThreads), 0, 0, a, b, n); });
    std::printf("copy   %8.1f GB/s (read + write)\n", 2.0 * n * sizeof(float4) / t / 1e9);
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(of));
    CHECK(hipFree(od));
    return 0;
}
