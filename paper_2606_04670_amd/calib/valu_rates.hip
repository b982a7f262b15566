// Throughput calibration for the rooflines of the kernels: each lane runs 16
// independent dependency chains of one VALU instruction kind (or each wave 4
// chains of one MFMA), the kernel is timed with hip events and the rate
// reported in lane-operations (FLOP for the MFMA) per second.
//   valu_rates [blocks]   rates (default 4096 blocks x 256 threads, about 16
//                         waves per SIMD on 256 CUs)
//   valu_rates copy       a plain 1 GiB device-to-device copy kernel, run
//                         twice: the reference for the HBM byte counters
//                         (FETCH_SIZE / WRITE_SIZE) of rocprofv3.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CH 16

#define OP_KERNEL(NAME, TYPE, ASM)                                                      \
    __global__ void __launch_bounds__(256) NAME(TYPE *out, int iters, TYPE b)          \
    {                                                                                   \
        TYPE a[CH];                                                                     \
        for (int j = 0; j < CH; ++j) a[j] = (TYPE)(threadIdx.x + j);                    \
        for (int it = 0; it < iters; ++it) {                                            \
            _Pragma("unroll") for (int j = 0; j < CH; ++j) asm volatile(ASM : "+v"(a[j]) : "v"(b)); \
        }                                                                               \
        TYPE s = 0;                                                                     \
        for (int j = 0; j < CH; ++j) s += a[j];                                         \
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;                                 \
    }

OP_KERNEL(k_add_f32, float, "v_add_f32 %0, %0, %1")
OP_KERNEL(k_sub_f32, float, "v_sub_f32 %0, %0, %1")
OP_KERNEL(k_fma_f32, float, "v_fma_f32 %0, %0, %1, %1")
OP_KERNEL(k_max_f32, float, "v_max_f32 %0, %0, %1")
OP_KERNEL(k_med3_f32, float, "v_med3_f32 %0, %0, %1, %1")
OP_KERNEL(k_min3_f32, float, "v_min3_f32 %0, %0, %1, %1")
OP_KERNEL(k_sqrt_f32, float, "v_sqrt_f32 %0, %1")
OP_KERNEL(k_minimum3_f32, float, "v_minimum3_f32 %0, %0, %1, %1")
OP_KERNEL(k_add_f64, double, "v_add_f64 %0, %0, %1")
OP_KERNEL(k_fma_f64, double, "v_fma_f64 %0, %0, %1, %1")
OP_KERNEL(k_mul_f64, double, "v_mul_f64 %0, %0, %1")
OP_KERNEL(k_max_f64, double, "v_max_f64 %0, %0, %1")

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// 4 independent accumulator chains of v_mfma_f32_32x32x16_bf16 per wave.
__global__ void __launch_bounds__(256) k_mfma_bf16(float *out, int iters, float b)
{
    bf16x8 x;
    for (int e = 0; e < 8; ++e) x[e] = (__bf16)(b * (float)(threadIdx.x + e));
    f32x16 acc[4] = {};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, x, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
    for (int c = 0; c < 4; ++c)
        for (int e = 0; e < 16; ++e) s += acc[c][e];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_copy(const float4 *a, float4 *b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

static void check(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        exit(1);
    }
}

template <typename T, void (*K)(T *, int, T)>
static void run(const char *name, int blocks, int iters)
{
    T *out = nullptr;
    check(hipMalloc(&out, sizeof(T) * (size_t)blocks * 256), "hipMalloc");
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "event");
    check(hipEventCreate(&e1), "event");
    hipLaunchKernelGGL(K, dim3(blocks), dim3(256), 0, 0, out, 16, (T)1);
    check(hipDeviceSynchronize(), "warm-up");
    check(hipEventRecord(e0), "record");
    hipLaunchKernelGGL(K, dim3(blocks), dim3(256), 0, 0, out, iters, (T)1);
    check(hipEventRecord(e1), "record");
    check(hipEventSynchronize(e1), "sync");
    float ms = 0;
    check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    const double ops = (double)blocks * 256 * iters * CH;
    printf("%-9s blocks=%d  %8.3f ms  %8.3f T lane-ops/s\n", name, blocks, ms, ops / ms / 1e9);
    check(hipFree(out), "hipFree");
}

static void copy_reference()
{
    const size_t bytes = 1ull << 30, n = bytes / sizeof(float4);
    float4 *a = nullptr, *b = nullptr;
    check(hipMalloc(&a, bytes), "hipMalloc");
    check(hipMalloc(&b, bytes), "hipMalloc");
    check(hipMemset(a, 0, bytes), "memset");
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "event");
    check(hipEventCreate(&e1), "event");
    for (int r = 0; r < 2; ++r) {
        check(hipEventRecord(e0), "record");
        hipLaunchKernelGGL(k_copy, dim3(8192), dim3(256), 0, 0, a, b, n);
        check(hipEventRecord(e1), "record");
        check(hipEventSynchronize(e1), "sync");
        float ms = 0;
        check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        printf("copy run %d: %zu bytes read, %zu bytes written, %.3f ms, %.1f GB/s\n", r, bytes,
               bytes, ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
    }
    check(hipFree(a), "free");
    check(hipFree(b), "free");
}

static void run_mfma(int blocks, int iters)
{
    float *out = nullptr;
    check(hipMalloc(&out, sizeof(float) * (size_t)blocks * 256), "hipMalloc");
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "event");
    check(hipEventCreate(&e1), "event");
    hipLaunchKernelGGL(k_mfma_bf16, dim3(blocks), dim3(256), 0, 0, out, 16, 1.0f);
    check(hipDeviceSynchronize(), "warm-up");
    check(hipEventRecord(e0), "record");
    hipLaunchKernelGGL(k_mfma_bf16, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0f);
    check(hipEventRecord(e1), "record");
    check(hipEventSynchronize(e1), "sync");
    float ms = 0;
    check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    const double flop = (double)blocks * 4 /* waves */ * iters * 4 /* chains */ * 32.0 * 32 * 16 * 2;
    printf("%-12s %8.3f ms  %8.2f TFLOP/s\n", "mfma_bf16_32x32x16", ms, flop / (ms * 1e-3) / 1e12);
    check(hipFree(out), "free");
}

int main(int argc, char **argv)
{
    if (argc > 1 && argv[1][0] == 'c') {
        copy_reference();
        return 0;
    }
    const int blocks = argc > 1 ? atoi(argv[1]) : 4096;
    if (blocks < 1 || blocks > 65536) return 2;
    hipDeviceProp_t p;
    check(hipGetDeviceProperties(&p, 0), "props");
    printf("%s CUs=%d clock=%d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
    run<float, k_add_f32>("add_f32", blocks, 20000);
    run<float, k_sub_f32>("sub_f32", blocks, 20000);
    run<float, k_fma_f32>("fma_f32", blocks, 20000);
    run<float, k_max_f32>("max_f32", blocks, 20000);
    run<float, k_med3_f32>("med3_f32", blocks, 20000);
    run<float, k_min3_f32>("min3_f32", blocks, 20000);
    run<float, k_sqrt_f32>("sqrt_f32", blocks, 5000);
    run<float, k_minimum3_f32>("minimum3_f32", blocks, 20000);
    run<double, k_add_f64>("add_f64", blocks, 10000);
    run<double, k_fma_f64>("fma_f64", blocks, 10000);
    run<double, k_mul_f64>("mul_f64", blocks, 10000);
    run<double, k_max_f64>("max_f64", blocks, 10000);
    run_mfma(blocks, 2000);
    return 0;
}
