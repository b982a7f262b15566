// VALU throughput calibration for the roofline of the bound kernels: each
// lane runs 16 independent dependency chains of one instruction kind, the
// kernel is timed with hip events and the rate reported in lane-operations
// per second.  Usage: valu_rates [blocks]   (default 4096 blocks x 256 threads,
// about 16 waves per SIMD on 256 CUs).
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
OP_KERNEL(k_add_f64, double, "v_add_f64 %0, %0, %1")
OP_KERNEL(k_fma_f64, double, "v_fma_f64 %0, %0, %1, %1")
OP_KERNEL(k_mul_f64, double, "v_mul_f64 %0, %0, %1")
OP_KERNEL(k_max_f64, double, "v_max_f64 %0, %0, %1")

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

int main(int argc, char **argv)
{
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
    run<double, k_add_f64>("add_f64", blocks, 10000);
    run<double, k_fma_f64>("fma_f64", blocks, 10000);
    run<double, k_mul_f64>("mul_f64", blocks, 10000);
    run<double, k_max_f64>("max_f64", blocks, 10000);
    return 0;
}
