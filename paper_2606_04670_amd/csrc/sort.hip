// Ascending in-place sort of 64-bit keys (bitonic network): one kernel sorts
// blocks of kSortBlock keys in LDS, then each merge stage runs its
// long-distance steps over the whole array (two steps per pass where it has
// two, each thread holding four keys) and finishes its steps below
// kSortBlock in LDS.  Deterministic; used for the (y, index) order of the
// BF16 l2 path and the spatial (Morton code, index) orders of the kNN pass
// and of the queries.
#include "lip_internal.hpp"

namespace lip {
namespace {

constexpr int kSortBlock = 4096;   // keys per LDS block (32 KiB)
constexpr int kSortThreads = 1024; // threads per LDS block; each takes 2 pairs a step

__device__ __forceinline__ void cswap(unsigned long long &a, unsigned long long &b, bool asc)
{
    if ((a > b) == asc) {
        const unsigned long long t = a;
        a = b;
        b = t;
    }
}

// Bitonic network, ascending overall: a pair (i, i + j) inside a run of
// length k is ordered ascending when bit k of i is clear.

// Steps j = j0, j0 / 2, ..., 1 of stage k on the block's keys in LDS.
__device__ __forceinline__ void lds_steps(unsigned long long *s, int64_t base, int64_t k, int j0)
{
    for (int j = j0; j > 0; j >>= 1) {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < kSortBlock / 2 / kSortThreads; ++h) {
            const int t = threadIdx.x + h * kSortThreads;
            const int i = (t / j) * 2 * j + (t % j);
            cswap(s[i], s[i + j], ((base + i) & k) == 0);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void lds_load(unsigned long long *s, const unsigned long long *keys,
                                         int64_t base)
{
    for (int e = threadIdx.x; e < kSortBlock; e += kSortThreads) s[e] = keys[base + e];
}

__device__ __forceinline__ void lds_store(const unsigned long long *s, unsigned long long *keys,
                                          int64_t base)
{
    for (int e = threadIdx.x; e < kSortBlock; e += kSortThreads) keys[base + e] = s[e];
}

// All stages k <= kSortBlock inside one block of kSortBlock keys.
__global__ void __launch_bounds__(kSortThreads) bitonic_local_kernel(unsigned long long *keys)
{
    __shared__ unsigned long long s[kSortBlock];
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    lds_load(s, keys, base);
    for (int k = 2; k <= kSortBlock; k <<= 1) lds_steps(s, base, k, k >> 1);
    lds_store(s, keys, base);
}

// One stage-k step of distance j >= kSortBlock over the whole array.
__global__ void bitonic_global_kernel(unsigned long long *keys, int64_t P, int64_t k, int64_t j)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P / 2; t += stride) {
        const int64_t i = (t / j) * 2 * j + (t % j);
        unsigned long long a = keys[i], b = keys[i + j];
        cswap(a, b, (i & k) == 0);
        keys[i] = a;
        keys[i + j] = b;
    }
}

// Two steps of stage k, distances 2 h and h (h >= kSortBlock), in one pass:
// the keys i, i + h, i + 2 h, i + 3 h (bits h and 2 h of i clear) meet only
// each other in both steps, and all four have the same direction (k > 2 h).
__global__ void bitonic_global2_kernel(unsigned long long *keys, int64_t P, int64_t k, int64_t h)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P / 4; t += stride) {
        const int64_t i = (t / h) * 4 * h + (t % h);
        unsigned long long a0 = keys[i], a1 = keys[i + h], a2 = keys[i + 2 * h],
                           a3 = keys[i + 3 * h];
        const bool asc = (i & k) == 0;
        cswap(a0, a2, asc);
        cswap(a1, a3, asc);
        cswap(a0, a1, asc);
        cswap(a2, a3, asc);
        keys[i] = a0;
        keys[i + h] = a1;
        keys[i + 2 * h] = a2;
        keys[i + 3 * h] = a3;
    }
}

// The steps j < kSortBlock of stage k inside one block.
__global__ void __launch_bounds__(kSortThreads) bitonic_merge_kernel(unsigned long long *keys,
                                                                    int64_t k)
{
    __shared__ unsigned long long s[kSortBlock];
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    lds_load(s, keys, base);
    lds_steps(s, base, k, kSortBlock / 2);
    lds_store(s, keys, base);
}

}  // namespace

int64_t sort_len(int64_t n)
{
    int64_t P = kSortBlock;
    while (P < n) P *= 2;
    return P;
}

hipError_t launch_sort_u64(unsigned long long *keys, int64_t P, hipStream_t s)
{
    if (P < kSortBlock || (P & (P - 1)) != 0) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)(P / kSortBlock);
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(nblk), dim3(kSortThreads), 0, s, keys);
    int64_t g = P / 2 / 256, g2 = P / 4 / 256;
    if (g > 65536) g = 65536;
    if (g2 > 65536) g2 = 65536;
    for (int64_t k = 2 * kSortBlock; k <= P; k *= 2) {
        int64_t j = k / 2;
        for (; j >= 2 * kSortBlock; j /= 4)
            hipLaunchKernelGGL(bitonic_global2_kernel, dim3((unsigned)g2), dim3(256), 0, s, keys,
                               P, k, j / 2);
        if (j >= kSortBlock)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3((unsigned)g), dim3(256), 0, s, keys, P,
                               k, j);
        hipLaunchKernelGGL(bitonic_merge_kernel, dim3(nblk), dim3(kSortThreads), 0, s, keys, k);
    }
    return hipGetLastError();
}

}  // namespace lip
