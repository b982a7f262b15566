// Ascending in-place sort of 64-bit keys (bitonic network): one kernel sorts
// blocks of 1024 keys in LDS, then each merge stage runs its long-distance
// steps over the whole array and finishes its steps below 1024 in LDS.
// Deterministic; used for the (y, index) order of the BF16 l2 path and the
// spatial (Morton code, index) order of the kNN pass.
#include "lip_internal.hpp"

namespace lip {
namespace {

constexpr int kSortBlock = 1024;

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

// All stages k <= kSortBlock inside one block of kSortBlock keys.
__global__ void __launch_bounds__(512) bitonic_local_kernel(unsigned long long *keys)
{
    __shared__ unsigned long long s[kSortBlock];
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    const int t = threadIdx.x;
    s[t] = keys[base + t];
    s[t + 512] = keys[base + t + 512];
    for (int k = 2; k <= kSortBlock; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            const int i = (t / j) * 2 * j + (t % j);
            cswap(s[i], s[i + j], ((base + i) & k) == 0);
        }
    }
    __syncthreads();
    keys[base + t] = s[t];
    keys[base + t + 512] = s[t + 512];
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

// The steps j < kSortBlock of stage k inside one block.
__global__ void __launch_bounds__(512) bitonic_merge_kernel(unsigned long long *keys, int64_t k)
{
    __shared__ unsigned long long s[kSortBlock];
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    const int t = threadIdx.x;
    s[t] = keys[base + t];
    s[t + 512] = keys[base + t + 512];
    for (int j = kSortBlock / 2; j > 0; j >>= 1) {
        __syncthreads();
        const int i = (t / j) * 2 * j + (t % j);
        cswap(s[i], s[i + j], ((base + i) & k) == 0);
    }
    __syncthreads();
    keys[base + t] = s[t];
    keys[base + t + 512] = s[t + 512];
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
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(nblk), dim3(512), 0, s, keys);
    int64_t g = P / 2 / 256;
    if (g > 65536) g = 65536;
    for (int64_t k = 2 * kSortBlock; k <= P; k *= 2) {
        for (int64_t j = k / 2; j >= kSortBlock; j /= 2)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3((unsigned)g), dim3(256), 0, s, keys, P,
                               k, j);
        hipLaunchKernelGGL(bitonic_merge_kernel, dim3(nblk), dim3(512), 0, s, keys, k);
    }
    return hipGetLastError();
}

}  // namespace lip
