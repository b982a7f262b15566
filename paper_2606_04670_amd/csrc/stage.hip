// Small helper kernels of the bound path: data staging, partial combine,
// fills and the optional finite-value scan.
#include <climits>

#include "lip_device.hpp"
#include "lip_internal.hpp"

namespace lip {

// ---- coordinate origin ------------------------------------------------------
//
// Per coordinate, the mid-range of the data, o = fl(min / 2 + max / 2), an
// FP32 value in [min, max] (halving is exact for normal numbers and the
// rounded sum of two values in [min / 2, max / 2] stays in [min, max]).
// Pass 1: each of G workgroups reduces a strided part of the rows to
// partial (min, max) per coordinate; pass 2 (one workgroup) combines the G
// partials and writes origin[j] for the permuted coordinate j.  Rows are
// read whole, so the loads are coalesced for any d.

__global__ void __launch_bounds__(256) origin_partial_kernel(const float *x, int64_t n, int d,
                                                             float *part)
{
    __shared__ float smin[256], smax[256];
    for (int j = 0; j < d; ++j) {
        float mn = __builtin_inff(), mx = -__builtin_inff();
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
             k += (int64_t)gridDim.x * blockDim.x) {
            const float v = x[k * d + j];
            mn = fminf(mn, v);
            mx = fmaxf(mx, v);
        }
        smin[threadIdx.x] = mn;
        smax[threadIdx.x] = mx;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + h]);
                smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + h]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[((int64_t)blockIdx.x * kMaxDim + j) * 2] = smin[0];
            part[((int64_t)blockIdx.x * kMaxDim + j) * 2 + 1] = smax[0];
        }
        __syncthreads();
    }
}

struct OriginPerm {
    int32_t perm[kMaxDim];
};

// One workgroup: per coordinate, its threads take the partials in turn and
// reduce them in LDS (minima and maxima do not depend on the order).
__global__ void __launch_bounds__(256) origin_final_kernel(const float *part, int n_part, int d,
                                                           OriginPerm pm, float *origin)
{
    __shared__ float smin[256], smax[256];
    const int t = threadIdx.x;
    for (int j = 0; j < kMaxDim; ++j) {
        if (j >= d) {
            if (t == 0) origin[j] = 0.0f;
            continue;
        }
        const int c = pm.perm[j];
        float mn = __builtin_inff(), mx = -__builtin_inff();
        for (int b = t; b < n_part; b += blockDim.x) {
            mn = fminf(mn, part[((int64_t)b * kMaxDim + c) * 2]);
            mx = fmaxf(mx, part[((int64_t)b * kMaxDim + c) * 2 + 1]);
        }
        smin[t] = mn;
        smax[t] = mx;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if (t < h) {
                smin[t] = fminf(smin[t], smin[t + h]);
                smax[t] = fmaxf(smax[t], smax[t + h]);
            }
            __syncthreads();
        }
        if (t == 0) origin[j] = origin_of_range(smin[0], smax[0]);
        __syncthreads();
    }
}

// Stage the data set into records [x'_0..x'_{D-1} | y | M | yU] (see
// lip_device.hpp), padding up to n_pad by repeating the last datum.  A
// repeated record has the same candidates as the datum it copies and a
// higher index, so it never wins a tie.
template <int D>
__global__ void stage_kernel(StageArgs a)
{
    constexpr int S = Rec<D>::S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_pad; k += stride) {
        const int64_t src = k < a.n ? k : a.n - 1;
        const float *xs = a.x + src * D;
        float *o = a.out + k * S;
        float xv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) xv[j] = xf_coord(a.xf, xs, j);
        const float y = a.y[src];
        const float m = a.Mk ? a.Mk[src] : a.M;
        // l1 with monotone coordinates: yU = y - M * sum_mon x'_i (summed in
        // index order, like the per-query sum Qm).
        float yu = y;
        if (a.l1_mon > 0) {
            float s = 0.0f;
            bool first = true;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                if (j >= D - a.l1_mon) {
                    s = first ? xv[j] : s + xv[j];
                    first = false;
                }
            }
            yu = fmaf(-m, s, y);
        }
#pragma unroll
        for (int j = 0; j < D; ++j) o[j] = xv[j];
        o[Rec<D>::Y] = y;
        o[Rec<D>::M] = m;
        o[Rec<D>::YU] = yu;
    }
}

// Reduce per-chunk partials in chunk order: strict comparisons keep the
// earlier chunk (lower indices) on ties.  Writes the final outputs.
__global__ void combine_kernel(CombineArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.q; j += stride) {
        float bu = a.part_v[j];
        int iu = a.part_i[j];
        float bl = a.part_v[(int64_t)a.n_chunks * a.q + j];
        int il = a.part_i[(int64_t)a.n_chunks * a.q + j];
        for (int c = 1; c < a.n_chunks; ++c) {
            const float vu = a.part_v[(int64_t)c * a.q + j];
            const float vl = a.part_v[((int64_t)a.n_chunks + c) * a.q + j];
            if (vu < bu) {
                bu = vu;
                iu = a.part_i[(int64_t)c * a.q + j];
            }
            if (vl > bl) {
                bl = vl;
                il = a.part_i[((int64_t)a.n_chunks + c) * a.q + j];
            }
        }
        const int64_t o = a.qorder ? (int64_t)(uint32_t)a.qorder[j] : j;
        if (a.g) a.g[o] = 0.5f * (bu + bl);
        if (a.h_up) a.h_up[o] = bu;
        if (a.h_lo) a.h_lo[o] = bl;
        if (a.arg_up) a.arg_up[o] = iu;
        if (a.arg_lo) a.arg_lo[o] = il;
    }
}

// Sets flag[0] to 1 if any of the n floats is NaN or +-Inf (exponent bits
// all ones; tested on the bit pattern).
__global__ void nonfinite_kernel(const float *v, int64_t n, int *flag)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t b = __float_as_uint(v[i]);
        bad |= ((b & 0x7f800000u) == 0x7f800000u);
    }
    if (bad) atomicOr(flag, 1);
}

__global__ void fill_i32_kernel(int *p, int64_t n, int v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_stage(int d, const StageArgs &a, hipStream_t s)
{
    const int block = 256;
    const int grid = grid_for(a.n_pad, block);
    switch (d) {
#define LIP_STAGE_CASE(DD) \
    case DD: hipLaunchKernelGGL(stage_kernel<DD>, dim3(grid), dim3(block), 0, s, a); break;
        LIP_STAGE_CASE(1) LIP_STAGE_CASE(2) LIP_STAGE_CASE(3) LIP_STAGE_CASE(4)
        LIP_STAGE_CASE(5) LIP_STAGE_CASE(6) LIP_STAGE_CASE(7) LIP_STAGE_CASE(8)
        LIP_STAGE_CASE(9) LIP_STAGE_CASE(10) LIP_STAGE_CASE(11) LIP_STAGE_CASE(12)
        LIP_STAGE_CASE(13) LIP_STAGE_CASE(14) LIP_STAGE_CASE(15) LIP_STAGE_CASE(16)
#undef LIP_STAGE_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_origin(const float *x, int64_t n, int d, const int32_t *perm, float *area,
                         hipStream_t s)
{
    if (n < 1 || d < 1 || d > kMaxDim) return hipErrorInvalidValue;
    OriginPerm pm{};
    for (int j = 0; j < kMaxDim; ++j) pm.perm[j] = j < d ? perm[j] : 0;
    int64_t g = (n + 255) / 256;
    if (g > kOriginBlocks) g = kOriginBlocks;
    float *part = area + kMaxDim * 4;
    hipLaunchKernelGGL(origin_partial_kernel, dim3((unsigned)g), dim3(256), 0, s, x, n, d, part);
    hipLaunchKernelGGL(origin_final_kernel, dim3(1), dim3(256), 0, s, (const float *)part, (int)g,
                       d, pm, area);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs &a, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(combine_kernel, dim3(grid_for(a.q, block)), dim3(block), 0, s, a);
    return hipGetLastError();
}

// Spatial order of the queries: Morton code of the coordinates quantised to
// 32 / d bits (at least 1, at most 16) inside the queries' bounding box,
// packed as (code << 32 | index); positions q..P-1 are padding (~0).  Used
// by kernels whose waves do better on spatially close queries (the filtered
// l2 forward, the step-function forward); results do not depend on it.
constexpr int kBoxBlocks = 256;  // workgroups of the query bounding-box reduction

__device__ inline unsigned int f32_key(float v)
{
    const unsigned int b = __float_as_uint(v);
    return (b >> 31) ? ~b : (b | 0x80000000u);
}

__device__ inline float f32_unkey(unsigned int k)
{
    return __uint_as_float((k >> 31) ? (k & 0x7FFFFFFFu) : ~k);
}

__global__ void qbox_init_kernel(unsigned int *bb, int d)
{
    const int j = threadIdx.x;
    if (j < d) {
        bb[j] = ~0u;
        bb[kMaxDim + j] = 0u;
    }
}

// Bounding box of the queries as order keys: every thread keeps the minimum
// and maximum key of each coordinate over whole query rows (contiguous
// loads), the workgroup reduces them (shuffles, then LDS across its waves)
// and adds one atomic per coordinate and side.
__global__ void __launch_bounds__(256) qbox_kernel(const float *xq, int64_t q, int d,
                                                   unsigned int *bb)
{
    __shared__ unsigned int slo[4][kMaxDim], shi[4][kMaxDim];
    unsigned int lo[kMaxDim], hi[kMaxDim];
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        lo[j] = ~0u;
        hi[j] = 0u;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < q; k += stride) {
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) {
            if (j < d) {
                const unsigned int key = f32_key(xq[k * d + j]);
                lo[j] = key < lo[j] ? key : lo[j];
                hi[j] = key > hi[j] ? key : hi[j];
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        if (j < d) {
            unsigned int a = lo[j], b = hi[j];
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned int c = __shfl_xor(a, off), e = __shfl_xor(b, off);
                a = c < a ? c : a;
                b = e > b ? e : b;
            }
            if (lane == 0) {
                slo[wv][j] = a;
                shi[wv][j] = b;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < d) {
        const int j = threadIdx.x;
        unsigned int a = ~0u, b = 0u;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a = slo[w][j] < a ? slo[w][j] : a;
            b = shi[w][j] > b ? shi[w][j] : b;
        }
        atomicMin(bb + j, a);
        atomicMax(bb + kMaxDim + j, b);
    }
}

__global__ void qmorton_kernel(const float *xq, int64_t q, int d, int64_t P, const unsigned int *bb,
                               unsigned long long *keys)
{
    const int bits = 32 / d > 0 ? (32 / d < 16 ? 32 / d : 16) : 1;
    const float cells = (float)(1u << bits);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += stride) {
        if (k >= q) {
            keys[k] = ~0ull;
            continue;
        }
        unsigned long long code = 0;
        unsigned int c[kMaxDim];
        for (int j = 0; j < d; ++j) {
            const float lo = f32_unkey(bb[j]), hi = f32_unkey(bb[kMaxDim + j]);
            float t = hi > lo ? (xq[k * d + j] - lo) / (hi - lo) * cells : 0.0f;
            t = t < 0.0f ? 0.0f : (t > cells - 1.0f ? cells - 1.0f : t);  // NaN -> cells - 1
            c[j] = (unsigned int)t;
        }
        for (int b = bits - 1; b >= 0; --b)
            for (int j = 0; j < d; ++j) code = (code << 1) | ((c[j] >> b) & 1u);
        keys[k] = (code << 32) | (unsigned int)k;
    }
}

// Rows of the queries in their visiting order (one thread per float).
__global__ void query_gather_kernel(const float *xq, int64_t q, int d,
                                    const unsigned long long *keys, float *out)
{
    const int64_t total = q * d;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t p = e / d, j = e - p * d;
        out[e] = xq[(int64_t)(uint32_t)keys[p] * d + j];
    }
}

hipError_t launch_query_gather(const float *xq, int64_t q, int d, const unsigned long long *keys,
                               float *out, hipStream_t s)
{
    int64_t g = (q * d + 255) / 256;
    if (g > 65535) g = 65535;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(query_gather_kernel, dim3((unsigned)g), dim3(256), 0, s, xq, q, d, keys, out);
    return hipGetLastError();
}

hipError_t launch_query_order(const float *xq, int64_t q, int d, unsigned int *bb,
                              unsigned long long *keys, int64_t P, hipStream_t s)
{
    hipLaunchKernelGGL(qbox_init_kernel, dim3(1), dim3(64), 0, s, bb, d);
    int64_t gq = (q + 255) / 256;
    if (gq > kBoxBlocks) gq = kBoxBlocks;
    if (gq < 1) gq = 1;
    hipLaunchKernelGGL(qbox_kernel, dim3((unsigned)gq), dim3(256), 0, s, xq, q, d, bb);
    int64_t gp = (P + 255) / 256;
    if (gp > 65535) gp = 65535;
    hipLaunchKernelGGL(qmorton_kernel, dim3((unsigned)gp), dim3(256), 0, s, xq, q, d, P,
                       (const unsigned int *)bb, keys);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sort_u64(keys, P, s);
}

hipError_t launch_nonfinite(const float *v, int64_t n, int *flag, hipStream_t s)
{
    if (n <= 0 || !v) return hipSuccess;
    const int block = 256;
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n, block)), dim3(block), 0, s, v, n, flag);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int64_t n, int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, block)), dim3(block), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace lip
