// Penalty objective of the smoothing problem (Sec. 4.4, Eq. 7) and its
// gradient, as one fused pass over all ordered pairs (no distance matrix):
//     a_ik = z_i - z_k - M_k dist_up(x^i, x^k)        (constraint of Eq. 5)
//     b_ik = z_k - z_i - M_k dist_lo(x^i, x^k)        (constraint of Eq. 6)
//     F    = (1/p) ||eps||^2 + sum_{i != k} (a_ik)_+^2 + (b_ik)_+^2,   z = y + eps
//     dF/d eps_i = 2 eps_i / p + sum_k [ 2 (a_ik)_+ - 2 (b_ik)_+ - 2 (a_ki)_+ + 2 (b_ki)_+ ].
// Row i's pass over every k forms the pair's two directional distances once
// and gets both of its roles from them: dist_up(x^k, x^i) = dist_lo(x^i, x^k),
// so a_ki = z_k - z_i - M_i dist_lo(x^i, x^k) and b_ki = z_i - z_k - M_i
// dist_up(x^i, x^k).  With one global M, a_ki = b_ik and b_ki = a_ik, and the
// row's gradient is 4 (a_ik)_+ - 4 (b_ik)_+ per pair.  The diagonal k = i
// contributes exactly zero (both distances and differences are 0).
//
// Arithmetic: the pair terms in FP32 (distances with the bound path's FP32
// arithmetic on its staged coordinates), summed in FP32 over one tile of 64
// columns and then in FP64; per-chunk row partials are combined in chunk
// order and the objective is reduced over rows in a fixed order, so repeated
// calls give identical results.
//
// Work split: a lane owns R rows (queries of the bound path's layout), a
// wave 64 R rows and one column chunk; columns arrive four at a time through
// scalar loads of records [x'_0..x'_{D-1} | z | M_k].
#pragma once

#include "local_fwd.hpp"

namespace lip {

constexpr int kSmoothMaxChunks = 32;
constexpr int kSmoothTile = 64;

struct SmoothArgs {
    const float *rec;      // [npad][D + 2]: x' (bound-path transform), z = y + eps, M_k
    int64_t n, npad;
    int32_t n_chunks;
    int32_t pad0;
    int64_t chunk_cols;    // multiple of kSmoothTile
    double *pF, *pG;       // [n_chunks][n] row partials
};

template <int D, int DM, int NORM, bool LOCAL>
__global__ void __launch_bounds__(256) smooth_kernel(SmoothArgs A)
{
    constexpr int R = rows_for_dim(D);
    constexpr int S = D + 2;
    constexpr int G = 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % A.n_chunks;
    const int64_t rb = (int64_t)(blockIdx.x / A.n_chunks) * (blockDim.x >> 6) + wave;
    const int64_t r0 = rb * 64 * R;
    if (r0 >= A.n) return;
    const int lane = threadIdx.x & 63;
    float xr[R][D], zr[R], mr[R], f32[R], g32[R];
    double f64[R], g64[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = r0 + r * 64 + lane;
        i = i < A.n ? i : A.n - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.rec[i * S + j];
        zr[r] = A.rec[i * S + D];
        mr[r] = A.rec[i * S + D + 1];
        f32[r] = 0.0f;
        g32[r] = 0.0f;
        f64[r] = 0.0;
        g64[r] = 0.0;
    }
    const int64_t c0 = (int64_t)chunk * A.chunk_cols;
    int64_t c1 = c0 + A.chunk_cols;
    c1 = c1 < A.n ? c1 : A.n;
    const cfloat_ptr rec = as_const(A.rec);
#pragma unroll 1
    for (int64_t t0 = c0; t0 < c1; t0 += kSmoothTile) {
        const int64_t t1 = t0 + kSmoothTile < c1 ? t0 + kSmoothTile : c1;
#pragma unroll 1
        for (int64_t g0 = t0; g0 < t1; g0 += G) {
            float v[G * S];
#pragma unroll
            for (int e = 0; e < G * S; ++e) v[e] = rec[g0 * S + e];
#pragma unroll
            for (int c = 0; c < G; ++c) {
                if (g0 + c >= t1) break;  // wave-uniform
                const float *xk = v + c * S;
                const float zk = xk[D], mk = xk[D + 1];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float du, dl;
                    step_dist32<D, DM, NORM>(xr[r], xk, du, dl);
                    const float dz = zr[r] - zk;
                    const float a = fmaxf(fmaf(-mk, du, dz), 0.0f);
                    const float b = fmaxf(fmaf(-mk, dl, -dz), 0.0f);
                    f32[r] = fmaf(a, a, fmaf(b, b, f32[r]));
                    if constexpr (LOCAL) {
                        const float a2 = fmaxf(fmaf(-mr[r], dl, -dz), 0.0f);  // a_ki
                        const float b2 = fmaxf(fmaf(-mr[r], du, dz), 0.0f);   // b_ki
                        g32[r] = g32[r] + ((a - b) + (b2 - a2));
                    } else {
                        g32[r] = g32[r] + (a - b);
                    }
                }
            }
        }
        // one tile of 64 columns in FP32, then into the FP64 row sums
#pragma unroll
        for (int r = 0; r < R; ++r) {
            f64[r] += (double)f32[r];
            g64[r] += (double)g32[r];
            f32[r] = 0.0f;
            g32[r] = 0.0f;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = r0 + r * 64 + lane;
        if (i >= A.n) continue;
        A.pF[(int64_t)chunk * A.n + i] = f64[r];
        A.pG[(int64_t)chunk * A.n + i] = (LOCAL ? 2.0 : 4.0) * g64[r];
    }
}

typedef void (*SmoothLaunch)(const SmoothArgs &, dim3, dim3, hipStream_t);

template <int NORM, int D, int DM>
void launch_smooth_global(const SmoothArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((smooth_kernel<D, DM, NORM, false>), g, b, 0, s, a);
}

template <int NORM, int D, int DM>
void launch_smooth_local(const SmoothArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((smooth_kernel<D, DM, NORM, true>), g, b, 0, s, a);
}

template <int NORM, int D, int... DMs>
constexpr std::array<SmoothLaunch, 2 * (D + 1)> smooth_row(std::integer_sequence<int, DMs...>)
{
    return {{&launch_smooth_global<NORM, D, DMs>..., &launch_smooth_local<NORM, D, DMs>...}};
}

template <int NORM>
SmoothLaunch smooth_table(int d, int dm, bool local)
{
    if (dm < 0 || dm > d) return nullptr;
    switch (d) {
#define LIP_SM_CASE(DD)                                                                     \
    case DD: {                                                                              \
        constexpr auto row = smooth_row<NORM, DD>(std::make_integer_sequence<int, DD + 1>{}); \
        return row[(local ? DD + 1 : 0) + dm];                                              \
    }
        LIP_SM_CASE(1) LIP_SM_CASE(2) LIP_SM_CASE(3) LIP_SM_CASE(4)
        LIP_SM_CASE(5) LIP_SM_CASE(6) LIP_SM_CASE(7) LIP_SM_CASE(8)
        LIP_SM_CASE(9) LIP_SM_CASE(10) LIP_SM_CASE(11) LIP_SM_CASE(12)
        LIP_SM_CASE(13) LIP_SM_CASE(14) LIP_SM_CASE(15) LIP_SM_CASE(16)
#undef LIP_SM_CASE
    default: return nullptr;
    }
}

SmoothLaunch smooth_l1(int d, int dm, bool local);
SmoothLaunch smooth_l2(int d, int dm, bool local);
SmoothLaunch smooth_linf(int d, int dm, bool local);

}  // namespace lip
