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
// scalar loads of records [x'_0..x'_{D-1} | z | M_k] (with the pre-screening
// also [.. | y | c M_k]).
//
// Pre-screening (Sec. 5, PRUNE): the ordered pair (i, k) leaves the sums when
//     y_i - y_k <= c M_k dist_up(x^i, x^k)  and  y_k - y_i <= c M_k dist_lo(x^i, x^k),
// on the given y.  Which pairs leave is a yes / no answer decided by floating
// point, so it is decided as by the definition: FP64 distances formed in
// index order (the consistency check's arithmetic), products left to right.
// The FP32 pass decides all but a sliver of the pairs: with
//     m = max(fma(-cM_k, du32, dy32), fma(-cM_k, dl32, -dy32))
// each of e_u = DY - cM du and e_l = -DY - cM dl is within
//     2^-17 (|DY| + cM t) + cM alpha
// of its FP32 value (FP32 distance error rho t + alpha with rho = 2^-18 and
// alpha as in the step-function forward; one rounding each of dy, cM and the
// fma).  With cM t = DY - e_u that is at most 2^-16 |dy| + 2^-17 |e| + cM
// alpha, so |e| > tol = 2^-14 |dy32| + 2 cM alpha fixes the sign of e, and
// |m| > tol fixes the sign of m (if m > tol, the larger one is certainly
// positive; if m < -tol, both are certainly negative).  A pair with
// |m| <= tol is deferred: if some lane of
// the wave has one, the wave decides those pairs in FP64 and adds the kept
// ones right after the column, so every row's sum keeps its column order.
// (The diagonal, m = 0, is always deferred and dropped: its terms are zero.)
#pragma once

#include "local_fwd.hpp"

namespace lip {

constexpr int kSmoothMaxChunks = 32;
constexpr int kSmoothTile = 64;

struct SmoothArgs {
    const float *rec;      // [npad][smooth_stride]: x' (bound-path transform), z = y + eps, M_k
                           // (pre-screening: then y, c M_k)
    int64_t n, npad;
    int32_t n_chunks;
    int32_t pad0;
    int64_t chunk_cols;    // multiple of kSmoothTile
    double *pF, *pG;       // [n_chunks][n] row partials
    // pre-screening
    double c;              // fraction c > 0
    const float *alpha;    // [1] absolute error term of the FP32 distances
    const double *X;       // FP64 d-major data [D + 2][npad64] (consistency-check staging)
    int64_t npad64;
    const double *wf;      // [2][kMaxDim]: weights, then free (1) / monotone (0) selectors
};

template <bool PRUNE>
constexpr int smooth_extra() { return PRUNE ? 4 : 2; }

// Rows per lane: the bound path's, halved with the pre-screening (each row
// then also holds y_i, c M_i and the filter's terms).
constexpr int smooth_rows(int D, bool prune)
{
    return prune ? (rows_for_dim(D) / 2 > 0 ? rows_for_dim(D) / 2 : 1) : rows_for_dim(D);
}

// FP64 decisions of the pre-screening for row i and column k: bit 0 set
// when the pair (i, k) stays (with M_k), bit 1 when (k, i) stays (with the
// row's M_i; dist_up(x^k, x^i) = dist_lo(x^i, x^k) and the reverse).  The
// distances follow the consistency check's operation sequence and the tests
// are the oracle's expressions; everything is read from memory, so the
// caller can loop over its deferred rows without unrolling.
template <int D, int NORM, bool MON>
__device__ __forceinline__ unsigned smooth_decide64(const SmoothArgs &A, int64_t i, int64_t k)
{
    constexpr int S = D + 4;
    double su = 0.0, sl = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double d = A.X[(int64_t)j * A.npad64 + i] - A.X[(int64_t)j * A.npad64 + k];
        if (j == 0) ds_step<NORM, true, MON, true>(A.wf[kMaxDim + j], A.wf[j], d, su, sl);
        else ds_step<NORM, true, MON, false>(A.wf[kMaxDim + j], A.wf[j], d, su, sl);
    }
    if (NORM == kNormL2) {
        su = sqrt(su);
        if (MON) sl = sqrt(sl);
    }
    if (!MON) sl = su;
    const float mi = A.rec[i * S + D + 1], yi = A.rec[i * S + D + 2];
    const float mk = A.rec[k * S + D + 1], yk = A.rec[k * S + D + 2];
    const double dy = (double)yi - (double)yk;
    const double c1 = A.c * (double)mk, c2 = A.c * (double)mi;
    const bool keep1 = !(dy <= c1 * su && -dy <= c1 * sl);
    const bool keep2 = !(-dy <= c2 * sl && dy <= c2 * su);
    return (keep1 ? 1u : 0u) | (keep2 ? 2u : 0u);
}

// One column k for the lane's R rows.
template <int D, int DM, int NORM, bool LOCAL, bool PRUNE, int R>
__device__ __forceinline__ void smooth_column(const SmoothArgs &A, const float *xk, int64_t k,
                                              int64_t r0, int lane, const float (&xr)[R][D],
                                              const float (&zr)[R], const float (&mr)[R],
                                              const float (&yr)[R], const float (&cr)[R],
                                              const float (&kr)[R], float s_alpha2,
                                              float (&f32)[R], float (&g32)[R])
{
    const float zk = xk[D], mk = xk[D + 1];
    float yk = 0.0f, ck = 0.0f, ka = 0.0f;
    if constexpr (PRUNE) {
        yk = xk[D + 2];
        ck = xk[D + 3];
        ka = ck * s_alpha2;  // the absolute part of the datum's tolerance
    }
    unsigned defer = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float du, dl;
        step_dist32<D, DM, NORM>(xr[r], xk, du, dl);
        const float dz = zr[r] - zk;
        float a = fmaxf(fmaf(-mk, du, dz), 0.0f);
        float b = fmaxf(fmaf(-mk, dl, -dz), 0.0f);
        float a2 = 0.0f, b2 = 0.0f;
        if constexpr (LOCAL) {
            a2 = fmaxf(fmaf(-mr[r], dl, -dz), 0.0f);  // a_ki
            b2 = fmaxf(fmaf(-mr[r], du, dz), 0.0f);   // b_ki
        }
        if constexpr (PRUNE) {
            const float dy = yr[r] - yk;
            const float m1 = fmaxf(fmaf(-ck, du, dy), fmaf(-ck, dl, -dy));
            bool u = fabsf(m1) <= fmaf(0x1p-14f, fabsf(dy), ka);
            bool keep1 = m1 > 0.0f;
            bool keep2 = true;
            if constexpr (LOCAL) {
                const float m2 = fmaxf(fmaf(-cr[r], dl, -dy), fmaf(-cr[r], du, dy));
                u = u || fabsf(m2) <= fmaf(0x1p-14f, fabsf(dy), kr[r]);
                keep2 = m2 > 0.0f;
            }
            if (u) defer |= 1u << r;
            if (u || !keep1) {
                a = 0.0f;
                b = 0.0f;
            }
            if (LOCAL && (u || !keep2)) {
                a2 = 0.0f;
                b2 = 0.0f;
            }
        }
        f32[r] = fmaf(a, a, fmaf(b, b, f32[r]));
        if constexpr (LOCAL) g32[r] = g32[r] + ((a - b) + (b2 - a2));
        else g32[r] = g32[r] + (a - b);
    }
    if constexpr (PRUNE) {
        if (__builtin_amdgcn_ballot_w64(defer != 0u) == 0) return;
        // decisions: one rolled loop over the lane's deferred rows
        unsigned keep = 0u, left = defer;
#pragma unroll 1
        while (left != 0u) {
            const int r = __builtin_ctz(left);
            left &= left - 1u;
            int64_t i = r0 + r * 64 + lane;
            i = i < A.n ? i : A.n - 1;
            keep |= smooth_decide64<D, NORM, (DM > 0)>(A, i, k) << (2 * r);
        }
        // the kept terms, in the main loop's arithmetic
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!((defer >> r) & 1u)) continue;
            float du, dl;
            step_dist32<D, DM, NORM>(xr[r], xk, du, dl);
            const float dz = zr[r] - zk;
            const bool keep1 = (keep >> (2 * r)) & 1u;
            const float a = keep1 ? fmaxf(fmaf(-mk, du, dz), 0.0f) : 0.0f;
            const float b = keep1 ? fmaxf(fmaf(-mk, dl, -dz), 0.0f) : 0.0f;
            f32[r] = fmaf(a, a, fmaf(b, b, f32[r]));
            if constexpr (LOCAL) {
                const bool keep2 = (keep >> (2 * r + 1)) & 1u;
                const float a2 = keep2 ? fmaxf(fmaf(-mr[r], dl, -dz), 0.0f) : 0.0f;
                const float b2 = keep2 ? fmaxf(fmaf(-mr[r], du, dz), 0.0f) : 0.0f;
                g32[r] = g32[r] + ((a - b) + (b2 - a2));
            } else {
                g32[r] = g32[r] + (a - b);
            }
        }
    }
}

template <int D, int DM, int NORM, bool LOCAL, bool PRUNE>
__global__ void __launch_bounds__(256) smooth_kernel(SmoothArgs A)
{
    constexpr int R = smooth_rows(D, PRUNE);
    constexpr int S = D + smooth_extra<PRUNE>();
    constexpr int G = 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % A.n_chunks;
    const int64_t rb = (int64_t)(blockIdx.x / A.n_chunks) * (blockDim.x >> 6) + wave;
    const int64_t r0 = rb * 64 * R;
    if (r0 >= A.n) return;
    const int lane = threadIdx.x & 63;
    float xr[R][D], zr[R], mr[R], yr[R], cr[R], kr[R], f32[R], g32[R];
    double f64[R], g64[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = r0 + r * 64 + lane;
        i = i < A.n ? i : A.n - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.rec[i * S + j];
        zr[r] = A.rec[i * S + D];
        mr[r] = A.rec[i * S + D + 1];
        yr[r] = PRUNE ? A.rec[i * S + D + 2] : 0.0f;
        cr[r] = PRUNE ? A.rec[i * S + D + 3] : 0.0f;
        f32[r] = 0.0f;
        g32[r] = 0.0f;
        f64[r] = 0.0;
        g64[r] = 0.0;
    }
    const float s_alpha2 = PRUNE ? 2.0f * A.alpha[0] : 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) kr[r] = cr[r] * s_alpha2;
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
                smooth_column<D, DM, NORM, LOCAL, PRUNE, R>(A, v + c * S, g0 + c, r0, lane, xr, zr,
                                                            mr, yr, cr, kr, s_alpha2, f32, g32);
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

template <int NORM, int D, int DM, bool LOCAL, bool PRUNE>
void launch_smooth(const SmoothArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((smooth_kernel<D, DM, NORM, LOCAL, PRUNE>), g, b, 0, s, a);
}

// [global | local] x [all pairs | pre-screened] x monotone count
template <int NORM, int D, int... DMs>
constexpr std::array<SmoothLaunch, 4 * (D + 1)> smooth_row(std::integer_sequence<int, DMs...>)
{
    return {{&launch_smooth<NORM, D, DMs, false, false>...,
             &launch_smooth<NORM, D, DMs, true, false>...,
             &launch_smooth<NORM, D, DMs, false, true>...,
             &launch_smooth<NORM, D, DMs, true, true>...}};
}

template <int NORM>
SmoothLaunch smooth_table(int d, int dm, bool local, bool prune)
{
    if (dm < 0 || dm > d) return nullptr;
    switch (d) {
#define LIP_SM_CASE(DD)                                                                     \
    case DD: {                                                                              \
        constexpr auto row = smooth_row<NORM, DD>(std::make_integer_sequence<int, DD + 1>{}); \
        return row[((prune ? 2 : 0) + (local ? 1 : 0)) * (DD + 1) + dm];                    \
    }
        LIP_SM_CASE(1) LIP_SM_CASE(2) LIP_SM_CASE(3) LIP_SM_CASE(4)
        LIP_SM_CASE(5) LIP_SM_CASE(6) LIP_SM_CASE(7) LIP_SM_CASE(8)
        LIP_SM_CASE(9) LIP_SM_CASE(10) LIP_SM_CASE(11) LIP_SM_CASE(12)
        LIP_SM_CASE(13) LIP_SM_CASE(14) LIP_SM_CASE(15) LIP_SM_CASE(16)
#undef LIP_SM_CASE
    default: return nullptr;
    }
}

SmoothLaunch smooth_l1(int d, int dm, bool local, bool prune);
SmoothLaunch smooth_l2(int d, int dm, bool local, bool prune);
SmoothLaunch smooth_linf(int d, int dm, bool local, bool prune);

}  // namespace lip
