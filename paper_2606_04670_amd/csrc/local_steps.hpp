// Step-function local constants of Sec. 4.3: the per-datum table
// (d1, V_0..V_{K+1}) over all pairs (steps_build), in FP64 with the
// operation order of the other data-side passes (symmetric distance,
// coordinates in index order), and the arguments shared with the bound
// kernel of local_fwd.hpp.
//
// M_k(t) is V_0 for t <= d1_k, V_s for the first knot with t <= q_s, and
// V_{K+1} beyond the last knot.
//
// Work split of the builder: a lane owns kDsRows rows, a wave 64 kDsRows
// rows and one column chunk; chunk partials are merged by steps_combine.
#pragma once

#include "data_side.hpp"

namespace lip {

constexpr int kMaxKnots = 8;
constexpr int kStepMaxChunks = 8;

// The smallest float >= v.
__device__ inline float round_up_f32(double v)
{
    float f = (float)v;
    if ((double)f < v) f = nextafterf(f, __builtin_inff());
    return f;
}

struct StepArgs {
    DsArgs ds;                 // staged data (X, n, npad), weights, free/monotone selectors, chunks
    int32_t K;                 // number of knots
    int32_t pad0;
    double knot[kMaxKnots];    // knots q_s (padded with +inf): the builder's radii
    double knotS[kMaxKnots];   // forward decision thresholds (l2: largest S with sqrt(S) <= q_s)
    // builder: chunk partials and outputs
    double *p_d1, *p_v0, *p_v;  // [n_chunks][n], [n_chunks][n], [n_chunks][KB + 1][n]
    int32_t *p_inf;             // [n_chunks][n]
    double *d1;                 // [n]
    double *V64;                // [n][K + 2] or NULL
    float *V32;                 // [n][K + 2] or NULL
    // forward
    const float *rec;           // [npad][D + 4] FP32 records (local_fwd.hpp)
    const double *T1;           // [npad] first-segment threshold (l2: largest S with sqrt(S) <= d1)
    const float *Vs;            // [K + 2][npad] segment-major table
    const float *xq;            // [q][D]
    int64_t q;
    const unsigned long long *qorder;  // queries in spatial order: (Morton code << 32 | index)
    Xform xf;                   // FP32 query transform (weights, signs, free coordinates first)
    float qsign[kMaxDim];       // -1 for a decreasing coordinate (as in the FP64 staging)
    float *g, *h_up, *h_lo;
    int32_t *arg_up, *arg_lo;
    float *part_v;              // [2][n_chunks][q]
    int32_t *part_i;
};

// ---- table builder ------------------------------------------------------------

// One group of kDsGroup columns for the lane's kDsRows rows.  A pair can
// only raise the first-segment value when its distance is <= the current d1,
// or a maximum v_j (knot j at or beyond its distance, or the overall one)
// when its slope exceeds it; the smallest of those maxima, vf, decides (the
// maxima are nested: v_j <= v_{j+1} <= v_all).  dy / t > vf is decided
// exactly by the sign of fma(-vf, t, dy), so the FP64 division and the
// updates run only for pairs that pass (a wave-uniform branch per pair).
template <int D, int NORM, bool HASW, int KB, bool MASK>
__device__ __forceinline__ void steps_group(const StepArgs &A, cdouble_ptr X, int64_t g0,
                                            const double (&xr)[kDsRows][D],
                                            const double (&yr)[kDsRows], const int (&ir)[kDsRows],
                                            double (&d1)[kDsRows], double (&v0)[kDsRows],
                                            double (&v)[KB + 1][kDsRows], bool (&inf)[kDsRows])
{
    double su[kDsGroup][kDsRows], sl[kDsGroup][kDsRows];
    ds_dist_group<D, NORM, HASW, false, kDsRows>(A.ds, X, g0, xr, su, sl);
    double yk[kDsGroup];
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c) yk[c] = X[(int64_t)D * A.ds.npad + g0 + c];
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
        for (int r = 0; r < kDsRows; ++r) {
            const int64_t k = g0 + c;
            const bool use = !MASK || (k != ir[r] && k < A.ds.n);
            double t = su[c][r];
            if (NORM == 2) t = sqrt(t);
            const double dy = fabs(yr[r] - yk[c]);
            inf[r] = inf[r] || (use && t == 0.0 && dy != 0.0);
            const bool pos = use && t > 0.0;
            double vf = v[KB][r];
#pragma unroll
            for (int j = KB - 1; j >= 0; --j) vf = t <= A.knot[j] ? v[j][r] : vf;
            const bool need = pos && (t <= d1[r] || fma(-vf, t, dy) > 0.0);
            if (__builtin_amdgcn_ballot_w64(need) == 0) continue;
            const double s = need ? dy / t : 0.0;
            const bool lt = need && t < d1[r];
            const bool eq = need && t == d1[r];
            v0[r] = lt ? s : ((eq && s > v0[r]) ? s : v0[r]);
            d1[r] = lt ? t : d1[r];
#pragma unroll
            for (int j = 0; j < KB; ++j)
                v[j][r] = (need && t <= A.knot[j] && s > v[j][r]) ? s : v[j][r];
            v[KB][r] = (need && s > v[KB][r]) ? s : v[KB][r];
        }
}

template <int D, int NORM, bool HASW, int KB>
__global__ void __launch_bounds__(256) steps_build_kernel(StepArgs A)
{
    constexpr int RW = 64 * kDsRows;
    WaveRange w;
    if (!wave_range(A.ds, RW, w)) return;
    const int lane = threadIdx.x & 63;
    double xr[kDsRows][D], yr[kDsRows], d1[kDsRows], v0[kDsRows], v[KB + 1][kDsRows];
    int ir[kDsRows];
    bool valid[kDsRows], inf[kDsRows];
#pragma unroll
    for (int r = 0; r < kDsRows; ++r) {
        int64_t i = w.r0 + r * 64 + lane;
        valid[r] = i < A.ds.n;
        i = i < A.ds.n ? i : A.ds.n - 1;
        ir[r] = (int)i;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.ds.X[(int64_t)j * A.ds.npad + i];
        yr[r] = A.ds.X[(int64_t)D * A.ds.npad + i];
        d1[r] = __builtin_inf();
        v0[r] = 0.0;
#pragma unroll
        for (int j = 0; j <= KB; ++j) v[j][r] = 0.0;
        inf[r] = false;
    }
    const cdouble_ptr X = (cdouble_ptr)(A.ds.X);
#pragma unroll 1
    for (int64_t g0 = w.c0; g0 < w.c1; g0 += kDsGroup) {
        // the diagonal (k == i) and the end of the data need a mask
        const bool masked = (g0 + kDsGroup > A.ds.n) || (g0 < w.r1 && g0 + kDsGroup > w.r0);
        if (masked)
            steps_group<D, NORM, HASW, KB, true>(A, X, g0, xr, yr, ir, d1, v0, v, inf);
        else
            steps_group<D, NORM, HASW, KB, false>(A, X, g0, xr, yr, ir, d1, v0, v, inf);
    }
#pragma unroll
    for (int r = 0; r < kDsRows; ++r) {
        if (!valid[r]) continue;
        const int64_t o = (int64_t)w.chunk * A.ds.n + ir[r];
        A.p_d1[o] = d1[r];
        A.p_v0[o] = v0[r];
        A.p_inf[o] = inf[r] ? 1 : 0;
#pragma unroll
        for (int j = 0; j <= KB; ++j)
            A.p_v[((int64_t)w.chunk * (KB + 1) + j) * A.ds.n + ir[r]] = v[j][r];
    }
}

// ---- launcher tables -----------------------------------------------------------

typedef void (*StepLaunch)(const StepArgs &, dim3, dim3, hipStream_t);

struct StepLaunchers {
    StepLaunch build;
};

template <int D, int NORM, bool HASW, int KB>
StepLaunchers step_launchers_for()
{
    StepLaunchers L;
    L.build = [](const StepArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((steps_build_kernel<D, NORM, HASW, KB>), g, b, 0, s, a);
    };
    return L;
}

template <int NORM>
bool step_table(int d, bool hasw, int kb, StepLaunchers *L)
{
    switch (d) {
#define LIP_SL_CASE(DD)                                                                  \
    case DD:                                                                             \
        if (kb == 4)                                                                     \
            *L = hasw ? step_launchers_for<DD, NORM, true, 4>()                          \
                      : step_launchers_for<DD, NORM, false, 4>();                        \
        else                                                                             \
            *L = hasw ? step_launchers_for<DD, NORM, true, 8>()                          \
                      : step_launchers_for<DD, NORM, false, 8>();                        \
        return true;
        LIP_SL_CASE(1) LIP_SL_CASE(2) LIP_SL_CASE(3) LIP_SL_CASE(4)
        LIP_SL_CASE(5) LIP_SL_CASE(6) LIP_SL_CASE(7) LIP_SL_CASE(8)
        LIP_SL_CASE(9) LIP_SL_CASE(10) LIP_SL_CASE(11) LIP_SL_CASE(12)
        LIP_SL_CASE(13) LIP_SL_CASE(14) LIP_SL_CASE(15) LIP_SL_CASE(16)
#undef LIP_SL_CASE
    default: return false;
    }
}

bool step_table_l1(int d, bool hasw, int kb, StepLaunchers *L);
bool step_table_l2(int d, bool hasw, int kb, StepLaunchers *L);
bool step_table_linf(int d, bool hasw, int kb, StepLaunchers *L);

}  // namespace lip
