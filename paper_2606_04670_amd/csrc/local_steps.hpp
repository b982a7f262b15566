// Step-function local constants of Sec. 4.3 (kernel templates):
//  * steps_build  - the per-datum table (d1, V_0..V_{K+1}) over all pairs,
//                   in FP64 with the operation order of the other data-side
//                   passes (symmetric distance, coordinates in index order);
//  * steps_fwd    - the bounds of Eq. (2) with M_k(dist) in place of M.
//
// M_k(t) is V_0 for t <= d1_k, V_s for the first knot with t <= q_s, and
// V_{K+1} beyond the last knot.  The segment of a pair is an integer decided
// by floating point, so the forward decides it on the FP64 distance formed
// exactly like the definition's (the same staged d-major FP64 data and the
// same per-coordinate step as the consistency pass), not on the FP32 value
// it multiplies.  For l2 the comparison t <= q is made on the sum of squares
// S against the largest double S* with sqrt(S*) <= q (correctly rounded
// root), which is the same decision without a root per pair.  The bound
// candidate itself is FP32: y_k + M fl32(t) (l2: the FP32 root of fl32(S)).
//
// Work split.  steps_build: a lane owns kDsRows rows, a wave 64 kDsRows rows
// and one column chunk; chunk partials are merged by steps_combine.
// steps_fwd: a lane owns R queries, a wave 64 R queries and one column
// chunk; columns come in groups of kDsGroup through scalar loads of the
// d-major data, the step table is staged segment-major (V[s][npad]) so one
// scalar load brings one segment of the whole group.  Argmin / argmax keep
// the index per pair (strict comparisons, columns ascending), and chunk
// partials are reduced in chunk order, so ties go to the lowest index.
#pragma once

#include "data_side.hpp"

namespace lip {

constexpr int kMaxKnots = 8;
constexpr int kStepMaxChunks = 8;

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
    const double *T1;           // [npad] first-segment threshold (l2: largest S with sqrt(S) <= d1)
    const float *Vs;            // [KB + 2][npad] segment-major table
    const float *xq;            // [q][D]
    int64_t q;
    float qsign[kMaxDim];       // -1 for a decreasing coordinate (as in the staging)
    float *g, *h_up, *h_lo;
    int32_t *arg_up, *arg_lo;
    float *part_v;              // [2][n_chunks][q]
    int32_t *part_i;
};

// ---- table builder ------------------------------------------------------------

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
            const double s = pos ? dy / t : 0.0;
            const bool lt = pos && t < d1[r];
            const bool eq = pos && t == d1[r];
            v0[r] = lt ? s : ((eq && s > v0[r]) ? s : v0[r]);
            d1[r] = lt ? t : d1[r];
#pragma unroll
            for (int j = 0; j < KB; ++j)
                v[j][r] = (pos && t <= A.knot[j] && s > v[j][r]) ? s : v[j][r];
            v[KB][r] = (pos && s > v[KB][r]) ? s : v[KB][r];
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

// ---- bounds with M_k(dist) -----------------------------------------------------

// Queries per lane: the FP64 coordinates of R queries stay in VGPRs.
constexpr int step_rows(int D) { return D <= 4 ? 4 : (D <= 8 ? 2 : 1); }

// M_k(t) for one column: vc[0..KB+1] are its table entries (the entries past
// the K-th knot repeat V_{K+1}, whose padded knots are +inf).
template <int KB>
__device__ __forceinline__ float step_M(const StepArgs &A, double t, double t1,
                                        const float (&vc)[KB + 2])
{
    float m = vc[KB + 1];
#pragma unroll
    for (int s = KB - 1; s >= 0; --s) m = t <= A.knotS[s] ? vc[s + 1] : m;
    return t <= t1 ? vc[0] : m;
}

template <int D, int NORM, bool HASW, bool MON, int KB, bool MASK>
__device__ __forceinline__ void step_fwd_group(const StepArgs &A, cdouble_ptr X, int64_t g0,
                                               const double (&xr)[step_rows(D)][D],
                                               float (&hu)[step_rows(D)], float (&hl)[step_rows(D)],
                                               int (&au)[step_rows(D)], int (&al)[step_rows(D)])
{
    constexpr int R = step_rows(D);
    double su[kDsGroup][R], sl[kDsGroup][R];
    ds_dist_group<D, NORM, HASW, MON, R>(A.ds, X, g0, xr, su, sl);
    const cdouble_ptr T1 = (cdouble_ptr)(A.T1);
    const cfloat_ptr Vs = as_const(A.Vs);
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c) {
        const int64_t k = g0 + c;
        const float yk = (float)X[(int64_t)D * A.ds.npad + k];
        const double t1 = T1[k];
        float vc[KB + 2];
#pragma unroll
        for (int s = 0; s < KB + 2; ++s) vc[s] = Vs[(int64_t)s * A.ds.npad + k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double tu = su[c][r];
            const double tl = MON ? sl[c][r] : tu;
            const float mu = step_M<KB>(A, tu, t1, vc);
            const float ml = MON ? step_M<KB>(A, tl, t1, vc) : mu;
            float fu = (float)tu, fl = (float)tl;
            if (NORM == 2) {
                fu = __builtin_amdgcn_sqrtf(fu);
                fl = MON ? __builtin_amdgcn_sqrtf(fl) : fu;
            }
            float u = fmaf(mu, fu, yk);
            float l = fmaf(-ml, fl, yk);
            if (MASK && k >= A.ds.n) {
                u = __builtin_inff();
                l = -__builtin_inff();
            }
            const bool bu = u < hu[r], bl = l > hl[r];
            hu[r] = bu ? u : hu[r];
            au[r] = bu ? (int)k : au[r];
            hl[r] = bl ? l : hl[r];
            al[r] = bl ? (int)k : al[r];
        }
    }
}

template <int D, int NORM, bool HASW, bool MON, int KB>
__global__ void __launch_bounds__(256) steps_fwd_kernel(StepArgs A)
{
    constexpr int R = step_rows(D);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % A.ds.n_chunks;
    const int64_t qb = (int64_t)(blockIdx.x / A.ds.n_chunks) * (blockDim.x >> 6) + wave;
    const int64_t q0 = qb * 64 * R;
    if (q0 >= A.q) return;
    const int lane = threadIdx.x & 63;
    double xr[R][D];
    float hu[R], hl[R];
    int au[R], al[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t qi = q0 + r * 64 + lane;
        qi = qi < A.q ? qi : A.q - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = (double)(A.qsign[j] * A.xq[qi * D + j]);
        hu[r] = __builtin_inff();
        hl[r] = -__builtin_inff();
        au[r] = -1;
        al[r] = -1;
    }
    const int64_t c0 = (int64_t)chunk * A.ds.chunk_cols;
    int64_t c1 = c0 + A.ds.chunk_cols;
    c1 = c1 < A.ds.n ? c1 : A.ds.n;
    const cdouble_ptr X = (cdouble_ptr)(A.ds.X);
#pragma unroll 1
    for (int64_t g0 = c0; g0 < c1; g0 += kDsGroup) {
        if (g0 + kDsGroup > A.ds.n)
            step_fwd_group<D, NORM, HASW, MON, KB, true>(A, X, g0, xr, hu, hl, au, al);
        else
            step_fwd_group<D, NORM, HASW, MON, KB, false>(A, X, g0, xr, hu, hl, au, al);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t qi = q0 + r * 64 + lane;
        if (qi >= A.q) continue;
        if (A.ds.n_chunks == 1) {
            if (A.g) A.g[qi] = 0.5f * (hu[r] + hl[r]);
            if (A.h_up) A.h_up[qi] = hu[r];
            if (A.h_lo) A.h_lo[qi] = hl[r];
            if (A.arg_up) A.arg_up[qi] = au[r];
            if (A.arg_lo) A.arg_lo[qi] = al[r];
        } else {
            const int64_t nc = A.ds.n_chunks;
            A.part_v[(int64_t)chunk * A.q + qi] = hu[r];
            A.part_i[(int64_t)chunk * A.q + qi] = au[r];
            A.part_v[(nc + chunk) * A.q + qi] = hl[r];
            A.part_i[(nc + chunk) * A.q + qi] = al[r];
        }
    }
}

// ---- launcher tables -----------------------------------------------------------

typedef void (*StepLaunch)(const StepArgs &, dim3, dim3, hipStream_t);

struct StepLaunchers {
    StepLaunch build, fwd, fwd_mon;
};

template <int D, int NORM, bool HASW, int KB>
StepLaunchers step_launchers_for()
{
    StepLaunchers L;
    L.build = [](const StepArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((steps_build_kernel<D, NORM, HASW, KB>), g, b, 0, s, a);
    };
    L.fwd = [](const StepArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((steps_fwd_kernel<D, NORM, HASW, false, KB>), g, b, 0, s, a);
    };
    L.fwd_mon = [](const StepArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((steps_fwd_kernel<D, NORM, HASW, true, KB>), g, b, 0, s, a);
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
