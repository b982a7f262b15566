// Bounds of Eq. (2) with the step-function constants of Sec. 4.3:
//     u_k = y_k + M_k(dist_up) dist_up,   l_k = y_k - M_k(dist_lo) dist_lo.
//
// The segment of M_k a pair falls in is an integer decided by floating
// point, so it is decided exactly as by the definition: on the FP64 distance
// formed coordinate by coordinate in index order (the operation sequence of
// the consistency check), compared with the FP64 knots (l2: the sum of
// squares against the largest S whose rounded root is <= the knot).  The
// bound value itself is FP32: y_k + M fl32-distance (the same FP32 distance
// arithmetic as the scalar-M path, on coordinates staged with the weights
// and signs applied).
//
// Most pairs cannot change the running min / max, and they are recognised
// without the FP64 work: with t32 the FP32 distance,
//     u_k = fma(M, t32, y_k) >= fma(M_lb, t32, y_k)   for every M >= M_lb,
// since the fused multiply-add is monotone in M for t32 >= 0.  M_lb is the
// smallest table entry of the datum, or, when t32 exceeds the record's
// threshold D1hi (so that the FP64 distance is certainly beyond the first
// segment, see below), the smallest entry past the first segment.  If no
// lane of the wave has fma(M_lb, t32, y) < H_up or the mirror test for H_lo
// on a datum, the datum is skipped: its candidates cannot win.  Otherwise the
// wave evaluates that datum exactly (FP64 distance, segment, FP32 bound) for
// the queries of every row (one query per lane) in which some lane passed.  The skip changes no result, ties included (a skipped
// candidate is >= the running minimum, and minima are strict).
//
// D1hi.  |t32 - t64| <= rho t64 + alpha with rho = 2^-18 (the FP32
// distance's relative rounding, (d + 6) 2^-24 at most, with margin) and
// alpha = 2^-21 sum_j max|x'_j| + 2^-70: the staged coordinates
// x' = fl(fl(x - o) c) carry two roundings each, relative to the centred
// coordinates rather than to their difference, so a coordinate difference
// of a query and a datum errs by at most (2^-23 + 2^-48) (|q'_j| + |x'_j|)
// <= 2^-22 max|x'_j| (the maximum taken over the data and the queries);
// any of the three norms passes this on to the distance with factor <= 1
// per coordinate; the factor 2 is margin; 2^-70 covers FP32 underflow of
// squares.  So t32 > D1hi = up(d1 (1 + rho) + alpha) implies t64 > d1.
//
// The queries are processed in spatial (Morton) order, so that the queries
// of one wave are close together and few data can beat their running bounds.
//
// Layout: records [x'_0..x'_{D-1} | y | VL0 | VL1 | D1hi] (free coordinates
// first, then the monotone ones, as in the scalar-M path) read four at a
// time with scalar loads; the exact step reads the d-major FP64 data, the
// first-segment threshold T1 and the segment-major table of local_steps.hpp.
#pragma once

#include "lip_device.hpp"
#include "local_steps.hpp"

namespace lip {

constexpr int kStepRec = 4;  // extra floats per record: y, VL0, VL1, D1hi
constexpr float kStepRho = 0x1p-18f;

template <int D>
constexpr int step_rec_stride() { return D + kStepRec; }

// Queries per lane: half of the scalar-M path's, so that the exact step's
// FP64 registers fit.  Each row of a wave is a run of 64 consecutive queries
// in spatial order and is voted on separately, so a row whose queries cannot
// take a datum skips its exact evaluation.
constexpr int step_rows(int D) { return rows_for_dim(D) / 2 > 0 ? rows_for_dim(D) / 2 : 1; }

// FP32 directional distances of one pair: D coordinates, the last DM
// monotone (increasing after the staging's sign flip), Eq. (4) for the upper
// and its mirror for the lower distance.
template <int D, int DM, int NORM>
__device__ __forceinline__ void step_dist32(const float (&q)[D], const float *xk, float &tu,
                                            float &tl)
{
    constexpr int DF = D - DM;
    if constexpr (NORM == kNormL1) {
        float f = 0.0f, p = 0.0f, m = 0.0f;
#pragma unroll
        for (int i = 0; i < DF; ++i) f = i == 0 ? fabsf(q[i] - xk[i]) : f + fabsf(q[i] - xk[i]);
#pragma unroll
        for (int i = DF; i < D; ++i) {
            const float d = q[i] - xk[i];
            p = i == DF ? fmaxf(d, 0.0f) : p + fmaxf(d, 0.0f);
            m = i == DF ? fmaxf(-d, 0.0f) : m + fmaxf(-d, 0.0f);
        }
        tu = DF == 0 ? p : (DM == 0 ? f : f + p);
        tl = DF == 0 ? m : (DM == 0 ? f : f + m);
    } else if constexpr (NORM == kNormLinf) {
        float f = 0.0f, p = 0.0f, m = 0.0f;
#pragma unroll
        for (int i = 0; i < DF; ++i) f = fmaxf(f, fabsf(q[i] - xk[i]));
#pragma unroll
        for (int i = DF; i < D; ++i) {
            const float d = q[i] - xk[i];
            p = fmaxf(p, d);
            m = fmaxf(m, -d);
        }
        tu = fmaxf(f, p);
        tl = fmaxf(f, m);
    } else {
        float f = 0.0f, p = 0.0f, m = 0.0f;
#pragma unroll
        for (int i = 0; i < DF; ++i) {
            const float d = q[i] - xk[i];
            f = fmaf(d, d, f);
        }
#pragma unroll
        for (int i = DF; i < D; ++i) {
            const float d = q[i] - xk[i];
            const float pp = fmaxf(d, 0.0f);
            const float nn = d - pp;  // min(d, 0), exactly
            p = fmaf(pp, pp, p);
            m = fmaf(nn, nn, m);
        }
        tu = __builtin_amdgcn_sqrtf(DM == 0 ? f : f + p);
        tl = DM == 0 ? tu : __builtin_amdgcn_sqrtf(f + m);
    }
}

// M_k(t) for the FP64 decision quantity t (l2: sum of squares); the table
// column k is read from the segment-major staging (runtime K, exact path).
__device__ __forceinline__ float step_M_exact(const StepArgs &A, double t, double t1, int64_t k)
{
    const int K = A.K;
    if (t <= t1) return A.Vs[k];
    int s = 1;
    while (s <= K && !(t <= A.knotS[s - 1])) ++s;
    return A.Vs[(int64_t)s * A.ds.npad + k];
}

// Exact evaluation of datum k for the queries of the lane in the rows set in
// `rows` (wave-uniform: the rows where some lane's lower-bound test passed;
// in the others the candidate cannot win).
template <int D, int NORM, bool MON, int R>
__device__ __forceinline__ void step_exact(const StepArgs &A, int64_t k, float yk, unsigned rows,
                                           const int (&qi)[R], const float (&tu)[R],
                                           const float (&tl)[R], float (&hu)[R], float (&hl)[R],
                                           int (&au)[R], int (&al)[R])
{
    const double t1 = A.T1[k];
    double xc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xc[i] = A.ds.X[(int64_t)i * A.ds.npad + k];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!((rows >> r) & 1u)) continue;
        const int64_t j = qi[r];
        double su = 0.0, sl = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double d = (double)(A.qsign[i] * A.xq[j * D + i]) - xc[i];
            if (i == 0) ds_step<NORM, true, MON, true>(A.ds.fsel[i], A.ds.w[i], d, su, sl);
            else ds_step<NORM, true, MON, false>(A.ds.fsel[i], A.ds.w[i], d, su, sl);
        }
        if (!MON) sl = su;
        const float mu = step_M_exact(A, su, t1, k);
        const float ml = MON ? step_M_exact(A, sl, t1, k) : mu;
        const float u = fmaf(mu, tu[r], yk);
        const float l = fmaf(-ml, tl[r], yk);
        if (u < hu[r]) {
            hu[r] = u;
            au[r] = (int)k;
        }
        if (l > hl[r]) {
            hl[r] = l;
            al[r] = (int)k;
        }
    }
}

template <int D, int DM, int NORM>
__global__ void __launch_bounds__(256) steps_fwd32_kernel(StepArgs A)
{
    constexpr int R = step_rows(D);
    constexpr int S = step_rec_stride<D>();
    constexpr int G = 4;
    constexpr bool MON = DM > 0;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % A.ds.n_chunks;
    const int64_t qb = (int64_t)(blockIdx.x / A.ds.n_chunks) * (blockDim.x >> 6) + wave;
    const int64_t q0 = qb * 64 * R;
    if (q0 >= A.q) return;
    const int lane = threadIdx.x & 63;
    float qv[R][D], hu[R], hl[R];
    int au[R], al[R], qi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t p = q0 + r * 64 + lane;
        p = p < A.q ? p : A.q - 1;
        const int64_t j = (int64_t)(uint32_t)(A.qorder[p] & 0xFFFFFFFFull);
        qi[r] = (int)j;
#pragma unroll
        for (int i = 0; i < D; ++i) qv[r][i] = xf_coord(A.xf, A.xq + j * D, i);
        hu[r] = __builtin_inff();
        hl[r] = -__builtin_inff();
        au[r] = -1;
        al[r] = -1;
    }
    const int64_t c0 = (int64_t)chunk * A.ds.chunk_cols;
    int64_t c1 = c0 + A.ds.chunk_cols;
    c1 = c1 < A.ds.n ? c1 : A.ds.n;
    const cfloat_ptr rec = as_const(A.rec);
#pragma unroll 1
    for (int64_t g0 = c0; g0 < c1; g0 += G) {
        float v[G * S];
#pragma unroll
        for (int e = 0; e < G * S; ++e) v[e] = rec[g0 * S + e];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int64_t k = g0 + c;
            if (k >= c1) break;  // wave-uniform
            const float *xk = v + c * S;
            const float yk = xk[D], vl0 = xk[D + 1], vl1 = xk[D + 2], d1hi = xk[D + 3];
            float tu[R], tl[R];
            unsigned rows = 0u;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                step_dist32<D, DM, NORM>(qv[r], xk, tu[r], tl[r]);
                const float mu = tu[r] > d1hi ? vl1 : vl0;
                const float ml = tl[r] > d1hi ? vl1 : vl0;
                const bool need = fmaf(mu, tu[r], yk) < hu[r] || fmaf(-ml, tl[r], yk) > hl[r];
                if (__builtin_amdgcn_ballot_w64(need) != 0) rows |= 1u << r;
            }
            if (rows != 0u)
                step_exact<D, NORM, MON, R>(A, k, yk, rows, qi, tu, tl, hu, hl, au, al);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (q0 + r * 64 + lane >= A.q) continue;
        const int64_t j = qi[r];
        if (A.ds.n_chunks == 1) {
            if (A.g) A.g[j] = 0.5f * (hu[r] + hl[r]);
            if (A.h_up) A.h_up[j] = hu[r];
            if (A.h_lo) A.h_lo[j] = hl[r];
            if (A.arg_up) A.arg_up[j] = au[r];
            if (A.arg_lo) A.arg_lo[j] = al[r];
        } else {
            const int64_t nc = A.ds.n_chunks;
            A.part_v[(int64_t)chunk * A.q + j] = hu[r];
            A.part_i[(int64_t)chunk * A.q + j] = au[r];
            A.part_v[(nc + chunk) * A.q + j] = hl[r];
            A.part_i[(nc + chunk) * A.q + j] = al[r];
        }
    }
}

template <int NORM, int D, int DM>
void launch_step_fwd(const StepArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    hipLaunchKernelGGL((steps_fwd32_kernel<D, DM, NORM>), grid, block, 0, s, a);
}

template <int NORM, int D, int... DMs>
constexpr std::array<StepLaunch, D + 1> step_fwd_row(std::integer_sequence<int, DMs...>)
{
    return {{&launch_step_fwd<NORM, D, DMs>...}};
}

template <int NORM>
StepLaunch step_fwd_table(int d, int dm)
{
    if (dm < 0 || dm > d) return nullptr;
    switch (d) {
#define LIP_SF_CASE(DD)                                                                       \
    case DD: {                                                                                \
        constexpr auto row = step_fwd_row<NORM, DD>(std::make_integer_sequence<int, DD + 1>{}); \
        return row[dm];                                                                       \
    }
        LIP_SF_CASE(1) LIP_SF_CASE(2) LIP_SF_CASE(3) LIP_SF_CASE(4)
        LIP_SF_CASE(5) LIP_SF_CASE(6) LIP_SF_CASE(7) LIP_SF_CASE(8)
        LIP_SF_CASE(9) LIP_SF_CASE(10) LIP_SF_CASE(11) LIP_SF_CASE(12)
        LIP_SF_CASE(13) LIP_SF_CASE(14) LIP_SF_CASE(15) LIP_SF_CASE(16)
#undef LIP_SF_CASE
    default: return nullptr;
    }
}

StepLaunch step_fwd_l1(int d, int dm);
StepLaunch step_fwd_l2(int d, int dm);
StepLaunch step_fwd_linf(int d, int dm);

}  // namespace lip
