// Bounds of Eq. (2)-(3) with monotonicity on parts of the domain (Sec. 4.2):
// the pair kernel, instantiated per norm in bounds_reg_{l1,l2,linf}.hip.
//
// Every coordinate carries the two intervals where f is not decreasing (ND)
// and not increasing (NI) (kinds 0 / +1 / -1 are the cases where these are
// everything or nothing; an empty interval is stored as [0, 0]).  With
// c(v) = w (clamp(v, s, t) - o) the clamped, weighted coordinate (o the
// data's mid-range in that coordinate, so that rounding happens at the scale
// of the data's extent rather than of |v|; see lip_device.hpp), the travelled
// length inside [s, t] is |c(q) - c(x)|, and the difference a = c_ND(q) -
// c_ND(x) is positive when moving towards larger values, negative otherwise
// (likewise b for NI).  So the upper component (length where f may rise in
// the direction of travel: inside ND moving up, inside NI moving down) is
// max(a, -b), and the lower one max(b, -a).  A free coordinate (both
// intervals unbounded) gives |q - x| to both, so the DF free coordinates come
// first, stored once, and their part of the norm is shared by the upper and
// the lower distance (as in the fused kernel); the restricted ones follow as
// (c_ND, c_NI) pairs.  The clamped data coordinates are staged per datum and
// the query's formed once per query, so a restricted coordinate costs two
// subtractions and two maxima per pair, a free one a subtraction.
//
// A lane owns R queries, a wave 64 R queries and one data chunk; records
// [w x_free.. | c_ND, c_NI per restricted coordinate | y | M_k] come four at
// a time through scalar loads.  The inner loop keeps only the running min /
// max; at the end of every tile of kRegTile records a query notes the tile if
// its value strictly improved there, and afterwards re-scans that one tile
// with the same arithmetic for the first index that attains the final value
// (so ties resolve to the lowest index, as in the definition).  Chunk
// partials go through the bound path's combine.
#pragma once

#include "bounds_fwd.hpp"  // l2f_record: per-record constants of the root-free l2 filter
#include "host_common.hpp"
#include "lip_device.hpp"

namespace lip {

struct RegArgs {
    const float *rec;  // [npad][2 D - DF + 2]
    int64_t n, npad;
    int32_t n_chunks;
    int32_t pad0;
    int64_t chunk_cols;
    // per position (free coordinates first): source coordinate, intervals, weight
    int32_t perm[kMaxDim];
    float nd_s[kMaxDim], nd_t[kMaxDim], ni_s[kMaxDim], ni_t[kMaxDim], w[kMaxDim];
    const float *origin;  // device [kMaxDim], per position
    const float *xq;
    int64_t q;
    float *g, *h_up, *h_lo;
    int32_t *arg_up, *arg_lo;
    float *part_v;
    int32_t *part_i;
};

constexpr int kRegTile = 64;  // records per tile; chunks are whole tiles

constexpr int reg_rows(int D) { return rows_for_dim(D) / 2 > 0 ? rows_for_dim(D) / 2 : 1; }

// w (clamp(v, s, t) - o) (s <= t; the median of three needs no
// canonicalisation)
__device__ __forceinline__ float reg_clamp(float v, float s, float t, float w, float o)
{
    return w * (__builtin_amdgcn_fmed3f(v, s, t) - o);
}

// Upper and lower distances of one pair: q and xk hold the DF free weighted
// coordinates, then (c_ND, c_NI) for each restricted coordinate.
template <int D, int DF, int NORM>
__device__ __forceinline__ void reg_dist(const float (&q)[2 * D - DF], const float *xk, float &tu,
                                         float &tl)
{
    float f = 0.0f;
#pragma unroll
    for (int i = 0; i < DF; ++i) {
        const float d = q[i] - xk[i];
        if (NORM == kNormL1) f = i == 0 ? fabsf(d) : f + fabsf(d);
        else if (NORM == kNormL2) f = i == 0 ? d * d : fmaf(d, d, f);
        else f = i == 0 ? fabsf(d) : fmaxf(f, fabsf(d));
    }
    float su = f, sl = f;
#pragma unroll
    for (int j = 0; j < D - DF; ++j) {
        const int e = DF + 2 * j;
        const float a = q[e] - xk[e];          // signed length inside ND
        const float b = q[e + 1] - xk[e + 1];  // signed length inside NI
        const float cu = fmaxf(a, -b), cl = fmaxf(b, -a);
        const bool first = DF == 0 && j == 0;
        if (NORM == kNormL1) {
            su = first ? cu : su + cu;
            sl = first ? cl : sl + cl;
        } else if (NORM == kNormL2) {
            su = first ? cu * cu : fmaf(cu, cu, su);
            sl = first ? cl * cl : fmaf(cl, cl, sl);
        } else {
            su = first ? cu : fmaxf(su, cu);
            sl = first ? cl : fmaxf(sl, cl);
        }
    }
    if (NORM == kNormL2) {
        su = __builtin_amdgcn_sqrtf(su);
        sl = DF == D ? su : __builtin_amdgcn_sqrtf(sl);
    }
    tu = su;
    tl = sl;
}

// l2: root-free bounds of one pair's candidates from the largest component
// of each distance, as in the bound kernel's filter (the same argument
// holds: the exact path squares exactly these components, sums
// non-negative terms with monotone rounding and takes v_sqrt_f32 of the
// sum, and its candidates are fma(M_k, dist, y_k)).  The components are all
// non-negative: a and b have the sign of the coordinate difference, so one
// of a and -b is >= 0.
template <int D, int DF>
__device__ __forceinline__ void reg_l2_root_free(const float (&q)[2 * D - DF], const float *xk,
                                                 const L2fRec &c, float &ulb, float &lub)
{
    float f = 0.0f;
#pragma unroll
    for (int i = 0; i < DF; ++i) f = fmaxf(f, fabsf(q[i] - xk[i]));
    float su = f, sl = f;
#pragma unroll
    for (int j = 0; j < D - DF; ++j) {
        const int e = DF + 2 * j;
        const float a = q[e] - xk[e], b = q[e + 1] - xk[e + 1];
        su = fmaxf(su, fmaxf(a, -b));
        sl = fmaxf(sl, fmaxf(b, -a));
    }
    ulb = fmaf(c.ms, su, c.ylo);
    lub = fmaf(-c.ms, sl, c.yhi);
}

template <int D, int DF, int NORM>
__global__ void __launch_bounds__(256) bounds_reg_kernel(RegArgs A)
{
    constexpr int R = reg_rows(D);
    constexpr int E = 2 * D - DF;  // coordinate values per record
    constexpr int S = E + 2;
    constexpr int G = 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % A.n_chunks;
    const int64_t qb = (int64_t)(blockIdx.x / A.n_chunks) * (blockDim.x >> 6) + wave;
    const int64_t q0 = qb * 64 * R;
    if (q0 >= A.q) return;
    const int lane = threadIdx.x & 63;
    float qv[R][E], hu[R], hl[R], pu[R], pl[R];
    int tu[R], tl[R];
    const int64_t c0 = (int64_t)chunk * A.chunk_cols;
    int64_t c1 = c0 + A.chunk_cols;
    c1 = c1 < A.n ? c1 : A.n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t j = q0 + r * 64 + lane;
        j = j < A.q ? j : A.q - 1;
#pragma unroll
        for (int i = 0; i < DF; ++i) qv[r][i] = A.w[i] * (A.xq[j * D + A.perm[i]] - A.origin[i]);
#pragma unroll
        for (int i = DF; i < D; ++i) {
            const float v = A.xq[j * D + A.perm[i]];
            qv[r][DF + 2 * (i - DF)] = reg_clamp(v, A.nd_s[i], A.nd_t[i], A.w[i], A.origin[i]);
            qv[r][DF + 2 * (i - DF) + 1] = reg_clamp(v, A.ni_s[i], A.ni_t[i], A.w[i], A.origin[i]);
        }
        hu[r] = __builtin_inff();
        hl[r] = -__builtin_inff();
        pu[r] = hu[r];
        pl[r] = hl[r];
        tu[r] = (int)(c0 / kRegTile);
        tl[r] = tu[r];
    }
    const cfloat_ptr rec = as_const(A.rec);
    // min / max as medians with an opaque infinity: no re-quieting of the
    // running values each pair
    const float big = opaque_inf(), nbig = -big;
    constexpr int gpt = kRegTile / G;  // groups per tile
    int left = gpt;
    int t = (int)(c0 / kRegTile);
#pragma unroll 1
    for (int64_t g0 = c0; g0 < c1; g0 += G) {
        float v[G * S];
#pragma unroll
        for (int e = 0; e < G * S; ++e) v[e] = rec[g0 * S + e];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            if (g0 + c >= c1) break;  // wave-uniform
            const float *xk = v + c * S;
            const float yk = xk[E], mk = xk[E + 1];
            if constexpr (NORM == kNormL2) {
                // exact distances (two square roots) only for the rows of 64
                // queries where some lane could improve
                const L2fRec rc = l2f_record(yk, mk);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float ulb, lub;
                    reg_l2_root_free<D, DF>(qv[r], xk, rc, ulb, lub);
                    if (__builtin_amdgcn_ballot_w64((ulb < hu[r]) | (lub > hl[r]))) {
                        float du, dl;
                        reg_dist<D, DF, NORM>(qv[r], xk, du, dl);
                        hu[r] = __builtin_amdgcn_fmed3f(hu[r], fmaf(mk, du, yk), nbig);
                        hl[r] = __builtin_amdgcn_fmed3f(hl[r], fmaf(-mk, dl, yk), big);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float du, dl;
                    reg_dist<D, DF, NORM>(qv[r], xk, du, dl);
                    hu[r] = __builtin_amdgcn_fmed3f(hu[r], fmaf(mk, du, yk), nbig);
                    hl[r] = __builtin_amdgcn_fmed3f(hl[r], fmaf(-mk, dl, yk), big);
                }
            }
        }
        if (--left == 0 || g0 + G >= c1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                tu[r] = hu[r] < pu[r] ? t : tu[r];
                tl[r] = hl[r] > pl[r] ? t : tl[r];
                pu[r] = hu[r];
                pl[r] = hl[r];
            }
            left = gpt;
            ++t;
        }
    }
    // first attaining index: descending re-scan of the last improving tile
    int au[R], al[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t bu = (int64_t)tu[r] * kRegTile, bl = (int64_t)tl[r] * kRegTile;
        const int64_t eu = bu + kRegTile < c1 ? bu + kRegTile : c1;
        const int64_t el = bl + kRegTile < c1 ? bl + kRegTile : c1;
        int iu = -1, il = -1;
#pragma unroll 1
        for (int64_t k = eu - 1; k >= bu; --k) {
            const float *xk = A.rec + k * S;
            float du, dl;
            reg_dist<D, DF, NORM>(qv[r], xk, du, dl);
            iu = fmaf(xk[E + 1], du, xk[E]) == hu[r] ? (int)k : iu;
        }
#pragma unroll 1
        for (int64_t k = el - 1; k >= bl; --k) {
            const float *xk = A.rec + k * S;
            float du, dl;
            reg_dist<D, DF, NORM>(qv[r], xk, du, dl);
            il = fmaf(-xk[E + 1], dl, xk[E]) == hl[r] ? (int)k : il;
        }
        au[r] = iu;
        al[r] = il;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = q0 + r * 64 + lane;
        if (j >= A.q) continue;
        if (A.n_chunks == 1) {
            if (A.g) A.g[j] = 0.5f * (hu[r] + hl[r]);
            if (A.h_up) A.h_up[j] = hu[r];
            if (A.h_lo) A.h_lo[j] = hl[r];
            if (A.arg_up) A.arg_up[j] = au[r];
            if (A.arg_lo) A.arg_lo[j] = al[r];
        } else {
            const int64_t nc = A.n_chunks;
            A.part_v[(int64_t)chunk * A.q + j] = hu[r];
            A.part_i[(int64_t)chunk * A.q + j] = au[r];
            A.part_v[(nc + chunk) * A.q + j] = hl[r];
            A.part_i[(nc + chunk) * A.q + j] = al[r];
        }
    }
}

typedef void (*RegLaunch)(const RegArgs &, dim3, dim3, hipStream_t);

template <int NORM, int D, int DF>
void launch_reg(const RegArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((bounds_reg_kernel<D, DF, NORM>), g, b, 0, s, a);
}

template <int NORM, int D, int... DFs>
constexpr std::array<RegLaunch, D + 1> reg_row(std::integer_sequence<int, DFs...>)
{
    return {{&launch_reg<NORM, D, DFs>...}};
}

template <int NORM>
RegLaunch reg_table(int d, int df)
{
    if (df < 0 || df > d) return nullptr;
    switch (d) {
#define LIP_RG_CASE(DD)                                                                   \
    case DD: {                                                                            \
        constexpr auto row = reg_row<NORM, DD>(std::make_integer_sequence<int, DD + 1>{}); \
        return row[df];                                                                   \
    }
        LIP_RG_CASE(1) LIP_RG_CASE(2) LIP_RG_CASE(3) LIP_RG_CASE(4)
        LIP_RG_CASE(5) LIP_RG_CASE(6) LIP_RG_CASE(7) LIP_RG_CASE(8)
        LIP_RG_CASE(9) LIP_RG_CASE(10) LIP_RG_CASE(11) LIP_RG_CASE(12)
        LIP_RG_CASE(13) LIP_RG_CASE(14) LIP_RG_CASE(15) LIP_RG_CASE(16)
#undef LIP_RG_CASE
    default: return nullptr;
    }
}

RegLaunch reg_l1(int d, int df);
RegLaunch reg_l2(int d, int df);
RegLaunch reg_linf(int d, int df);

}  // namespace lip
