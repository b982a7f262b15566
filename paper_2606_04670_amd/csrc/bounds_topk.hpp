// The k best bounds with weights (Sec. 5, k > 1): for every query the k
// smallest upper candidates u_(1) <= .. <= u_(k) and the k largest lower
// candidates l_[1] >= .. >= l_[k] of Eq. (2), and
//     H_up = sum_j w_j u_(j),   H_lo = sum_j w_j l_[j],   g = (H_up + H_lo) / 2.
//
// Same work decomposition and pair arithmetic as the fused bound kernel
// (pair_bounds on the staged records, queries in VGPRs, records from SGPRs).
// Each query keeps its KL best values per bound in registers, sorted, with
// the list length KL the smallest of 4, 8, 16, 32 that holds k (so k <=
// kTopKMax).  A candidate enters only if it beats the current KL-th value;
// the test is one compare per bound and pair, and the insertion (a min into
// the last slot and one compare-exchange pass) runs per candidate only when
// some lane of the wave improves one of its two lists (a wave-uniform branch:
// after the first data, few candidates improve any list; the number of
// insertions per query grows like KL log(n / KL)).  The k values form a
// multiset, so no index rule is needed; for l2 with monotone coordinates
// the forward's root-free bounds skip the records that cannot enter a row's
// lists (identical results); records past n (the staging's
// padding repeats the last datum) are masked, so every datum counts once.
// Split chunks write their sorted lists; a merge kernel takes the KL
// smallest / largest of all of them.  Longer lists would leave too few
// registers for the queries; larger k would take a threshold pass (the k-th
// value of a subset bounds the k-th value of all data), a pass collecting
// the candidates beyond it, and a sort per query.
#pragma once

#include "bounds_fwd.hpp"

namespace lip {

constexpr int kTopKMax = 32;

// List length for k: 4, 8, 16 or 32.
constexpr int topk_list_len(int k) { return k <= 4 ? 4 : (k <= 8 ? 8 : (k <= 16 ? 16 : 32)); }

// Queries per lane: the fused kernel's rows divided by KL / 2, at least one,
// since each query also holds its two sorted lists of KL values.
constexpr int topk_rows(int D, int KL)
{
    return rows_for_dim(D) * 2 / KL > 0 ? rows_for_dim(D) * 2 / KL : 1;
}

struct TopkArgs {
    FwdArgs f;             // staged records, n, queries, transform, outputs g / h_up / h_lo
    int32_t k;
    float wk[kTopKMax];    // weights, zero past k
    int64_t chunk_recs;    // records per chunk (multiple of the group size)
    float *part;           // [2][n_chunks][q][KL] sorted partial lists (n_chunks > 1)
};

// Ascending list: the new value replaces the last slot if smaller, then one
// compare-exchange pass from the end restores the order.
template <int KL>
__device__ __forceinline__ void topk_insert_up(float (&s)[KL], float v)
{
    s[KL - 1] = fminf(s[KL - 1], v);
#pragma unroll
    for (int j = KL - 1; j > 0; --j) {
        const float a = fminf(s[j - 1], s[j]), b = fmaxf(s[j - 1], s[j]);
        s[j - 1] = a;
        s[j] = b;
    }
}

// Descending list, the mirror.
template <int KL>
__device__ __forceinline__ void topk_insert_lo(float (&s)[KL], float v)
{
    s[KL - 1] = fmaxf(s[KL - 1], v);
#pragma unroll
    for (int j = KL - 1; j > 0; --j) {
        const float a = fmaxf(s[j - 1], s[j]), b = fminf(s[j - 1], s[j]);
        s[j - 1] = a;
        s[j] = b;
    }
}

template <int D, int DM, int NORM, int KL>
__global__ void __launch_bounds__(256) bounds_topk_kernel(TopkArgs A)
{
    constexpr int S = Rec<D>::S;
    constexpr int R = topk_rows(D, KL);
    constexpr int G = group_for_dim(D);
    const FwdArgs &a = A.f;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % a.n_chunks;
    const int64_t qblock = (int64_t)(blockIdx.x / a.n_chunks) * (blockDim.x >> 6) + wave;
    const int lane = threadIdx.x & 63;
    const int64_t q0 = qblock * (64 * R);
    if (q0 >= a.q) return;

    const float big = opaque_inf();
    float qv[R][D], qm[R], U[R][KL], L[R][KL];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t qi = q0 + r * 64 + lane;
        qi = qi < a.q ? qi : a.q - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) qv[r][j] = xf_coord(a.xf, a.xq + qi * D, j);
        qm[r] = query_mon_sum<D, DM>(qv[r]);
#pragma unroll
        for (int j = 0; j < KL; ++j) {
            U[r][j] = __builtin_inff();
            L[r][j] = -__builtin_inff();
        }
    }
    const int64_t c0 = (int64_t)chunk * A.chunk_recs;
    int64_t c1 = c0 + A.chunk_recs;
    c1 = c1 < a.n ? c1 : a.n;
    const cfloat_ptr base = as_const(a.data);
#pragma unroll 1
    for (int64_t g0 = c0; g0 < c1; g0 += G) {
        float v[G * S];
        load_group<D>(base + g0 * S, v);
#pragma unroll
        for (int c = 0; c < G; ++c) {
            float xk[D];
#pragma unroll
            for (int j = 0; j < D; ++j) xk[j] = v[c * S + j];
            if (g0 + c >= c1) break;  // wave-uniform
            if constexpr (NORM == kNormL2 && DM > 0) {
                // l2 with monotone coordinates: the forward's root-free
                // bounds first (ulb <= u, lub >= l); a record that cannot
                // enter any lane's lists is skipped for the row
                const L2fRec cr = l2f_record(v[c * S + Rec<D>::Y], v[c * S + Rec<D>::M]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float ulb, lub;
                    l2f_bounds<D, DM>(qv[r], xk, cr, ulb, lub);
                    if (__builtin_amdgcn_ballot_w64(ulb < U[r][KL - 1] || lub > L[r][KL - 1]) ==
                        0)
                        continue;
                    float u, l;
                    pair_bounds<D, DM, NORM>(qv[r], qm[r], xk, v[c * S + Rec<D>::Y],
                                             v[c * S + Rec<D>::M], v[c * S + Rec<D>::YU], big, u,
                                             l);
                    if (__builtin_amdgcn_ballot_w64(u < U[r][KL - 1] || l > L[r][KL - 1]) != 0) {
                        topk_insert_up<KL>(U[r], u);
                        topk_insert_lo<KL>(L[r], l);
                    }
                }
                continue;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float u, l;
                pair_bounds<D, DM, NORM>(qv[r], qm[r], xk, v[c * S + Rec<D>::Y],
                                         v[c * S + Rec<D>::M], v[c * S + Rec<D>::YU], big, u, l);
                // insert only where some lane of the wave improves a list
                // (an insertion that improves nothing leaves the list as it is)
                if (__builtin_amdgcn_ballot_w64(u < U[r][KL - 1] || l > L[r][KL - 1]) != 0) {
                    topk_insert_up<KL>(U[r], u);
                    topk_insert_lo<KL>(L[r], l);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t qi = q0 + r * 64 + lane;
        if (qi >= a.q) continue;
        if (a.n_chunks == 1) {
            float hu = 0.0f, hl = 0.0f;
#pragma unroll
            for (int j = 0; j < KL; ++j) {
                if (j < A.k) {
                    hu = fmaf(A.wk[j], U[r][j], hu);
                    hl = fmaf(A.wk[j], L[r][j], hl);
                }
            }
            if (a.g) a.g[qi] = 0.5f * (hu + hl);
            if (a.h_up) a.h_up[qi] = hu;
            if (a.h_lo) a.h_lo[qi] = hl;
        } else {
            float *pu = A.part + (((int64_t)chunk * a.q + qi) * KL);
            float *pl = A.part + ((((int64_t)a.n_chunks + chunk) * a.q + qi) * KL);
#pragma unroll
            for (int j = 0; j < KL; ++j) {
                pu[j] = U[r][j];
                pl[j] = L[r][j];
            }
        }
    }
}

typedef void (*TopkLaunch)(const TopkArgs &, dim3, dim3, hipStream_t);

template <int NORM, int KL, int D, int DM>
void launch_topk(const TopkArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((bounds_topk_kernel<D, DM, NORM, KL>), g, b, 0, s, a);
}

template <int NORM, int KL, int D, int... DMs>
constexpr std::array<TopkLaunch, D + 1> topk_row(std::integer_sequence<int, DMs...>)
{
    return {{&launch_topk<NORM, KL, D, DMs>...}};
}

template <int NORM, int KL>
TopkLaunch topk_table(int d, int dm)
{
    if (dm < 0 || dm > d) return nullptr;
    switch (d) {
#define LIP_TK_CASE(DD)                                                                        \
    case DD: {                                                                                 \
        constexpr auto row = topk_row<NORM, KL, DD>(std::make_integer_sequence<int, DD + 1>{}); \
        return row[dm];                                                                        \
    }
        LIP_TK_CASE(1) LIP_TK_CASE(2) LIP_TK_CASE(3) LIP_TK_CASE(4)
        LIP_TK_CASE(5) LIP_TK_CASE(6) LIP_TK_CASE(7) LIP_TK_CASE(8)
        LIP_TK_CASE(9) LIP_TK_CASE(10) LIP_TK_CASE(11) LIP_TK_CASE(12)
        LIP_TK_CASE(13) LIP_TK_CASE(14) LIP_TK_CASE(15) LIP_TK_CASE(16)
#undef LIP_TK_CASE
    default: return nullptr;
    }
}

// The kernel for list length kl (4, 8, 16, 32), else NULL.
template <int NORM>
TopkLaunch topk_table_kl(int d, int dm, int kl)
{
    switch (kl) {
    case 4: return topk_table<NORM, 4>(d, dm);
    case 8: return topk_table<NORM, 8>(d, dm);
    case 16: return topk_table<NORM, 16>(d, dm);
    case 32: return topk_table<NORM, 32>(d, dm);
    default: return nullptr;
    }
}

TopkLaunch topk_l1(int d, int dm, int kl);
TopkLaunch topk_l2(int d, int dm, int kl);
TopkLaunch topk_linf(int d, int dm, int kl);

}  // namespace lip
