// Device-side building blocks shared by the bound kernels (gfx950 / CDNA4).
//
// Staged data layout in HBM (written by the staging kernel, read by every
// bound kernel): one record of STRIDE = D + 3 floats per data point,
//     [ x'_0 .. x'_{D-1} | y | M | yU ]
// where x'_j = c_j * (x[perm_j] - o_j): the unconstrained coordinates come
// first, then the monotone ones; o_j is the mid-range of coordinate perm_j
// over the data (an FP32 value inside the data's range), and c_j folds in
// the distance weight w and the sign -1 of a decreasing coordinate (which
// turns it into an increasing one).  yU is the value the l1 upper bound
// starts from (see pair_bounds); it equals y for the other norms and without
// monotone coordinates.  Queries get the same transform when they are loaded
// into registers.
//
// Why the origin.  Eq. (2) depends on the coordinates only through
// x - x^k.  Rounding w x (or sums of coordinates) at the magnitude of the
// coordinates would put an error proportional to |x| into every candidate,
// which cancels later and is large when the data sit far from 0.  With the
// origin inside the data's range, |x - o| is at most the data's extent for a
// datum, and at most the query-datum distance plus that extent for a query;
// the subtraction is exact when x and o are within a factor 2 of each other
// (Sterbenz), and otherwise errs by half an ulp of |x - o|.  Every FP32 error
// of the bound path is therefore bounded by a small multiple of
// 2^-24 (|y_k| + M_k (dist + sum_i w_i ext_i)), ext_i the data's extent in
// coordinate i, whatever the position of the data.
//
// A wave reads one record at a time with a wave-uniform address, so the
// compiler emits scalar (SMEM) loads through the constant address space and
// the VALU takes the datum straight from SGPRs; the queries stay in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lip {

constexpr int kMaxDim = 16;
constexpr int kNormL1 = 1, kNormL2 = 2, kNormLinf = 3;

template <int D>
struct Rec {
    static constexpr int S = D + 3;  // record stride in floats
    static constexpr int Y = D, M = D + 1, YU = D + 2;
};

// Pointer into the constant address space: uniform loads become s_load.
typedef const float __attribute__((address_space(4))) *cfloat_ptr;

__device__ __forceinline__ cfloat_ptr as_const(const float *p) { return (cfloat_ptr)(p); }

// Per-coordinate transform applied to queries (data are staged with it):
// staged coordinate j = scale[j] * (x[perm[j]] - origin[j]).  `origin` is a
// device array of kMaxDim floats in the permuted order, written on the
// stream by launch_origin before any kernel that reads it.
struct Xform {
    int32_t perm[kMaxDim];
    float scale[kMaxDim];
    const float *origin;
};

// The origin of a coordinate whose data lie in [mn, mx]: the mid-range,
// with -0 turned into +0 (so that every path that reduces the same data gets
// the same bits) and 0 for a non-finite range (NaN / Inf inputs are outside
// the contract).
__device__ __forceinline__ float origin_of_range(float mn, float mx)
{
    const float o = (0.5f * mn + 0.5f * mx) + 0.0f;
    return __builtin_isfinite(o) ? o : 0.0f;
}

// Staged value of coordinate j of the row `row` (an untransformed [D] row).
__device__ __forceinline__ float xf_coord(const Xform &xf, const float *row, int j)
{
    return (row[xf.perm[j]] - xf.origin[j]) * xf.scale[j];
}

// Per-query constant of the l1 form with monotone coordinates:
// Qm = sum over the monotone coordinates of q'_i (in index order).
template <int D, int DM>
__device__ __forceinline__ float query_mon_sum(const float (&q)[D])
{
    float s = 0.0f;
    if constexpr (DM > 0) {
        s = q[D - DM];
#pragma unroll
        for (int i = D - DM + 1; i < D; ++i) s = s + q[i];
    }
    return s;
}

// max(a, b) for finite a, b as the median of (a, b, big) with big = +inf.
// fmaxf in the kernels' IEEE mode would first quiet (canonicalize) each
// operand loaded from memory, costing extra VALU work per pair; v_med3_f32
// needs none.  `big` must come from opaque_inf() so that the compiler cannot
// fold the median back into a max.
__device__ __forceinline__ float max_of_pair(float a, float b, float big)
{
    return __builtin_amdgcn_fmed3f(a, b, big);
}

// +inf in a VGPR, hidden from constant folding.
__device__ __forceinline__ float opaque_inf()
{
    float v = __builtin_inff();
    asm volatile("" : "+v"(v));
    return v;
}

// Bound candidates of Eq. (2) for one (query, datum) pair:
//     u = y + M dist_up(q, x^k),   l = y - M dist_lo(q, x^k),
// D coordinates of which the last DM are (increasing) monotone, Eq. (4) for
// the upper bound and its mirror for the lower bound.
//
//  l1:   su = F + sum_mon (q_i - x_i)_+,  sl = F + sum_mon (x_i - q_i)_+,
//        F = sum_free |q_i - x_i|.  Since (q - x)_+ = max(q, x) - x and
//        (x - q)_+ = max(q, x) - q, with G = sum_mon max(q_i, x_i),
//        S = F + G, X = sum_mon x_i and Qm = sum_mon q_i:
//            u = (y - M X) + M S = yU + M S,   l = y + M (Qm - S).
//        yU is staged per datum, Qm is computed once per query; `big` is
//        opaque_inf() (used by max_of_pair).
//  linf: F = max_free |d|;  su = max(F, max_mon d),  sl = max(F, max_mon -d)
//        (with no free coordinate, 0 joins the max: the positive part).
//  l2:   su = sqrt(sum_free d^2 + sum_mon ((d)_+)^2),
//        sl = sqrt(sum_free d^2 + sum_mon (min(d,0))^2).
// The operation order is fixed: every caller that must reproduce a value
// bit for bit (the argmin re-scan, the batched kernel, the BF16 re-scoring)
// calls this function with the same staged record.
template <int D, int DM, int NORM>
__device__ __forceinline__ void pair_bounds(const float (&q)[D], float qm, const float (&xk)[D],
                                            float yk, float mk, float yuk, float big, float &u,
                                            float &l)
{
    constexpr int DF = D - DM;
    if constexpr (NORM == kNormL1) {
        float s;
        if constexpr (DF > 0) {
            s = fabsf(q[0] - xk[0]);
#pragma unroll
            for (int i = 1; i < DF; ++i) s = s + fabsf(q[i] - xk[i]);
        }
        if constexpr (DM > 0) {
            float gsum = max_of_pair(q[DF], xk[DF], big);
#pragma unroll
            for (int i = DF + 1; i < D; ++i) gsum = gsum + max_of_pair(q[i], xk[i], big);
            if constexpr (DF > 0) s = s + gsum;
            else s = gsum;
            u = fmaf(mk, s, yuk);
            l = fmaf(mk, qm - s, yk);
        } else {
            u = fmaf(mk, s, yk);
            l = fmaf(-mk, s, yk);
        }
    } else if constexpr (NORM == kNormLinf) {
        float f = 0.0f;
        if constexpr (DF > 0) {
            f = fabsf(q[0] - xk[0]);
#pragma unroll
            for (int i = 1; i < DF; ++i) f = fmaxf(f, fabsf(q[i] - xk[i]));
        }
        float su = f, sl = f;
        if constexpr (DM > 0) {
#pragma unroll
            for (int i = DF; i < D; ++i) {
                const float dl = q[i] - xk[i];
                su = fmaxf(su, dl);
                sl = fmaxf(sl, -dl);
            }
        }
        u = fmaf(mk, su, yk);
        l = fmaf(-mk, sl, yk);
    } else {
        float f = 0.0f;
        if constexpr (DF > 0) {
            const float d0 = q[0] - xk[0];
            f = d0 * d0;
#pragma unroll
            for (int i = 1; i < DF; ++i) {
                const float di = q[i] - xk[i];
                f = fmaf(di, di, f);
            }
        }
        if constexpr (DM > 0) {
            float a = f, b = f;
#pragma unroll
            for (int i = DF; i < D; ++i) {
                const float dl = q[i] - xk[i];
                // max(dl, 0) and min(dl, 0) as medians (no operand
                // canonicalisation; the same values up to the sign of a
                // zero, which the squares drop)
                const float pp = __builtin_amdgcn_fmed3f(dl, 0.0f, big);
                const float nn = __builtin_amdgcn_fmed3f(dl, 0.0f, -big);
                a = fmaf(pp, pp, a);
                b = fmaf(nn, nn, b);
            }
            u = fmaf(mk, __builtin_amdgcn_sqrtf(a), yk);
            l = fmaf(-mk, __builtin_amdgcn_sqrtf(b), yk);
        } else {
            const float s = __builtin_amdgcn_sqrtf(f);
            u = fmaf(mk, s, yk);
            l = fmaf(-mk, s, yk);
        }
    }
}

// Order-preserving map of a float to uint32 (for packed (value, index) keys).
__device__ __forceinline__ uint32_t f32_order_key(float v)
{
    uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Packed keys of a result: min of (key(value) << 32 | index) is the smallest
// value with the lowest index; the lower bound stores (key(value) << 32 |
// ~index) complemented, so that its maximum with the lowest index is a
// minimum too (one fill value initialises both).  Adding +0 maps -0 to +0,
// so values that compare equal have equal keys.
__device__ __forceinline__ unsigned long long up_key(float v, int idx)
{
    return ((unsigned long long)f32_order_key(v + 0.0f) << 32) | (uint32_t)idx;
}
__device__ __forceinline__ unsigned long long lo_key(float v, int idx)
{
    return ~(((unsigned long long)f32_order_key(v + 0.0f) << 32) | (uint32_t)(~(uint32_t)idx));
}
__device__ __forceinline__ float f32_from_order_key(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ __forceinline__ void decode_keys(unsigned long long ku, unsigned long long kl_stored,
                                            float &hu, int &au, float &hl, int &al)
{
    const unsigned long long kl = ~kl_stored;
    hu = f32_from_order_key((uint32_t)(ku >> 32));
    hl = f32_from_order_key((uint32_t)(kl >> 32));
    au = (int)(uint32_t)ku;
    al = (int)(~(uint32_t)kl);
}

}  // namespace lip
