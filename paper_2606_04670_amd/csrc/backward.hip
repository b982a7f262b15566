// Subgradients of g (and of H_up, H_lo) through the saved attaining indices:
// the chain rule applied to Eq. (2)-(3) with a = arg_up[j], b = arg_lo[j]:
//   H_up = y_a + M_a dist_up(x, x^a),   H_lo = y_b - M_b dist_lo(x, x^b).
// One thread per query; O(q d) work.  Distances and their gradients are
// recomputed in the original coordinate order with the original weights and
// monotonicity, with the zero subgradient at kinks (|.|'(0) = 0,
// (.)_+'(0) = 0, l2 at distance 0 -> 0, linf -> lowest maximal coordinate).
//
// Accumulation of dy / dM: hardware FP32 atomic adds (global_atomic_add_f32 on
// device memory, no compare-and-swap loop), or with LIP_FLAG_DETERMINISTIC
// int64 fixed-point atomics (integer addition is associative, so the sum is
// independent of the order): pass 1 finds the largest |contribution|, pass 2
// adds round(contribution * 2^s) with s chosen so that q of them cannot
// overflow, pass 3 converts back and adds into the caller's arrays.
#include <climits>

#include "host_common.hpp"

namespace lip {

struct BwdArgs {
    const float *x, *Mk, *xq;
    float M;
    int32_t norm;
    int64_t n, q;
    const int32_t *arg_up, *arg_lo;
    const float *dg, *dh_up, *dh_lo;
    float *dxq, *dy, *dM;
    float w[kMaxDim];
    int32_t mon[kMaxDim];
    // deterministic mode
    int32_t fixed;              // 0: FP32 atomics, 1: pass 1 (max), 2: pass 2 (accumulate)
    unsigned int *maxbits;      // [1] max |contribution| as float bits
    unsigned long long *acc_y;  // [n] fixed-point dy
    unsigned long long *acc_m;  // [n] or [1] fixed-point dM
};

template <int D>
__device__ __forceinline__ float dist_and_grad(const BwdArgs &a, const float *xq, const float *xk,
                                               bool up, float (&grad)[D])
{
    float s = 0.0f;
    float cmax = -1.0f;
    int jmax = -1;
    float c[D], dc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float dl = xq[i] - xk[i];
        const int m = a.mon[i];
        float ci, di;
        if (m == 0) {
            ci = fabsf(dl);
            di = dl > 0.0f ? 1.0f : (dl < 0.0f ? -1.0f : 0.0f);
        } else if ((m > 0) == up) {  // component (delta)_+
            ci = dl > 0.0f ? dl : 0.0f;
            di = dl > 0.0f ? 1.0f : 0.0f;
        } else {  // component (-delta)_+
            ci = dl < 0.0f ? -dl : 0.0f;
            di = dl < 0.0f ? -1.0f : 0.0f;
        }
        c[i] = a.w[i] * ci;
        dc[i] = a.w[i] * di;
        if (a.norm == 1) {
            s = s + c[i];
        } else if (a.norm == 2) {
            s = fmaf(c[i], c[i], s);
        } else {
            if (c[i] > cmax) {
                cmax = c[i];
                jmax = i;
            }
        }
    }
    if (a.norm == 2) s = sqrtf(s);
    if (a.norm == 3) s = cmax;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (a.norm == 1)
            grad[i] = dc[i];
        else if (a.norm == 2)
            grad[i] = s > 0.0f ? c[i] * dc[i] / s : 0.0f;
        else
            grad[i] = (i == jmax) ? dc[i] : 0.0f;
    }
    return s;
}

__device__ __forceinline__ long long to_fixed(float v, int shift)
{
    return (long long)rint(ldexp((double)v, shift));
}

// Adds (v1, v2) into (p1[idx], p2[idx]) for every active lane, first summing
// the lanes of the wave that share an index (the attaining data points of
// neighbouring queries coincide often, and same-address atomics serialise).
// The lane-set of each sum is fixed by the data and the butterfly order by
// the lane numbers, so a wave's contribution does not depend on timing.
template <typename T, typename AddFn>
__device__ __forceinline__ void wave_scatter_add(bool active, int idx, T v1, T v2, T *p1, T *p2,
                                                 AddFn add)
{
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int lidx = __shfl(idx, leader);
        const bool mine = active && idx == lidx;
        T s1 = mine ? v1 : T(0), s2 = mine ? v2 : T(0);
        for (int off = 32; off > 0; off >>= 1) {
            s1 += __shfl_xor(s1, off);
            s2 += __shfl_xor(s2, off);
        }
        if (lane == leader) {
            if (p1) add(p1 + lidx, s1);
            if (p2) add(p2 + lidx, s2);
        }
        pending &= ~__ballot(mine);
        active = active && !mine;
    }
}

struct FloatAtomic {
    __device__ void operator()(float *p, float v) const { unsafeAtomicAdd(p, v); }
};
template <int D>
__global__ void __launch_bounds__(256) backward_kernel(BwdArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // indices outside [0, n) (not produced by the forward) are skipped
    const bool valid = j < a.q && a.arg_up[j] >= 0 && a.arg_up[j] < a.n && a.arg_lo[j] >= 0 &&
                       a.arg_lo[j] < a.n;
    int ia = 0, ib = 0;
    float Gu = 0.0f, Gl = 0.0f, cu_m = 0.0f, cl_m = 0.0f;
    if (valid) {
        ia = a.arg_up[j];
        ib = a.arg_lo[j];
        const float *xj = a.xq + j * D;
        float xr[D];
#pragma unroll
        for (int i = 0; i < D; ++i) xr[i] = xj[i];
        const float hg = a.dg ? 0.5f * a.dg[j] : 0.0f;
        Gu = hg + (a.dh_up ? a.dh_up[j] : 0.0f);
        Gl = hg + (a.dh_lo ? a.dh_lo[j] : 0.0f);
        float gu[D], gl[D];
        const float du = dist_and_grad<D>(a, xr, a.x + (int64_t)ia * D, true, gu);
        const float dl = dist_and_grad<D>(a, xr, a.x + (int64_t)ib * D, false, gl);
        const float Ma = a.Mk ? a.Mk[ia] : a.M;
        const float Mb = a.Mk ? a.Mk[ib] : a.M;
        if (a.fixed != 1 && a.dxq) {
#pragma unroll
            for (int i = 0; i < D; ++i) a.dxq[j * D + i] = Gu * Ma * gu[i] - Gl * Mb * gl[i];
        }
        cu_m = Gu * du;
        cl_m = -(Gl * dl);
    }
    if (a.fixed == 0) {
        float *py = a.dy, *pm = (a.dM && a.Mk) ? a.dM : nullptr;
        if (py || pm) {
            wave_scatter_add<float>(valid, ia, Gu, cu_m, py, pm, FloatAtomic());
            wave_scatter_add<float>(valid, ib, Gl, cl_m, py, pm, FloatAtomic());
        }
        if (a.dM && !a.Mk) {
            // global M: one sum per wave
            float v = cu_m + cl_m;
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(a.dM, v);
        }
    } else if (a.fixed == 1) {
        if (valid) {
            const float mx = fmaxf(fmaxf(fabsf(Gu), fabsf(Gl)), fmaxf(fabsf(cu_m), fabsf(cl_m)));
            atomicMax(a.maxbits, __float_as_uint(mx));
        }
    } else {
        const float mx = __uint_as_float(*a.maxbits);
        // 2^shift * mx * 2q < 2^63: no int64 overflow
        int e = 0;
        frexpf(mx > 0.0f ? mx : 1.0f, &e);
        int qbits = 0;
        frexp((double)(a.q > 0 ? a.q : 1), &qbits);
        const int shift = 61 - e - qbits;
        const long long fu = valid ? to_fixed(Gu, shift) : 0, fl = valid ? to_fixed(Gl, shift) : 0;
        const long long mu = valid ? to_fixed(cu_m, shift) : 0;
        const long long ml = valid ? to_fixed(cl_m, shift) : 0;
        unsigned long long *py = a.dy ? a.acc_y : nullptr;
        unsigned long long *pm = (a.dM && a.Mk) ? a.acc_m : nullptr;
        if (py || pm) {
            wave_scatter_add<long long>(valid, ia, fu, mu, (long long *)py, (long long *)pm,
                                        [](long long *p, long long v) {
                                            atomicAdd((unsigned long long *)p,
                                                      (unsigned long long)v);
                                        });
            wave_scatter_add<long long>(valid, ib, fl, ml, (long long *)py, (long long *)pm,
                                        [](long long *p, long long v) {
                                            atomicAdd((unsigned long long *)p,
                                                      (unsigned long long)v);
                                        });
        }
        if (a.dM && !a.Mk) {
            long long v = mu + ml;
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if ((threadIdx.x & 63) == 0) atomicAdd(a.acc_m, (unsigned long long)v);
        }
    }
}

__global__ void fixed_to_float_kernel(const unsigned long long *acc, int64_t n,
                                      const unsigned int *maxbits, int64_t q, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float mx = __uint_as_float(*maxbits);
    int e = 0;
    frexpf(mx > 0.0f ? mx : 1.0f, &e);
    int qbits = 0;
    frexp((double)(q > 0 ? q : 1), &qbits);
    const int shift = 61 - e - qbits;
    const double v = ldexp((double)(long long)acc[i], -shift);
    out[i] = (float)((double)out[i] + v);
}

__global__ void zero_u64_kernel(unsigned long long *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

typedef void (*BwdLaunch)(const BwdArgs &, dim3, dim3, hipStream_t);

template <int D>
void launch_bwd(const BwdArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL(backward_kernel<D>, g, b, 0, s, a);
}

static BwdLaunch bwd_table(int d)
{
    static const BwdLaunch t[kMaxDim + 1] = {
        nullptr,         &launch_bwd<1>,  &launch_bwd<2>,  &launch_bwd<3>,  &launch_bwd<4>,
        &launch_bwd<5>,  &launch_bwd<6>,  &launch_bwd<7>,  &launch_bwd<8>,  &launch_bwd<9>,
        &launch_bwd<10>, &launch_bwd<11>, &launch_bwd<12>, &launch_bwd<13>, &launch_bwd<14>,
        &launch_bwd<15>, &launch_bwd<16>};
    return (d >= 1 && d <= kMaxDim) ? t[d] : nullptr;
}

size_t backward_ws_bytes(int64_t n) { return align_up((size_t)(2 * n + 2) * 8, 256) + 256; }

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_fit_backward(const lip_metric *metric, const float *x, const float *y,
                                       int64_t n, float M, const float *Mk, const float *xq,
                                       int64_t q, const int32_t *arg_up, const int32_t *arg_lo,
                                       const float *dg, const float *dh_up, const float *dh_lo,
                                       float *dxq, float *dy, float *dM, void *ws, size_t ws_bytes,
                                       uint32_t flags, lip_stream stream)
{
    (void)y;
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~(LIP_FLAG_DETERMINISTIC | LIP_FLAG_CHECK_FINITE)) return LIP_E_ARG;
    if (n <= 0 || q < 0) return LIP_E_SHAPE;
    if (n > kMaxIndex || q > kMaxIndex) return LIP_E_SHAPE;
    if (!x || (q > 0 && (!xq || !arg_up || !arg_lo))) return LIP_E_ARG;
    if (!Mk && (!(M >= 0.0f) || !__builtin_isfinite(M))) return LIP_E_VALUE;
    const bool det = (flags & LIP_FLAG_DETERMINISTIC) != 0;
    const bool chk = (flags & LIP_FLAG_CHECK_FINITE) != 0;
    if ((det || chk) && (!ws || ws_bytes < backward_ws_bytes(n))) return LIP_E_WORKSPACE;
    if (q == 0) return LIP_OK;
    hipStream_t s = (hipStream_t)stream;
    if (chk) {
        const float *arr[6] = {x, Mk, xq, dg, dh_up, dh_lo};
        const int64_t cnt[6] = {n * mi.d, Mk ? n : 0, q * mi.d, dg ? q : 0, dh_up ? q : 0,
                                dh_lo ? q : 0};
        st = check_finite(arr, cnt, 6, ws, s);
        if (st != LIP_OK) return st;
    }
    BwdArgs a{};
    a.x = x;
    a.Mk = Mk;
    a.xq = xq;
    a.M = M;
    a.norm = mi.norm;
    a.n = n;
    a.q = q;
    a.arg_up = arg_up;
    a.arg_lo = arg_lo;
    a.dg = dg;
    a.dh_up = dh_up;
    a.dh_lo = dh_lo;
    a.dxq = dxq;
    a.dy = dy;
    a.dM = dM;
    for (int i = 0; i < kMaxDim; ++i) {
        a.w[i] = i < mi.d ? (float)mi.w[i] : 1.0f;
        a.mon[i] = i < mi.d ? mi.mon[i] : 0;
    }
    BwdLaunch launch = bwd_table(mi.d);
    const dim3 block(256), grid((unsigned)((q + 255) / 256));
    if (!det) {
        a.fixed = 0;
        launch(a, grid, block, s);
        return dev_status(hipGetLastError());
    }
    // deterministic: max pass, fixed-point accumulation, conversion
    char *p = (char *)ws;
    a.maxbits = (unsigned int *)p;
    a.acc_m = (unsigned long long *)(p + 256);
    a.acc_y = a.acc_m + (Mk ? n : 1);
    const int64_t nacc = (Mk ? n : 1) + n;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, (unsigned long long *)p, (int64_t)1);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((nacc + 255) / 256 > 4096 ? 4096 : (nacc + 255) / 256)),
                       dim3(256), 0, s, a.acc_m, nacc);
    a.fixed = 1;
    launch(a, grid, block, s);
    a.fixed = 2;
    launch(a, grid, block, s);
    if (dM) {
        const int64_t nm = Mk ? n : 1;
        hipLaunchKernelGGL(fixed_to_float_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s,
                           (const unsigned long long *)a.acc_m, nm, (const unsigned int *)a.maxbits, q, dM);
    }
    if (dy) {
        hipLaunchKernelGGL(fixed_to_float_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const unsigned long long *)a.acc_y, n, (const unsigned int *)a.maxbits, q, dy);
    }
    return dev_status(hipGetLastError());
}
