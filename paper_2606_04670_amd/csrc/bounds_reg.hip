// Bounds of Eq. (2)-(3) with monotonicity on parts of the domain (Sec. 4.2)
// and the host side of that path.
//
// Every coordinate carries the two intervals where f is not decreasing (ND)
// and not increasing (NI) (kinds 0 / +1 / -1 are the cases where these are
// everything or nothing; an empty interval is stored as [0, 0]).  With
// c(v) = w clamp(v, s, t) the clamped, weighted coordinate, the travelled
// length inside [s, t] is |c(q) - c(x)|, and the difference a = c_ND(q) -
// c_ND(x) is positive when moving towards larger values, negative otherwise
// (likewise b for NI).  So the upper component (length where f may rise in
// the direction of travel: inside ND moving up, inside NI moving down) is
// max(a, -b), and the lower one max(b, -a).  The clamped data coordinates are
// staged per datum and the clamped query coordinates formed once per query,
// so a pair costs two subtractions and two maxima per coordinate, then the
// norm, as in the fused kernel.  A lane owns R queries, a wave 64 R queries
// and one data chunk; records [c_ND(x_0), c_NI(x_0), .. | y | M_k] come four
// at a time through scalar loads; the first index of the running min / max is
// kept per pair (strict comparisons, data in ascending order), chunk
// partials go through the bound path's combine.
#include "host_common.hpp"
#include "lip_device.hpp"

namespace lip {

namespace {

struct RegArgs {
    const float *rec;  // [npad][2 D + 2]
    int64_t n, npad;
    int32_t n_chunks;
    int32_t pad0;
    int64_t chunk_cols;
    float nd_s[kMaxDim], nd_t[kMaxDim], ni_s[kMaxDim], ni_t[kMaxDim], w[kMaxDim];
    const float *xq;
    int64_t q;
    float *g, *h_up, *h_lo;
    int32_t *arg_up, *arg_lo;
    float *part_v;
    int32_t *part_i;
};

constexpr int reg_rows(int D) { return rows_for_dim(D) / 2 > 0 ? rows_for_dim(D) / 2 : 1; }

// w clamp(v, s, t) (s <= t; the median of three needs no canonicalisation)
__device__ __forceinline__ float reg_clamp(float v, float s, float t, float w)
{
    return w * __builtin_amdgcn_fmed3f(v, s, t);
}

template <int D, int NORM>
__device__ __forceinline__ void reg_dist(const float (&q)[2 * D], const float *xk, float &tu,
                                         float &tl)
{
    float su = 0.0f, sl = 0.0f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float a = q[2 * i] - xk[2 * i];          // signed length inside ND
        const float b = q[2 * i + 1] - xk[2 * i + 1];  // signed length inside NI
        const float cu = fmaxf(a, -b), cl = fmaxf(b, -a);
        if (NORM == kNormL1) {
            su = i == 0 ? cu : su + cu;
            sl = i == 0 ? cl : sl + cl;
        } else if (NORM == kNormL2) {
            su = i == 0 ? cu * cu : fmaf(cu, cu, su);
            sl = i == 0 ? cl * cl : fmaf(cl, cl, sl);
        } else {
            su = i == 0 ? cu : fmaxf(su, cu);
            sl = i == 0 ? cl : fmaxf(sl, cl);
        }
    }
    if (NORM == kNormL2) {
        su = __builtin_amdgcn_sqrtf(su);
        sl = __builtin_amdgcn_sqrtf(sl);
    }
    tu = su;
    tl = sl;
}

template <int D, int NORM>
__global__ void __launch_bounds__(256) bounds_reg_kernel(RegArgs A)
{
    constexpr int R = reg_rows(D);
    constexpr int S = 2 * D + 2;
    constexpr int G = 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = blockIdx.x % A.n_chunks;
    const int64_t qb = (int64_t)(blockIdx.x / A.n_chunks) * (blockDim.x >> 6) + wave;
    const int64_t q0 = qb * 64 * R;
    if (q0 >= A.q) return;
    const int lane = threadIdx.x & 63;
    float qv[R][2 * D], hu[R], hl[R];
    int au[R], al[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t j = q0 + r * 64 + lane;
        j = j < A.q ? j : A.q - 1;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float v = A.xq[j * D + i];
            qv[r][2 * i] = reg_clamp(v, A.nd_s[i], A.nd_t[i], A.w[i]);
            qv[r][2 * i + 1] = reg_clamp(v, A.ni_s[i], A.ni_t[i], A.w[i]);
        }
        hu[r] = __builtin_inff();
        hl[r] = -__builtin_inff();
        au[r] = -1;
        al[r] = -1;
    }
    const int64_t c0 = (int64_t)chunk * A.chunk_cols;
    int64_t c1 = c0 + A.chunk_cols;
    c1 = c1 < A.n ? c1 : A.n;
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
            const float yk = xk[2 * D], mk = xk[2 * D + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float tu, tl;
                reg_dist<D, NORM>(qv[r], xk, tu, tl);
                const float u = fmaf(mk, tu, yk), l = fmaf(-mk, tl, yk);
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

__global__ void reg_stage_kernel(const float *x, const float *y, const float *Mk, float M, int d,
                                 int64_t n, int64_t npad, RegArgs A, float *rec)
{
    const int S = 2 * d + 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        float *o = rec + k * S;
        const bool in = k < n;
        for (int j = 0; j < d; ++j) {
            const float v = in ? x[k * d + j] : 0.0f;
            o[2 * j] = reg_clamp(v, A.nd_s[j], A.nd_t[j], A.w[j]);
            o[2 * j + 1] = reg_clamp(v, A.ni_s[j], A.ni_t[j], A.w[j]);
        }
        o[2 * d] = in ? y[k] : 0.0f;
        o[2 * d + 1] = in ? (Mk ? Mk[k] : M) : 0.0f;
    }
}

typedef void (*RegLaunch)(const RegArgs &, dim3, dim3, hipStream_t);

template <int D, int NORM>
void launch_reg(const RegArgs &a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((bounds_reg_kernel<D, NORM>), g, b, 0, s, a);
}

template <int NORM>
RegLaunch reg_table(int d)
{
    switch (d) {
#define LIP_RG_CASE(DD) \
    case DD: return &launch_reg<DD, NORM>;
        LIP_RG_CASE(1) LIP_RG_CASE(2) LIP_RG_CASE(3) LIP_RG_CASE(4)
        LIP_RG_CASE(5) LIP_RG_CASE(6) LIP_RG_CASE(7) LIP_RG_CASE(8)
        LIP_RG_CASE(9) LIP_RG_CASE(10) LIP_RG_CASE(11) LIP_RG_CASE(12)
        LIP_RG_CASE(13) LIP_RG_CASE(14) LIP_RG_CASE(15) LIP_RG_CASE(16)
#undef LIP_RG_CASE
    default: return nullptr;
    }
}

constexpr int kRegMaxChunks = 16;

int64_t reg_npad(int64_t n) { return (n + 63) / 64 * 64; }

}  // namespace

size_t reg_ws_bytes(int64_t n, int64_t q, int d)
{
    return align_up((size_t)reg_npad(n) * (size_t)(2 * d + 2) * 4, 256) + partial_bytes(q) + 256;
}

lip_status run_bounds_reg(const MetricInfo &mi, const float *x, const float *y, int64_t n,
                          float M, const float *Mk, const float *xq, int64_t q, float *g,
                          float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws,
                          size_t ws_bytes, hipStream_t s)
{
    if (ws_bytes < reg_ws_bytes(n, q, mi.d)) return LIP_E_WORKSPACE;
    RegLaunch launch = mi.norm == LIP_L1   ? reg_table<kNormL1>(mi.d)
                       : mi.norm == LIP_L2 ? reg_table<kNormL2>(mi.d)
                                           : reg_table<kNormLinf>(mi.d);
    if (!launch) return LIP_E_UNSUPPORTED;
    RegArgs A{};
    A.n = n;
    A.npad = reg_npad(n);
    for (int i = 0; i < kMaxDim; ++i) {
        const bool in = i < mi.d;
        float nds = in ? mi.nd_s[i] : 0.0f, ndt = in ? mi.nd_t[i] : 0.0f;
        float nis = in ? mi.ni_s[i] : 0.0f, nit = in ? mi.ni_t[i] : 0.0f;
        // an empty region clamps everything to one point: zero length
        if (!(nds <= ndt)) nds = ndt = 0.0f;
        if (!(nis <= nit)) nis = nit = 0.0f;
        A.nd_s[i] = nds;
        A.nd_t[i] = ndt;
        A.ni_s[i] = nis;
        A.ni_t[i] = nit;
        A.w[i] = in ? (float)mi.w[i] : 1.0f;
    }
    float *rec = (float *)ws;
    char *p = (char *)ws + align_up((size_t)A.npad * (size_t)(2 * mi.d + 2) * 4, 256);
    A.rec = rec;
    A.xq = xq;
    A.q = q;
    A.g = g;
    A.h_up = h_up;
    A.h_lo = h_lo;
    A.arg_up = arg_up;
    A.arg_lo = arg_lo;
    const int R = reg_rows(mi.d);
    const int64_t qwaves = (q + 64 * R - 1) / (64 * R);
    int nc = 1;
    while (nc < kRegMaxChunks && qwaves * nc < 16384 && n >= (int64_t)nc * 2 * 64 &&
           (int64_t)nc * 2 * q <= kMaxPartials)
        nc *= 2;
    int64_t cols = (n + nc - 1) / nc;
    cols = (cols + 63) / 64 * 64;
    A.chunk_cols = cols;
    A.n_chunks = (int)((n + cols - 1) / cols);
    if (A.n_chunks > 1) {
        const int64_t entries = (int64_t)A.n_chunks * q;
        A.part_v = (float *)p;
        A.part_i = (int32_t *)(p + align_up((size_t)entries * 2 * sizeof(float), 256));
    }
    int64_t gs = (A.npad + 255) / 256;
    if (gs > 65536) gs = 65536;
    hipLaunchKernelGGL(reg_stage_kernel, dim3((unsigned)gs), dim3(256), 0, s, x, y, Mk, M, mi.d,
                       n, A.npad, A, rec);
    const unsigned grid = (unsigned)(((qwaves + 3) / 4) * A.n_chunks);
    launch(A, dim3(grid), dim3(256), s);
    if (hipGetLastError() != hipSuccess) return LIP_E_DEVICE;
    if (A.n_chunks > 1) {
        CombineArgs c{};
        c.part_v = A.part_v;
        c.part_i = A.part_i;
        c.q = q;
        c.n_chunks = A.n_chunks;
        c.g = g;
        c.h_up = h_up;
        c.h_lo = h_lo;
        c.arg_up = arg_up;
        c.arg_lo = arg_lo;
        if (launch_combine(c, s) != hipSuccess) return LIP_E_DEVICE;
    }
    return dev_status(hipGetLastError());
}

}  // namespace lip
