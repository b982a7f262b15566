// Host entry points of the step-function local constants of Sec. 4.3
// (lip_local_knots, lip_local_steps, lip_fit_eval_steps) and their small
// helper kernels; the pair kernels are in local_steps.hpp (tables) and
// local_fwd.hpp (bounds), instantiated per norm in local_steps_*.hip and
// local_fwd_*.hip.
#include <math.h>

#include "local_fwd.hpp"

namespace lip {

namespace {

constexpr int64_t kMaxKnotSample = 1ll << 26;

__host__ __device__ inline unsigned long long dbits(double v)
{
    unsigned long long b;
    __builtin_memcpy(&b, &v, sizeof b);
    return b;
}

__host__ __device__ inline double from_bits(unsigned long long b)
{
    double v;
    __builtin_memcpy(&v, &b, sizeof v);
    return v;
}

// Largest double S >= 0 whose correctly rounded square root is <= q, for
// q >= 0: the l2 decision sqrt(S) <= q is exactly S <= sq_threshold(q),
// because the rounded root is non-decreasing in S.  Starts at fl(q * q),
// which is within a few units of the answer, and steps one double at a time
// (bounded loops).
__host__ __device__ inline double sq_threshold(double q)
{
    if (!(q > 0.0)) return 0.0;
    if (!(q < __builtin_inf())) return __builtin_inf();
    double s = q * q;
    for (int it = 0; it < 64 && s > 0.0 && sqrt(s) > q; ++it) s = from_bits(dbits(s) - 1);
    for (int it = 0; it < 64 && sqrt(from_bits(dbits(s) + 1)) <= q; ++it)
        s = from_bits(dbits(s) + 1);
    return s;
}

struct Weights {
    double w[kMaxDim];
};

// Sampled pair distances (symmetric distance, FP64, coordinates in index
// order, weight applied to each component) as sort keys: a non-negative
// double orders like its bit pattern.  Positions m..P-1 are padding (~0).
__global__ void knot_dist_kernel(const float *x, int d, int norm, Weights w,
                                 const long long *pairs, int64_t m, int64_t P,
                                 unsigned long long *keys)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < P; s += stride) {
        if (s >= m) {
            keys[s] = ~0ull;
            continue;
        }
        const int64_t i = pairs[2 * s], j = pairs[2 * s + 1];
        double acc = 0.0;
        for (int c = 0; c < d; ++c) {
            const double a = w.w[c] * fabs((double)x[i * d + c] - (double)x[j * d + c]);
            if (norm == 1) acc = acc + a;
            else if (norm == 2) acc = acc + a * a;
            else acc = a > acc ? a : acc;
        }
        if (norm == 2) acc = sqrt(acc);
        keys[s] = dbits(acc);
    }
}

struct Ranks {
    int64_t r[kMaxKnots];
};

__global__ void knot_pick_kernel(const unsigned long long *keys, Ranks rk, int K, double *knots)
{
    const int j = threadIdx.x;
    if (j < K) knots[j] = from_bits(keys[rk.r[j]]);
}

// Merge of the builder's chunk partials: nearest distance (min), its slope
// (max over the chunks that attain the min), the knot maxima (max); then the
// table: V_0, V_s = max(v_s, V_0) (a knot below d1 adds nothing beyond the
// nearest data), V_{K+1} = max(v_all, V_0); +inf rows for infinite slopes.
__global__ void steps_combine_kernel(StepArgs A, int KB)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = A.ds.n;
    if (i >= n) return;
    const int nc = A.ds.n_chunks;
    double d1 = __builtin_inf();
    int inf = 0;
    for (int c = 0; c < nc; ++c) {
        const double v = A.p_d1[(int64_t)c * n + i];
        d1 = v < d1 ? v : d1;
        inf |= A.p_inf[(int64_t)c * n + i];
    }
    double v0 = 0.0;
    for (int c = 0; c < nc; ++c) {
        const double v = A.p_v0[(int64_t)c * n + i];
        if (A.p_d1[(int64_t)c * n + i] == d1 && v > v0) v0 = v;
    }
    A.d1[i] = d1;
    const int K = A.K;
    for (int s = 0; s < K + 2; ++s) {
        const int j = s == 0 ? -1 : (s <= K ? s - 1 : KB);
        double v = v0;
        if (j >= 0) {
            for (int c = 0; c < nc; ++c) {
                const double pv = A.p_v[((int64_t)c * (KB + 1) + j) * n + i];
                v = pv > v ? pv : v;
            }
        }
        if (inf) v = __builtin_inf();
        if (A.V64) A.V64[i * (K + 2) + s] = v;
        if (A.V32) A.V32[i * (K + 2) + s] = round_up_f32(v);
    }
}

// Forward staging, part 1: first-segment threshold per datum and the table
// in segment-major order (K + 2 rows).
__global__ void steps_stage_kernel(const double *d1, const float *V, int K, int norm, int64_t n,
                                   int64_t npad, double *T1, float *Vs)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        const bool in = k < n;
        T1[k] = in ? (norm == 2 ? sq_threshold(d1[k]) : d1[k]) : 0.0;
        for (int s = 0; s < K + 2; ++s) Vs[(int64_t)s * npad + k] = in ? V[k * (K + 2) + s] : 0.0f;
    }
}

// Largest |x'_j| over the data and the queries (x' = the FP32 transform of
// the bound path: origin, weights, signs, free coordinates first), as float
// bits (non-negative floats order like their bit patterns).
__global__ void steps_amax_kernel(const float *x, int64_t n, const float *xq, int64_t q, int d,
                                  Xform xf, unsigned int *amax)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = n + q;
    for (int j = 0; j < d; ++j) {
        float m = 0.0f;
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
            const float v = k < n ? xf_coord(xf, x + k * d, j) : xf_coord(xf, xq + (k - n) * d, j);
            m = fmaxf(m, fabsf(v));
        }
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0) atomicMax(amax + j, __float_as_uint(m));
    }
}

__global__ void zero_u32_kernel(unsigned int *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Forward staging, part 2: the FP32 records [x' | y | VL0 | VL1 | D1hi] of
// local_fwd.hpp.  VL0 / VL1 are the smallest table entries overall and past
// the first segment; D1hi = up(d1 (1 + rho) + alpha), alpha from amax.
__global__ void steps_rec_kernel(const float *x, const float *y, const double *d1, const float *V,
                                 int K, int d, int64_t n, int64_t npad, Xform xf,
                                 const unsigned int *amax, float *rec)
{
    const int S = d + kStepRec;
    double asum = 0.0;
    for (int j = 0; j < d; ++j) asum += (double)__uint_as_float(amax[j]);
    const double alpha = 0x1p-21 * asum + 0x1p-70;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        float *o = rec + k * S;
        if (k >= n) {
            for (int j = 0; j < S; ++j) o[j] = 0.0f;
            continue;
        }
        for (int j = 0; j < d; ++j) o[j] = xf_coord(xf, x + k * d, j);
        o[d] = y[k];
        float v0 = V[k * (K + 2)], v1 = V[k * (K + 2) + 1];
        for (int s = 1; s < K + 2; ++s) {
            const float v = V[k * (K + 2) + s];
            v1 = v < v1 ? v : v1;
        }
        v0 = v1 < v0 ? v1 : v0;
        o[d + 1] = v0;
        o[d + 2] = v1;
        const double t = d1[k] * (1.0 + (double)kStepRho) + alpha;
        o[d + 3] = round_up_f32(t);
    }
}

StepLaunch get_step_fwd(int norm, int d, int dm)
{
    switch (norm) {
    case LIP_L1: return step_fwd_l1(d, dm);
    case LIP_L2: return step_fwd_l2(d, dm);
    case LIP_LINF: return step_fwd_linf(d, dm);
    default: return nullptr;
    }
}

bool get_steps(int norm, int d, bool hasw, int kb, StepLaunchers *L)
{
    switch (norm) {
    case LIP_L1: return step_table_l1(d, hasw, kb, L);
    case LIP_L2: return step_table_l2(d, hasw, kb, L);
    case LIP_LINF: return step_table_linf(d, hasw, kb, L);
    default: return false;
    }
}

lip_status check_knots(const double *knots, int32_t K)
{
    if (K < 0 || K > kMaxKnots) return LIP_E_SHAPE;
    if (K > 0 && !knots) return LIP_E_ARG;
    for (int j = 0; j < K; ++j) {
        if (!(knots[j] >= 0.0)) return LIP_E_VALUE;
        if (j > 0 && !(knots[j] >= knots[j - 1])) return LIP_E_VALUE;
    }
    return LIP_OK;
}

unsigned grid1d(int64_t work)
{
    int64_t g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)(g < 1 ? 1 : g);
}

size_t builder_partial_bytes(int64_t n)
{
    return align_up((size_t)kStepMaxChunks * (size_t)n * (8 + 8 + 4 + 8 * (kMaxKnots + 1)), 256);
}

}  // namespace

size_t local_ws_bytes(int64_t n, int64_t q, int d)
{
    const int64_t npad = ds_npad(n);
    const size_t staged = align_up((size_t)npad * (size_t)(d + 2) * 8, 256) +
                          align_up((size_t)npad * 8, 256) +
                          align_up((size_t)npad * (kMaxKnots + 2) * 4, 256) +
                          align_up((size_t)npad * (size_t)(d + kStepRec) * 4, 256) + 256 +
                          align_up((size_t)sort_len(q > 0 ? q : 1) * 8, 256) + 256;
    size_t part = builder_partial_bytes(n);
    const size_t fwd = partial_bytes(q);
    const size_t knots = align_up((size_t)sort_len(n) * 8, 256) + align_up((size_t)n * 16, 256);
    if (fwd > part) part = fwd;
    if (knots > part) part = knots;
    return staged + part + 4096;
}

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_local_knots(const lip_metric *metric, const float *x, int64_t n,
                                      const int64_t *pairs, int64_t m, const double *probs,
                                      int32_t K, double *knots, void *ws, size_t ws_bytes,
                                      uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || n > kMaxIndex - kDsTile) return LIP_E_SHAPE;
    if (m < 1 || m > kMaxKnotSample || K < 0 || K > kMaxKnots) return LIP_E_SHAPE;
    if (!x || !pairs || (K > 0 && (!probs || !knots))) return LIP_E_ARG;
    for (int j = 0; j < K; ++j) {
        if (!(probs[j] > 0.0 && probs[j] <= 1.0)) return LIP_E_VALUE;
        if (j > 0 && !(probs[j] >= probs[j - 1])) return LIP_E_VALUE;
    }
    for (int64_t s = 0; s < 2 * m; ++s)
        if (pairs[s] < 0 || pairs[s] >= n) return LIP_E_VALUE;
    const int64_t P = sort_len(m);
    const size_t need = align_up((size_t)P * 8, 256) + align_up((size_t)m * 16, 256);
    if (!ws || ws_bytes < need) return LIP_E_WORKSPACE;
    if (K == 0) return LIP_OK;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[1] = {x};
        const int64_t cnt[1] = {n * mi.d};
        st = check_finite(arr, cnt, 1, ws, s);
        if (st != LIP_OK) return st;
    }
    unsigned long long *keys = (unsigned long long *)ws;
    long long *dpairs = (long long *)((char *)ws + align_up((size_t)P * 8, 256));
    if (hipMemcpyAsync(dpairs, pairs, (size_t)m * 16, hipMemcpyHostToDevice, s) != hipSuccess)
        return LIP_E_DEVICE;
    Weights w{};
    for (int i = 0; i < kMaxDim; ++i) w.w[i] = i < mi.d ? mi.w[i] : 1.0;
    hipLaunchKernelGGL(knot_dist_kernel, dim3(grid1d(P)), dim3(256), 0, s, x, mi.d, mi.norm, w,
                       (const long long *)dpairs, m, P, keys);
    if (launch_sort_u64(keys, P, s) != hipSuccess) return LIP_E_DEVICE;
    Ranks rk{};
    for (int j = 0; j < K; ++j) {
        int64_t c = (int64_t)ceil(probs[j] * (double)m) - 1;
        rk.r[j] = c < 0 ? 0 : (c > m - 1 ? m - 1 : c);
    }
    hipLaunchKernelGGL(knot_pick_kernel, dim3(1), dim3(64), 0, s, (const unsigned long long *)keys,
                       rk, K, knots);
    return dev_status(hipGetLastError());
}

extern "C" lip_status lip_local_steps(const lip_metric *metric, const float *x, const float *y,
                                      int64_t n, const double *knots, int32_t K, double *d1,
                                      double *V64, float *V32, void *ws, size_t ws_bytes,
                                      uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || n > kMaxIndex - kDsTile) return LIP_E_SHAPE;
    st = check_knots(knots, K);
    if (st != LIP_OK) return st;
    if (!x || !y || !d1) return LIP_E_ARG;
    if (!ws || ws_bytes < local_ws_bytes(n, 0, mi.d)) return LIP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[2] = {x, y};
        const int64_t cnt[2] = {n * mi.d, n};
        st = check_finite(arr, cnt, 2, ws, s);
        if (st != LIP_OK) return st;
    }
    StepArgs A{};
    Signs sg{};
    const bool hasw = fill_ds_metric(mi, false, &A.ds, &sg);
    const int KB = K <= 4 ? 4 : 8;
    StepLaunchers L;
    if (!get_steps(mi.norm, mi.d, hasw, KB, &L)) return LIP_E_UNSUPPORTED;
    A.K = K;
    for (int j = 0; j < kMaxKnots; ++j) A.knot[j] = j < K ? knots[j] : __builtin_inf();
    A.ds.n = n;
    A.ds.npad = ds_npad(n);
    A.ds.norm = mi.norm;
    double *X = (double *)ws;
    A.ds.X = X;
    char *p = (char *)ws + align_up((size_t)A.ds.npad * (size_t)(mi.d + 2) * 8, 256) +
              align_up((size_t)A.ds.npad * 8, 256) +
              align_up((size_t)A.ds.npad * (kMaxKnots + 2) * 4, 256) +
              align_up((size_t)A.ds.npad * (size_t)(mi.d + kStepRec) * 4, 256) + 256;
    choose_chunks(n, 64 * kDsRows, kStepMaxChunks, &A.ds);
    const size_t e = (size_t)A.ds.n_chunks * (size_t)n;
    A.p_d1 = (double *)p;
    A.p_v0 = A.p_d1 + e;
    A.p_v = A.p_v0 + e;
    A.p_inf = (int32_t *)(A.p_v + e * (KB + 1));
    A.d1 = d1;
    A.V64 = V64;
    A.V32 = V32;
    if (launch_stage64(mi.d, x, y, nullptr, 0.0f, n, A.ds.npad, sg, X, s) != hipSuccess)
        return LIP_E_DEVICE;
    L.build(A, dim3(grid_for_rows(n, 64 * kDsRows, A.ds.n_chunks)), dim3(256), s);
    hipLaunchKernelGGL(steps_combine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A,
                       KB);
    return dev_status(hipGetLastError());
}

extern "C" lip_status lip_fit_eval_steps(const lip_metric *metric, const float *x, const float *y,
                                         int64_t n, const lip_steps *steps, const float *xq,
                                         int64_t q, float *g, float *h_up, float *h_lo,
                                         int32_t *arg_up, int32_t *arg_lo, void *ws,
                                         size_t ws_bytes, uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & LIP_FLAG_BF16) return LIP_E_UNSUPPORTED;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || q < 0 || n > kMaxIndex - kDsTile || q > kMaxIndex) return LIP_E_SHAPE;
    if (!steps) return LIP_E_ARG;
    st = check_knots(steps->knots, steps->K);
    if (st != LIP_OK) return st;
    if (!x || !y || !steps->d1 || !steps->V || (q > 0 && !xq)) return LIP_E_ARG;
    if (!ws || ws_bytes < kOriginBytes + local_ws_bytes(n, q, mi.d)) return LIP_E_WORKSPACE;
    if (q == 0) return LIP_OK;
    hipStream_t s = (hipStream_t)stream;
    const int K = steps->K;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[4] = {x, y, steps->V, xq};
        const int64_t cnt[4] = {n * mi.d, n, n * (K + 2), q * mi.d};
        st = check_finite(arr, cnt, 4, ws, s);
        if (st != LIP_OK) return st;
    }
    StepArgs A{};
    Signs sg{};
    (void)fill_ds_metric(mi, true, &A.ds, &sg);
    StepLaunch launch = get_step_fwd(mi.norm, mi.d, mi.dm);
    if (!launch) return LIP_E_UNSUPPORTED;
    A.K = K;
    for (int j = 0; j < kMaxKnots; ++j) {
        const double kq = j < K ? steps->knots[j] : __builtin_inf();
        A.knot[j] = kq;
        A.knotS[j] = mi.norm == LIP_L2 ? sq_threshold(kq) : kq;
    }
    for (int j = 0; j < kMaxDim; ++j) A.qsign[j] = sg.s[j];
    A.xf = mi.xf;
    st = origin_for(x, n, mi.d, A.xf, ws, s);
    if (st != LIP_OK) return st;
    ws = (char *)ws + kOriginBytes;
    A.ds.n = n;
    A.ds.npad = ds_npad(n);
    A.ds.norm = mi.norm;
    double *X = (double *)ws;
    char *p = (char *)ws + align_up((size_t)A.ds.npad * (size_t)(mi.d + 2) * 8, 256);
    double *T1 = (double *)p;
    p += align_up((size_t)A.ds.npad * 8, 256);
    float *Vs = (float *)p;
    p += align_up((size_t)A.ds.npad * (kMaxKnots + 2) * 4, 256);
    float *rec = (float *)p;
    p += align_up((size_t)A.ds.npad * (size_t)(mi.d + kStepRec) * 4, 256);
    unsigned int *amax = (unsigned int *)p;
    p += 256;
    const int64_t PQ = sort_len(q);
    unsigned long long *qorder = (unsigned long long *)p;
    p += align_up((size_t)PQ * 8, 256);
    unsigned int *qbb = (unsigned int *)p;
    p += 256;
    A.qorder = qorder;
    A.ds.X = X;
    A.T1 = T1;
    A.Vs = Vs;
    A.rec = rec;
    A.xq = xq;
    A.q = q;
    A.g = g;
    A.h_up = h_up;
    A.h_lo = h_lo;
    A.arg_up = arg_up;
    A.arg_lo = arg_lo;
    // column split when the queries alone do not fill the chip
    const int R = step_rows(mi.d);
    const int64_t qwaves = (q + 64 * R - 1) / (64 * R);
    int nc = 1;
    while (nc < kStepMaxChunks * 2 && qwaves * nc < 8192 && n >= (int64_t)nc * 2 * kDsTile &&
           (int64_t)nc * 2 * q <= kMaxPartials)
        nc *= 2;
    int64_t cols = (n + nc - 1) / nc;
    cols = (cols + kDsTile - 1) / kDsTile * kDsTile;
    A.ds.chunk_cols = cols;
    A.ds.n_chunks = (int)((n + cols - 1) / cols);
    if (A.ds.n_chunks > 1) {
        const int64_t entries = (int64_t)A.ds.n_chunks * q;
        A.part_v = (float *)p;
        A.part_i = (int32_t *)(p + align_up((size_t)entries * 2 * sizeof(float), 256));
    }
    if (launch_stage64(mi.d, x, y, nullptr, 0.0f, n, A.ds.npad, sg, X, s) != hipSuccess)
        return LIP_E_DEVICE;
    hipLaunchKernelGGL(steps_stage_kernel, dim3(grid1d(A.ds.npad)), dim3(256), 0, s, steps->d1,
                       steps->V, K, mi.norm, n, A.ds.npad, T1, Vs);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, amax, mi.d);
    int64_t ga = (n + q + 255) / 256;
    if (ga > 1024) ga = 1024;
    hipLaunchKernelGGL(steps_amax_kernel, dim3((unsigned)ga), dim3(256), 0, s, x, n, xq, q, mi.d,
                       A.xf, amax);
    hipLaunchKernelGGL(steps_rec_kernel, dim3(grid1d(A.ds.npad)), dim3(256), 0, s, x, y,
                       steps->d1, steps->V, K, mi.d, n, A.ds.npad, A.xf,
                       (const unsigned int *)amax, rec);
    if (launch_query_order(xq, q, mi.d, qbb, qorder, PQ, s) != hipSuccess) return LIP_E_DEVICE;
    const unsigned grid = (unsigned)(((qwaves + 3) / 4) * A.ds.n_chunks);
    launch(A, dim3(grid), dim3(256), s);
    if (hipGetLastError() != hipSuccess) return LIP_E_DEVICE;
    if (A.ds.n_chunks > 1) {
        CombineArgs c{};
        c.part_v = A.part_v;
        c.part_i = A.part_i;
        c.q = q;
        c.n_chunks = A.ds.n_chunks;
        c.g = g;
        c.h_up = h_up;
        c.h_lo = h_lo;
        c.arg_up = arg_up;
        c.arg_lo = arg_lo;
        if (launch_combine(c, s) != hipSuccess) return LIP_E_DEVICE;
    }
    return dev_status(hipGetLastError());
}
