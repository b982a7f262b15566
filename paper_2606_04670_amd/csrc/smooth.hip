// Host entry point of the smoothing objective (lip_smooth_objective) and its
// staging / reduction kernels; the pair kernel is in smooth.hpp,
// instantiated per norm in smooth_{l1,l2,linf}.hip.
#include "smooth.hpp"

namespace lip {

namespace {

// Records [x' | z = y + eps | M_k] with the bound path's coordinate
// transform, with the pre-screening (c > 0) followed by [y | fl32(c M_k)];
// padded records are zero (never read as columns).
__global__ void smooth_stage_kernel(const float *x, const float *y, const float *eps,
                                    const float *Mk, float M, double c, int d, int64_t n,
                                    int64_t npad, Xform xf, float *rec)
{
    const int S = d + (c > 0.0 ? 4 : 2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        float *o = rec + k * S;
        if (k >= n) {
            for (int j = 0; j < S; ++j) o[j] = 0.0f;
            continue;
        }
        for (int j = 0; j < d; ++j) o[j] = xf_coord(xf, x + k * d, j);
        o[d] = y[k] + eps[k];
        const float m = Mk ? Mk[k] : M;
        o[d + 1] = m;
        if (c > 0.0) {
            o[d + 2] = y[k];
            o[d + 3] = (float)(c * (double)m);
        }
    }
}

// Largest staged coordinate magnitude per coordinate (bit patterns of
// non-negative floats order as integers; amax starts at zero).
__global__ void smooth_amax_kernel(const float *x, int64_t n, int d, Xform xf, unsigned int *amax)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int j = 0; j < d; ++j) {
        float m = 0.0f;
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
            m = fmaxf(m, fabsf(xf_coord(xf, x + k * d, j)));
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0) atomicMax(amax + j, __float_as_uint(m));
    }
}

// alpha = 2^-21 sum_j max |x'_j| + 2^-70, rounded up: the absolute part of
// the FP32 distance's error against the FP64 one (the staged coordinates
// fl(fl(x - o) c) carry two roundings relative to the centred coordinates,
// not to their difference: at most 2^-22 max |x'_j| per coordinate
// difference, doubled for margin; plus underflow of FP32 squares).  Runs as
// one wave.
__global__ void smooth_alpha_kernel(unsigned int *amax, int d, float *alpha)
{
    if (threadIdx.x != 0) return;
    double a = 0.0;
    for (int j = 0; j < d; ++j) a += (double)__uint_as_float(amax[j]);
    alpha[0] = round_up_f32(0x1p-21 * a + 0x1p-70);
}

__global__ void smooth_zero_kernel(unsigned int *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Weights and free / monotone selectors of the FP64 decisions, [2][kMaxDim].
struct WeightsSel {
    double v[2 * kMaxDim];
};

__global__ void smooth_wf_kernel(WeightsSel ws, double *wf)
{
    if ((int)threadIdx.x < 2 * kMaxDim) wf[threadIdx.x] = ws.v[threadIdx.x];
}

// Per row: the chunk partials in chunk order plus the (1/p) eps^2 term and
// its derivative.
__global__ void smooth_rows_kernel(const double *pF, const double *pG, int n_chunks, int64_t n,
                                   const float *eps, double p, double *rowF, float *grad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double f = 0.0, g = 0.0;
    for (int c = 0; c < n_chunks; ++c) {
        f += pF[(int64_t)c * n + i];
        g += pG[(int64_t)c * n + i];
    }
    const double e = (double)eps[i];
    rowF[i] = f + e * e / p;
    if (grad) grad[i] = (float)(g + 2.0 * e / p);
}

// F = sum of the row values in a fixed order: thread t adds rows t, t + 1024,
// ... in turn, then a fixed tree over the 1024 partial sums.
__global__ void __launch_bounds__(1024) smooth_reduce_kernel(const double *rowF, int64_t n,
                                                             double *F)
{
    __shared__ double s[1024];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) a += rowF[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) F[0] = s[0];
}

SmoothLaunch get_smooth(int norm, int d, int dm, bool local, bool prune)
{
    switch (norm) {
    case LIP_L1: return smooth_l1(d, dm, local, prune);
    case LIP_L2: return smooth_l2(d, dm, local, prune);
    case LIP_LINF: return smooth_linf(d, dm, local, prune);
    default: return nullptr;
    }
}

int64_t smooth_npad(int64_t n) { return (n + kSmoothTile - 1) / kSmoothTile * kSmoothTile; }

}  // namespace

size_t smooth_ws_bytes(int64_t n, int d)
{
    const int64_t npad = smooth_npad(n);
    return align_up((size_t)npad * (size_t)(d + 4) * 4, 256) +
           2 * align_up((size_t)kSmoothMaxChunks * (size_t)n * 8, 256) +
           align_up((size_t)n * 8, 256) + align_up((size_t)ds_npad(n) * (size_t)(d + 2) * 8, 256) +
           768;
}

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_smooth_objective(const lip_metric *metric, const float *x,
                                           const float *y, int64_t n, float M, const float *Mk,
                                           const float *eps, double p, double prune, double *F,
                                           float *grad, void *ws, size_t ws_bytes, uint32_t flags,
                                           lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || n > kMaxIndex - kSmoothTile) return LIP_E_SHAPE;
    if (!x || !y || !eps) return LIP_E_ARG;
    if (!Mk && (!(M >= 0.0f) || !__builtin_isfinite(M))) return LIP_E_VALUE;
    if (!(p > 0.0) || !__builtin_isfinite(p)) return LIP_E_VALUE;
    if (!(prune >= 0.0) || !__builtin_isfinite(prune)) return LIP_E_VALUE;
    if (!ws || ws_bytes < kOriginBytes + smooth_ws_bytes(n, mi.d)) return LIP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[4] = {x, y, eps, Mk};
        const int64_t cnt[4] = {n * mi.d, n, n, Mk ? n : 0};
        st = check_finite(arr, cnt, 4, ws, s);
        if (st != LIP_OK) return st;
    }
    const bool pr = prune > 0.0;
    SmoothLaunch launch = get_smooth(mi.norm, mi.d, mi.dm, Mk != nullptr, pr);
    if (!launch) return LIP_E_UNSUPPORTED;
    SmoothArgs A{};
    A.n = n;
    A.npad = smooth_npad(n);
    A.c = prune;
    Xform xf = mi.xf;
    st = origin_for(x, n, mi.d, xf, ws, s);
    if (st != LIP_OK) return st;
    char *p0 = (char *)ws + kOriginBytes;
    float *rec = (float *)p0;
    p0 += align_up((size_t)A.npad * (size_t)(mi.d + 4) * 4, 256);
    const int R = smooth_rows(mi.d, pr);
    const int64_t row_waves = (n + 64 * R - 1) / (64 * R);
    int64_t nc = (8192 + row_waves - 1) / row_waves;
    if (nc > kSmoothMaxChunks) nc = kSmoothMaxChunks;
    if (nc < 1) nc = 1;
    int64_t cols = (n + nc - 1) / nc;
    cols = (cols + kSmoothTile - 1) / kSmoothTile * kSmoothTile;
    A.chunk_cols = cols;
    A.n_chunks = (int)((n + cols - 1) / cols);
    A.rec = rec;
    A.pF = (double *)p0;
    p0 += align_up((size_t)kSmoothMaxChunks * (size_t)n * 8, 256);
    A.pG = (double *)p0;
    p0 += align_up((size_t)kSmoothMaxChunks * (size_t)n * 8, 256);
    double *rowF = (double *)p0;
    p0 += align_up((size_t)n * 8, 256);
    double *X = (double *)p0;
    p0 += align_up((size_t)ds_npad(n) * (size_t)(mi.d + 2) * 8, 256);
    unsigned int *amax = (unsigned int *)p0;  // [kMaxDim]
    float *alpha = (float *)(p0 + 256);
    double *wf = (double *)(p0 + 512);        // [2][kMaxDim]
    int64_t gs = (A.npad + 255) / 256;
    if (gs > 65536) gs = 65536;
    hipLaunchKernelGGL(smooth_stage_kernel, dim3((unsigned)gs), dim3(256), 0, s, x, y, eps, Mk, M,
                       prune, mi.d, n, A.npad, xf, rec);
    if (pr) {
        DsArgs ds{};
        Signs sg{};
        (void)fill_ds_metric(mi, true, &ds, &sg);
        WeightsSel wsel{};
        for (int j = 0; j < kMaxDim; ++j) {
            wsel.v[j] = ds.w[j];
            wsel.v[kMaxDim + j] = ds.fsel[j];
        }
        A.X = X;
        A.npad64 = ds_npad(n);
        A.wf = wf;
        if (launch_stage64(mi.d, x, y, nullptr, 0.0f, n, A.npad64, sg, X, s) != hipSuccess)
            return LIP_E_DEVICE;
        hipLaunchKernelGGL(smooth_wf_kernel, dim3(1), dim3(64), 0, s, wsel, wf);
        int64_t ga = (n + 255) / 256;
        if (ga > 1024) ga = 1024;
        hipLaunchKernelGGL(smooth_zero_kernel, dim3(1), dim3(64), 0, s, amax, kMaxDim);
        hipLaunchKernelGGL(smooth_amax_kernel, dim3((unsigned)ga), dim3(256), 0, s, x, n, mi.d,
                           xf, amax);
        hipLaunchKernelGGL(smooth_alpha_kernel, dim3(1), dim3(64), 0, s, amax, mi.d, alpha);
        A.alpha = alpha;
    }
    const unsigned grid = (unsigned)(((row_waves + 3) / 4) * A.n_chunks);
    launch(A, dim3(grid), dim3(256), s);
    hipLaunchKernelGGL(smooth_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const double *)A.pF, (const double *)A.pG, A.n_chunks, n, eps, p, rowF,
                       grad);
    if (F)
        hipLaunchKernelGGL(smooth_reduce_kernel, dim3(1), dim3(1024), 0, s, (const double *)rowF,
                           n, F);
    return dev_status(hipGetLastError());
}
