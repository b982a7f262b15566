// Data-side passes over all pairs of data points, in FP64:
//  * lip_consistency - the Lipschitz condition of Sec. 1 with the
//    monotonicity constraints of Sec. 4.1, in the pairwise form of
//    Eqs. (5)-(6) with zero corrections;
//  * lip_estimate_M  - the largest pairwise slope (Sec. 5) and the per-datum
//    slope over the K nearest data (Sec. 4.3, scalar form).
//
// Every pair is evaluated in double precision from the FP32 inputs with a
// fixed operation order: per coordinate in index order, delta = x_i - x_k,
// the component (|delta|, or a positive part on a monotone coordinate) times
// the weight, then accumulated (sum, sum of squares, or max) from 0; l2 takes
// the square root; bounds are y_k + M_k * dist (product, then sum).  All of
// these operations are correctly rounded, so the decisions that produce the
// integer outputs (violation counts, partners, neighbour ranks) are
// reproducible by any implementation that follows the same order.
//
// Data are first staged as FP64 records [x_0 .. x_{D-1} | y | M] so that the
// column loop reads them with scalar loads and the VALU uses them straight
// from SGPR pairs.  A lane owns R rows; columns are streamed.
#include <climits>
#include <float.h>

#include "host_common.hpp"

namespace lip {

struct DsArgs {
    const double *rec;  // staged [n][D + 2]
    int64_t n;
    int32_t norm;
    int32_t has_w;
    double w[kMaxDim];
    int32_t kind[kMaxDim];  // 0 free, 1 increasing, -1 decreasing
    double tol;
    // consistency outputs
    double *slack_up, *slack_lo;
    int32_t *partner_up, *partner_lo;
    unsigned long long *counts;  // [2]
    // estimate-M outputs
    double *row_best;     // [n] per-row best slope (global mode)
    int32_t *row_arg;     // [n] its column, -1 none
    int32_t *row_dup;     // [n] first coincident column with different y, -1 none
    int32_t knn;
    double *M64;
    float *M32;
};

template <int D>
__global__ void stage64_kernel(const float *x, const float *y, const float *Mk, float M, int64_t n,
                               double *out)
{
    constexpr int S = D + 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
#pragma unroll
        for (int j = 0; j < D; ++j) out[k * S + j] = (double)x[k * D + j];
        out[k * S + D] = (double)y[k];
        out[k * S + D + 1] = Mk ? (double)Mk[k] : (double)M;
    }
}

// Directional distances between row point a and column point b, FP64, the
// fixed order described above.  With sym the monotonicity is ignored.
template <int D, bool sym>
__device__ __forceinline__ void dist64(const DsArgs &A, const double (&a)[D], const double *b,
                                       double &su, double &sl)
{
    su = 0.0;
    sl = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const double dl = a[i] - b[i];
        double cu, cl;
        const int kd = sym ? 0 : A.kind[i];
        if (kd == 0) {
            cu = fabs(dl);
            cl = cu;
        } else if (kd > 0) {
            cu = dl > 0.0 ? dl : 0.0;
            cl = dl < 0.0 ? -dl : 0.0;
        } else {
            cu = dl < 0.0 ? -dl : 0.0;
            cl = dl > 0.0 ? dl : 0.0;
        }
        if (A.has_w) {
            cu = A.w[i] * cu;
            cl = A.w[i] * cl;
        }
        if (A.norm == 1) {
            su = su + cu;
            if (!sym) sl = sl + cl;
        } else if (A.norm == 2) {
            su = su + cu * cu;
            if (!sym) sl = sl + cl * cl;
        } else {
            su = cu > su ? cu : su;
            if (!sym) sl = cl > sl ? cl : sl;
        }
    }
    if (sym) sl = su;
}

typedef const double __attribute__((address_space(4))) *cdouble_ptr;

// ---- consistency -------------------------------------------------------------

__global__ void zero_counts_kernel(unsigned long long *c)
{
    if (threadIdx.x < 2) c[threadIdx.x] = 0ull;
}

constexpr int kDsRows = 2;

template <int D, bool self_check>
__device__ __forceinline__ void consistency_cols(const DsArgs &A, cdouble_ptr rec, int64_t k0,
                                                 int64_t k1, const double (&xr)[kDsRows][D],
                                                 const double (&yr)[kDsRows],
                                                 const int64_t (&ir)[kDsRows], double (&bu)[kDsRows],
                                                 double (&bl)[kDsRows], int (&pu)[kDsRows],
                                                 int (&pl)[kDsRows], int (&cu)[kDsRows],
                                                 int (&cl)[kDsRows])
{
    constexpr int S = D + 2;
    for (int64_t k = k0; k < k1; ++k) {
        double xk[S];
#pragma unroll
        for (int j = 0; j < S; ++j) xk[j] = rec[k * S + j];
        const double yk = xk[D], mk = xk[D + 1];
#pragma unroll
        for (int r = 0; r < kDsRows; ++r) {
            double du, dl;
            dist64<D, false>(A, xr[r], xk, du, dl);
            if (A.norm == 2) {
                du = sqrt(du);
                dl = sqrt(dl);
            }
            const double tu = (yk + mk * du) - yr[r];
            const double tl = yr[r] - (yk - mk * dl);
            const bool ok = !self_check || (k != ir[r]);
            if (ok && tu < bu[r]) {
                bu[r] = tu;
                pu[r] = (int)k;
            }
            if (ok && tl < bl[r]) {
                bl[r] = tl;
                pl[r] = (int)k;
            }
            cu[r] += (ok && tu < -A.tol) ? 1 : 0;
            cl[r] += (ok && tl < -A.tol) ? 1 : 0;
        }
    }
}

template <int D>
__global__ void __launch_bounds__(256) consistency_kernel(DsArgs A)
{
    constexpr int S = D + 2;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * (64 * kDsRows);
    if (r0 >= A.n) return;
    int64_t r1 = r0 + 64 * kDsRows;
    r1 = r1 < A.n ? r1 : A.n;
    double xr[kDsRows][D], yr[kDsRows];
    int64_t ir[kDsRows];
    double bu[kDsRows], bl[kDsRows];
    int pu[kDsRows], pl[kDsRows], cu[kDsRows], cl[kDsRows];
#pragma unroll
    for (int r = 0; r < kDsRows; ++r) {
        int64_t i = r0 + r * 64 + lane;
        ir[r] = i;
        i = i < A.n ? i : A.n - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.rec[i * S + j];
        yr[r] = A.rec[i * S + D];
        bu[r] = __builtin_inf();
        bl[r] = __builtin_inf();
        pu[r] = pl[r] = -1;
        cu[r] = cl[r] = 0;
    }
    const cdouble_ptr rec = (cdouble_ptr)(A.rec);
    consistency_cols<D, false>(A, rec, 0, r0, xr, yr, ir, bu, bl, pu, pl, cu, cl);
    consistency_cols<D, true>(A, rec, r0, r1, xr, yr, ir, bu, bl, pu, pl, cu, cl);
    consistency_cols<D, false>(A, rec, r1, A.n, xr, yr, ir, bu, bl, pu, pl, cu, cl);
    unsigned long long tu = 0, tl = 0;
#pragma unroll
    for (int r = 0; r < kDsRows; ++r) {
        const int64_t i = ir[r];
        if (i >= A.n) continue;
        if (A.slack_up) A.slack_up[i] = bu[r];
        if (A.slack_lo) A.slack_lo[i] = bl[r];
        if (A.partner_up) A.partner_up[i] = pu[r];
        if (A.partner_lo) A.partner_lo[i] = pl[r];
        tu += (unsigned long long)cu[r];
        tl += (unsigned long long)cl[r];
    }
    for (int off = 32; off > 0; off >>= 1) {
        tu += __shfl_xor(tu, off);
        tl += __shfl_xor(tl, off);
    }
    if (lane == 0) {
        atomicAdd(A.counts, tu);
        atomicAdd(A.counts + 1, tl);
    }
}

// ---- global M: max over i < k of |y_i - y_k| / dist ------------------------------

constexpr int kMRows = 2;

template <int D, bool diag>
__device__ __forceinline__ void slope_cols(const DsArgs &A, cdouble_ptr rec, int64_t k0, int64_t k1,
                                           const double (&xr)[kMRows][D], const double (&yr)[kMRows],
                                           const int64_t (&ir)[kMRows], double (&best)[kMRows],
                                           int (&arg)[kMRows], int (&dup)[kMRows])
{
    constexpr int S = D + 2;
    for (int64_t k = k0; k < k1; ++k) {
        double xk[S];
#pragma unroll
        for (int j = 0; j < D + 1; ++j) xk[j] = rec[k * S + j];
#pragma unroll
        for (int r = 0; r < kMRows; ++r) {
            if (diag && !(k > ir[r])) continue;
            double du, dl;
            dist64<D, true>(A, xr[r], xk, du, dl);
            if (A.norm == 2) du = sqrt(du);
            const double dy = fabs(yr[r] - xk[D]);
            if (du == 0.0) {
                if (dy != 0.0 && dup[r] < 0) dup[r] = (int)k;
                continue;
            }
            // dy / du > best  <=>  dy - best * du > 0, decided exactly by the
            // sign of one fused multiply-add; only then form the quotient.
            if (best[r] < 0.0 || fma(-best[r], du, dy) > 0.0) {
                const double s = dy / du;
                if (s > best[r]) {
                    best[r] = s;
                    arg[r] = (int)k;
                }
            }
        }
    }
}

template <int D>
__global__ void __launch_bounds__(256) slope_kernel(DsArgs A)
{
    constexpr int S = D + 2;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * (64 * kMRows);
    if (r0 >= A.n) return;
    int64_t r1 = r0 + 64 * kMRows;
    r1 = r1 < A.n ? r1 : A.n;
    double xr[kMRows][D], yr[kMRows], best[kMRows];
    int64_t ir[kMRows];
    int arg[kMRows], dup[kMRows];
#pragma unroll
    for (int r = 0; r < kMRows; ++r) {
        int64_t i = r0 + r * 64 + lane;
        ir[r] = i;
        i = i < A.n ? i : A.n - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.rec[i * S + j];
        yr[r] = A.rec[i * S + D];
        best[r] = -1.0;
        arg[r] = -1;
        dup[r] = -1;
    }
    const cdouble_ptr rec = (cdouble_ptr)(A.rec);
    slope_cols<D, true>(A, rec, r0, r1, xr, yr, ir, best, arg, dup);
    slope_cols<D, false>(A, rec, r1, A.n, xr, yr, ir, best, arg, dup);
#pragma unroll
    for (int r = 0; r < kMRows; ++r) {
        const int64_t i = ir[r];
        if (i >= A.n) continue;
        A.row_best[i] = best[r];
        A.row_arg[i] = arg[r];
        A.row_dup[i] = dup[r];
    }
}

// Single-workgroup reduction of the per-row results: the first row (lowest
// i) with a coincident pair of different values wins outright; otherwise the
// largest slope, lowest i on ties (each row already holds its lowest k).
__global__ void slope_reduce_kernel(DsArgs A, int64_t *pair)
{
    __shared__ double sb[1024];
    __shared__ long long si[1024];
    __shared__ long long sd[1024];
    double best = -1.0;
    long long bi = -1, di = LLONG_MAX;
    for (int64_t i = threadIdx.x; i < A.n; i += blockDim.x) {
        if (A.row_dup[i] >= 0 && i < di) di = i;
        if (A.row_arg[i] >= 0 && (A.row_best[i] > best || (A.row_best[i] == best && i < bi))) {
            best = A.row_best[i];
            bi = i;
        }
    }
    sb[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    sd[threadIdx.x] = di;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const int o = threadIdx.x + s;
            if (sd[o] < sd[threadIdx.x]) sd[threadIdx.x] = sd[o];
            const bool take = si[o] >= 0 &&
                              (si[threadIdx.x] < 0 || sb[o] > sb[threadIdx.x] ||
                               (sb[o] == sb[threadIdx.x] && si[o] < si[threadIdx.x]));
            if (take) {
                sb[threadIdx.x] = sb[o];
                si[threadIdx.x] = si[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double M;
        long long p0, p1;
        if (sd[0] != LLONG_MAX) {
            M = __builtin_inf();
            p0 = sd[0];
            p1 = A.row_dup[sd[0]];
        } else if (si[0] >= 0) {
            M = sb[0];
            p0 = si[0];
            p1 = A.row_arg[si[0]];
        } else {
            M = 0.0;
            p0 = p1 = -1;
        }
        if (A.M64) A.M64[0] = M;
        if (A.M32) {
            float f = (float)M;
            if ((double)f < M) f = nextafterf(f, __builtin_inff());
            A.M32[0] = f;
        }
        if (pair) {
            pair[0] = p0;
            pair[1] = p1;
        }
    }
}

// ---- local M from the K nearest data ---------------------------------------------

// Keeps the K smallest (key, index) of the row in ascending order.  Columns
// arrive in increasing index order, so a strict comparison ranks the lower
// index first among equal keys.
template <int K>
__device__ __forceinline__ void knn_insert(double (&key)[K], int (&idx)[K], double kv, int j)
{
    key[K - 1] = kv;
    idx[K - 1] = j;
#pragma unroll
    for (int t = K - 1; t > 0; --t) {
        const bool sw = key[t] < key[t - 1];
        const double a = key[t], b = key[t - 1];
        const int ia = idx[t], ib = idx[t - 1];
        key[t] = sw ? b : a;
        key[t - 1] = sw ? a : b;
        idx[t] = sw ? ib : ia;
        idx[t - 1] = sw ? ia : ib;
    }
}

template <int D, int K>
__global__ void __launch_bounds__(256) knn_kernel(DsArgs A)
{
    constexpr int S = D + 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ic = i < A.n ? i : A.n - 1;
    double xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xr[j] = A.rec[ic * S + j];
    double key[K];
    int idx[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        key[t] = __builtin_inf();
        idx[t] = -1;
    }
    // Only the first knn (<= K) slots matter; thr is the knn-th smallest key.
    const int kk = A.knn;
    double thr = __builtin_inf();
    const cdouble_ptr rec = (cdouble_ptr)(A.rec);
    for (int64_t k = 0; k < A.n; ++k) {
        double xk[D];
#pragma unroll
        for (int j = 0; j < D; ++j) xk[j] = rec[k * S + j];
        double du, dl;
        dist64<D, true>(A, xr, xk, du, dl);
        // rank by the distance (l2: by the sum of squares)
        if (k != ic && du < thr) {
            knn_insert<K>(key, idx, du, (int)k);
#pragma unroll
            for (int t = 0; t < K; ++t)
                if (t == kk - 1) thr = key[t];
        }
    }
    if (i >= A.n) return;
    const double yi = A.rec[ic * S + D];
    double best = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        if (t >= kk || idx[t] < 0) continue;
        const double *xk = A.rec + (int64_t)idx[t] * S;
        double du, dl;
        double xx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) xx[j] = xk[j];
        dist64<D, true>(A, xr, xx, du, dl);
        if (A.norm == 2) du = sqrt(du);
        const double dy = fabs(yi - xk[D]);
        if (du == 0.0) {
            if (dy != 0.0) best = __builtin_inf();
            continue;
        }
        const double s = dy / du;
        if (s > best) best = s;
    }
    if (A.M64) A.M64[i] = best;
    if (A.M32) {
        float f = (float)best;
        if ((double)f < best) f = nextafterf(f, __builtin_inff());
        A.M32[i] = f;
    }
}

// ---- host side ------------------------------------------------------------------

size_t data_side_ws_bytes(int64_t n, int d)
{
    return align_up((size_t)n * (size_t)(d + 2) * 8, 256) + align_up((size_t)n * 16, 256) + 512;
}

struct DsLaunchers {
    void (*stage)(const float *, const float *, const float *, float, int64_t, double *, hipStream_t);
    void (*consistency)(const DsArgs &, dim3, dim3, hipStream_t);
    void (*slope)(const DsArgs &, dim3, dim3, hipStream_t);
    void (*knn16)(const DsArgs &, dim3, dim3, hipStream_t);
    void (*knn32)(const DsArgs &, dim3, dim3, hipStream_t);
};

template <int D>
static DsLaunchers ds_launchers()
{
    DsLaunchers L;
    L.stage = [](const float *x, const float *y, const float *Mk, float M, int64_t n, double *out,
                 hipStream_t s) {
        int64_t g = (n + 255) / 256;
        if (g > 65536) g = 65536;
        hipLaunchKernelGGL(stage64_kernel<D>, dim3((unsigned)g), dim3(256), 0, s, x, y, Mk, M, n, out);
    };
    L.consistency = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL(consistency_kernel<D>, g, b, 0, s, a);
    };
    L.slope = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL(slope_kernel<D>, g, b, 0, s, a);
    };
    L.knn16 = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_kernel<D, 16>), g, b, 0, s, a);
    };
    L.knn32 = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_kernel<D, 32>), g, b, 0, s, a);
    };
    return L;
}

static bool get_ds(int d, DsLaunchers *L)
{
    switch (d) {
#define LIP_DS_CASE(DD) \
    case DD: *L = ds_launchers<DD>(); return true;
        LIP_DS_CASE(1) LIP_DS_CASE(2) LIP_DS_CASE(3) LIP_DS_CASE(4)
        LIP_DS_CASE(5) LIP_DS_CASE(6) LIP_DS_CASE(7) LIP_DS_CASE(8)
        LIP_DS_CASE(9) LIP_DS_CASE(10) LIP_DS_CASE(11) LIP_DS_CASE(12)
        LIP_DS_CASE(13) LIP_DS_CASE(14) LIP_DS_CASE(15) LIP_DS_CASE(16)
#undef LIP_DS_CASE
    default: return false;
    }
}

static void fill_ds_metric(const MetricInfo &mi, bool use_mon, DsArgs *A)
{
    A->norm = mi.norm;
    A->has_w = 0;
    for (int i = 0; i < kMaxDim; ++i) {
        A->w[i] = i < mi.d ? mi.w[i] : 1.0;
        A->kind[i] = (use_mon && i < mi.d) ? mi.mon[i] : 0;
        if (i < mi.d && mi.w[i] != 1.0) A->has_w = 1;
    }
}

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_consistency(const lip_metric *metric, const float *x, const float *y,
                                      int64_t n, float M, const float *Mk, double tol,
                                      int64_t *counts, double *slack_up, double *slack_lo,
                                      int32_t *partner_up, int32_t *partner_lo, void *ws,
                                      size_t ws_bytes, uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || n > kMaxIndex) return LIP_E_SHAPE;
    if (!x || !y || !counts) return LIP_E_ARG;
    if (!Mk && (!(M >= 0.0f) || !__builtin_isfinite(M))) return LIP_E_VALUE;
    if (!(tol >= 0.0) || !__builtin_isfinite(tol)) return LIP_E_VALUE;
    if (!ws || ws_bytes < data_side_ws_bytes(n, mi.d)) return LIP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[3] = {x, y, Mk};
        const int64_t cnt[3] = {n * mi.d, n, Mk ? n : 0};
        st = check_finite(arr, cnt, 3, ws, s);
        if (st != LIP_OK) return st;
    }
    DsLaunchers L;
    if (!get_ds(mi.d, &L)) return LIP_E_UNSUPPORTED;
    DsArgs A{};
    A.rec = (const double *)ws;
    A.n = n;
    A.tol = tol;
    fill_ds_metric(mi, true, &A);
    A.slack_up = slack_up;
    A.slack_lo = slack_lo;
    A.partner_up = partner_up;
    A.partner_lo = partner_lo;
    A.counts = (unsigned long long *)counts;
    L.stage(x, y, Mk, M, n, (double *)ws, s);
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, s, A.counts);
    const int64_t waves = (n + 64 * kDsRows - 1) / (64 * kDsRows);
    const int64_t blocks = (waves + 3) / 4;
    L.consistency(A, dim3((unsigned)blocks), dim3(256), s);
    return dev_status(hipGetLastError());
}

extern "C" lip_status lip_estimate_M(const lip_metric *metric, const float *x, const float *y,
                                     int64_t n, int32_t mode, int32_t knn, double *M64, float *M32,
                                     int64_t *pair, void *ws, size_t ws_bytes, uint32_t flags,
                                     lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || n > kMaxIndex) return LIP_E_SHAPE;
    if (!x || !y) return LIP_E_ARG;
    if (mode != LIP_M_GLOBAL && mode != LIP_M_LOCAL_KNN) return LIP_E_ARG;
    if (mode == LIP_M_LOCAL_KNN && (knn < 1 || knn > LIP_MAX_KNN)) return LIP_E_VALUE;
    if (!ws || ws_bytes < data_side_ws_bytes(n, mi.d)) return LIP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[2] = {x, y};
        const int64_t cnt[2] = {n * mi.d, n};
        st = check_finite(arr, cnt, 2, ws, s);
        if (st != LIP_OK) return st;
    }
    DsLaunchers L;
    if (!get_ds(mi.d, &L)) return LIP_E_UNSUPPORTED;
    DsArgs A{};
    A.rec = (const double *)ws;
    A.n = n;
    fill_ds_metric(mi, false, &A);
    A.M64 = M64;
    A.M32 = M32;
    L.stage(x, y, nullptr, 0.0f, n, (double *)ws, s);
    if (mode == LIP_M_GLOBAL) {
        char *p = (char *)ws + align_up((size_t)n * (size_t)(mi.d + 2) * 8, 256);
        A.row_best = (double *)p;
        A.row_arg = (int32_t *)(p + (size_t)n * 8);
        A.row_dup = A.row_arg + n;
        const int64_t waves = (n + 64 * kMRows - 1) / (64 * kMRows);
        L.slope(A, dim3((unsigned)((waves + 3) / 4)), dim3(256), s);
        hipLaunchKernelGGL(slope_reduce_kernel, dim3(1), dim3(1024), 0, s, A, pair);
    } else {
        A.knn = knn;
        const dim3 grid((unsigned)((n + 255) / 256)), block(256);
        if (knn <= 16)
            L.knn16(A, grid, block, s);
        else
            L.knn32(A, grid, block, s);
    }
    return dev_status(hipGetLastError());
}
