// Host entry points of the FP64 data-side passes (lip_consistency,
// lip_estimate_M) and their small helper kernels; the pair kernels are in
// data_side.hpp, instantiated per norm in data_side_{l1,l2,linf}.hip.
#include "data_side.hpp"

namespace lip {

// d-major FP64 staging: X[j * npad + k]; padded columns hold zeros and are
// masked out by every kernel.  Coordinates with sign -1 (monotone
// decreasing) are negated, which is exact and turns them into increasing
// ones: the pair components (x_i - x_k)_+ and (x_k - x_i)_+ swap roles.
template <int D>
__global__ void stage64_kernel(const float *x, const float *y, const float *Mk, float M, int64_t n,
                               int64_t npad, Signs sg, double *X)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        const bool in = k < n;
#pragma unroll
        for (int j = 0; j < D; ++j)
            X[(int64_t)j * npad + k] = in ? (double)(sg.s[j] * x[k * D + j]) : 0.0;
        X[(int64_t)D * npad + k] = in ? (double)y[k] : 0.0;
        X[(int64_t)(D + 1) * npad + k] = in ? (Mk ? (double)Mk[k] : (double)M) : 0.0;
    }
}

hipError_t launch_stage64(int d, const float *x, const float *y, const float *Mk, float M,
                          int64_t n, int64_t npad, const Signs &sg, double *X, hipStream_t s)
{
    int64_t g = (npad + 255) / 256;
    if (g > 65536) g = 65536;
    switch (d) {
#define LIP_ST_CASE(DD)                                                                          \
    case DD:                                                                                     \
        hipLaunchKernelGGL(stage64_kernel<DD>, dim3((unsigned)g), dim3(256), 0, s, x, y, Mk, M, \
                           n, npad, sg, X);                                                      \
        break;
        LIP_ST_CASE(1) LIP_ST_CASE(2) LIP_ST_CASE(3) LIP_ST_CASE(4)
        LIP_ST_CASE(5) LIP_ST_CASE(6) LIP_ST_CASE(7) LIP_ST_CASE(8)
        LIP_ST_CASE(9) LIP_ST_CASE(10) LIP_ST_CASE(11) LIP_ST_CASE(12)
        LIP_ST_CASE(13) LIP_ST_CASE(14) LIP_ST_CASE(15) LIP_ST_CASE(16)
#undef LIP_ST_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- spatial order of the data for the kNN pass ----------------------------------
//
// Morton (bit-interleaved) code of the coordinates quantised to b bits each
// (b = 32 / d, at least 1) inside the data's bounding box, packed as
// (code << 32 | index) and sorted: consecutive positions are spatial
// neighbours.  Only the order of the rows and the threshold pass depend on
// it; every kNN list is still formed from all columns in index order.

__device__ __forceinline__ unsigned long long f64_key(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double f64_unkey(unsigned long long k)
{
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k));
}

__global__ void bbox_init_kernel(unsigned long long *bb, int d)
{
    const int j = threadIdx.x;
    if (j < d) {
        bb[j] = ~0ull;  // min keys
        bb[kMaxDim + j] = 0ull;  // max keys
    }
}

// Workgroups of the small reductions over the rows (bounding boxes, the FP32
// error bound, the worst pair): one per compute unit.
constexpr int kReduceBlocks = 256;

// Bounding box of the staged coordinates as order keys: per-thread minima
// and maxima over a strided part of the rows, reduced in the workgroup
// (shuffles, then LDS across its waves), one atomic per coordinate and side.
__global__ void __launch_bounds__(256) bbox_kernel(const double *X, int64_t n, int64_t npad,
                                                   int d, unsigned long long *bb)
{
    __shared__ double slo[4][kMaxDim], shi[4][kMaxDim];
    double lo[kMaxDim], hi[kMaxDim];
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        lo[j] = __builtin_inf();
        hi[j] = -__builtin_inf();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) {
            if (j < d) {
                const double v = X[(int64_t)j * npad + k];
                lo[j] = fmin(lo[j], v);
                hi[j] = fmax(hi[j], v);
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        if (j < d) {
            double a = lo[j], b = hi[j];
            for (int off = 32; off > 0; off >>= 1) {
                a = fmin(a, __shfl_xor(a, off));
                b = fmax(b, __shfl_xor(b, off));
            }
            if (lane == 0) {
                slo[wv][j] = a;
                shi[wv][j] = b;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < d) {
        const int j = threadIdx.x;
        double a = __builtin_inf(), b = -__builtin_inf();
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a = fmin(a, slo[w][j]);
            b = fmax(b, shi[w][j]);
        }
        atomicMin(bb + j, f64_key(a));
        atomicMax(bb + kMaxDim + j, f64_key(b));
    }
}

__global__ void morton_kernel(const double *X, int64_t n, int64_t npad, int d, int64_t P,
                              const unsigned long long *bb, unsigned long long *keys)
{
    const int bits = 32 / d > 0 ? (32 / d < 16 ? 32 / d : 16) : 1;
    const double cells = (double)(1u << bits);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += stride) {
        if (k >= n) {
            keys[k] = ~0ull;
            continue;
        }
        uint32_t q[kMaxDim];
        for (int j = 0; j < d; ++j) {
            const double lo = f64_unkey(bb[j]), hi = f64_unkey(bb[kMaxDim + j]);
            double t = hi > lo ? (X[(int64_t)j * npad + k] - lo) / (hi - lo) * cells : 0.0;
            t = t < 0.0 ? 0.0 : (t > cells - 1.0 ? cells - 1.0 : t);  // NaN -> cells - 1
            q[j] = (uint32_t)t;
        }
        unsigned long long code = 0;
        for (int b = bits - 1; b >= 0; --b)
            for (int j = 0; j < d; ++j) code = (code << 1) | ((q[j] >> b) & 1u);
        keys[k] = (code << 32) | (uint32_t)k;
    }
}

// FP32 records of the consistency filter: [npad][d + 2] = (signed x, y, M_k),
// all exact copies of the FP32 inputs (padding zero, masked by the kernel).
__global__ void stage32_kernel(const float *x, const float *y, const float *Mk, float M, int64_t n,
                               int64_t npad, int d, Signs sg, float *c32)
{
    const int S = d + 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        const bool in = k < n;
        for (int j = 0; j < d; ++j) c32[k * S + j] = in ? sg.s[j] * x[k * d + j] : 0.0f;
        c32[k * S + d] = in ? y[k] : 0.0f;
        c32[k * S + d + 1] = in ? (Mk ? Mk[k] : M) : 0.0f;
    }
}

// E = 2^-18 (max M_k * max pairwise distance + 2 max |y|) + max M_k 2^-60
// + 2^-126, the bound on |FP32 slack - FP64 slack| used by the filtered
// consistency kernel (the distance bound is the norm of the weighted
// bounding-box extent).  Data whose FP32 evaluation could overflow (extent
// >= 2^60 or bounds >= 2^100), or non-finite values, give +inf, which sends
// every pair to FP64.
//
// Pass 1 (kReduceBlocks workgroups): max |y|, max M_k and the per-coordinate
// minima and maxima, reduced in each workgroup and combined with atomics on
// order keys in kb[2 + 2 kMaxDim] (max |y|, max M_k, minima, maxima; set up
// by cons_bound_init_kernel).  Pass 2 (one thread) forms E.
__global__ void cons_bound_init_kernel(unsigned long long *kb)
{
    const int t = threadIdx.x;
    if (t < 2 + 2 * kMaxDim) kb[t] = (t >= 2 && t < 2 + kMaxDim) ? ~0ull : 0ull;
}

__global__ void __launch_bounds__(256) cons_bound_kernel(const float *c32, int64_t n, int d,
                                                         unsigned long long *kb)
{
    __shared__ double red[2 + 2 * kMaxDim][4];
    const int S = d + 2;
    double ymax = 0.0, mmax = 0.0, lo[kMaxDim], hi[kMaxDim];
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        lo[j] = __builtin_inf();
        hi[j] = -__builtin_inf();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        ymax = fmax(ymax, fabs((double)c32[k * S + d]));
        mmax = fmax(mmax, (double)c32[k * S + d + 1]);
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) {
            if (j < d) {
                const double v = c32[k * S + j];
                lo[j] = fmin(lo[j], v);
                hi[j] = fmax(hi[j], v);
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    auto wmax = [&](double v) {
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        return v;
    };
    ymax = wmax(ymax);
    mmax = wmax(mmax);
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        if (j < d) {
            lo[j] = -wmax(-lo[j]);
            hi[j] = wmax(hi[j]);
        }
    }
    if (lane == 0) {
        red[0][wv] = ymax;
        red[1][wv] = mmax;
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) {
            if (j < d) {
                red[2 + j][wv] = lo[j];
                red[2 + kMaxDim + j][wv] = hi[j];
            }
        }
    }
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    const int t = threadIdx.x;
    if (t < 2) {
        double m = 0.0;
        for (int q = 0; q < nw; ++q) m = fmax(m, red[t][q]);
        atomicMax(kb + t, f64_key(m));
    } else if (t < 2 + d) {
        const int j = t - 2;
        double l = __builtin_inf(), h = -__builtin_inf();
        for (int q = 0; q < nw; ++q) {
            l = fmin(l, red[2 + j][q]);
            h = fmax(h, red[2 + kMaxDim + j][q]);
        }
        atomicMin(kb + 2 + j, f64_key(l));
        atomicMax(kb + 2 + kMaxDim + j, f64_key(h));
    }
}

__global__ void cons_bound_final_kernel(const unsigned long long *kb, int d, DsArgs A, double *E)
{
    if (threadIdx.x != 0) return;
    const double ym = f64_unkey(kb[0]), mm = f64_unkey(kb[1]);
    double dist = 0.0;
    for (int j = 0; j < d; ++j) {
        const double l = f64_unkey(kb[2 + j]), h = f64_unkey(kb[2 + kMaxDim + j]);
        const double span = A.w[j] * (h - l);
        // l1: sum; l2: root of the sum of squares; linf: max
        if (span > 0.0)
            dist = A.norm == 1 ? dist + span : (A.norm == 2 ? dist + span * span : fmax(dist, span));
    }
    if (A.norm == 2) dist = sqrt(dist);
    // relative part; the absolute part covers FP32 underflow of squared
    // components (a distance error of at most 2^-72) and of the sums
    double e = 0x1p-18 * (mm * dist + 2.0 * ym) + mm * 0x1p-60 + 0x1p-126;
    // FP32 squares and bounds must stay finite: components below 2^60,
    // bounds below 2^100; otherwise every pair goes to FP64
    if (!(dist < 0x1p60) || !(mm * dist + ym < 0x1p100) || !(e < 0x1p100)) e = __builtin_inf();
    E[0] = e;
}

__global__ void zero_counts_kernel(unsigned long long *c)
{
    if (threadIdx.x < 2) c[threadIdx.x] = 0ull;
}

__global__ void consistency_combine_kernel(DsArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    double bu = __builtin_inf(), bl = __builtin_inf();
    int pu = -1, pl = -1;
    for (int c = 0; c < A.n_chunks; ++c) {
        const int64_t o = (int64_t)c * A.n + i;
        if (A.pv_up[o] < bu) {
            bu = A.pv_up[o];
            pu = A.pi_up[o];
        }
        if (A.pv_lo[o] < bl) {
            bl = A.pv_lo[o];
            pl = A.pi_lo[o];
        }
    }
    if (A.slack_up) A.slack_up[i] = bu;
    if (A.slack_lo) A.slack_lo[i] = bl;
    if (A.partner_up) A.partner_up[i] = pu;
    if (A.partner_lo) A.partner_lo[i] = pl;
}

// Smallest slack over all rows and both bounds, with the pair attaining it:
// (value, row i, partner k) compared lexicographically, so ties go to the
// lowest i, then the lowest k.  No pair at all (n == 1): +inf and (-1, -1).
// Pass 1 (up to kReduceBlocks workgroups) writes one candidate per
// workgroup, pass 2 (one workgroup) reduces them; the minimum of a total
// order does not depend on how the rows are split.
struct WorstRec {
    double v;
    long long i, k;
};

__device__ __forceinline__ bool worst_better(double v, long long i, long long k, double bv,
                                             long long bi, long long bk)
{
    if (k < 0) return false;
    if (bk < 0) return true;
    if (v != bv) return v < bv;
    if (i != bi) return i < bi;
    return k < bk;
}

// Workgroup reduction of (v, i, k) (256 threads); thread 0 gets the result.
__device__ __forceinline__ void worst_block_reduce(double &bv, long long &bi, long long &bk)
{
    __shared__ double sv[256];
    __shared__ long long si[256], sk[256];
    const int t = threadIdx.x;
    sv[t] = bv;
    si[t] = bi;
    sk[t] = bk;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (t < h && worst_better(sv[t + h], si[t + h], sk[t + h], sv[t], si[t], sk[t])) {
            sv[t] = sv[t + h];
            si[t] = si[t + h];
            sk[t] = sk[t + h];
        }
        __syncthreads();
    }
    bv = sv[0];
    bi = si[0];
    bk = sk[0];
}

__global__ void __launch_bounds__(256) worst_partial_kernel(const double *su, const double *sl,
                                                            const int32_t *pu,
                                                            const int32_t *pl, int64_t n,
                                                            WorstRec *part)
{
    double bv = __builtin_inf();
    long long bi = -1, bk = -1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double vu = su[i], vl = sl[i];
        const long long ku = pu[i], kl = pl[i];
        if (worst_better(vu, i, ku, bv, bi, bk)) {
            bv = vu;
            bi = i;
            bk = ku;
        }
        if (worst_better(vl, i, kl, bv, bi, bk)) {
            bv = vl;
            bi = i;
            bk = kl;
        }
    }
    worst_block_reduce(bv, bi, bk);
    if (threadIdx.x == 0) part[blockIdx.x] = WorstRec{bv, bi, bk};
}

__global__ void __launch_bounds__(256) worst_final_kernel(const WorstRec *part, int n_part,
                                                          double *worst, int64_t *pair)
{
    double bv = __builtin_inf();
    long long bi = -1, bk = -1;
    for (int b = threadIdx.x; b < n_part; b += blockDim.x) {
        const WorstRec r = part[b];
        if (worst_better(r.v, r.i, r.k, bv, bi, bk)) {
            bv = r.v;
            bi = r.i;
            bk = r.k;
        }
    }
    worst_block_reduce(bv, bi, bk);
    if (threadIdx.x == 0) {
        if (worst) worst[0] = bk >= 0 ? bv : __builtin_inf();
        if (pair) {
            pair[0] = bk >= 0 ? bi : -1;
            pair[1] = bk >= 0 ? bk : -1;
        }
    }
}

// Sets flag[0] to 1 if any of the n values (FP64 when v64, else FP32) is
// +inf (an infinite slope).
__global__ void any_inf_kernel(const double *v64, const float *v32, int64_t n, int *flag)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad |= v64 ? (v64[i] == __builtin_inf()) : (v32[i] == __builtin_inff());
    if (bad) atomicOr(flag, 1);
}

// Single-workgroup reduction over all (chunk, row) slope partials.  Order: a
// coincident pair with different values (lowest i, then lowest k) wins
// outright; otherwise the largest slope, then the lowest i, then the lowest
// k.  Every wave writes all of its rows for its chunk (a chunk left of the
// rows has no usable column: best -1, arg -1, dup -1).
struct SlopeKey {
    double v;
    long long i, k, di, dk;
};

__device__ __forceinline__ bool better_dup(const SlopeKey &a, const SlopeKey &b)
{
    if (a.di < 0) return false;
    if (b.di < 0) return true;
    return a.di < b.di || (a.di == b.di && a.dk < b.dk);
}

__device__ __forceinline__ bool better_slope(const SlopeKey &a, const SlopeKey &b)
{
    if (a.i < 0) return false;
    if (b.i < 0) return true;
    if (a.v != b.v) return a.v > b.v;
    return a.i < b.i || (a.i == b.i && a.k < b.k);
}

__global__ void slope_reduce_kernel(DsArgs A, int64_t *pair)
{
    __shared__ SlopeKey sk[1024];
    SlopeKey me{-1.0, -1, -1, -1, -1};
    const int64_t total = (int64_t)A.n_chunks * A.n;
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
        const int64_t i = e % A.n;
        const SlopeKey cand{A.row_best[e], A.row_arg[e] >= 0 ? i : -1, A.row_arg[e], -1, -1};
        if (better_slope(cand, me)) {
            me.v = cand.v;
            me.i = cand.i;
            me.k = cand.k;
        }
        if (A.row_dup[e] >= 0) {
            const SlopeKey dd{0.0, -1, -1, i, A.row_dup[e]};
            if (better_dup(dd, me)) {
                me.di = dd.di;
                me.dk = dd.dk;
            }
        }
    }
    sk[threadIdx.x] = me;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const SlopeKey a = sk[threadIdx.x], b = sk[threadIdx.x + s];
            SlopeKey r = better_slope(b, a) ? b : a;
            const SlopeKey &dsrc = better_dup(b, a) ? b : a;
            r.di = dsrc.di;
            r.dk = dsrc.dk;
            sk[threadIdx.x] = r;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const SlopeKey r = sk[0];
        double M;
        long long p0, p1;
        if (r.di >= 0) {
            M = __builtin_inf();
            p0 = r.di;
            p1 = r.dk;
        } else if (r.i >= 0) {
            M = r.v;
            p0 = r.i;
            p1 = r.k;
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

int64_t ds_npad(int64_t n) { return (n + kDsTile - 1) / kDsTile * kDsTile; }

// Small fixed area of the consistency workspace: E at 0, the error bound's
// order keys at 64, the worst-pair partials at 512.
constexpr size_t kConsAuxKeys = 64, kConsAuxWorst = 512;
constexpr size_t kConsAuxBytes = kConsAuxWorst + align_up(kReduceBlocks * sizeof(WorstRec), 256);
static_assert(kConsAuxKeys + (2 + 2 * kMaxDim) * 8 <= kConsAuxWorst, "aux layout");

size_t data_side_ws_bytes(int64_t n, int d)
{
    const size_t staged = align_up((size_t)ds_npad(n) * (size_t)(d + 2) * 8, 256);
    int cc = cons_chunks(n, d, LIP_L1);
    if (cons_chunks(n, d, LIP_L2) > cc) cc = cons_chunks(n, d, LIP_L2);
    if (cc < kDsMaxChunks) cc = kDsMaxChunks;  // the slope pass uses up to kDsMaxChunks here
    const size_t cons = align_up((size_t)cc * (size_t)n * 24, 256) +
                        align_up((size_t)ds_npad(n) * (size_t)(d + 2) * 4, 256) + kConsAuxBytes +
                        align_up((size_t)n * 24, 256);
    const size_t knn = align_up((size_t)n * 4, 256) + align_up((size_t)n * kKnnCap * 4, 256) +
                       align_up((size_t)sort_len(n) * 8, 256) + align_up((size_t)n * 8, 256) +
                       2 * kMaxDim * 8;
    const size_t part = cons > knn ? cons : knn;
    return staged + align_up(part, 256) + 4096;
}

static bool get_ds(const MetricInfo &mi, bool hasw, DsLaunchers *L)
{
    switch (mi.norm) {
    case LIP_L1: return ds_table_l1(mi.d, hasw, L);
    case LIP_L2: return ds_table_l2(mi.d, hasw, L);
    case LIP_LINF: return ds_table_linf(mi.d, hasw, L);
    default: return false;
    }
}

bool fill_ds_metric(const MetricInfo &mi, bool use_mon, DsArgs *A, Signs *sg)
{
    bool hasw = false;
    for (int i = 0; i < kMaxDim; ++i) {
        A->w[i] = i < mi.d ? mi.w[i] : 1.0;
        const int m = (use_mon && i < mi.d) ? mi.mon[i] : 0;
        A->fsel[i] = m != 0 ? 0.0 : 1.0;
        if (i < mi.d && m == 0) A->fmask |= 1 << i;
        sg->s[i] = m < 0 ? -1.0f : 1.0f;
        if (i < mi.d && mi.w[i] != 1.0) hasw = true;
    }
    return hasw;
}

// Column split: enough waves to fill the chip, chunks a multiple of the
// partner tile, at most max_chunks of them.
void choose_chunks(int64_t n, int rows_per_wave, int max_chunks, DsArgs *A, int64_t target_waves)
{
    const int64_t row_waves = (n + rows_per_wave - 1) / rows_per_wave;
    int64_t nc = (target_waves + row_waves - 1) / row_waves;
    if (nc > max_chunks) nc = max_chunks;
    if (nc < 1) nc = 1;
    int64_t cols = (n + nc - 1) / nc;
    cols = (cols + kDsTile - 1) / kDsTile * kDsTile;
    A->chunk_cols = cols;
    A->n_chunks = (int)((n + cols - 1) / cols);
}

int cons_chunks(int64_t n, int d, int norm)
{
    DsArgs A{};
    const int rows = 64 * (norm == LIP_L2 ? c32_rows(d) : ds_cons_rows(d));
    choose_chunks(n, rows, kConsMaxChunks, &A, kConsTargetWaves);
    return A.n_chunks;
}

unsigned grid_for_rows(int64_t n, int rows_per_wave, int n_chunks)
{
    const int64_t waves = (n + rows_per_wave - 1) / rows_per_wave;
    return (unsigned)(((waves + 3) / 4) * n_chunks);
}

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_consistency(const lip_metric *metric, const float *x, const float *y,
                                      int64_t n, float M, const float *Mk, double tol,
                                      int64_t *counts, double *worst_slack, int64_t *worst_pair,
                                      double *slack_up, double *slack_lo, int32_t *partner_up,
                                      int32_t *partner_lo, void *ws, size_t ws_bytes,
                                      uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || n > kMaxIndex - kDsTile) return LIP_E_SHAPE;
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
    DsArgs A{};
    Signs sg{};
    const bool hasw = fill_ds_metric(mi, true, &A, &sg);
    DsLaunchers L;
    if (!get_ds(mi, hasw, &L)) return LIP_E_UNSUPPORTED;
    A.n = n;
    A.npad = ds_npad(n);
    A.X = (const double *)ws;
    A.tol = tol;
    // l2 runs the FP32-filtered kernel (c32_rows(d) rows per lane), l1 / linf
    // the FP64 kernel (ds_cons_rows(d))
    const int rows = 64 * (mi.norm == LIP_L2 ? c32_rows(mi.d) : ds_cons_rows(mi.d));
    choose_chunks(n, rows, kConsMaxChunks, &A, kConsTargetWaves);
    char *p = (char *)ws + align_up((size_t)A.npad * (size_t)(mi.d + 2) * 8, 256);
    const size_t e = (size_t)A.n_chunks * (size_t)n;
    A.pv_up = (double *)p;
    A.pv_lo = A.pv_up + e;
    A.pi_up = (int32_t *)(A.pv_lo + e);
    A.pi_lo = A.pi_up + e;
    char *q = p + align_up(e * 24, 256);
    float *c32 = (float *)q;
    q += align_up((size_t)A.npad * (size_t)(mi.d + 2) * 4, 256);
    double *cE = (double *)q;
    unsigned long long *cons_keys = (unsigned long long *)(q + kConsAuxKeys);
    WorstRec *worst_part = (WorstRec *)(q + kConsAuxWorst);
    q += kConsAuxBytes;
    A.c32 = c32;
    A.cE = cE;
    // the worst pair needs every row's slacks and partners: rows the caller
    // did not ask for go to the workspace
    const bool worst = worst_slack || worst_pair;
    double *row_v = (double *)q;
    int32_t *row_i = (int32_t *)(row_v + 2 * n);
    A.slack_up = slack_up ? slack_up : (worst ? row_v : nullptr);
    A.slack_lo = slack_lo ? slack_lo : (worst ? row_v + n : nullptr);
    A.partner_up = partner_up ? partner_up : (worst ? row_i : nullptr);
    A.partner_lo = partner_lo ? partner_lo : (worst ? row_i + n : nullptr);
    A.counts = (unsigned long long *)counts;
    if (launch_stage64(mi.d, x, y, Mk, M, n, A.npad, sg, (double *)ws, s) != hipSuccess)
        return LIP_E_DEVICE;
    if (mi.norm == LIP_L2) {
        int64_t g32 = (A.npad + 255) / 256;
        if (g32 > 65536) g32 = 65536;
        hipLaunchKernelGGL(stage32_kernel, dim3((unsigned)g32), dim3(256), 0, s, x, y, Mk, M, n,
                           A.npad, mi.d, sg, c32);
        A.norm = mi.norm;
        int64_t gb = (n + 255) / 256;
        if (gb > kReduceBlocks) gb = kReduceBlocks;
        hipLaunchKernelGGL(cons_bound_init_kernel, dim3(1), dim3(64), 0, s, cons_keys);
        hipLaunchKernelGGL(cons_bound_kernel, dim3((unsigned)gb), dim3(256), 0, s,
                           (const float *)c32, n, mi.d, cons_keys);
        hipLaunchKernelGGL(cons_bound_final_kernel, dim3(1), dim3(64), 0, s,
                           (const unsigned long long *)cons_keys, mi.d, A, cE);
    }
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, s, A.counts);
    (mi.dm > 0 ? L.consistency_mon : L.consistency)(A, dim3(grid_for_rows(n, rows, A.n_chunks)),
                                                    dim3(256), s);
    const bool rows_out = A.slack_up || A.slack_lo || A.partner_up || A.partner_lo;
    if (mi.norm != LIP_L2) {
        // the FP64 kernel leaves per-chunk minima and tiles; the finish
        // kernel combines them and finds the partners
        if (rows_out)
            (mi.dm > 0 ? L.cons_finish_mon : L.cons_finish)(
                A, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), s);
    } else if (A.n_chunks > 1 && rows_out) {
        hipLaunchKernelGGL(consistency_combine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256),
                           0, s, A);
    }
    if (worst) {
        int64_t gw = (n + 255) / 256;
        if (gw > kReduceBlocks) gw = kReduceBlocks;
        hipLaunchKernelGGL(worst_partial_kernel, dim3((unsigned)gw), dim3(256), 0, s,
                           (const double *)A.slack_up, (const double *)A.slack_lo,
                           (const int32_t *)A.partner_up, (const int32_t *)A.partner_lo, n,
                           worst_part);
        hipLaunchKernelGGL(worst_final_kernel, dim3(1), dim3(256), 0, s,
                           (const WorstRec *)worst_part, (int)gw, worst_slack, worst_pair);
    }
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
    if (n <= 0 || n > kMaxIndex - kDsTile) return LIP_E_SHAPE;
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
    DsArgs A{};
    Signs sg{};
    const bool hasw = fill_ds_metric(mi, false, &A, &sg);
    DsLaunchers L;
    if (!get_ds(mi, hasw, &L)) return LIP_E_UNSUPPORTED;
    A.n = n;
    A.npad = ds_npad(n);
    A.X = (const double *)ws;
    A.M64 = M64;
    A.M32 = M32;
    char *p = (char *)ws + align_up((size_t)A.npad * (size_t)(mi.d + 2) * 8, 256);
    if (launch_stage64(mi.d, x, y, nullptr, 0.0f, n, A.npad, sg, (double *)ws, s) != hipSuccess)
        return LIP_E_DEVICE;
    if (mode == LIP_M_GLOBAL) {
        choose_chunks(n, 64 * kDsRows, kDsMaxChunks, &A);
        const size_t e = (size_t)A.n_chunks * (size_t)n;
        A.row_best = (double *)p;
        A.row_arg = (int32_t *)(A.row_best + e);
        A.row_dup = A.row_arg + e;
        L.slope(A, dim3(grid_for_rows(n, 64 * kDsRows, A.n_chunks)), dim3(256), s);
        hipLaunchKernelGGL(slope_reduce_kernel, dim3(1), dim3(1024), 0, s, A, pair);
    } else {
        A.knn = knn;
        const int K = knn <= 16 ? 16 : 32;
        char *q = p;
        A.kcnt = (int32_t *)q;
        q += align_up((size_t)n * 4, 256);
        A.kcand = (int32_t *)q;
        q += align_up((size_t)n * kKnnCap * 4, 256);
        const int64_t P = sort_len(n);
        unsigned long long *order = (unsigned long long *)q;
        q += align_up((size_t)P * 8, 256);
        A.tau = (double *)q;
        q += align_up((size_t)n * 8, 256);
        unsigned long long *bb = (unsigned long long *)q;
        A.x32 = x;
        // spatial order of the rows and the per-row threshold pass
        int64_t gb = (n + 255) / 256;
        if (gb > kReduceBlocks) gb = kReduceBlocks;
        hipLaunchKernelGGL(bbox_init_kernel, dim3(1), dim3(64), 0, s, bb, mi.d);
        hipLaunchKernelGGL(bbox_kernel, dim3((unsigned)gb), dim3(256), 0, s, A.X, n, A.npad, mi.d,
                           bb);
        int64_t gm = (P + 255) / 256;
        if (gm > 65536) gm = 65536;
        hipLaunchKernelGGL(morton_kernel, dim3((unsigned)gm), dim3(256), 0, s, A.X, n, A.npad,
                           mi.d, P, bb, order);
        if (launch_sort_u64(order, P, s) != hipSuccess) return LIP_E_DEVICE;
        A.order = order;
        (K == 16 ? L.tau16 : L.tau32)(A, dim3((unsigned)((n + 63) / 64)), dim3(64), s);
        // FP32 candidate scan over all pairs, then the exact ranking per row
        if (launch_fill_i32(A.kcnt, n, 0, s) != hipSuccess) return LIP_E_DEVICE;
        const int rows = 64 * rows_for_dim(mi.d);
        choose_chunks(n, rows, kKnnMaxChunks, &A);
        L.scan(A, dim3(grid_for_rows(n, rows, A.n_chunks)), dim3(256), s);
        (K == 16 ? L.select16 : L.select32)(A, dim3((unsigned)((n + 255) / 256)), dim3(256), s);
    }
    if (hipGetLastError() != hipSuccess) return LIP_E_DEVICE;
    // with the synchronous checks: an infinite estimate (coincident data with
    // different values) is reported as LIP_E_VALUE
    if ((flags & LIP_FLAG_CHECK_FINITE) && (M64 || M32)) {
        int *flag = (int *)((char *)ws + data_side_ws_bytes(n, mi.d) - 256);
        const int64_t cnt = mode == LIP_M_GLOBAL ? 1 : n;
        if (launch_fill_i32(flag, 1, 0, s) != hipSuccess) return LIP_E_DEVICE;
        int64_t g = (cnt + 255) / 256;
        if (g > 1024) g = 1024;
        hipLaunchKernelGGL(any_inf_kernel, dim3((unsigned)g), dim3(256), 0, s,
                           (const double *)M64, (const float *)M32, cnt, flag);
        int host = 0;
        if (hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return LIP_E_DEVICE;
        if (host) return LIP_E_VALUE;
    }
    return LIP_OK;
}
