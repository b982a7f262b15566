// Data-side passes over all pairs of data points, in FP64 (kernel templates):
//  * consistency - the Lipschitz condition of Sec. 1 with the monotonicity
//    constraints of Sec. 4.1, in the pairwise form of Eqs. (5)-(6) with zero
//    corrections;
//  * slope       - the largest pairwise slope (Sec. 5, global constant);
//  * knn         - the per-datum slope over the K nearest data (Sec. 4.3,
//    scalar form).
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
// Layout.  The data are staged d-major in FP64: X[j * npad + k] for
// j = 0..D-1 (coordinates), j = D (y) and j = D + 1 (M_k), npad a multiple of
// 64.  The column loop handles groups of 4 consecutive columns: one scalar
// load brings the 4 values of one coordinate into SGPRs, and the uniform
// branch on that coordinate's monotonicity is taken once per 4 columns x R
// rows instead of once per pair.
//
// Work split.  A lane owns R rows; a wave owns 64 R rows and one chunk of the
// columns, so that the grid has several waves per SIMD even when n is only
// ~1e5; per-chunk partial results are combined in chunk (= column) order.
// Workgroups are numbered chunk-fastest (blockIdx % 8 picks the XCD).
//
// Partners without per-pair index tracking: the column loop keeps running
// minima only and notes, per tile of kDsTile columns, whether they strictly
// improved; the last improving tile is re-scanned with the same arithmetic
// to find the first attaining column (for the FP64 consistency kernel in a
// separate pass over the rows, and only in the chunk that holds the
// minimum).  Violation counts are wave-uniform:
// ballot + popcount into scalar registers.
#pragma once

#include <array>
#include <climits>
#include <float.h>
#include <type_traits>
#include <utility>

#include "host_common.hpp"

namespace lip {

constexpr int kDsRows = 2;        // rows per lane (slope)
// Rows per lane of the FP64 consistency kernel: 2, and 1 above d = 12 where
// two rows of FP64 coordinates would leave one wave per SIMD.
constexpr int ds_cons_rows(int D) { return D <= 12 ? 2 : 1; }
constexpr int kDsTile = 64;       // columns per partner tile
constexpr int kDsGroup = 4;       // columns per scalar-load group
constexpr int kDsMaxChunks = 16;  // column chunks (consistency, slope)
constexpr int kKnnMaxChunks = 32; // column chunks (kNN candidate scan)
constexpr int kKnnWin = 192;      // spatial-order window of the kNN threshold pass
constexpr int64_t kDsTargetWaves = 8192;

struct DsArgs {
    const double *X;  // staged d-major [D + 2][npad]
    int64_t n, npad;
    double w[kMaxDim];
    double fsel[kMaxDim];   // 1 free, 0 monotone (decreasing ones negated at staging)
    double tol;
    int32_t fmask;          // bit i: coordinate i free (consistency with monotone coordinates)
    int32_t norm;           // 1 l1, 2 l2, 3 linf
    int32_t n_chunks;
    int32_t knn;
    int64_t chunk_cols;  // columns per chunk (multiple of kDsTile)
    // consistency: partials [n_chunks][n] and final outputs
    double *pv_up, *pv_lo;
    int32_t *pi_up, *pi_lo;
    double *slack_up, *slack_lo;
    int32_t *partner_up, *partner_lo;
    unsigned long long *counts;  // [2]
    const float *c32;   // FP32 records [npad][D + 2] (signed x, y, M_k) for the FP32 filter
    const double *cE;   // [1] error bound E of the FP32 slack
    // global slope: partials [n_chunks][n]
    double *row_best;
    int32_t *row_arg;
    int32_t *row_dup;
    // kNN: per-row candidate counters [n] and lists [n][kKnnCap]
    const float *x32;  // the caller's x [n][D] (FP32 candidate scan)
    int32_t *kcnt;
    int32_t *kcand;
    const unsigned long long *order;  // kNN row order: (Morton code << 32 | index), sorted
    double *tau;                       // [n] per-row bound on the knn-th smallest key
    double *M64;
    float *M32;
};

typedef const double __attribute__((address_space(4))) *cdouble_ptr;

// max(v, 0) and max(-v, 0) in FP64.  Written as instructions so that the
// compiler does not first quiet (canonicalize) the operand, which the IEEE
// mode of the kernels would otherwise require for fmax; v is always the
// result of an arithmetic instruction here.  Equal to the definition's
// (v > 0 ? v : 0) up to the sign of a zero, which no later step can observe
// (sums, squares and comparisons ignore it).
__device__ __forceinline__ double pos_part(double v)
{
    double r;
    asm("v_max_f64 %0, %1, 0" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ double neg_part(double v)
{
    double r;
    asm("v_max_f64 %0, -%1, 0" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ double max2(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// max(s, |v|) and max(s, -v), s >= 0 (same conventions).
__device__ __forceinline__ double max_abs(double s, double v)
{
    double r;
    asm("v_max_f64 %0, %1, |%2|" : "=v"(r) : "v"(s), "v"(v));
    return r;
}
__device__ __forceinline__ double max_neg(double s, double v)
{
    double r;
    asm("v_max_f64 %0, %1, -%2" : "=v"(r) : "v"(s), "v"(v));
    return r;
}

// The running norm value after the first component c (FIRST) or after
// adding one more component to s.  Starting from c instead of 0 + c
// differs at most in the sign of a zero.
template <int NORM, bool FIRST>
__device__ __forceinline__ double ds_acc(double s, double c)
{
    if constexpr (NORM == 1) return FIRST ? c : s + c;
    else if constexpr (NORM == 2) return FIRST ? c * c : s + c * c;
    else return FIRST ? c : max2(s, c);
}

// Accumulate coordinate i of one pair.  A free coordinate contributes |d|
// to both distances, a monotone one (d)_+ to the upper and (-d)_+ to the
// lower distance (decreasing coordinates were negated at staging, which maps
// them onto increasing ones exactly).  Without monotone coordinates (MON
// false, and for the symmetric distance) only su is formed.  With them the
// step is branch-free: with p = (d)_+, q = (-d)_+ and f = 1 for a free
// coordinate, 0 for a monotone one (wave-uniform),
//     c_up = f q + p,  c_lo = f p + q,
// each a single fused multiply-add of exact terms (one of p, q is zero and f
// is 0 or 1), hence exactly the component of the definition.
template <int NORM, bool HASW, bool MON, bool FIRST>
__device__ __forceinline__ void ds_step(double f, double w, double d, double &su, double &sl)
{
    if (!MON) {
        double a = fabs(d);
        if (HASW) a = w * a;
        su = ds_acc<NORM, FIRST>(su, a);
    } else {
        const double p = pos_part(d), q = neg_part(d);
        double cu = fma(f, q, p), cl = fma(f, p, q);
        if (HASW) {
            cu = w * cu;
            cl = w * cl;
        }
        su = ds_acc<NORM, FIRST>(su, cu);
        sl = ds_acc<NORM, FIRST>(sl, cl);
    }
}

// One pair, the column's staged values given by col(j) (j < D coordinates):
// the same operation sequence as the grouped loops below.  Without MON,
// sl = su.
template <int D, int NORM, bool HASW, bool MON, class Col>
__device__ __forceinline__ void ds_dist_col(const DsArgs &A, const double (&xr)[D], Col col,
                                            double &su, double &sl)
{
    su = 0.0;
    sl = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const double d = xr[i] - col(i);
        if (i == 0)
            ds_step<NORM, HASW, MON, true>(A.fsel[i], A.w[i], d, su, sl);
        else
            ds_step<NORM, HASW, MON, false>(A.fsel[i], A.w[i], d, su, sl);
    }
    if (NORM == 2) {
        su = sqrt(su);
        if (MON) sl = sqrt(sl);
    }
    if (!MON) sl = su;
}

// One pair, column k read from the staged data (per-lane vector loads).
template <int D, int NORM, bool HASW, bool MON>
__device__ __forceinline__ void ds_dist1(const DsArgs &A, const double (&xr)[D], int64_t k,
                                         double &su, double &sl)
{
    ds_dist_col<D, NORM, HASW, MON>(
        A, xr, [&](int j) { return A.X[(int64_t)j * A.npad + k]; }, su, sl);
}

// Component step with the coordinate's kind known at compile time: a free
// coordinate adds |d| to both distances, a monotone one (d)_+ to the upper
// and (-d)_+ to the lower one.  Bit for bit the values of the branch-free
// ds_step (fma(1, q, p) = p + q = |d| and fma(0, q, p) = p exactly, since
// one of p, q is zero).
template <int NORM, bool HASW, bool FREE, bool FIRST>
__device__ __forceinline__ void ds_step_kind(double w, double d, double &su, double &sl)
{
    if constexpr (FREE) {
        double a = fabs(d);
        if (HASW) a = w * a;
        su = ds_acc<NORM, FIRST>(su, a);
        sl = ds_acc<NORM, FIRST>(sl, a);
    } else {
        double p = pos_part(d), q = neg_part(d);
        if (HASW) {
            p = w * p;
            q = w * q;
        }
        su = ds_acc<NORM, FIRST>(su, p);
        sl = ds_acc<NORM, FIRST>(sl, q);
    }
}

// Distances of R rows to the columns g0 .. g0 + kDsGroup - 1 (scalar
// loads of one coordinate of the whole group at a time).  For l2 the sums
// of squares are returned (no root); without MON only su is formed.  FM >= 0
// gives the free / monotone kind of every coordinate at compile time (bit i
// set: coordinate i free); FM < 0 reads it from A.fsel at run time.
template <int D, int NORM, bool HASW, bool MON, int R, int FM = -1>
__device__ __forceinline__ void ds_dist_group(const DsArgs &A, cdouble_ptr X, int64_t g0,
                                              const double (&xr)[R][D],
                                              double (&su)[kDsGroup][R],
                                              double (&sl)[kDsGroup][R])
{
    if constexpr (NORM == 3 && MON && FM >= 0) {
        // linf with the kinds known: a maximum is exact in any order, so the
        // free coordinates go first into f = max |w d| (>= 0, 0 without free
        // coordinates), shared by both distances; then, since f >= 0,
        // max(s, w (d)_+) = max(s, w d) and max(s, w (-d)_+) = max(s, -w d)
        // for each monotone coordinate: one maximum per free coordinate and
        // two per monotone one instead of two and four, with the
        // definition's values (up to the sign of a zero).
        double f[kDsGroup][R];
#pragma unroll
        for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) f[c][r] = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (!((FM >> i) & 1)) continue;
            double xc[kDsGroup];
#pragma unroll
            for (int c = 0; c < kDsGroup; ++c) xc[c] = X[(int64_t)i * A.npad + g0 + c];
            const double w = A.w[i];
#pragma unroll
            for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double e = xr[r][i] - xc[c];
                    if (HASW) e = w * e;
                    f[c][r] = max_abs(f[c][r], e);
                }
        }
#pragma unroll
        for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) su[c][r] = sl[c][r] = f[c][r];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if ((FM >> i) & 1) continue;
            double xc[kDsGroup];
#pragma unroll
            for (int c = 0; c < kDsGroup; ++c) xc[c] = X[(int64_t)i * A.npad + g0 + c];
            const double w = A.w[i];
#pragma unroll
            for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double e = xr[r][i] - xc[c];
                    if (HASW) e = w * e;
                    su[c][r] = max2(su[c][r], e);
                    sl[c][r] = max_neg(sl[c][r], e);
                }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double xc[kDsGroup];
#pragma unroll
        for (int c = 0; c < kDsGroup; ++c) xc[c] = X[(int64_t)i * A.npad + g0 + c];
        const double w = A.w[i], f = A.fsel[i];
#pragma unroll
        for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double d = xr[r][i] - xc[c];
                if constexpr (MON && FM >= 0) {
                    const bool fr = (FM >> i) & 1;
                    if (i == 0) {
                        if (fr) ds_step_kind<NORM, HASW, true, true>(w, d, su[c][r], sl[c][r]);
                        else ds_step_kind<NORM, HASW, false, true>(w, d, su[c][r], sl[c][r]);
                    } else {
                        if (fr) ds_step_kind<NORM, HASW, true, false>(w, d, su[c][r], sl[c][r]);
                        else ds_step_kind<NORM, HASW, false, false>(w, d, su[c][r], sl[c][r]);
                    }
                } else if (i == 0) {
                    ds_step<NORM, HASW, MON, true>(f, w, d, su[c][r], sl[c][r]);
                } else {
                    ds_step<NORM, HASW, MON, false>(f, w, d, su[c][r], sl[c][r]);
                }
            }
    }
}

// Work coordinates of a wave: rows [r0, r1), columns [c0, c1).
struct WaveRange {
    int64_t r0, r1, c0, c1;
    int chunk;
};

__device__ __forceinline__ bool wave_range(const DsArgs &A, int rows_per_wave, WaveRange &w)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    w.chunk = blockIdx.x % A.n_chunks;
    const int64_t rb = (int64_t)(blockIdx.x / A.n_chunks) * (blockDim.x >> 6) + wave;
    w.r0 = rb * rows_per_wave;
    if (w.r0 >= A.n) return false;
    w.r1 = w.r0 + rows_per_wave < A.n ? w.r0 + rows_per_wave : A.n;
    w.c0 = (int64_t)w.chunk * A.chunk_cols;
    w.c1 = w.c0 + A.chunk_cols < A.n ? w.c0 + A.chunk_cols : A.n;
    return true;
}

// ---- consistency -------------------------------------------------------------

// One group of kDsGroup columns for the R rows of each lane.  MASK: the group
// holds columns past n or the rows' own columns (such pairs are skipped);
// FULLW: every row of the wave exists, so the violation ballots need no row
// mask.  Violations are counted in 32 bits per tile (at most 64 R x 64 per
// tile) by the caller.
template <int D, int NORM, bool HASW, bool MON, bool MASK, int FM, int R, bool FULLW = false>
__device__ __forceinline__ void cons_group(const DsArgs &A, cdouble_ptr X, int64_t g0,
                                           const double (&xr)[R][D],
                                           const double (&yr)[R], const int (&ir)[R],
                                           const unsigned long long (&vmask)[R],
                                           double (&bu)[R], double (&bl)[R], unsigned &cu,
                                           unsigned &cl)
{
    double su[kDsGroup][R], sl[kDsGroup][R];
    ds_dist_group<D, NORM, HASW, MON, R, FM>(A, X, g0, xr, su, sl);
    double yk[kDsGroup], mk[kDsGroup];
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c) {
        yk[c] = X[(int64_t)D * A.npad + g0 + c];
        mk[c] = X[(int64_t)(D + 1) * A.npad + g0 + c];
    }
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double du = su[c][r], dl = MON ? sl[c][r] : su[c][r];
            if (NORM == 2) {
                du = sqrt(du);
                dl = MON ? sqrt(dl) : du;
            }
            double tu = fma(mk[c], du, yk[c]) - yr[r];
            double tl = yr[r] - fma(-mk[c], dl, yk[c]);
            if (MASK) {
                const int64_t k = g0 + c;
                const bool ok = k < A.n && k != ir[r];
                tu = ok ? tu : __builtin_inf();
                tl = ok ? tl : __builtin_inf();
            }
            bu[r] = fmin(bu[r], tu);
            bl[r] = fmin(bl[r], tl);
            // lanes past the last row are removed with the wave-uniform mask
            // (scalar work) instead of a per-pair vector condition
            if constexpr (FULLW) {
                cu += __popcll(__ballot(tu < -A.tol));
                cl += __popcll(__ballot(tl < -A.tol));
            } else {
                cu += __popcll(__ballot(tu < -A.tol) & vmask[r]);
                cl += __popcll(__ballot(tl < -A.tol) & vmask[r]);
            }
        }
}

// Slacks of one pair (row values xr, yr; column values col(j): coordinates,
// then y_k at j = D and M_k at j = D + 1).
template <int D, int NORM, bool HASW, bool MON, class Col>
__device__ __forceinline__ void cons_pair_col(const DsArgs &A, const double (&xr)[D], double yr,
                                              Col col, double &tu, double &tl)
{
    double du, dl;
    ds_dist_col<D, NORM, HASW, MON>(A, xr, col, du, dl);
    const double yk = col(D), mk = col(D + 1);
    tu = fma(mk, du, yk) - yr;
    tl = yr - fma(-mk, dl, yk);
}

template <int D, int NORM, bool HASW, bool MON>
__device__ __forceinline__ void cons_pair(const DsArgs &A, const double (&xr)[D], double yr,
                                          int64_t k, double &tu, double &tl)
{
    cons_pair_col<D, NORM, HASW, MON>(
        A, xr, yr, [&](int j) { return A.X[(int64_t)j * A.npad + k]; }, tu, tl);
}

template <int D, int NORM, bool HASW, bool MON, int FM = -1>
__global__ void __launch_bounds__(256) consistency_kernel(DsArgs A)
{
    constexpr int R = ds_cons_rows(D);
    constexpr int RW = 64 * R;
    WaveRange w;
    if (!wave_range(A, RW, w)) return;
    const int lane = threadIdx.x & 63;
    double xr[R][D], yr[R], bu[R], bl[R];
    int ir[R], tu_t[R], tl_t[R];
    bool valid[R];
    unsigned long long vmask[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = w.r0 + r * 64 + lane;
        valid[r] = i < A.n;
        vmask[r] = __ballot(valid[r]);
        i = i < A.n ? i : A.n - 1;
        ir[r] = (int)i;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.X[(int64_t)j * A.npad + i];
        yr[r] = A.X[(int64_t)D * A.npad + i];
        bu[r] = __builtin_inf();
        bl[r] = __builtin_inf();
        tu_t[r] = tl_t[r] = -1;
    }
    const cdouble_ptr X = (cdouble_ptr)(A.X);
    unsigned long long cu = 0, cl = 0;
    const bool fullw = w.r0 + RW <= A.n;
    int t = 0;
    for (int64_t tb = w.c0; tb < w.c1; tb += kDsTile, ++t) {
        const int64_t te = tb + kDsTile < w.c1 ? tb + kDsTile : w.c1;
        double pu[R], pl[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pu[r] = bu[r];
            pl[r] = bl[r];
        }
        unsigned tcu = 0, tcl = 0;
#pragma unroll 1
        for (int64_t g0 = tb; g0 < te; g0 += kDsGroup) {
            const bool masked = (g0 + kDsGroup > A.n) || (g0 < w.r1 && g0 + kDsGroup > w.r0);
            if (masked)
                cons_group<D, NORM, HASW, MON, true, FM, R>(A, X, g0, xr, yr, ir, vmask, bu, bl,
                                                            tcu, tcl);
            else if (fullw)
                cons_group<D, NORM, HASW, MON, false, FM, R, true>(A, X, g0, xr, yr, ir, vmask,
                                                                   bu, bl, tcu, tcl);
            else
                cons_group<D, NORM, HASW, MON, false, FM, R>(A, X, g0, xr, yr, ir, vmask, bu, bl,
                                                             tcu, tcl);
        }
        cu += tcu;
        cl += tcl;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            tu_t[r] = bu[r] < pu[r] ? t : tu_t[r];
            tl_t[r] = bl[r] < pl[r] ? t : tl_t[r];
        }
    }
    // per chunk and row: the smallest slacks and the last tile where they
    // improved; consistency_finish_kernel finds the partners from them
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!valid[r]) continue;
        const int64_t o = (int64_t)w.chunk * A.n + ir[r];
        A.pv_up[o] = bu[r];
        A.pv_lo[o] = bl[r];
        A.pi_up[o] = tu_t[r];
        A.pi_lo[o] = tl_t[r];
    }
    if (lane == 0) {
        atomicAdd(A.counts, cu);
        atomicAdd(A.counts + 1, cl);
    }
}

// Per row, after consistency_kernel: the smallest slack of each bound over
// the chunks (the first chunk on ties, i.e. the lower columns) and its
// partner, the first column of that chunk's last improving tile attaining
// it, found with the column loop's arithmetic.  Only the winning chunk's
// tile is re-scanned, in a kernel of its own where many rows keep the loads
// in flight.  A tile starts below n at a multiple of kDsTile and npad is a
// multiple of kDsTile, so all its columns are inside the staged
// (zero-padded) data: they are evaluated unconditionally and the conditions
// only decide which results count.
constexpr int kFinishChunks = 32;  // column chunks the finish pass reads (at most)

template <int D, int NORM, bool HASW, bool MON>
__global__ void __launch_bounds__(256) consistency_finish_kernel(DsArgs A)
{
    // two threads per row, one per bound (more rows' loads in flight)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> 1;
    const int side = (int)(t & 1);
    if (i >= A.n) return;
    double xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xr[j] = A.X[(int64_t)j * A.npad + i];
    const double yr = A.X[(int64_t)D * A.npad + i];
    const double *pv = side ? A.pv_lo : A.pv_up;
    const int32_t *pt = side ? A.pi_lo : A.pi_up;
    // all chunks' minima loaded before any is compared (independent loads)
    double v[kFinishChunks];
#pragma unroll
    for (int c = 0; c < kFinishChunks; ++c)
        v[c] = c < A.n_chunks ? pv[(int64_t)c * A.n + i] : __builtin_inf();
    double best = __builtin_inf();
    int cb = -1;
#pragma unroll
    for (int c = 0; c < kFinishChunks; ++c) {
        if (v[c] < best) {
            best = v[c];
            cb = c;
        }
    }
    const int tb = cb >= 0 ? pt[(int64_t)cb * A.n + i] : -1;
    int part = -1;
    if (tb >= 0) {
        const int64_t base = (int64_t)cb * A.chunk_cols + (int64_t)tb * kDsTile;
        int64_t c1 = (int64_t)(cb + 1) * A.chunk_cols;
        c1 = c1 < A.n ? c1 : A.n;
#pragma unroll 8
        for (int k = kDsTile - 1; k >= 0; --k) {
            const int64_t col = base + k;
            double tu, tl;
            cons_pair<D, NORM, HASW, MON>(A, xr, yr, col, tu, tl);
            if (((side ? tl : tu) == best) & (col < c1) & (col != i)) part = (int)col;
        }
    }
    double *sv = side ? A.slack_lo : A.slack_up;
    int32_t *sp = side ? A.partner_lo : A.partner_up;
    if (sv) sv[i] = best;
    if (sp) sp[i] = part;
}

// ---- global M: max over i < k of |y_i - y_k| / dist ------------------------------

template <int D, int NORM, bool HASW, bool MASK>
__device__ __forceinline__ void slope_group(const DsArgs &A, cdouble_ptr X, int64_t g0,
                                            const double (&xr)[kDsRows][D],
                                            const double (&yr)[kDsRows], const int (&ir)[kDsRows],
                                            double (&best)[kDsRows], int (&arg)[kDsRows],
                                            int (&dup)[kDsRows])
{
    double su[kDsGroup][kDsRows], sl[kDsGroup][kDsRows];
    ds_dist_group<D, NORM, HASW, false, kDsRows>(A, X, g0, xr, su, sl);
    double yk[kDsGroup];
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c) yk[c] = X[(int64_t)D * A.npad + g0 + c];
#pragma unroll
    for (int c = 0; c < kDsGroup; ++c)
#pragma unroll
        for (int r = 0; r < kDsRows; ++r) {
            const int64_t k = g0 + c;
            if (MASK && !(k > ir[r] && k < A.n)) continue;
            double du = su[c][r];
            if (NORM == 2) du = sqrt(du);
            const double dy = fabs(yr[r] - yk[c]);
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

template <int D, int NORM, bool HASW>
__global__ void __launch_bounds__(256) slope_kernel(DsArgs A)
{
    constexpr int RW = 64 * kDsRows;
    WaveRange w;
    if (!wave_range(A, RW, w)) return;
    const int lane = threadIdx.x & 63;
    double xr[kDsRows][D], yr[kDsRows], best[kDsRows];
    int ir[kDsRows], arg[kDsRows], dup[kDsRows];
    bool valid[kDsRows];
#pragma unroll
    for (int r = 0; r < kDsRows; ++r) {
        int64_t i = w.r0 + r * 64 + lane;
        valid[r] = i < A.n;
        i = i < A.n ? i : A.n - 1;
        ir[r] = (int)i;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.X[(int64_t)j * A.npad + i];
        yr[r] = A.X[(int64_t)D * A.npad + i];
        best[r] = -1.0;
        arg[r] = -1;
        dup[r] = -1;
    }
    const cdouble_ptr X = (cdouble_ptr)(A.X);
    // only columns k > i: groups left of the wave's rows are skipped, groups
    // overlapping them (or the end of the data) are masked per pair.
    const int64_t gstart = w.c0 > (w.r0 / kDsGroup) * kDsGroup ? w.c0 : (w.r0 / kDsGroup) * kDsGroup;
#pragma unroll 1
    for (int64_t g0 = gstart; g0 < w.c1; g0 += kDsGroup) {
        const bool masked = (g0 + kDsGroup > A.n) || (g0 < w.r1);
        if (masked)
            slope_group<D, NORM, HASW, true>(A, X, g0, xr, yr, ir, best, arg, dup);
        else
            slope_group<D, NORM, HASW, false>(A, X, g0, xr, yr, ir, best, arg, dup);
    }
#pragma unroll
    for (int r = 0; r < kDsRows; ++r) {
        if (!valid[r]) continue;
        const int64_t o = (int64_t)w.chunk * A.n + ir[r];
        A.row_best[o] = best[r];
        A.row_arg[o] = arg[r];
        A.row_dup[o] = dup[r];
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

// M_i = max over the neighbour list of |y_i - y_j| / dist (coincident
// neighbours: skipped with equal y, infinite slope otherwise).
template <int D, int NORM, bool HASW, int K>
__device__ __forceinline__ void knn_finish(const DsArgs &A, int64_t i, const double (&xr)[D],
                                           const int (&idx)[K])
{
    const double yi = A.X[(int64_t)D * A.npad + i];
    double best = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        if (t >= A.knn || idx[t] < 0) continue;
        double du, dl;
        ds_dist1<D, NORM, HASW, false>(A, xr, idx[t], du, dl);
        const double dy = fabs(yi - A.X[(int64_t)D * A.npad + idx[t]]);
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

// Smallest double above a finite t.
__device__ __forceinline__ double next_up(double t)
{
    const long long b = __double_as_longlong(t);
    if (t == 0.0) return __longlong_as_double(1ll);
    return __longlong_as_double(t > 0.0 ? b + 1 : b - 1);
}

// Threshold pass.  A wave takes 64 consecutive rows of the spatial (Morton)
// order and the kKnnWin data around them in that order, staged in LDS; each
// row keeps the knn smallest keys over that window (itself excluded).  The
// knn-th of them bounds the knn-th smallest key over all data from above, so
// the full scan can skip every column above it.  Keys are formed with the
// same operation sequence as in the full scan.
template <int D, int NORM, bool HASW, int K>
__global__ void __launch_bounds__(64) knn_tau_kernel(DsArgs A)
{
    __shared__ double win[D][kKnnWin];
    __shared__ int32_t wid[kKnnWin];
    const int lane = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    int64_t wlo = r0 - (kKnnWin - 64) / 2;
    if (wlo + kKnnWin > A.n) wlo = A.n - kKnnWin;
    if (wlo < 0) wlo = 0;
    const int nw = (int)(A.n - wlo < kKnnWin ? A.n - wlo : kKnnWin);
    for (int t = lane; t < nw; t += 64) {
        const int64_t c = (int64_t)(uint32_t)(A.order[wlo + t] & 0xFFFFFFFFull);
        wid[t] = (int32_t)c;
#pragma unroll
        for (int j = 0; j < D; ++j) win[j][t] = A.X[(int64_t)j * A.npad + c];
    }
    __syncthreads();
    const int64_t pos = r0 + lane;
    if (pos >= A.n) return;
    const int64_t i = (int64_t)(uint32_t)(A.order[pos] & 0xFFFFFFFFull);
    double xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xr[j] = A.X[(int64_t)j * A.npad + i];
    double key[K];
    int idx[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        key[t] = __builtin_inf();
        idx[t] = -1;
    }
    const int kk = A.knn;
    double thr = __builtin_inf();
#pragma unroll 1
    for (int t = 0; t < nw; ++t) {
        double su = 0.0, sl = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double dd = xr[j] - win[j][t];
            if (j == 0)
                ds_step<NORM, HASW, false, true>(1.0, A.w[j], dd, su, sl);
            else
                ds_step<NORM, HASW, false, false>(1.0, A.w[j], dd, su, sl);
        }
        if (wid[t] != (int32_t)i && su < thr) {
            knn_insert<K>(key, idx, su, wid[t]);
#pragma unroll
            for (int q = 0; q < K; ++q)
                if (q == kk - 1) thr = key[q];
        }
    }
    A.tau[i] = thr;
}

// Candidate scan.  In FP32, every pair (row i, column k) of the rows' spatial
// order x the chunk's columns is tested against the row's bound from the
// threshold pass, tau32 >= tau (1 + 2^-17) + 2^-120.  The FP32 key (the same
// sum / sum of squares / max as the FP64 key, each operation rounded to
// FP32) is within (d + 3) 2^-24 relative of the exact value, so every column
// whose FP64 key is <= tau passes.  Passing columns (a few dozen per row)
// are appended to the row's candidate list with an atomic counter; the
// select pass ranks them exactly.  Rows per lane follow the FP32 bound
// kernel; columns come through scalar loads in double-buffered groups.
constexpr int kKnnCap = 512;  // candidate slots per row (a few dozen are typical)

constexpr int knn_group(int D) { return D <= 4 ? 4 : (D <= 8 ? 2 : 1); }

__device__ __forceinline__ float knn_tau32(double t)
{
    if (!(t < __builtin_inf())) return __builtin_inff();
    const double v = t * (1.0 + 0x1p-17) + 0x1p-120;
    float f = (float)v;
    if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);  // v >= 0: next float up
    return f;
}

template <int D, int NORM, bool HASW>
__device__ __forceinline__ float knn_key32(const float (&xr)[D], const float *v, const float (&w)[D])
{
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float a = fabsf(xr[j] - v[j]);
        if (HASW) a = a * w[j];
        if (NORM == 1) s = j == 0 ? a : s + a;
        else if (NORM == 2) s = j == 0 ? a * a : fmaf(a, a, s);
        else s = j == 0 ? a : fmaxf(s, a);
    }
    return s;
}

template <int D, int NORM, bool HASW>
__global__ void __launch_bounds__(256) knn_scan_kernel(DsArgs A)
{
    constexpr int R = rows_for_dim(D);
    constexpr int G = knn_group(D);
    WaveRange w;
    if (!wave_range(A, 64 * R, w)) return;
    const int lane = threadIdx.x & 63;
    float xr[R][D], tr[R];
    int32_t ir[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p0 = w.r0 + r * 64 + lane;
        const bool valid = p0 < A.n;
        const int64_t pc = valid ? p0 : A.n - 1;
        const int64_t i = (int64_t)(uint32_t)(A.order[pc] & 0xFFFFFFFFull);
        ir[r] = (int32_t)i;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.x32[i * D + j];
        tr[r] = valid ? knn_tau32(A.tau[i]) : -1.0f;  // an invalid lane never passes
    }
    float wv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) wv[j] = (float)A.w[j];
    const cfloat_ptr xc = as_const(A.x32);

    auto hits = [&](int64_t g, const float (&v)[G * D]) {
        bool any = false;
        float key[G][R];
#pragma unroll
        for (int c = 0; c < G; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                key[c][r] = knn_key32<D, NORM, HASW>(xr[r], v + c * D, wv);
                any = any || key[c][r] <= tr[r];
            }
        if (__builtin_amdgcn_ballot_w64(any) == 0) return;
#pragma unroll
        for (int c = 0; c < G; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t k = g + c;
                if (key[c][r] <= tr[r] && k < w.c1) {
                    const int slot = atomicAdd(A.kcnt + ir[r], 1);
                    if (slot < kKnnCap) A.kcand[(int64_t)ir[r] * kKnnCap + slot] = (int32_t)k;
                }
            }
    };
    auto load = [&](int64_t g, float (&v)[G * D]) {
        if (g + G <= A.n) {
#pragma unroll
            for (int e = 0; e < G * D; ++e) v[e] = xc[g * D + e];
        } else {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                const int64_t k = g + c < A.n ? g + c : A.n - 1;
#pragma unroll
                for (int j = 0; j < D; ++j) v[c * D + j] = xc[k * D + j];
            }
        }
    };
    // two groups per iteration, the next one requested before use
    float va[G * D], vb[G * D];
    int64_t g = w.c0;
    if (g < w.c1) load(g, va);
#pragma unroll 1
    for (; g + G < w.c1; g += 2 * G) {
        load(g + G, vb);
        hits(g, va);
        if (g + 2 * G < w.c1) load(g + 2 * G, va);
        hits(g + G, vb);
    }
    if (g < w.c1) hits(g, va);
}

// K smallest (key, index) pairs in lexicographic order (candidates arrive
// in any order).
template <int K>
__device__ __forceinline__ void knn_insert_lex(double (&key)[K], int (&idx)[K], double kv, int j)
{
    if (!(kv < key[K - 1] || (kv == key[K - 1] && j < idx[K - 1]))) return;
    key[K - 1] = kv;
    idx[K - 1] = j;
#pragma unroll
    for (int t = K - 1; t > 0; --t) {
        const bool sw = key[t] < key[t - 1] || (key[t] == key[t - 1] && idx[t] < idx[t - 1]);
        const double a = key[t], b = key[t - 1];
        const int ia = idx[t], ib = idx[t - 1];
        key[t] = sw ? b : a;
        key[t - 1] = sw ? a : b;
        idx[t] = sw ? ib : ia;
        idx[t - 1] = sw ? ia : ib;
    }
}

// FP64 key of one pair with the operation sequence of ds_dist_group (l2:
// the sum of squares).
template <int D, int NORM, bool HASW>
__device__ __forceinline__ double knn_key64(const DsArgs &A, const double (&xr)[D], int64_t k)
{
    double su = 0.0, sl = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double dd = xr[j] - A.X[(int64_t)j * A.npad + k];
        if (j == 0) ds_step<NORM, HASW, false, true>(1.0, A.w[j], dd, su, sl);
        else ds_step<NORM, HASW, false, false>(1.0, A.w[j], dd, su, sl);
    }
    return su;
}

// Exact ranking: the row's candidates (or, if they overflowed the list,
// every column) by (FP64 key, index), then M_i over the first knn.
template <int D, int NORM, bool HASW, int K>
__global__ void __launch_bounds__(256) knn_select_kernel(DsArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    double xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xr[j] = A.X[(int64_t)j * A.npad + i];
    double key[K];
    int idx[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        key[t] = __builtin_inf();
        idx[t] = -1;
    }
    const int cnt = A.kcnt[i];
    if (cnt <= kKnnCap) {
        for (int t = 0; t < cnt; ++t) {
            const int k = A.kcand[i * kKnnCap + t];
            if (k == (int)i) continue;
            knn_insert_lex<K>(key, idx, knn_key64<D, NORM, HASW>(A, xr, k), k);
        }
    } else {
        for (int64_t k = 0; k < A.n; ++k) {
            if (k == i) continue;
            knn_insert_lex<K>(key, idx, knn_key64<D, NORM, HASW>(A, xr, k), (int)k);
        }
    }
    knn_finish<D, NORM, HASW, K>(A, i, xr, idx);
}

// ---- consistency with an FP32 filter -----------------------------------------
//
// The same outputs as consistency_kernel, bit for bit, with most pairs
// decided in FP32.  For a pair, t32 (the slack evaluated in FP32 from the
// same inputs: distance components, weights, sum / sum of squares + square
// root / max, then fma(M_k, dist, y_k) - y_i) differs from the FP64 slack by
// at most E = 2^-18 (max M_k * max dist + 2 max |y|) + max M_k 2^-60 + 2^-126
// (at most (d + 8) 2^-24 relative in the distance, three more roundings in
// the bound, a factor two spare; the absolute terms cover FP32 underflow).
// Data whose FP32 evaluation could overflow get E = +inf.  With V- <= -tol - E and V+ >= -tol + E (FP32, rounded outwards):
//   t32 <  V-             : a violation (t < -tol) for certain;
//   t32 >= V+             : no violation for certain;
//   otherwise             : ambiguous, decided in FP64;
//   t32 <= U + E (FP32)   : may lower the running minimum U, evaluated in
//                            FP64 (strict improvement in column order keeps
//                            the lowest index, as the partner requires).
// Pairs that need FP64 are evaluated with cons_pair_col (the FP64 kernel's
// own operation sequence, on the column's FP32 record widened).  A NaN t32 or an infinite E sends the pair to FP64.
// Rows per lane of the FP32-filtered kernel: one.  The per-pair predicates of
// every (row, column) of a group are held as lane masks in scalar registers
// until the wave's FP64 branch; with more rows they overflow the scalar file
// and spill into vector lanes (at d = 4: 4 rows 15.4 ms, 2 rows 12.8 ms,
// 1 row 11.1 ms for the 1e10 ordered pairs of the benchmark data).
constexpr int c32_rows(int D) { return 1; }

constexpr int c32_group(int D) { return D <= 4 ? 2 : 1; }

// Neighbouring floats of a finite f (toward -inf / +inf).
__device__ __forceinline__ float f32_prev(float f)
{
    if (f == 0.0f) return -0x1p-149f;
    const uint32_t b = __float_as_uint(f);
    return __uint_as_float(f > 0.0f ? b - 1u : b + 1u);
}
__device__ __forceinline__ float f32_next(float f)
{
    if (f == 0.0f) return 0x1p-149f;
    const uint32_t b = __float_as_uint(f);
    return __uint_as_float(f > 0.0f ? b + 1u : b - 1u);
}

// v rounded to FP32 toward -inf / +inf (infinities and NaN pass through).
__device__ __forceinline__ float f32_down(double v)
{
    float f = (float)v;
    if ((double)f > v && __builtin_isfinite(f)) f = f32_prev(f);
    return f;
}

__device__ __forceinline__ float f32_up(double v)
{
    float f = (float)v;
    if ((double)f < v && __builtin_isfinite(f)) f = f32_next(f);
    return f;
}

// FP32 distance components of one pair: free coordinates |d| to both sums,
// monotone ones (d)_+ to the upper and (-d)_+ to the lower sum; FM >= 0 gives
// the kinds at compile time, FM < 0 reads A.fsel.
template <int D, int NORM, bool HASW, bool MON, int FM>
__device__ __forceinline__ void c32_dist(const DsArgs &A, const float (&xr)[D], const float *xc,
                                         float &du, float &dl)
{
    if constexpr (MON && FM >= 0) {
        // kinds known: the free coordinates first, into the part shared by
        // both sums (any order is within the error bound E), then the
        // monotone ones
        float f = 0.0f;
        bool first = true;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (!((FM >> j) & 1)) continue;
            float c = fabsf(xr[j] - xc[j]);
            if (HASW) c *= (float)A.w[j];
            if (NORM == 1) f = first ? c : f + c;
            else if (NORM == 2) f = first ? c * c : fmaf(c, c, f);
            else f = first ? c : fmaxf(f, c);
            first = false;
        }
        float su = f, sl = f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if ((FM >> j) & 1) continue;
            const float d = xr[j] - xc[j];
            float cu = fmaxf(d, 0.0f), cl = fmaxf(-d, 0.0f);
            if (HASW) {
                const float wj = (float)A.w[j];
                cu *= wj;
                cl *= wj;
            }
            if (NORM == 1) {
                su = first ? cu : su + cu;
                sl = first ? cl : sl + cl;
            } else if (NORM == 2) {
                su = first ? cu * cu : fmaf(cu, cu, su);
                sl = first ? cl * cl : fmaf(cl, cl, sl);
            } else {
                su = first ? cu : fmaxf(su, cu);
                sl = first ? cl : fmaxf(sl, cl);
            }
            first = false;
        }
        if (NORM == 2) {
            su = __builtin_amdgcn_sqrtf(su);
            sl = __builtin_amdgcn_sqrtf(sl);
        }
        du = su;
        dl = sl;
        return;
    }
    float su = 0.0f, sl = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const float d = xr[j] - xc[j];
        float cu, cl;
        bool fr;
        if constexpr (!MON) fr = true;
        else if constexpr (FM >= 0) fr = (FM >> j) & 1;
        else fr = false;
        if (fr) {
            cu = cl = fabsf(d);
        } else if constexpr (MON && FM >= 0) {
            cu = fmaxf(d, 0.0f);
            cl = fmaxf(-d, 0.0f);
        } else {
            const float f = (float)A.fsel[j];
            const float p = fmaxf(d, 0.0f), q = fmaxf(-d, 0.0f);
            cu = fmaf(f, q, p);
            cl = fmaf(f, p, q);
        }
        if (HASW) {
            const float wj = (float)A.w[j];
            cu *= wj;
            cl *= wj;
        }
        if (NORM == 1) {
            su = j == 0 ? cu : su + cu;
            if (MON) sl = j == 0 ? cl : sl + cl;
        } else if (NORM == 2) {
            su = j == 0 ? cu * cu : fmaf(cu, cu, su);
            if (MON) sl = j == 0 ? cl * cl : fmaf(cl, cl, sl);
        } else {
            su = j == 0 ? cu : fmaxf(su, cu);
            if (MON) sl = j == 0 ? cl : fmaxf(sl, cl);
        }
    }
    if (NORM == 2) {
        su = __builtin_amdgcn_sqrtf(su);
        if (MON) sl = __builtin_amdgcn_sqrtf(sl);
    }
    du = su;
    dl = MON ? sl : su;
}

template <int D, int NORM, bool HASW, bool MON, int FM = -1>
__global__ void __launch_bounds__(256) consistency32_kernel(DsArgs A)
{
    constexpr int R = c32_rows(D);
    constexpr int S = D + 2;
    constexpr int G = c32_group(D);
    WaveRange w;
    if (!wave_range(A, 64 * R, w)) return;
    const int lane = threadIdx.x & 63;
    const double E = A.cE[0];
    const float vlo = f32_down(-A.tol - E), vhi = f32_up(-A.tol + E);
    float xr[R][D], yr[R], umin[R], lmin[R];
    double bu[R], bl[R];
    int ir[R], pu[R], pl[R];
    bool valid[R];
    unsigned long long vmask[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = w.r0 + r * 64 + lane;
        valid[r] = i < A.n;
        vmask[r] = __ballot(valid[r]);
        i = valid[r] ? i : A.n - 1;
        ir[r] = (int)i;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[r][j] = A.c32[i * S + j];
        yr[r] = A.c32[i * S + D];
        bu[r] = bl[r] = __builtin_inf();
        umin[r] = lmin[r] = __builtin_inff();
        pu[r] = pl[r] = -1;
    }
    unsigned long long cu = 0, cl = 0;  // certain violations (wave-uniform)
    unsigned int xu = 0, xl = 0;        // violations decided in FP64 (per lane)
    const cfloat_ptr C = as_const(A.c32);

    // Per (column, row) the predicates are lane masks (one vector compare
    // each, the logic on the scalar unit): certain violations are counted
    // at once; au / al mark the ambiguous lanes, eu / el the lanes that need
    // the FP64 evaluation (ambiguous, or within E of the running minimum).
    auto visit = [&](int64_t g, const float (&v)[G * S], auto mask_tag) {
        constexpr bool MASK = decltype(mask_tag)::value;
        unsigned long long any = 0;
        unsigned long long eu[G][R], el[G][R], au[G][R], al[G][R];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const float yk = v[c * S + D], mk = v[c * S + D + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float du, dl;
                c32_dist<D, NORM, HASW, MON, FM>(A, xr[r], v + c * S, du, dl);
                const float tu = fmaf(mk, du, yk) - yr[r];
                const float tl = yr[r] - fmaf(-mk, dl, yk);
                // okm: the pair exists (column inside the data, not the
                // row's own); ok: also the row exists
                unsigned long long okm = ~0ull, ok = vmask[r];
                if (MASK) {
                    okm = __builtin_amdgcn_ballot_w64((g + c) < A.n && (int)(g + c) != ir[r]);
                    ok &= okm;
                }
                const unsigned long long su = __builtin_amdgcn_ballot_w64(tu < vlo);
                const unsigned long long sl = __builtin_amdgcn_ballot_w64(tl < vlo);
                const unsigned long long nu = __builtin_amdgcn_ballot_w64(tu >= vhi);
                const unsigned long long nl = __builtin_amdgcn_ballot_w64(tl >= vhi);
                cu += __popcll(su & ok);  // violations for certain
                cl += __popcll(sl & ok);
                au[c][r] = ok & ~su & ~nu;  // ambiguous
                al[c][r] = ok & ~sl & ~nl;
                eu[c][r] = au[c][r] | (okm & __builtin_amdgcn_ballot_w64(!(tu > umin[r])));
                el[c][r] = al[c][r] | (okm & __builtin_amdgcn_ballot_w64(!(tl > lmin[r])));
                any |= eu[c][r] | el[c][r];
            }
        }
        if (any == 0) return;
#pragma unroll
        for (int c = 0; c < G; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if ((eu[c][r] | el[c][r]) == 0) continue;  // wave-uniform
                const unsigned long long bit = 1ull << lane;
                if (!((eu[c][r] | el[c][r]) & bit)) continue;
                const int64_t k = g + c;
                // the FP64 row values are the FP32 inputs widened (exact),
                // formed here instead of being held for the whole scan
                double xd[D];
#pragma unroll
                for (int j = 0; j < D; ++j) xd[j] = (double)xr[r][j];
                // the column's FP64 values are its FP32 record widened
                // (both stagings hold the same FP32 numbers: the sign-flipped
                // coordinates, y_k and M_k), so they come from the scalar
                // registers of the group instead of a load of the FP64 copy
                const float *xc = v + c * S;
                double tu, tl;
                cons_pair_col<D, NORM, HASW, MON>(
                    A, xd, (double)yr[r], [&](int j) { return (double)xc[j]; }, tu, tl);
                if ((au[c][r] & bit) && tu < -A.tol) ++xu;
                if ((al[c][r] & bit) && tl < -A.tol) ++xl;
                if ((eu[c][r] & bit) && tu < bu[r]) {
                    bu[r] = tu;
                    pu[r] = (int)k;
                    umin[r] = f32_up(tu + E);
                }
                if ((el[c][r] & bit) && tl < bl[r]) {
                    bl[r] = tl;
                    pl[r] = (int)k;
                    lmin[r] = f32_up(tl + E);
                }
            }
    };
    auto load = [&](int64_t g, float (&v)[G * S]) {
#pragma unroll
        for (int e = 0; e < G * S; ++e) v[e] = C[g * S + e];
    };
    // Groups that overlap the end of the data or this wave's own rows check
    // bounds and the diagonal per pair.
    // (column indices fit in 32 bits: n < 2^31; 32-bit compares stay on the
    // scalar unit)
    const int32_t n32 = (int32_t)A.n, r0 = (int32_t)w.r0, r1 = (int32_t)w.r1;
    auto masked = [&](int64_t g) {
        const int32_t g32 = (int32_t)g;
        return g32 > n32 - G || (g32 < r1 && g32 > r0 - G);
    };
    float va[G * S], vb[G * S];
    int64_t g = w.c0;
    if (g < w.c1) load(g, va);
#pragma unroll 1
    for (; g + G < w.c1; g += 2 * G) {
        load(g + G, vb);
        if (masked(g)) visit(g, va, std::true_type{});
        else visit(g, va, std::false_type{});
        if (g + 2 * G < w.c1) load(g + 2 * G, va);
        if (masked(g + G)) visit(g + G, vb, std::true_type{});
        else visit(g + G, vb, std::false_type{});
    }
    if (g < w.c1) {
        if (masked(g)) visit(g, va, std::true_type{});
        else visit(g, va, std::false_type{});
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!valid[r]) continue;
        const int64_t i = ir[r];
        if (A.n_chunks == 1) {
            if (A.slack_up) A.slack_up[i] = bu[r];
            if (A.slack_lo) A.slack_lo[i] = bl[r];
            if (A.partner_up) A.partner_up[i] = pu[r];
            if (A.partner_lo) A.partner_lo[i] = pl[r];
        } else {
            const int64_t o = (int64_t)w.chunk * A.n + i;
            A.pv_up[o] = bu[r];
            A.pv_lo[o] = bl[r];
            A.pi_up[o] = pu[r];
            A.pi_lo[o] = pl[r];
        }
    }
    unsigned long long tu = xu, tl = xl;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        tu += __shfl_xor(tu, off);
        tl += __shfl_xor(tl, off);
    }
    if (lane == 0) {
        atomicAdd(A.counts, cu + tu);
        atomicAdd(A.counts + 1, cl + tl);
    }
}

// ---- launcher tables ------------------------------------------------------------

typedef void (*DsLaunch)(const DsArgs &, dim3, dim3, hipStream_t);

struct DsLaunchers {
    DsLaunch consistency, consistency_mon, slope, scan, select16, select32, tau16, tau32;
    // slacks and partners after the FP64 consistency kernel (l1, linf)
    DsLaunch cons_finish, cons_finish_mon;
};

// Dimensions up to which the consistency pass has one kernel per free /
// monotone pattern of the coordinates.
constexpr int kDsMaskDims = 4;

typedef void (*DsKernel)(DsArgs);

// Per-pattern kernels of the consistency pass: the FP32-filtered kernel for
// l2 (where FP32 saves the two FP64 square roots of every pair), the FP64
// kernel for l1 and linf (where the filter's bookkeeping costs about what it
// saves).
template <int D, int NORM, bool HASW, int... FMs>
constexpr std::array<DsKernel, sizeof...(FMs)> cons_mask_table(std::integer_sequence<int, FMs...>)
{
    if constexpr (NORM == 2)
        return {{&consistency32_kernel<D, NORM, HASW, true, FMs>...}};
    else
        return {{&consistency_kernel<D, NORM, HASW, true, FMs>...}};
}

template <int D, int NORM, bool HASW>
DsLaunchers ds_launchers_for()
{
    DsLaunchers L;
    L.consistency = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        if constexpr (NORM == 2)
            hipLaunchKernelGGL((consistency32_kernel<D, NORM, HASW, false>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((consistency_kernel<D, NORM, HASW, false>), g, b, 0, s, a);
    };
    L.consistency_mon = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        if constexpr (D <= kDsMaskDims) {
            // every free / monotone pattern of a low dimension has its own kernel
            constexpr auto tbl = cons_mask_table<D, NORM, HASW>(std::make_integer_sequence<int, (1 << D)>{});
            if (a.fmask >= 0 && a.fmask < (1 << D)) {
                hipLaunchKernelGGL(tbl[a.fmask], g, b, 0, s, a);
                return;
            }
        }
        if constexpr (NORM == 2)
            hipLaunchKernelGGL((consistency32_kernel<D, NORM, HASW, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((consistency_kernel<D, NORM, HASW, true>), g, b, 0, s, a);
    };
    if constexpr (NORM == 2) {
        L.cons_finish = L.cons_finish_mon = nullptr;
    } else {
        L.cons_finish = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
            hipLaunchKernelGGL((consistency_finish_kernel<D, NORM, HASW, false>), g, b, 0, s, a);
        };
        L.cons_finish_mon = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
            hipLaunchKernelGGL((consistency_finish_kernel<D, NORM, HASW, true>), g, b, 0, s, a);
        };
    }
    L.slope = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((slope_kernel<D, NORM, HASW>), g, b, 0, s, a);
    };
    L.scan = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_scan_kernel<D, NORM, HASW>), g, b, 0, s, a);
    };
    L.select16 = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_select_kernel<D, NORM, HASW, 16>), g, b, 0, s, a);
    };
    L.select32 = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_select_kernel<D, NORM, HASW, 32>), g, b, 0, s, a);
    };
    L.tau16 = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_tau_kernel<D, NORM, HASW, 16>), g, b, 0, s, a);
    };
    L.tau32 = [](const DsArgs &a, dim3 g, dim3 b, hipStream_t s) {
        hipLaunchKernelGGL((knn_tau_kernel<D, NORM, HASW, 32>), g, b, 0, s, a);
    };
    return L;
}

template <int NORM>
bool ds_table(int d, bool hasw, DsLaunchers *L)
{
    switch (d) {
#define LIP_DS_CASE(DD)                                                                         \
    case DD:                                                                                    \
        *L = hasw ? ds_launchers_for<DD, NORM, true>() : ds_launchers_for<DD, NORM, false>(); \
        return true;
        LIP_DS_CASE(1) LIP_DS_CASE(2) LIP_DS_CASE(3) LIP_DS_CASE(4)
        LIP_DS_CASE(5) LIP_DS_CASE(6) LIP_DS_CASE(7) LIP_DS_CASE(8)
        LIP_DS_CASE(9) LIP_DS_CASE(10) LIP_DS_CASE(11) LIP_DS_CASE(12)
        LIP_DS_CASE(13) LIP_DS_CASE(14) LIP_DS_CASE(15) LIP_DS_CASE(16)
#undef LIP_DS_CASE
    default: return false;
    }
}

// Host helpers of data_side.hip shared with the step-function passes.
// Per-coordinate signs of the FP64 staging (-1 for a decreasing coordinate).
struct Signs {
    float s[kMaxDim];
};
hipError_t launch_stage64(int d, const float *x, const float *y, const float *Mk, float M,
                          int64_t n, int64_t npad, const Signs &sg, double *X, hipStream_t s);
int64_t ds_npad(int64_t n);
bool fill_ds_metric(const MetricInfo &mi, bool use_mon, DsArgs *A, Signs *sg);
void choose_chunks(int64_t n, int rows_per_wave, int max_chunks, DsArgs *A,
                   int64_t target_waves = kDsTargetWaves);
// Column chunks of the consistency passes: finer than the other passes' so
// that the grid holds ~6 waves per SIMD slot and the last round is short.
constexpr int kConsMaxChunks = 32;
static_assert(kConsMaxChunks <= kFinishChunks, "the finish pass reads every chunk");
constexpr int64_t kConsTargetWaves = 24576;
int cons_chunks(int64_t n, int d, int norm);
unsigned grid_for_rows(int64_t n, int rows_per_wave, int n_chunks);

bool ds_table_l1(int d, bool hasw, DsLaunchers *L);
bool ds_table_l2(int d, bool hasw, DsLaunchers *L);
bool ds_table_linf(int d, bool hasw, DsLaunchers *L);

}  // namespace lip
