/*
 * lipfit.h - C ABI of the MI355X (gfx950) library for Lipschitz-optimal
 * scattered-data fitting: the all-pairs bound evaluation and its data-side
 * passes.
 *
 * Problem (paper, Sec. 1 and 3): data x^k in R^d with values y^k,
 * k = 0..n-1, a Lipschitz constant M (or one constant M_k per datum,
 * Sec. 4.3), a distance dist, optional monotonicity per coordinate
 * (Sec. 4.1), and query points x.  For every query
 *     H_up(x) = min_k ( y^k + M_k dist_up(x, x^k) )          Eq. (2)
 *     H_lo(x) = max_k ( y^k - M_k dist_lo(x, x^k) )          Eq. (2)
 *     g(x)    = ( H_up(x) + H_lo(x) ) / 2                    Eq. (3)
 * The distance is the weighted l1, l2 or linf norm of the per-coordinate
 * component vector c: for an unconstrained coordinate c_i = |x_i - x^k_i|
 * in both bounds; for an increasing coordinate the upper bound uses
 * (x_i - x^k_i)_+ (Eq. 4) and the lower bound its mirror (x^k_i - x_i)_+;
 * a decreasing coordinate swaps the two.  dist = || w (.) c ||_p.
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer owned by the caller, except
 *    the lip_metric fields w and mon, which are HOST arrays of length d.
 *  - Matrices are row-major: x is [n][d], xq is [q][d], dxq is [q][d].
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Argument validation is synchronous and happens before any
 *    device work: on an error status nothing has been enqueued and no HIP
 *    call has been made.  LIP_E_DEVICE reports a failed launch.
 *  - Output pointers documented as optional may be NULL to skip them.
 *  - Indices are int32 (n < 2^31).  Ties in a min / max go to the lowest
 *    index.  n == 0 is LIP_E_SHAPE; q == 0 is a successful no-op.
 *  - Scratch memory comes from the caller's workspace `ws` of `ws_bytes`
 *    bytes (at least lip_workspace_size(...)); no entry point allocates
 *    device memory, except lip_plan_create and lip_autotune.
 *  - NaN inputs give unspecified results unless LIP_FLAG_CHECK_FINITE is set,
 *    which scans the inputs first (synchronously) and returns
 *    LIP_E_NONFINITE.
 */
#ifndef LIPFIT_H
#define LIPFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LIP_OK = 0,
    LIP_E_ARG = 1,          /* NULL where required, bad enum, bad flag combination */
    LIP_E_SHAPE = 2,        /* n == 0, d outside 1..LIP_MAX_DIM, sizes too large */
    LIP_E_VALUE = 3,        /* M < 0, weight <= 0, unknown mon kind, a_i > b_i, tol < 0 */
    LIP_E_NONFINITE = 4,    /* NaN/Inf found by LIP_FLAG_CHECK_FINITE */
    LIP_E_UNSUPPORTED = 5,  /* e.g. LIP_FLAG_BF16 with l1/linf or monotone coordinates */
    LIP_E_WORKSPACE = 6,    /* ws is NULL or smaller than lip_workspace_size() */
    LIP_E_DEVICE = 7        /* a HIP call or kernel launch failed */
} lip_status;

typedef enum { LIP_L1 = 1, LIP_L2 = 2, LIP_LINF = 3 } lip_norm;

#define LIP_MAX_DIM 16
#define LIP_MAX_KNN 32

/* Flags (bitwise or). */
#define LIP_FLAG_CHECK_FINITE  (1u << 0)
/* l2 without monotone coordinates only: the cross term x . x^k in BF16 MFMA
 * with FP32 accumulation, then every candidate within the proven error bound
 * re-evaluated with the FP32 path's arithmetic, so the results (values and
 * indices) are identical to the FP32 path. */
#define LIP_FLAG_BF16          (1u << 1)
/* Backward: accumulate dy / dM without floating-point atomics, so repeated
 * calls give bitwise identical results. */
#define LIP_FLAG_DETERMINISTIC (1u << 2)

/* Monotonicity on parts of the domain (Sec. 4.2): with A: x_i <= a_i,
 * AB: a_i <= x_i <= b_i, B: x_i >= b_i, a coordinate of kind
 *   LIP_MON_CASE_I    is increasing on A and B, unrestricted on AB,
 *   LIP_MON_CASE_II   is decreasing on A and B, unrestricted on AB,
 *   LIP_MON_CASE_III  is decreasing on A, increasing on B, unrestricted on AB,
 *   LIP_MON_CASE_IV   is increasing on A, decreasing on B, unrestricted on AB.
 * Its distance components are the lengths of the part of the segment between
 * x^k_i and x_i on which f may rise (upper distance) or fall (lower distance)
 * in the direction of travel: moving towards larger x_i it may rise where it
 * is not decreasing and fall where it is not increasing, and the reverse
 * moving towards smaller x_i.  (Kinds +1 / -1 are the same rule with one
 * region covering everything: Eq. 4 and its mirror.)  Only lip_bounds and
 * lip_fit_eval accept these kinds; the other entry points return
 * LIP_E_UNSUPPORTED for them. */
#define LIP_MON_CASE_I   2
#define LIP_MON_CASE_II  3
#define LIP_MON_CASE_III 4
#define LIP_MON_CASE_IV  5

/* Distance definition (Sec. 3 "other distances", Sec. 4.1 monotonicity,
 * Sec. 4.2 monotonicity on parts of the domain). */
typedef struct {
    int32_t d;            /* dimension, 1..LIP_MAX_DIM */
    int32_t norm;         /* lip_norm */
    const float *w;       /* HOST [d] weights > 0, or NULL for all ones */
    const int8_t *mon;    /* HOST [d] in {-1, 0, +1} or LIP_MON_CASE_I..IV, or NULL for no
                             constraints */
    const float *a;       /* HOST [d] interval starts a_i (finite, used by the CASE kinds), or
                             NULL when no coordinate has such a kind */
    const float *b;       /* HOST [d] interval ends b_i >= a_i (finite), or NULL likewise */
} lip_metric;

typedef void *lip_stream; /* hipStream_t */

/* Bytes of workspace that the entry points taking `ws` need for these sizes
 * and flags (an upper bound; 0 is never returned). */
size_t lip_workspace_size(int64_t n, int64_t q, int32_t d, uint32_t flags);

/* Eq. (2): the upper and lower Lipschitz bounds at q query points and the
 * data points that attain them.
 *   x [n][d], y [n]       data set D (Sec. 1)
 *   M                     global Lipschitz constant (>= 0, finite); ignored
 *                         when Mk != NULL
 *   Mk [n] or NULL        per-datum constants (Sec. 4.3, scalar per datum);
 *                         each pair uses the datum's own M_k
 *   xq [q][d]             query points
 *   h_up, h_lo [q]        optional outputs (FP32)
 *   arg_up, arg_lo [q]    optional outputs: attaining data index, lowest on ties
 * Arithmetic is FP32 (FP32 with a BF16 cross term under LIP_FLAG_BF16, with
 * identical results).  The forward is bitwise deterministic. */
lip_status lip_bounds(const lip_metric *metric, const float *x, const float *y, int64_t n,
                      float M, const float *Mk, const float *xq, int64_t q,
                      float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo,
                      void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

/* Eq. (3): the optimal interpolant g = (H_up + H_lo)/2 at the queries, plus
 * the optional bound outputs of lip_bounds (all of g, h_up, h_lo, arg_up,
 * arg_lo are optional).  Same arguments and rules as lip_bounds. */
lip_status lip_fit_eval(const lip_metric *metric, const float *x, const float *y, int64_t n,
                        float M, const float *Mk, const float *xq, int64_t q,
                        float *g, float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo,
                        void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

/* lip_fit_eval for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments without ws / ws_bytes, the same results
 * bit for bit.  Scratch memory is a 64 MiB device array of the library (one
 * per GPU, held until the process ends); nothing is allocated per call.
 * Limits: the staged data, (n + 256) (d + 3) 4 bytes plus about 31 KiB,
 * must fit in 64 MiB (n up to about 2.39e6 at d = 4, 0.88e6 at d = 16),
 * else LIP_E_SHAPE; the data split is reduced until its partial results fit
 * too.  flags must be 0 and the LIP_MON_CASE kinds are not accepted
 * (LIP_E_UNSUPPORTED).  Calls that overlap on one GPU (different streams or
 * threads without ordering) share the array and race; calls on one stream
 * are safe. */
lip_status lip_fit_eval_noalloc(const lip_metric *metric, const float *x, const float *y,
                                int64_t n, float M, const float *Mk, const float *xq, int64_t q,
                                float *g, float *h_up, float *h_lo, int32_t *arg_up,
                                int32_t *arg_lo, uint32_t flags, lip_stream stream);

/* Subgradients of g (and of H_up, H_lo) through the indices a = arg_up[j],
 * b = arg_lo[j] saved by the forward (the chain rule applied to Eq. 2-3):
 *   G_up = dg/2 + dh_up,  G_lo = dg/2 + dh_lo    (missing arrays count 0)
 *   dxq[j]  = G_up M_a grad_x dist_up(x, x^a) - G_lo M_b grad_x dist_lo(x, x^b)
 *   dy[a]  += G_up,  dy[b] += G_lo
 *   dM[0]  += G_up dist_up - G_lo dist_lo              (global M, Mk == NULL)
 *   dM[a]  += G_up dist_up,  dM[b] -= G_lo dist_lo     (per-datum M_k)
 * Kinks take the zero subgradient: |.|'(0) = 0, (.)_+'(0) = 0, grad l2 at
 * distance 0 = 0; linf picks the lowest coordinate among the largest.
 *   dg, dh_up, dh_lo [q]  upstream gradients, any may be NULL
 *   dxq [q][d]            optional, overwritten
 *   dy [n]                optional, ACCUMULATED (the caller zeroes it)
 *   dM [1] or [n]         optional, ACCUMULATED
 * Uses FP32 atomics for dy / dM unless LIP_FLAG_DETERMINISTIC, which takes
 * ws (>= lip_workspace_size) and gives bitwise reproducible sums.
 * LIP_FLAG_CHECK_FINITE (needs ws too) scans x, Mk, xq and the upstream
 * gradients first. */
lip_status lip_fit_backward(const lip_metric *metric, const float *x, const float *y, int64_t n,
                            float M, const float *Mk, const float *xq, int64_t q,
                            const int32_t *arg_up, const int32_t *arg_lo,
                            const float *dg, const float *dh_up, const float *dh_lo,
                            float *dxq, float *dy, float *dM,
                            void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

/* Data-side consistency check in FP64: can the data be interpolated by a
 * function that satisfies the Lipschitz condition (Sec. 1) and the
 * monotonicity constraints (Sec. 4.1)?  Pairwise form of Eqs. (5)-(6) with
 * zero corrections; for each row i and every k != i:
 *   t_up(i,k) = (y_k + M_k dist_up(x^i, x^k)) - y_i
 *   t_lo(i,k) = y_i - (y_k - M_k dist_lo(x^i, x^k))
 * all evaluated in double precision from the FP32 inputs, in this order,
 * coordinates accumulated in index order, the bound y_k +- M_k dist as one
 * fused multiply-add, correctly rounded operations (an l-infinity distance,
 * a maximum, is exact in any order).
 *   counts [2] (int64, required)  number of ordered pairs with t_up < -tol
 *                                 and with t_lo < -tol (overwritten)
 *   worst_slack [1] (FP64), worst_pair [2] (int64), optional: the smallest
 *                                 t_up or t_lo over all ordered pairs and the
 *                                 pair (i, k) attaining it, lowest i then
 *                                 lowest k on ties (+inf and (-1, -1) if
 *                                 n == 1); the data are consistent with
 *                                 tolerance tol iff worst_slack >= -tol
 *   slack_up, slack_lo [n]        optional: min_k t_up, min_k t_lo (+inf if n == 1)
 *   partner_up, partner_lo [n]    optional: the k attaining them (lowest on ties)
 * Equality (|y_i - y_k| = M dist) is consistent.  Needs ws. */
lip_status lip_consistency(const lip_metric *metric, const float *x, const float *y, int64_t n,
                           float M, const float *Mk, double tol, int64_t *counts,
                           double *worst_slack, int64_t *worst_pair,
                           double *slack_up, double *slack_lo,
                           int32_t *partner_up, int32_t *partner_lo,
                           void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

#define LIP_M_GLOBAL 0
#define LIP_M_LOCAL_KNN 1

/* Lipschitz constants estimated from the data, with the symmetric distance
 * (monotonicity in metric->mon is ignored), in FP64 from the FP32 inputs.
 * LIP_M_GLOBAL (Sec. 5, the max of |y_i - y_k| / dist(x^i, x^k) over all
 * pairs; no distance matrix is stored):
 *   M64 [1] optional, M32 [1] optional (M64 rounded up to FP32, so that the
 *   data stay consistent with it), pair [2] optional (int64, lowest (i, k)
 *   with i < k among ties).
 * LIP_M_LOCAL_KNN (Sec. 4.3, scalar per datum): for each i, the knn nearest
 *   j != i (ranked by dist, l2 by the sum of squares; ties rank the lower j
 *   first), M_i = max over them of |y_i - y_j| / dist:
 *   M64 [n] optional, M32 [n] optional (rounded up), pair unused.
 * Coincident points with equal y are skipped; coincident points with
 * different y make the slope infinite: the result is +inf (and, for
 * LIP_M_GLOBAL, pair names the lowest such pair).  The call is asynchronous,
 * so it reports an infinite estimate through the outputs; with
 * LIP_FLAG_CHECK_FINITE it also synchronises at the end and returns
 * LIP_E_VALUE when an estimate written to M64 or M32 is infinite (the
 * outputs are written either way).  knn in 1..LIP_MAX_KNN.  Needs ws. */
lip_status lip_estimate_M(const lip_metric *metric, const float *x, const float *y, int64_t n,
                          int32_t mode, int32_t knn, double *M64, float *M32, int64_t *pair,
                          void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

/* ---- k best bounds with weights (Sec. 5, k > 1) ------------------------------
 * Both bounds from the k best candidates of Eq. (2): with the upper
 * candidates sorted ascending u_(1) <= u_(2) <= .. and the lower ones
 * descending l_[1] >= l_[2] >= ..,
 *     h_up = sum_j wk[j] u_(j+1),   h_lo = sum_j wk[j] l_[j+1],   g = (h_up + h_lo) / 2.
 * The paper's weights add to 1 (not enforced); the result does not
 * interpolate the data for k > 1.
 *   k          1..LIP_MAX_K, and k <= n
 *   wk [k]     HOST weights >= 0 (finite)
 *   g, h_up, h_lo [q]   optional outputs (FP32)
 * Other arguments and rules as in lip_fit_eval (LIP_FLAG_BF16 unsupported).
 * Candidates are FP32 as in lip_fit_eval (k = 1 with wk = {1} gives its
 * h_up / h_lo bit for bit); the k values are a multiset, so no index rule.
 * Needs ws. */
#define LIP_MAX_K 32
lip_status lip_fit_eval_k(const lip_metric *metric, const float *x, const float *y, int64_t n,
                          float M, const float *Mk, int32_t k, const float *wk, const float *xq,
                          int64_t q, float *g, float *h_up, float *h_lo, void *ws,
                          size_t ws_bytes, uint32_t flags, lip_stream stream);

/* ---- step-function local constants (Sec. 4.3) ----------------------------
 * Each datum k gets a non-decreasing, piecewise constant M_k(t) of the
 * distance t, built from the data:
 *   knots     q_1 <= ... <= q_K (K <= LIP_MAX_KNOTS), shared by all data:
 *             quantiles of the inter-point distance distribution, estimated
 *             from a sample of pairs (lip_local_knots);
 *   d1_k      the distance from x^k to its nearest other datum;
 *   M_k(t)  = V_k,0   for t <= d1_k  (largest slope among the data at
 *                                      distance <= d1_k),
 *           = V_k,s   for the first s with t <= q_s (largest slope among the
 *                                      data at distance <= max(q_s, d1_k)),
 *           = V_k,K+1 for t > q_K     (largest slope over all data),
 * where a slope is |y_k - y_j| / dist(x^k, x^j) with the symmetric distance
 * (monotonicity ignored) and an empty set gives 0.  The bounds of Eq. (2)
 * then use u_k = y_k + M_k(dist_up) dist_up, l_k = y_k - M_k(dist_lo) dist_lo.
 * With the symmetric distance the result interpolates the data. */
#define LIP_MAX_KNOTS 8

/* Knots as quantiles of sampled inter-point distances, in FP64 from the
 * FP32 inputs (symmetric distance, coordinates accumulated in index order).
 *   pairs [m][2]   HOST int64 indices into x (the random sample is the
 *                  caller's; i == j is allowed and gives distance 0)
 *   probs [K]      HOST probabilities in (0, 1], non-decreasing
 *   knots [K]      DEVICE FP64 output: with the sampled distances sorted
 *                  ascending as r_0..r_{m-1}, knots[j] = r_c,
 *                  c = ceil(probs[j] * m) - 1 clamped to [0, m - 1]
 *                  (the inverse empirical distribution function).
 * 1 <= m <= 2^26.  Needs ws of lip_workspace_size(m, 0, d, 0) bytes; copies
 * pairs into it (a host-to-device copy on `stream`). */
lip_status lip_local_knots(const lip_metric *metric, const float *x, int64_t n,
                           const int64_t *pairs, int64_t m, const double *probs, int32_t K,
                           double *knots, void *ws, size_t ws_bytes, uint32_t flags,
                           lip_stream stream);

/* Per-datum step tables of M_k(t) in FP64 (all pairs, no distance matrix).
 *   knots [K]          HOST, non-decreasing, >= 0 (K = 0 allowed)
 *   d1 [n]             DEVICE FP64 output (required): nearest positive
 *                      distance, +inf when there is none
 *   V64 [n][K+2]       DEVICE FP64 output, optional: V_k,0 .. V_k,K+1
 *   V32 [n][K+2]       DEVICE FP32 output, optional: V64 rounded up (the
 *                      values lip_fit_eval_steps multiplies, so the data
 *                      stay interpolated)
 * Coincident data with equal values are skipped; with different values the
 * slope is infinite and the datum's whole row is +inf (such a table is not a
 * valid input of lip_fit_eval_steps).  Needs ws. */
lip_status lip_local_steps(const lip_metric *metric, const float *x, const float *y, int64_t n,
                           const double *knots, int32_t K, double *d1, double *V64, float *V32,
                           void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

/* The step tables as inputs of the bound evaluation. */
typedef struct {
    int32_t K;            /* number of knots, 0..LIP_MAX_KNOTS */
    const double *knots;  /* HOST [K], non-decreasing, >= 0 */
    const double *d1;     /* DEVICE [n], from lip_local_steps */
    const float *V;       /* DEVICE [n][K+2], finite, >= 0 */
} lip_steps;

/* Eq. (2)-(3) with M_k(dist) of the step tables in place of M.  Outputs and
 * rules as in lip_fit_eval (all optional, lowest index on ties).  Distances
 * are formed in FP64 (index order, as in the consistency check), so the
 * segment of every pair is decided exactly as by the definition; the bound
 * candidates are FP32: y_k + M fl32(dist) (l2: the FP32 root of the FP32
 * sum of squares).  LIP_FLAG_BF16 is not supported here. */
lip_status lip_fit_eval_steps(const lip_metric *metric, const float *x, const float *y, int64_t n,
                              const lip_steps *steps, const float *xq, int64_t q, float *g,
                              float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo,
                              void *ws, size_t ws_bytes, uint32_t flags, lip_stream stream);

/* ---- smoothing (Sec. 4.4) -------------------------------------------------
 * Penalty form of the smoothing problem, Eq. (7): with corrections eps and
 * z = y + eps, for every ordered pair i != k
 *     a_ik = z_i - z_k - M_k dist_up(x^i, x^k)     (Eq. 5 as a penalty)
 *     b_ik = z_k - z_i - M_k dist_lo(x^i, x^k)     (Eq. 6 as a penalty)
 *     F(eps) = (1/p) ||eps||^2 + sum_{i != k} (a_ik)_+^2 + (b_ik)_+^2
 * (M_k = M when Mk is NULL; directional distances on monotone coordinates as
 * in lip_consistency).  One fused pass over all pairs, no distance matrix.
 *   eps [n]      DEVICE FP32 corrections
 *   p            penalty parameter > 0 (finite)
 *   prune        pre-screening of Sec. 5: 0 keeps every pair; c > 0 drops the
 *                ordered pair (i, k) from both sums when, on the given y,
 *                y_i - y_k <= c M_k dist_up(x^i, x^k) and
 *                y_k - y_i <= c M_k dist_lo(x^i, x^k)  (the paper uses c = 1/3).
 *                Decided as in FP64 with the consistency check's distances
 *                and (c M_k) dist, so the dropped set is exact.  Negative or
 *                non-finite: LIP_E_VALUE.
 *   F [1]        DEVICE FP64 output, optional: the objective
 *   grad [n]     DEVICE FP32 output, optional: dF / d eps
 * Pair terms are FP32, sums FP64 in a fixed order (repeated calls give
 * identical results).  Meant to be called by an unconstrained minimiser
 * (L-BFGS); y + eps is then the smoothed data.  Needs ws. */
lip_status lip_smooth_objective(const lip_metric *metric, const float *x, const float *y,
                                int64_t n, float M, const float *Mk, const float *eps, double p,
                                double prune, double *F, float *grad, void *ws, size_t ws_bytes,
                                uint32_t flags, lip_stream stream);

/* ---- many independent fits in one launch ------------------------------------
 * One entry per data set: its own metric, data, constants, queries and
 * outputs (all device pointers except metric.w / metric.mon).  Outputs as in
 * lip_fit_eval; the results are identical to calling lip_fit_eval on each
 * set. */
typedef struct {
    lip_metric metric;
    const float *x;
    const float *y;
    int64_t n;
    float M;
    const float *Mk;
    const float *xq;
    int64_t q;
    float *g;
    float *h_up;
    float *h_lo;
    int32_t *arg_up;
    int32_t *arg_lo;
} lip_batch_desc;

typedef struct lip_plan lip_plan;

/* Builds a plan: copies the descriptors, allocates the plan's own device
 * memory (staged data, work list, counters), picks tile parameters from the
 * tuning table, orders the work longest-first and records one HIP graph that
 * runs every set.  The metric host arrays are copied; the device arrays
 * must stay valid while the plan is executed. */
lip_status lip_plan_create(lip_plan **plan, const lip_batch_desc *sets, int32_t n_sets,
                           uint32_t flags, lip_stream stream);
/* Launches the plan's graph on `stream` (asynchronous). */
lip_status lip_plan_execute(lip_plan *plan, lip_stream stream);
/* Releases the plan (synchronises with its last execution first). */
lip_status lip_plan_destroy(lip_plan *plan);

/* ---- tile parameters --------------------------------------------------------
 * Runtime choices of the bound kernels (lip_bounds, lip_fit_eval and the
 * sets of a plan) for a shape class (d, number of monotone coordinates,
 * norm) and a size class of (n, q): sizes within a factor of 4 of each other
 * (floor(log2 v) / 2 equal for n and for q) share an entry.  Results do not
 * depend on these choices, only the time does. */
typedef struct {
    int32_t tile;         /* data points per argmin tile (multiple of 8, 8..256) */
    int32_t split;        /* number of data chunks (1..64; 1 = no split) */
    int32_t waves;        /* waves per workgroup (1..8).  At d <= 8 the waves of a
                           * workgroup take the same queries and consecutive
                           * chunks and merge their results in LDS, so that
                           * only split / waves partial results per query go
                           * through HBM; at d >= 9 they take different
                           * queries and at most 4 are used (lip_bounds,
                           * lip_fit_eval; plans run one wave per work item) */
    int32_t flags;        /* LIP_TILE_* bits */
} lip_tile_cfg;

/* l2 with monotone coordinates: give every pair root-free bounds of its
 * candidates first (from the largest weighted component of each distance)
 * and form the exact candidates (two square roots) only for the rows of 64
 * queries where some query could improve.  Identical results; faster when
 * few data compete for each query (default on).  Without monotone
 * coordinates the flag is accepted and has no effect. */
#define LIP_TILE_L2_FILTER 1
/* Visit the queries in Morton order (a sort of the queries' codes per call,
 * in the workspace): a wave's queries are then close to each other, so the
 * l2 filter's decisions, taken for 64 queries at a time, are coherent.
 * Identical results (lip_bounds, lip_fit_eval; ignored by plans and by
 * lip_fit_eval_noalloc; default on with the filter for q >= 65536). */
#define LIP_TILE_QUERY_ORDER 2

/* The configuration the next call of these sizes will use: the table's
 * entry for the size class of (n, q), else the entry set for every size,
 * else the built-in default.  The first lookup loads the file named by the
 * environment variable LIPFIT_TUNE_CACHE, if it is set (see lip_tune_load). */
lip_status lip_tune_get(int32_t d, int32_t n_mon, int32_t norm, int64_t n, int64_t q,
                        lip_tile_cfg *cfg);
/* Stores cfg for the size class of (n, q), or for every size when n == 0 and
 * q == 0 (one of them 0 alone is LIP_E_SHAPE); cfg == NULL removes that
 * entry.  Invalid values: LIP_E_VALUE. */
lip_status lip_tune_set(int32_t d, int32_t n_mon, int32_t norm, int64_t n, int64_t q,
                        const lip_tile_cfg *cfg);
/* Times every candidate (tile 16/32/64/128 x split 1..32 x 1, 2, 4 or 8
 * waves up to the split, and for l2 with monotone coordinates without
 * flags, with LIP_TILE_L2_FILTER and with it and LIP_TILE_QUERY_ORDER) for
 * this shape class on synthetic data of the given sizes (allocates and frees
 * its own device memory, blocks), stores the fastest under the size class of
 * (n, q) and returns it; with LIPFIT_TUNE_CACHE set, the whole table is then
 * written to that file. */
lip_status lip_autotune(int32_t d, int32_t n_mon, int32_t norm, int64_t n, int64_t q,
                        lip_stream stream, lip_tile_cfg *best);
/* The table as a JSON file: {"format": "lipfit-tune-1", "entries": [{"arch":
 * "gfx950", "d", "n_mon", "norm", "n_class", "q_class", "tile", "split",
 * "waves", "flags"}, ...]} (class -1: every size; "flags" may be absent: 0).  Save writes every entry under the
 * architecture name `arch`; load adds the entries of architecture `arch`
 * (others are skipped) and changes nothing if the file does not parse
 * (LIP_E_VALUE).  arch == NULL means the current device's ("" without a
 * device: LIP_E_DEVICE).  An unreadable / unwritable path is LIP_E_ARG. */
lip_status lip_tune_save(const char *path, const char *arch);
lip_status lip_tune_load(const char *path, const char *arch);
/* Removes every entry. */
lip_status lip_tune_clear(void);

/* The tile parameters set number `set` of a plan (0-based, in the order
 * given to lip_plan_create) runs with: cfg->tile the argmin tile from the
 * tuning table at plan creation, cfg->split its number of data chunks,
 * cfg->waves the waves per workgroup. */
lip_status lip_plan_tiles(const lip_plan *plan, int32_t set, lip_tile_cfg *cfg);

const char *lip_status_string(lip_status status);

#ifdef __cplusplus
}
#endif

#endif /* LIPFIT_H */
