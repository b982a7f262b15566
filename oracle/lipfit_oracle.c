/*
 * Plain FP64 CPU oracle for the all-pairs Lipschitz bound evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or constant with the GPU library: it is written straight from the paper's
 * definitions, in double precision, with no blocking, tiling or pruning.
 * Inputs are the same float32 arrays the GPU reads, widened to double.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 *
 * Notation (paper, Sec. 1 and 3): data x^k in R^d, values y^k, k = 0..n-1
 * (0-based here), query point x, Lipschitz constant M (global) or M_k
 * (per datum, Sec. 4.3 applied with a scalar per datum), distance dist.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes):
 *  - Eq. (4) gives one directional distance ||(x - x^k)_+||.  It is used for
 *    the upper bound; the lower bound uses ||(x^k - x)_+||, the mirror image
 *    (f(x) <= f(max(x, x^k)) <= y^k + M||(x - x^k)_+|| and
 *    f(x) >= f(min(x, x^k)) >= y^k - M||(x^k - x)_+|| for increasing f).
 *  - Monotone-decreasing coordinates swap the two.  Unconstrained
 *    coordinates contribute |x_i - x^k_i| to both.  The norm is taken of the
 *    whole per-coordinate component vector, weighted: ||w (.) c||_p,
 *    p in {1, 2, inf}.
 *  - Ties in min/max go to the lowest index k (strict < and > scans from 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_L1 = 1, ORC_L2 = 2, ORC_LINF = 3 };

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Per-coordinate components of the directional distances between the point a
 * (the one being evaluated) and the datum b: delta = a_i - b_i.
 *   mon_i =  0: c_up = c_lo = |delta|
 *   mon_i = +1: c_up = (delta)_+,  c_lo = (-delta)_+      (Eq. 4 and mirror)
 *   mon_i = -1: c_up = (-delta)_+, c_lo = (delta)_+
 * mon == NULL means all coordinates unconstrained. */
static void components(int i, double delta, const signed char *mon, double *cu, double *cl)
{
    int m = mon ? mon[i] : 0;
    if (m == 0) {
        *cu = fabs(delta);
        *cl = *cu;
    } else if (m > 0) {
        *cu = delta > 0.0 ? delta : 0.0;
        *cl = delta < 0.0 ? -delta : 0.0;
    } else {
        *cu = delta < 0.0 ? -delta : 0.0;
        *cl = delta > 0.0 ? delta : 0.0;
    }
}

/* dist(a, b) for the upper and the lower bound (Eq. 2 with Eq. 4).  For l2,
 * *su_sq / *sl_sq (if not NULL) receive the sums of squares before the root.
 * Coordinates are accumulated in index order starting from 0.0. */
static void dist_pair(int d, int norm, const double *w, const signed char *mon,
                      const float *a, const float *b, double *dup, double *dlo,
                      double *su_sq, double *sl_sq)
{
    double su = 0.0, sl = 0.0;
    for (int i = 0; i < d; ++i) {
        double delta = (double)a[i] - (double)b[i];
        double cu, cl;
        components(i, delta, mon, &cu, &cl);
        cu = w[i] * cu;
        cl = w[i] * cl;
        if (norm == ORC_L1) {
            su = su + cu;
            sl = sl + cl;
        } else if (norm == ORC_L2) {
            su = su + cu * cu;
            sl = sl + cl * cl;
        } else {
            if (cu > su) su = cu;
            if (cl > sl) sl = cl;
        }
    }
    if (su_sq) *su_sq = su;
    if (sl_sq) *sl_sq = sl;
    if (norm == ORC_L2) {
        su = sqrt(su);
        sl = sqrt(sl);
    }
    *dup = su;
    *dlo = sl;
}

static double m_of(const float *Mk, double M, long k) { return Mk ? (double)Mk[k] : M; }

/* Eq. (2) and Eq. (3): for every query x,
 *   H_up(x) = min_k (y^k + M_k dist_up(x, x^k)),  H_lo(x) = max_k (y^k - M_k dist_lo(x, x^k)),
 *   g(x) = (H_up(x) + H_lo(x)) / 2,
 * with the lowest index among exact ties.  Any output pointer may be NULL. */
void orc_bounds(int d, int norm, const double *w, const signed char *mon,
                const float *x, const float *y, long n, double M, const float *Mk,
                const float *xq, long q,
                double *h_up, double *h_lo, double *g, long *arg_up, long *arg_lo)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < q; ++j) {
        const float *xj = xq + j * (long)d;
        double best_u = INFINITY, best_l = -INFINITY;
        long au = -1, al = -1;
        for (long k = 0; k < n; ++k) {
            double du, dl;
            dist_pair(d, norm, w, mon, xj, x + k * (long)d, &du, &dl, NULL, NULL);
            double mk = m_of(Mk, M, k);
            double u = (double)y[k] + mk * du;
            double l = (double)y[k] - mk * dl;
            if (u < best_u) { best_u = u; au = k; }
            if (l > best_l) { best_l = l; al = k; }
        }
        if (h_up) h_up[j] = best_u;
        if (h_lo) h_lo[j] = best_l;
        if (g) g[j] = 0.5 * (best_u + best_l);
        if (arg_up) arg_up[j] = au;
        if (arg_lo) arg_lo[j] = al;
    }
}

/* All candidates of Eq. (2) for one query: u[k] = y^k + M_k dist_up(x, x^k),
 * l[k] = y^k - M_k dist_lo(x, x^k), k = 0..n-1 (used to list near-ties). */
void orc_candidates(int d, int norm, const double *w, const signed char *mon,
                    const float *x, const float *y, long n, double M, const float *Mk,
                    const float *xq1, double *u, double *l)
{
    for (long k = 0; k < n; ++k) {
        double du, dl;
        dist_pair(d, norm, w, mon, xq1, x + k * (long)d, &du, &dl, NULL, NULL);
        double mk = m_of(Mk, M, k);
        u[k] = (double)y[k] + mk * du;
        l[k] = (double)y[k] - mk * dl;
    }
}

/* Data-side consistency check: whether the data can be interpolated by a
 * function with Lipschitz constant M (Sec. 1, the Lipschitz condition
 * |f(x) - f(z)| <= M d(x, z)) that also respects the monotonicity constraints
 * (Sec. 4.1), in the pairwise form of Eqs. (5)-(6) with eps = 0.
 * For each requested row i (all rows when rows == NULL), over k != i:
 *   t_up(i,k) = (y_k + M_k dist_up(x^i, x^k)) - y_i    (>= 0 when consistent)
 *   t_lo(i,k) = y_i - (y_k - M_k dist_lo(x^i, x^k))    (>= 0 when consistent)
 * evaluated in FP64 with the bound y_k +- M_k dist as one fused multiply-add
 * (one rounding) and then the difference with y_i.
 * slack_up[r] = min_k t_up, slack_lo[r] = min_k t_lo (lowest k on ties),
 * viol_up[r] / viol_lo[r] = number of k with t < -tol.
 * Equality |y_i - y_k| = M d is consistent (the condition is "<=").
 * With n == 1 the slacks are +inf and the partners -1. */
void orc_consistency(int d, int norm, const double *w, const signed char *mon,
                     const float *x, const float *y, long n, double M, const float *Mk,
                     double tol, const long *rows, long n_rows,
                     double *slack_up, double *slack_lo, long *partner_up, long *partner_lo,
                     long *viol_up, long *viol_lo)
{
    if (!rows) n_rows = n;
#pragma omp parallel for schedule(dynamic, 4)
    for (long r = 0; r < n_rows; ++r) {
        long i = rows ? rows[r] : r;
        const float *xi = x + i * (long)d;
        double yi = (double)y[i];
        double su = INFINITY, sl = INFINITY;
        long pu = -1, pl = -1, cu = 0, cl = 0;
        for (long k = 0; k < n; ++k) {
            if (k == i) continue;
            double du, dl;
            dist_pair(d, norm, w, mon, xi, x + k * (long)d, &du, &dl, NULL, NULL);
            double mk = m_of(Mk, M, k);
            double tu = fma(mk, du, (double)y[k]) - yi;
            double tl = yi - fma(-mk, dl, (double)y[k]);
            if (tu < su) { su = tu; pu = k; }
            if (tl < sl) { sl = tl; pl = k; }
            if (tu < -tol) ++cu;
            if (tl < -tol) ++cl;
        }
        if (slack_up) slack_up[r] = su;
        if (slack_lo) slack_lo[r] = sl;
        if (partner_up) partner_up[r] = pu;
        if (partner_lo) partner_lo[r] = pl;
        if (viol_up) viol_up[r] = cu;
        if (viol_lo) viol_lo[r] = cl;
    }
}

/* Global Lipschitz constant from the data (Sec. 5, lipschitz_constant):
 *   M = max over pairs i < k of |y_i - y_k| / dist(x^i, x^k),
 * with the symmetric distance (monotonicity ignored).  Pairs at distance 0
 * with equal y are skipped.  Returns 0, or 3 when two coincident points carry
 * different values (infinite slope; that pair is reported).  The maximising
 * pair is the lexicographically lowest (i, k) among exact ties; with no
 * usable pair M = 0 and pair = (-1, -1). */
int orc_estimate_M_global(int d, int norm, const double *w, const float *x, const float *y,
                          long n, double *M_out, long *pair)
{
    double *row_best = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    long *row_arg = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    long *row_dup = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 8)
    for (long i = 0; i < n; ++i) {
        double best = -1.0;
        long arg = -1, dup = -1;
        for (long k = i + 1; k < n; ++k) {
            double du, dl;
            dist_pair(d, norm, w, NULL, x + i * (long)d, x + k * (long)d, &du, &dl, NULL, NULL);
            double dy = fabs((double)y[i] - (double)y[k]);
            if (du == 0.0) {
                if (dy != 0.0 && dup < 0) dup = k;
                continue;
            }
            double r = dy / du;
            if (r > best) { best = r; arg = k; }
        }
        row_best[i] = best;
        row_arg[i] = arg;
        row_dup[i] = dup;
    }
    int status = 0;
    double best = -1.0;
    pair[0] = -1;
    pair[1] = -1;
    for (long i = 0; i < n; ++i) {
        if (row_dup[i] >= 0) {
            status = 3;
            pair[0] = i;
            pair[1] = row_dup[i];
            break;
        }
        if (row_arg[i] >= 0 && row_best[i] > best) {
            best = row_best[i];
            pair[0] = i;
            pair[1] = row_arg[i];
        }
    }
    *M_out = status ? INFINITY : (best < 0.0 ? 0.0 : best);
    free(row_best);
    free(row_arg);
    free(row_dup);
    return status;
}

typedef struct { double key; long j; } keyed;

static int keyed_cmp(const void *pa, const void *pb)
{
    const keyed *a = (const keyed *)pa, *b = (const keyed *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* Per-point Lipschitz constant from the K nearest data (the scalar form of
 * Sec. 4.3: M_i = max over the K nearest j != i of |y_i - y_j| / dist(x^i, x^j)).
 * Nearness uses the symmetric distance (monotonicity ignored); for l2 the
 * points are ranked by the sum of squares, which orders them like the
 * distance.  Ties rank the lower j first.  The ranking is a full sort of all
 * j != i.  Coincident neighbours with equal y are skipped; with different y
 * the function returns 3 and M_out[r] = +inf for that row.  nbr (if not
 * NULL) receives the K neighbour indices of each row in rank order (-1 when
 * n - 1 < K). */
int orc_estimate_M_knn(int d, int norm, const double *w, const float *x, const float *y,
                       long n, int K, const long *rows, long n_rows, double *M_out, long *nbr)
{
    if (!rows) n_rows = n;
    int status = 0;
#pragma omp parallel
    {
        keyed *buf = (keyed *)malloc(sizeof(keyed) * (size_t)(n > 1 ? n : 1));
#pragma omp for schedule(dynamic, 4) reduction(max : status)
        for (long r = 0; r < n_rows; ++r) {
            long i = rows ? rows[r] : r;
            long m = 0;
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double du, dl, sq, sq2;
                dist_pair(d, norm, w, NULL, x + i * (long)d, x + j * (long)d, &du, &dl, &sq, &sq2);
                buf[m].key = (norm == ORC_L2) ? sq : du;
                buf[m].j = j;
                ++m;
            }
            qsort(buf, (size_t)m, sizeof(keyed), keyed_cmp);
            long kk = m < K ? m : K;
            double best = 0.0;
            for (long t = 0; t < kk; ++t) {
                long j = buf[t].j;
                double du, dl;
                dist_pair(d, norm, w, NULL, x + i * (long)d, x + j * (long)d, &du, &dl, NULL, NULL);
                double dy = fabs((double)y[i] - (double)y[j]);
                if (du == 0.0) {
                    if (dy != 0.0) { best = INFINITY; status = 3; }
                    continue;
                }
                double s = dy / du;
                if (s > best) best = s;
            }
            M_out[r] = best;
            if (nbr) {
                for (long t = 0; t < K; ++t) nbr[r * (long)K + t] = t < kk ? buf[t].j : -1;
            }
        }
        free(buf);
    }
    return status;
}

/* Derivative of the component c_i with respect to delta_i = a_i - b_i, for the
 * upper (up = 1) or the lower (up = 0) distance.  Kinks take 0:
 * |.|'(0) = 0 and (.)_+'(0) = 0. */
static double dcomp(int i, double delta, const signed char *mon, int up)
{
    int m = mon ? mon[i] : 0;
    if (m == 0) return delta > 0.0 ? 1.0 : (delta < 0.0 ? -1.0 : 0.0);
    int pos = (m > 0) == (up != 0); /* component is (delta)_+ when pos, else (-delta)_+ */
    if (pos) return delta > 0.0 ? 1.0 : 0.0;
    return delta < 0.0 ? -1.0 : 0.0;
}

/* Gradient of dist_up (up = 1) or dist_lo (up = 0) with respect to the first
 * argument a.  l2 at distance 0 gives 0; linf takes the lowest coordinate
 * among the maximal weighted components. */
static void dist_grad(int d, int norm, const double *w, const signed char *mon,
                      const float *a, const float *b, int up, double dist, double *out)
{
    float cmax = -1.0f;
    int jmax = -1;
    for (int i = 0; i < d; ++i) {
        double delta = (double)a[i] - (double)b[i];
        double cu, cl;
        components(i, delta, mon, &cu, &cl);
        double c = w[i] * (up ? cu : cl);
        double dc = w[i] * dcomp(i, delta, mon, up);
        if (norm == ORC_L1) {
            out[i] = dc;
        } else if (norm == ORC_L2) {
            out[i] = dist > 0.0 ? c * dc / dist : 0.0;
        } else {
            /* Which coordinate carries the linf subgradient is an integer
             * decided by floating point: it is decided in single precision,
             * with the component formed as the evaluation precision forms it
             * (the single-precision difference, its absolute value or
             * positive part, times the weight), lowest coordinate on ties. */
            const float df = a[i] - b[i];
            double cu32, cl32;
            components(i, (double)df, mon, &cu32, &cl32);
            const float c32 = (float)w[i] * (float)(up ? cu32 : cl32);
            out[i] = 0.0;
            if (c32 > cmax) { cmax = c32; jmax = i; }
        }
    }
    if (norm == ORC_LINF && jmax >= 0) {
        double delta = (double)a[jmax] - (double)b[jmax];
        out[jmax] = w[jmax] * dcomp(jmax, delta, mon, up);
    }
}

/* Subgradients of g (and optionally of H_up, H_lo) through the selected data
 * points a = arg_up[j], b = arg_lo[j]:
 *   H_up = y_a + M_a dist_up(x, x^a),  H_lo = y_b - M_b dist_lo(x, x^b),  g = (H_up + H_lo)/2.
 * With G_up = dg/2 + dh_up and G_lo = dg/2 + dh_lo (missing arrays count 0):
 *   dxq[j]  = G_up M_a grad dist_up - G_lo M_b grad dist_lo
 *   dy[a]  += G_up,  dy[b] += G_lo
 *   dM     += G_up dist_up - G_lo dist_lo            (global M, dM[0])
 *   dM[a]  += G_up dist_up,  dM[b] -= G_lo dist_lo   (per-point M_k)
 * dy and dM are accumulated in query order; dxq is overwritten. */
void orc_grad(int d, int norm, const double *w, const signed char *mon,
              const float *x, const float *y, long n, double M, const float *Mk,
              const float *xq, long q, const long *arg_up, const long *arg_lo,
              const double *dg, const double *dh_up, const double *dh_lo,
              double *dxq, double *dy, double *dM)
{
    (void)y;
    (void)n;
    double *gu = (double *)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
    double *gl = (double *)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
    for (long j = 0; j < q; ++j) {
        const float *xj = xq + j * (long)d;
        long a = arg_up[j], b = arg_lo[j];
        double Gu = (dg ? 0.5 * dg[j] : 0.0) + (dh_up ? dh_up[j] : 0.0);
        double Gl = (dg ? 0.5 * dg[j] : 0.0) + (dh_lo ? dh_lo[j] : 0.0);
        double du, dl_unused, du_unused, dl;
        dist_pair(d, norm, w, mon, xj, x + a * (long)d, &du, &dl_unused, NULL, NULL);
        dist_pair(d, norm, w, mon, xj, x + b * (long)d, &du_unused, &dl, NULL, NULL);
        dist_grad(d, norm, w, mon, xj, x + a * (long)d, 1, du, gu);
        dist_grad(d, norm, w, mon, xj, x + b * (long)d, 0, dl, gl);
        double Ma = m_of(Mk, M, a), Mb = m_of(Mk, M, b);
        if (dxq) {
            for (int i = 0; i < d; ++i) dxq[j * (long)d + i] = Gu * Ma * gu[i] - Gl * Mb * gl[i];
        }
        if (dy) {
            dy[a] += Gu;
            dy[b] += Gl;
        }
        if (dM) {
            if (Mk) {
                dM[a] += Gu * du;
                dM[b] -= Gl * dl;
            } else {
                dM[0] += Gu * du - Gl * dl;
            }
        }
    }
    free(gu);
    free(gl);
}

/* ---- step-function local constants (Sec. 4.3) -------------------------------
 *
 * Reading used here (the section describes the construction in words only):
 *  - Knots q_1 <= ... <= q_K are shared by all data: quantiles of the
 *    distribution of inter-point distances, estimated from a sample of pairs
 *    (orc_knots).  The sample itself is an input.
 *  - For datum k, d1_k is the distance to its nearest other datum (positive
 *    distances only; coincident data with the same value are skipped).
 *  - M_k(t) is non-decreasing and piecewise constant:
 *        t <= d1_k                   -> V_k,0   = max slope over the data at distance <= d1_k
 *        otherwise, the first s with t <= q_s -> V_k,s = max slope over the data at
 *                                                 distance <= max(q_s, d1_k)
 *        t > q_K                     -> V_k,K+1 = max slope over all data
 *    where the slope of a pair is |y_k - y_j| / dist(x^k, x^j) with the
 *    symmetric distance (monotonicity ignored).  An empty set gives 0.
 *  - A coincident datum with a different value makes the slope infinite: the
 *    whole row is +inf and the function returns 3.
 *  - Bounds use the datum's function at the pair's own distance:
 *        u_k = y_k + M_k(dist_up) dist_up,   l_k = y_k - M_k(dist_lo) dist_lo.
 */

static int cmp_double(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/* Knots as quantiles of sampled inter-point distances: the m pairs
 * (pairs[2s], pairs[2s+1]) give distances with the symmetric distance, sorted
 * ascending as r_0 <= ... <= r_{m-1}; knot j is the inverse of the empirical
 * distribution function at probs[j]: r_c with c = ceil(probs[j] * m) - 1,
 * clamped to [0, m - 1]. */
void orc_knots(int d, int norm, const double *w, const float *x, const long *pairs, long m,
               const double *probs, int K, double *knots)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (long s = 0; s < m; ++s) {
        double du, dl;
        dist_pair(d, norm, w, NULL, x + pairs[2 * s] * (long)d, x + pairs[2 * s + 1] * (long)d,
                  &du, &dl, NULL, NULL);
        r[s] = du;
    }
    qsort(r, (size_t)m, sizeof(double), cmp_double);
    for (int j = 0; j < K; ++j) {
        long c = (long)ceil(probs[j] * (double)m) - 1;
        if (c < 0) c = 0;
        if (c > m - 1) c = m - 1;
        knots[j] = r[c];
    }
    free(r);
}

/* The step table of every requested row i (all rows when rows == NULL):
 * d1[r] and V[r * (K + 2) + s], s = 0..K+1, as defined above, written from
 * the definition: first the pair list of the row, then one pass per entry. */
int orc_local_steps(int d, int norm, const double *w, const float *x, const float *y, long n,
                    const double *knots, int K, const long *rows, long n_rows, double *d1,
                    double *V)
{
    if (!rows) n_rows = n;
    int status = 0;
#pragma omp parallel
    {
        double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *sl = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 4) reduction(max : status)
        for (long r = 0; r < n_rows; ++r) {
            long i = rows ? rows[r] : r;
            double *v = V + r * (long)(K + 2);
            int infinite = 0;
            /* pair list: distance and slope of every j != i with a positive distance */
            long m = 0;
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double du, dl;
                dist_pair(d, norm, w, NULL, x + i * (long)d, x + j * (long)d, &du, &dl, NULL, NULL);
                double dy = fabs((double)y[i] - (double)y[j]);
                if (du == 0.0) {
                    if (dy != 0.0) infinite = 1;
                    continue;
                }
                t[m] = du;
                sl[m] = dy / du;
                ++m;
            }
            double nn = INFINITY;
            for (long a = 0; a < m; ++a)
                if (t[a] < nn) nn = t[a];
            d1[r] = nn;
            for (int s = 0; s < K + 2; ++s) {
                /* radius of entry s: d1 (s = 0), max(q_s, d1) (1 <= s <= K), all (K + 1) */
                double rad = s == 0 ? nn : (s <= K ? (knots[s - 1] > nn ? knots[s - 1] : nn) : INFINITY);
                double best = 0.0;
                for (long a = 0; a < m; ++a)
                    if (t[a] <= rad && sl[a] > best) best = sl[a];
                v[s] = infinite ? INFINITY : best;
            }
            if (infinite) status = 3;
        }
        free(t);
        free(sl);
    }
    return status;
}

/* M_k(t) from the row's table (d1 and V[0..K+1], as float values widened). */
static double step_value(double t, double d1, const float *v, const double *knots, int K)
{
    if (t <= d1) return (double)v[0];
    for (int s = 1; s <= K; ++s)
        if (t <= knots[s - 1]) return (double)v[s];
    return (double)v[K + 1];
}

/* Eq. (2) and Eq. (3) with the step-function constants: the table is given as
 * d1 [n] (FP64) and V [n][K+2] (FP32, the values the bounds multiply).  Lowest
 * index among exact ties.  Any output pointer may be NULL. */
void orc_bounds_step(int d, int norm, const double *w, const signed char *mon, const float *x,
                     const float *y, long n, const double *knots, int K, const double *d1,
                     const float *V, const float *xq, long q, double *h_up, double *h_lo,
                     double *g, long *arg_up, long *arg_lo)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < q; ++j) {
        const float *xj = xq + j * (long)d;
        double best_u = INFINITY, best_l = -INFINITY;
        long au = -1, al = -1;
        for (long k = 0; k < n; ++k) {
            double du, dl;
            dist_pair(d, norm, w, mon, xj, x + k * (long)d, &du, &dl, NULL, NULL);
            const float *vk = V + k * (long)(K + 2);
            double u = (double)y[k] + step_value(du, d1[k], vk, knots, K) * du;
            double l = (double)y[k] - step_value(dl, d1[k], vk, knots, K) * dl;
            if (u < best_u) { best_u = u; au = k; }
            if (l > best_l) { best_l = l; al = k; }
        }
        if (h_up) h_up[j] = best_u;
        if (h_lo) h_lo[j] = best_l;
        if (g) g[j] = 0.5 * (best_u + best_l);
        if (arg_up) arg_up[j] = au;
        if (arg_lo) arg_lo[j] = al;
    }
}

/* Every candidate of one query under the step-function constants. */
void orc_candidates_step(int d, int norm, const double *w, const signed char *mon,
                         const float *x, const float *y, long n, const double *knots, int K,
                         const double *d1, const float *V, const float *xq1, double *u, double *l)
{
    for (long k = 0; k < n; ++k) {
        double du, dl;
        dist_pair(d, norm, w, mon, xq1, x + k * (long)d, &du, &dl, NULL, NULL);
        const float *vk = V + k * (long)(K + 2);
        u[k] = (double)y[k] + step_value(du, d1[k], vk, knots, K) * du;
        l[k] = (double)y[k] - step_value(dl, d1[k], vk, knots, K) * dl;
    }
}

/* ---- penalty form of the smoothing problem (Sec. 4.4, Eq. 7) --------------
 *
 * With corrections eps (z = y + eps) the data must satisfy, for every ordered
 * pair i != k, the two constraints of Eqs. (5)-(6); written with the
 * directional distances (Sec. 4.1) and the datum k's constant, as in the
 * consistency check:
 *     a_ik = z_i - z_k - M_k dist_up(x^i, x^k) <= 0          (Eq. 5)
 *     b_ik = z_k - z_i - M_k dist_lo(x^i, x^k) <= 0          (Eq. 6)
 * Eq. (7) minimises
 *     F(eps) = (1/p) ||eps||^2 + sum_{i != k} ( (a_ik)_+^2 + (b_ik)_+^2 ).
 * This returns F and its gradient: d/d eps_i of (a_ik)_+^2 is 2 (a_ik)_+ and
 * d/d eps_k is -2 (a_ik)_+; (b_ik)_+^2 gives the opposite signs.  Plain
 * serial loops over all ordered pairs.
 *
 * Pre-screening of Sec. 5 (c > 0): a pair whose data already satisfy both
 * constraints with a third of the allowance (c = 1/3 in the paper) is taken
 * out of the sums before the minimisation.  Here the ordered pair (i, k) is
 * dropped when, on the given y (not on z),
 *     y_i - y_k <= c M_k dist_up(x^i, x^k)  and  y_k - y_i <= c M_k dist_lo(x^i, x^k)
 * (products evaluated left to right); c = 0 keeps every pair. */
static int pruned(double c, double yi, double yk, double mk, double du, double dl)
{
    return c > 0.0 && yi - yk <= c * mk * du && yk - yi <= c * mk * dl;
}

void orc_smooth(int d, int norm, const double *w, const signed char *mon, const float *x,
                const float *y, long n, double M, const float *Mk, const double *eps, double p,
                double c, double *F, double *grad)
{
    double total = 0.0;
    for (long i = 0; i < n; ++i) grad[i] = 0.0;
    for (long i = 0; i < n; ++i) {
        for (long k = 0; k < n; ++k) {
            if (k == i) continue;
            double du, dl;
            dist_pair(d, norm, w, mon, x + i * (long)d, x + k * (long)d, &du, &dl, NULL, NULL);
            double mk = m_of(Mk, M, k);
            if (pruned(c, (double)y[i], (double)y[k], mk, du, dl)) continue;
            double zi = (double)y[i] + eps[i], zk = (double)y[k] + eps[k];
            double a = zi - zk - mk * du;
            double b = zk - zi - mk * dl;
            if (a > 0.0) {
                total += a * a;
                grad[i] += 2.0 * a;
                grad[k] -= 2.0 * a;
            }
            if (b > 0.0) {
                total += b * b;
                grad[k] += 2.0 * b;
                grad[i] -= 2.0 * b;
            }
        }
    }
    for (long i = 0; i < n; ++i) {
        total += eps[i] * eps[i] / p;
        grad[i] += 2.0 * eps[i] / p;
    }
    *F = total;
}

/* Error scale of the penalty objective, for comparisons only: the sum A of
 * the positive parts (a_ik)_+ + (b_ik)_+ over all ordered pairs that the
 * pre-screening keeps, and per row
 * i, over the four terms that move eps_i (a_ik, b_ik of the pairs (i, k) and
 * a_ki, b_ki of the pairs (k, i)), the sum of their gradient magnitudes
 * 2 (t)_+ (row_abs) and the number of them above -tau (row_cnt). */
void orc_smooth_scale(int d, int norm, const double *w, const signed char *mon, const float *x,
                      const float *y, long n, double M, const float *Mk, const double *eps,
                      double c, double tau, double *A, double *row_abs, long *row_cnt)
{
    double total = 0.0;
    for (long i = 0; i < n; ++i) {
        row_abs[i] = 0.0;
        row_cnt[i] = 0;
    }
    for (long i = 0; i < n; ++i) {
        for (long k = 0; k < n; ++k) {
            if (k == i) continue;
            double du, dl;
            dist_pair(d, norm, w, mon, x + i * (long)d, x + k * (long)d, &du, &dl, NULL, NULL);
            double mk = m_of(Mk, M, k);
            if (pruned(c, (double)y[i], (double)y[k], mk, du, dl)) continue;
            double zi = (double)y[i] + eps[i], zk = (double)y[k] + eps[k];
            double t[2] = {zi - zk - mk * du, zk - zi - mk * dl};
            for (int j = 0; j < 2; ++j) {
                double v = t[j] > 0.0 ? t[j] : 0.0;
                total += v;
                row_abs[i] += 2.0 * v;
                row_abs[k] += 2.0 * v;
                if (t[j] > -tau) {
                    ++row_cnt[i];
                    ++row_cnt[k];
                }
            }
        }
    }
    *A = total;
}

/* ---- k best bounds with weights (Sec. 5, k > 1) ------------------------------
 *
 * With k > 1 and weights wk[0..k-1], both bounds use the k best candidates
 * of Eq. (2): u sorted ascending u_(1) <= u_(2) <= ..., l sorted descending
 * l_[1] >= l_[2] >= ...;
 *     H_up = sum_j wk[j] u_(j+1),   H_lo = sum_j wk[j] l_[j+1],   g = (H_up + H_lo) / 2.
 * (The k values are a multiset: ties need no index rule.)  Requires k <= n. */
static int cmp_double_desc(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a < b) - (a > b);
}

void orc_bounds_k(int d, int norm, const double *w, const signed char *mon, const float *x,
                  const float *y, long n, double M, const float *Mk, int K, const double *wk,
                  const float *xq, long q, double *h_up, double *h_lo, double *g)
{
#pragma omp parallel
    {
        double *u = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *l = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 16)
        for (long j = 0; j < q; ++j) {
            const float *xj = xq + j * (long)d;
            for (long k = 0; k < n; ++k) {
                double du, dl;
                dist_pair(d, norm, w, mon, xj, x + k * (long)d, &du, &dl, NULL, NULL);
                double mk = m_of(Mk, M, k);
                u[k] = (double)y[k] + mk * du;
                l[k] = (double)y[k] - mk * dl;
            }
            qsort(u, (size_t)n, sizeof(double), cmp_double);
            qsort(l, (size_t)n, sizeof(double), cmp_double_desc);
            double su = 0.0, sl = 0.0;
            for (int t = 0; t < K; ++t) {
                su += wk[t] * u[t];
                sl += wk[t] * l[t];
            }
            if (h_up) h_up[j] = su;
            if (h_lo) h_lo[j] = sl;
            if (g) g[j] = 0.5 * (su + sl);
        }
        free(u);
        free(l);
    }
}

/* ---- monotonicity on parts of the domain (Sec. 4.2) -------------------------
 *
 * Per coordinate i a kind: 0 free, +1 / -1 increasing / decreasing everywhere,
 * and on the partition A: x_i <= a_i, AB: a_i <= x_i <= b_i, B: x_i >= b_i
 *   2 (case I)   increasing on A and B, unrestricted on AB,
 *   3 (case II)  decreasing on A and B, unrestricted on AB,
 *   4 (case III) decreasing on A, increasing on B, unrestricted on AB,
 *   5 (case IV)  increasing on A, decreasing on B, unrestricted on AB.
 * Reading (the section's formulas are not given): going from x^k to x along
 * coordinate i, f can rise only where it is not decreasing (moving right) or
 * not increasing (moving left), by at most M per unit length, and elsewhere
 * it cannot rise.  So the component of the upper distance is the length of
 * the part of the segment between x^k_i and x_i where f may rise in the
 * direction of travel, and that of the lower distance the length where it
 * may fall; with the regions "not decreasing" ND and "not increasing" NI:
 *     x_i >= x^k_i:  c_up = |seg ∩ ND|,  c_lo = |seg ∩ NI|
 *     x_i <  x^k_i:  c_up = |seg ∩ NI|,  c_lo = |seg ∩ ND|
 * For +1 (ND = everything, NI = nothing) these are (x_i - x^k_i)_+ and
 * (x^k_i - x_i)_+, Eq. (4) and its mirror.  The components are weighted and
 * combined by the norm as before. */

/* length of [lo, hi] ∩ [s, t] */
static double overlap(double lo, double hi, double s, double t)
{
    double a = lo > s ? lo : s;
    double b = hi < t ? hi : t;
    return b > a ? b - a : 0.0;
}

static void regions(int kind, double a, double b, double *nd_s, double *nd_t, double *ni_s,
                    double *ni_t)
{
    const double inf = INFINITY;
    double s1 = -inf, t1 = inf, s2 = -inf, t2 = inf; /* ND, NI: everything */
    switch (kind) {
    case 1: s2 = inf; t2 = -inf; break;                 /* NI empty */
    case -1: s1 = inf; t1 = -inf; break;                /* ND empty */
    case 2: s2 = a; t2 = b; break;                      /* NI = AB */
    case 3: s1 = a; t1 = b; break;                      /* ND = AB */
    case 4: s1 = a; t1 = inf; s2 = -inf; t2 = b; break; /* ND = AB u B, NI = A u AB */
    case 5: s1 = -inf; t1 = b; s2 = a; t2 = inf; break; /* ND = A u AB, NI = AB u B */
    default: break;                                     /* free */
    }
    *nd_s = s1;
    *nd_t = t1;
    *ni_s = s2;
    *ni_t = t2;
}

static void dist_pair_reg(int d, int norm, const double *w, const signed char *kind,
                          const double *ra, const double *rb, const float *x, const float *xk,
                          double *dup, double *dlo)
{
    double su = 0.0, sl = 0.0;
    for (int i = 0; i < d; ++i) {
        double xi = (double)x[i], ki = (double)xk[i];
        double nds, ndt, nis, nit;
        regions(kind ? kind[i] : 0, ra ? ra[i] : 0.0, rb ? rb[i] : 0.0, &nds, &ndt, &nis, &nit);
        double cu, cl;
        if (xi >= ki) {
            cu = overlap(ki, xi, nds, ndt);
            cl = overlap(ki, xi, nis, nit);
        } else {
            cu = overlap(xi, ki, nis, nit);
            cl = overlap(xi, ki, nds, ndt);
        }
        cu = w[i] * cu;
        cl = w[i] * cl;
        if (norm == ORC_L1) {
            su = su + cu;
            sl = sl + cl;
        } else if (norm == ORC_L2) {
            su = su + cu * cu;
            sl = sl + cl * cl;
        } else {
            if (cu > su) su = cu;
            if (cl > sl) sl = cl;
        }
    }
    if (norm == ORC_L2) {
        su = sqrt(su);
        sl = sqrt(sl);
    }
    *dup = su;
    *dlo = sl;
}

/* Eq. (2)-(3) with the regional components above; lowest index on ties. */
void orc_bounds_reg(int d, int norm, const double *w, const signed char *kind, const double *ra,
                    const double *rb, const float *x, const float *y, long n, double M,
                    const float *Mk, const float *xq, long q, double *h_up, double *h_lo,
                    double *g, long *arg_up, long *arg_lo)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < q; ++j) {
        const float *xj = xq + j * (long)d;
        double best_u = INFINITY, best_l = -INFINITY;
        long au = -1, al = -1;
        for (long k = 0; k < n; ++k) {
            double du, dl;
            dist_pair_reg(d, norm, w, kind, ra, rb, xj, x + k * (long)d, &du, &dl);
            double mk = m_of(Mk, M, k);
            double u = (double)y[k] + mk * du;
            double l = (double)y[k] - mk * dl;
            if (u < best_u) { best_u = u; au = k; }
            if (l > best_l) { best_l = l; al = k; }
        }
        if (h_up) h_up[j] = best_u;
        if (h_lo) h_lo[j] = best_l;
        if (g) g[j] = 0.5 * (best_u + best_l);
        if (arg_up) arg_up[j] = au;
        if (arg_lo) arg_lo[j] = al;
    }
}

void orc_candidates_reg(int d, int norm, const double *w, const signed char *kind,
                        const double *ra, const double *rb, const float *x, const float *y, long n,
                        double M, const float *Mk, const float *xq1, double *u, double *l)
{
    for (long k = 0; k < n; ++k) {
        double du, dl;
        dist_pair_reg(d, norm, w, kind, ra, rb, xq1, x + k * (long)d, &du, &dl);
        double mk = m_of(Mk, M, k);
        u[k] = (double)y[k] + mk * du;
        l[k] = (double)y[k] - mk * dl;
    }
}
