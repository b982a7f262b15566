// C-ABI entry points of the bound path (lip_bounds, lip_fit_eval), the
// workspace size, the tuning table and status strings.
#include <math.h>
#include <string.h>

#include "host_common.hpp"

namespace lip {

lip_status parse_metric(const lip_metric *m, MetricInfo *out, bool allow_regional)
{
    if (!m) return LIP_E_ARG;
    if (m->d < 1 || m->d > kMaxDim) return LIP_E_SHAPE;
    if (m->norm != LIP_L1 && m->norm != LIP_L2 && m->norm != LIP_LINF) return LIP_E_ARG;
    MetricInfo mi;
    mi.d = m->d;
    mi.norm = m->norm;
    const float inf = __builtin_inff();
    for (int i = 0; i < m->d; ++i) {
        const float w = m->w ? m->w[i] : 1.0f;
        if (!(w > 0.0f) || !__builtin_isfinite(w)) return LIP_E_VALUE;
        const int8_t mo = m->mon ? m->mon[i] : 0;
        if (mo < -1 || mo > LIP_MON_CASE_IV) return LIP_E_VALUE;
        mi.w[i] = (double)w;
        // regions where f is not decreasing / not increasing
        float nds = -inf, ndt = inf, nis = -inf, nit = inf;
        if (mo == 1) {
            nis = inf;
            nit = -inf;
        } else if (mo == -1) {
            nds = inf;
            ndt = -inf;
        } else if (mo >= LIP_MON_CASE_I) {
            if (!allow_regional) return LIP_E_UNSUPPORTED;
            if (!m->a || !m->b) return LIP_E_ARG;
            const float a = m->a[i], b = m->b[i];
            if (!__builtin_isfinite(a) || !__builtin_isfinite(b) || !(a <= b)) return LIP_E_VALUE;
            mi.regional = true;
            if (mo == LIP_MON_CASE_I) {
                nis = a;
                nit = b;
            } else if (mo == LIP_MON_CASE_II) {
                nds = a;
                ndt = b;
            } else if (mo == LIP_MON_CASE_III) {
                nds = a;
                nit = b;
            } else {
                ndt = b;
                nis = a;
            }
        }
        mi.nd_s[i] = nds;
        mi.nd_t[i] = ndt;
        mi.ni_s[i] = nis;
        mi.ni_t[i] = nit;
        mi.mon[i] = mo >= LIP_MON_CASE_I ? 0 : mo;
    }
    int k = 0;
    for (int i = 0; i < m->d; ++i) {
        if (mi.mon[i] == 0) {
            mi.xf.perm[k] = i;
            mi.xf.scale[k] = (float)mi.w[i];
            ++k;
        }
    }
    mi.dm = m->d - k;
    for (int i = 0; i < m->d; ++i) {
        if (mi.mon[i] != 0) {
            mi.xf.perm[k] = i;
            mi.xf.scale[k] = mi.mon[i] > 0 ? (float)mi.w[i] : -(float)mi.w[i];
            ++k;
        }
    }
    for (; k < kMaxDim; ++k) {
        mi.xf.perm[k] = 0;
        mi.xf.scale[k] = 0.0f;
    }
    *out = mi;
    return LIP_OK;
}

FwdLaunchers fwd_launchers(int norm, int d, int dm)
{
    switch (norm) {
    case LIP_L1: return fwd_launchers_l1(d, dm);
    case LIP_L2: return fwd_launchers_l2(d, dm);
    case LIP_LINF: return fwd_launchers_linf(d, dm);
    default: return FwdLaunchers{nullptr, nullptr};
    }
}

size_t staged_bytes(int64_t n, int d)
{
    // any tile <= kMaxTile pads n by less than kMaxTile records
    return align_up((size_t)(n + kMaxTile) * (size_t)(d + 3) * sizeof(float), 256);
}

size_t partial_bytes(int64_t q)
{
    int64_t entries = (int64_t)kMaxChunks * q;
    if (entries > kMaxPartials) entries = kMaxPartials;
    // two bounds x (value + index), values and indices in separate aligned blocks
    return align_up((size_t)entries * 2 * sizeof(float), 256) * 2;
}

lip_tile_cfg default_tile_cfg(int d, int dm, int norm, int64_t n, int64_t q)
{
    // About 16 waves per SIMD (256 CUs x 4 SIMDs) so that the last wave of
    // each SIMD starts early (small tail), data split in a power-of-two
    // number of chunks when the queries alone do not fill the chip.
    lip_tile_cfg c{};
    c.tile = 32;
    c.waves = 4;
    const int R = rows_for_dim(d);
    const int64_t qwaves = (q + 64 * R - 1) / (64 * R);
    const int64_t target = 16384;
    int split = 1;
    const int64_t tiles = (n + c.tile - 1) / c.tile;
    while (split < kMaxChunks && qwaves * split < target && tiles >= 4ll * split * 2 &&
           (int64_t)split * 2 * q <= kMaxPartials)
        split *= 2;
    c.split = split;
    // the root-free l2 filter halves the l2 forward with monotone
    // coordinates at d = 2..10 (N = 1e5, Q = 1e6, per-datum constants); with
    // it, queries in Morton order make a wave's filter decisions coherent on
    // the d = 4 benchmark data (27.3 against 30.1 ms, sorting included; not
    // measurable on uniform random data at other d, and not worth the sort
    // for few queries)
    if (norm == LIP_L2 && dm > 0) {
        c.flags = LIP_TILE_L2_FILTER;
        if (d <= 4 && q >= (int64_t(1) << 16)) c.flags |= LIP_TILE_QUERY_ORDER;
    }
    return c;
}

FwdPlan make_fwd_plan(const MetricInfo &mi, int64_t n, int64_t q, const lip_tile_cfg &cfg)
{
    FwdPlan p;
    p.R = rows_for_dim(mi.d);
    p.tile = cfg.tile;
    p.waves = cfg.waves;
    p.n_pad = (n + p.tile - 1) / p.tile * p.tile;
    p.n_tiles = p.n_pad / p.tile;
    int split = cfg.split < 1 ? 1 : cfg.split;
    if (split > kMaxChunks) split = kMaxChunks;
    while (split > 1 && (int64_t)split * q > kMaxPartials) split /= 2;
    if (split > p.n_tiles) split = (int)p.n_tiles;
    p.tiles_per_chunk = (int)((p.n_tiles + split - 1) / split);
    p.n_chunks = (int)((p.n_tiles + p.tiles_per_chunk - 1) / p.tiles_per_chunk);
    const int64_t qwaves = (q + 64 * p.R - 1) / (64 * p.R);
    if (mi.d <= kFwdMergeMaxDim) {
        // one workgroup per (query block, group of `waves` consecutive chunks)
        if (p.waves > p.n_chunks) p.waves = p.n_chunks;
        p.part_chunks = (p.n_chunks + p.waves - 1) / p.waves;
        p.n_chunks = p.part_chunks * p.waves;
        p.grid = qwaves * p.part_chunks;
    } else {
        // one workgroup per (`waves` query blocks, chunk), at most 4 waves
        if (p.waves > kFwdPlainMaxWaves) p.waves = kFwdPlainMaxWaves;
        p.part_chunks = p.n_chunks;
        p.grid = (qwaves + p.waves - 1) / p.waves * p.n_chunks;
    }
    return p;
}

lip_status check_finite(const float *const *arrays, const int64_t *counts, int n_arrays, void *ws,
                        hipStream_t stream)
{
    int *flag = (int *)ws;
    if (launch_fill_i32(flag, 1, 0, stream) != hipSuccess) return LIP_E_DEVICE;
    for (int i = 0; i < n_arrays; ++i)
        if (launch_nonfinite(arrays[i], counts[i], flag, stream) != hipSuccess) return LIP_E_DEVICE;
    int host = 0;
    if (hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return LIP_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return LIP_E_DEVICE;
    return host ? LIP_E_NONFINITE : LIP_OK;
}

lip_status run_bounds(const MetricInfo &mi, const float *x, const float *y, int64_t n, float M,
                      const float *Mk, const float *xq, int64_t q, float *g, float *h_up,
                      float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws, size_t ws_bytes,
                      const lip_tile_cfg &cfg, hipStream_t stream)
{
    const FwdPlan p = make_fwd_plan(mi, n, q, cfg);
    const size_t sb = staged_bytes(n, mi.d);
    const size_t pbytes = fwd_partial_bytes(p, q) / 2;
    const bool qord = (cfg.flags & LIP_TILE_QUERY_ORDER) != 0;
    const size_t need = kOriginBytes + sb + 2 * pbytes + (qord ? query_order_bytes(q, mi.d) : 0);
    if (ws_bytes < need) return LIP_E_WORKSPACE;
    FwdLauncher launch = fwd_launchers(mi.norm, mi.d, mi.dm).plain;
    if (!launch) return LIP_E_UNSUPPORTED;
    Xform xf = mi.xf;
    lip_status st = origin_for(x, n, mi.d, xf, ws, stream);
    if (st != LIP_OK) return st;
    ws = (char *)ws + kOriginBytes;
    float *staged = (float *)ws;

    StageArgs sa{};
    sa.x = x;
    sa.y = y;
    sa.Mk = Mk;
    sa.M = M;
    sa.l1_mon = mi.norm == LIP_L1 ? mi.dm : 0;
    sa.n = n;
    sa.n_pad = p.n_pad;
    sa.xf = xf;
    sa.out = staged;
    if (launch_stage(mi.d, sa, stream) != hipSuccess) return LIP_E_DEVICE;

    FwdArgs a{};
    a.data = staged;
    a.n = n;
    a.n_tiles = p.n_tiles;
    a.tile = p.tile;
    a.tiles_per_chunk = p.tiles_per_chunk;
    a.n_chunks = p.n_chunks;
    a.l2_filter = (cfg.flags & LIP_TILE_L2_FILTER) ? 1 : 0;
    a.xq = xq;
    a.q = q;
    a.xf = xf;
    a.g = g;
    a.h_up = h_up;
    a.h_lo = h_lo;
    a.arg_up = arg_up;
    a.arg_lo = arg_lo;
    if (p.part_chunks > 1) {
        char *pb = (char *)ws + sb;
        a.part_v = (float *)pb;
        a.part_i = (int32_t *)(pb + pbytes);
    }
    if (qord) {
        char *qb = (char *)ws + sb + 2 * pbytes;
        unsigned long long *keys = (unsigned long long *)qb;
        unsigned int *bb = (unsigned int *)(qb + align_up((size_t)sort_len(q) * 8, 256));
        float *xs = (float *)((char *)bb + 256);
        if (launch_query_order(xq, q, mi.d, bb, keys, sort_len(q), stream) != hipSuccess ||
            launch_query_gather(xq, q, mi.d, keys, xs, stream) != hipSuccess)
            return LIP_E_DEVICE;
        a.xq = xs;
        a.qorder = keys;
    }
    launch(a, dim3((unsigned)p.grid), dim3(64 * p.waves), stream);
    if (hipGetLastError() != hipSuccess) return LIP_E_DEVICE;
    if (p.part_chunks > 1) {
        CombineArgs c{};
        c.part_v = a.part_v;
        c.part_i = a.part_i;
        c.q = q;
        c.n_chunks = p.part_chunks;
        c.g = g;
        c.h_up = h_up;
        c.h_lo = h_lo;
        c.arg_up = arg_up;
        c.arg_lo = arg_lo;
        c.qorder = a.qorder;
        if (launch_combine(c, stream) != hipSuccess) return LIP_E_DEVICE;
    }
    return LIP_OK;
}

// Validation shared by lip_bounds / lip_fit_eval; no HIP call.
lip_status validate_bounds(const lip_metric *metric, const float *x, const float *y,
                                  int64_t n, float M, const float *Mk, const float *xq, int64_t q,
                                  uint32_t flags, MetricInfo *mi)
{
    lip_status st = parse_metric(metric, mi, true);
    if (st != LIP_OK) return st;
    if (flags & ~(LIP_FLAG_CHECK_FINITE | LIP_FLAG_BF16)) return LIP_E_ARG;
    if ((flags & LIP_FLAG_BF16) && mi->regional) return LIP_E_UNSUPPORTED;
    if (n <= 0 || q < 0) return LIP_E_SHAPE;
    if (n > kMaxIndex - kMaxTile || q > kMaxIndex) return LIP_E_SHAPE;
    if (!x || !y || (q > 0 && !xq)) return LIP_E_ARG;
    if (!Mk && (!(M >= 0.0f) || !__builtin_isfinite(M))) return LIP_E_VALUE;
    if ((flags & LIP_FLAG_BF16) && (mi->norm != LIP_L2 || mi->dm != 0)) return LIP_E_UNSUPPORTED;
    return LIP_OK;
}

}  // namespace lip

using namespace lip;

extern "C" {

size_t lip_workspace_size(int64_t n, int64_t q, int32_t d, uint32_t flags)
{
    (void)flags;
    if (n < 1) n = 1;
    if (q < 0) q = 0;
    if (d < 1) d = 1;
    if (d > kMaxDim) d = kMaxDim;
    size_t fwd = kOriginBytes + staged_bytes(n, d) + partial_bytes(q) + query_order_bytes(q, d) +
                 bf16_extra_bytes(n, q, d);
    size_t m = fwd;
    const size_t ds = data_side_ws_bytes(n, d);
    const size_t bwd = backward_ws_bytes(n);
    const size_t loc = local_ws_bytes(n, q, d);
    const size_t sm = smooth_ws_bytes(n, d);
    const size_t tk = topk_ws_bytes(n, q, d);
    const size_t rg = reg_ws_bytes(n, q, d);
    if (rg > m) m = rg;
    if (sm > m) m = sm;
    if (tk > m) m = tk;
    if (ds > m) m = ds;
    if (bwd > m) m = bwd;
    if (loc > m) m = loc;
    return m + 256;
}

lip_status lip_fit_eval(const lip_metric *metric, const float *x, const float *y, int64_t n,
                        float M, const float *Mk, const float *xq, int64_t q, float *g, float *h_up,
                        float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws, size_t ws_bytes,
                        uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = validate_bounds(metric, x, y, n, M, Mk, xq, q, flags, &mi);
    if (st != LIP_OK) return st;
    if (!ws) return LIP_E_WORKSPACE;
    if (q == 0) return LIP_OK;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[4] = {x, y, Mk, xq};
        const int64_t cnt[4] = {n * mi.d, n, Mk ? n : 0, q * mi.d};
        st = check_finite(arr, cnt, 4, ws, s);
        if (st != LIP_OK) return st;
    }
    if (mi.regional)
        return run_bounds_reg(mi, x, y, n, M, Mk, xq, q, g, h_up, h_lo, arg_up, arg_lo, ws,
                              ws_bytes, s);
    const lip_tile_cfg cfg = tune_lookup(mi.d, mi.dm, mi.norm, n, q);
    if (flags & LIP_FLAG_BF16) {
        return run_bounds_bf16(mi, x, y, n, M, Mk, xq, q, g, h_up, h_lo, arg_up, arg_lo, ws,
                               ws_bytes, s);
    }
    return run_bounds(mi, x, y, n, M, Mk, xq, q, g, h_up, h_lo, arg_up, arg_lo, ws, ws_bytes, cfg,
                      s);
}

lip_status lip_bounds(const lip_metric *metric, const float *x, const float *y, int64_t n, float M,
                      const float *Mk, const float *xq, int64_t q, float *h_up, float *h_lo,
                      int32_t *arg_up, int32_t *arg_lo, void *ws, size_t ws_bytes, uint32_t flags,
                      lip_stream stream)
{
    return lip_fit_eval(metric, x, y, n, M, Mk, xq, q, nullptr, h_up, h_lo, arg_up, arg_lo, ws,
                        ws_bytes, flags, stream);
}

const char *lip_status_string(lip_status status)
{
    switch (status) {
    case LIP_OK: return "ok";
    case LIP_E_ARG: return "invalid argument";
    case LIP_E_SHAPE: return "invalid shape";
    case LIP_E_VALUE: return "invalid value";
    case LIP_E_NONFINITE: return "non-finite input";
    case LIP_E_UNSUPPORTED: return "unsupported combination";
    case LIP_E_WORKSPACE: return "workspace missing or too small";
    case LIP_E_DEVICE: return "device error";
    default: return "unknown status";
    }
}

}  // extern "C"
