// Many independent fits in one graph launch (lip_plan_*) and the tile
// autotuner (lip_autotune).
//
// Plan.  Sets are grouped by shape class (norm, d, number of monotone
// coordinates).  Each set's queries are cut into waves of 64 R queries and
// its data into chunks of at most ~4M pairs per work item; the items of a
// class are sorted longest first and consumed by one persistent kernel per
// class (every wave pops the next item from a counter), so uneven set sizes
// balance across the chip.  Each set's argmin tile comes from the tuning
// table for its shape and size class (lip_autotune fills it); its data
// chunks follow from the work-item size, since the items of all sets fill
// the chip together.  Sets that need more than one data chunk merge
// their per-chunk results with atomic min on packed 64-bit (value, index)
// keys, decoded by a finalize kernel.  Staging, key initialisation, the class
// kernels and the finalize pass are recorded once into a HIP graph, and
// lip_plan_execute launches that graph.  Every item runs the wave body of the
// plain bound kernel, so results equal per-set lip_fit_eval calls.
#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "host_common.hpp"
#include "lip_device.hpp"

namespace lip {

// Staging of many sets in one launch: workgroup g handles sets g, g + G, ...
// Each set first gets its coordinate origin (the mid-range per coordinate,
// the same value launch_origin computes: minima and maxima are exact in any
// order), written to `origin` for the class kernels' query loads.
struct BatchStage {
    const float *x, *y, *Mk;
    float M;
    int32_t d;
    int32_t l1_mon;
    int32_t pad0;
    int64_t n, n_pad;
    Xform xf;
    float *origin;  // [kMaxDim], the array xf.origin points to
    float *out;
};

__global__ void __launch_bounds__(256) batched_stage_kernel(const BatchStage *st, int n_sets)
{
    __shared__ float smin[256], smax[256], org[kMaxDim];
    for (int s = blockIdx.x; s < n_sets; s += gridDim.x) {
        const BatchStage a = st[s];
        for (int j = 0; j < a.d; ++j) {
            float mn = __builtin_inff(), mx = -__builtin_inff();
            for (int64_t k = threadIdx.x; k < a.n; k += blockDim.x) {
                const float v = a.x[k * a.d + a.xf.perm[j]];
                mn = fminf(mn, v);
                mx = fmaxf(mx, v);
            }
            smin[threadIdx.x] = mn;
            smax[threadIdx.x] = mx;
            __syncthreads();
            for (int h = 128; h > 0; h >>= 1) {
                if ((int)threadIdx.x < h) {
                    smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + h]);
                    smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + h]);
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                const float o = origin_of_range(smin[0], smax[0]);
                org[j] = o;
                a.origin[j] = o;
            }
            __syncthreads();
        }
        if ((int)threadIdx.x >= a.d && threadIdx.x < kMaxDim) a.origin[threadIdx.x] = 0.0f;
        const int S = a.d + 3;
        for (int64_t k = threadIdx.x; k < a.n_pad; k += blockDim.x) {
            const int64_t src = k < a.n ? k : a.n - 1;
            const float *xs = a.x + src * a.d;
            float *o = a.out + k * S;
            const float y = a.y[src];
            const float m = a.Mk ? a.Mk[src] : a.M;
            float xm = 0.0f;
            for (int j = 0; j < a.d; ++j) {
                // xf_coord with the origin from LDS (same operations, same value)
                const float v = (xs[a.xf.perm[j]] - org[j]) * a.xf.scale[j];
                o[j] = v;
                if (j >= a.d - a.l1_mon) xm = (j == a.d - a.l1_mon) ? v : xm + v;
            }
            o[a.d] = y;
            o[a.d + 1] = m;
            o[a.d + 2] = a.l1_mon > 0 ? fmaf(-m, xm, y) : y;
        }
        __syncthreads();  // org and the reduction arrays are reused by the next set
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void fill_u32_kernel(unsigned int *p, int n, unsigned int v)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// Decodes the packed keys of the chunked sets (up_key / lo_key).
__global__ void batched_finalize_kernel(const FwdArgs *sets, const int32_t *chunked, int n_chunked)
{
    for (int c = blockIdx.x; c < n_chunked; c += gridDim.x) {
        const FwdArgs a = sets[chunked[c]];
        for (int64_t j = threadIdx.x; j < a.q; j += blockDim.x) {
            float hu, hl;
            int au, al;
            decode_keys(a.keys[j], a.keys[a.q + j], hu, au, hl, al);
            if (a.g) a.g[j] = 0.5f * (hu + hl);
            if (a.h_up) a.h_up[j] = hu;
            if (a.h_lo) a.h_lo[j] = hl;
            if (a.arg_up) a.arg_up[j] = au;
            if (a.arg_lo) a.arg_lo[j] = al;
        }
    }
}

}  // namespace lip

using namespace lip;

struct lip_plan {
    int device = 0;
    void *mem = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<lip_tile_cfg> tiles;  // per set: argmin tile, data chunks, waves per workgroup
};

namespace {

struct SetPlan {
    MetricInfo mi;
    int R = 0, tile = 32, flags = 0;
    int64_t n_pad = 0, n_tiles = 0, qblocks = 0;
    int tiles_per_chunk = 0, n_chunks = 1;
    size_t staged_off = 0, keys_off = 0, origin_off = 0;
};

constexpr int64_t kItemPairs = int64_t(1) << 22;  // target pairs per work item

lip_status validate_set(const lip_batch_desc &s, MetricInfo *mi)
{
    lip_status st = parse_metric(&s.metric, mi);
    if (st != LIP_OK) return st;
    if (s.n <= 0 || s.q < 0 || s.n > kMaxIndex - kMaxTile || s.q > kMaxIndex) return LIP_E_SHAPE;
    if (!s.x || !s.y || (s.q > 0 && !s.xq)) return LIP_E_ARG;
    if (!s.Mk && (!(s.M >= 0.0f) || !__builtin_isfinite(s.M))) return LIP_E_VALUE;
    return LIP_OK;
}

void free_plan(lip_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

}  // namespace

extern "C" lip_status lip_plan_create(lip_plan **plan, const lip_batch_desc *sets, int32_t n_sets,
                                      uint32_t flags, lip_stream stream)
{
    (void)stream;
    if (!plan) return LIP_E_ARG;
    *plan = nullptr;
    if (n_sets < 0 || (n_sets > 0 && !sets)) return LIP_E_ARG;
    if (flags != 0) return LIP_E_ARG;
    std::vector<SetPlan> sp(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        lip_status st = validate_set(sets[s], &sp[s].mi);
        if (st != LIP_OK) return st;
        if (!fwd_launchers(sp[s].mi.norm, sp[s].mi.d, sp[s].mi.dm).batched) return LIP_E_UNSUPPORTED;
    }
    // geometry and memory layout
    size_t off = 0;
    std::vector<int32_t> chunked;
    for (int s = 0; s < n_sets; ++s) {
        SetPlan &p = sp[s];
        const lip_batch_desc &d = sets[s];
        const lip_tile_cfg cfg = tune_lookup(p.mi.d, p.mi.dm, p.mi.norm, d.n, d.q);
        p.R = rows_for_dim(p.mi.d);
        p.tile = cfg.tile;
        p.flags = cfg.flags & LIP_TILE_L2_FILTER;  // plans visit queries in index order
        p.n_pad = (d.n + p.tile - 1) / p.tile * p.tile;
        p.n_tiles = p.n_pad / p.tile;
        int64_t chunk_records = kItemPairs / (64 * p.R);
        int64_t tpc = chunk_records / p.tile;
        if (tpc < 1) tpc = 1;
        if (tpc > p.n_tiles) tpc = p.n_tiles;
        p.tiles_per_chunk = (int)tpc;
        p.n_chunks = (int)((p.n_tiles + tpc - 1) / tpc);
        p.qblocks = (d.q + 64 * p.R - 1) / (64 * p.R);
        p.staged_off = off;
        off += align_up((size_t)p.n_pad * (size_t)(p.mi.d + 3) * sizeof(float), 256);
        p.origin_off = off;
        off += align_up(kMaxDim * sizeof(float), 256);
        if (p.n_chunks > 1 && d.q > 0) chunked.push_back(s);
    }
    size_t keys_begin = off;
    for (int32_t s : chunked) {
        sp[s].keys_off = off;
        off += align_up((size_t)sets[s].q * 2 * sizeof(unsigned long long), 256);
    }
    size_t keys_end = off;
    // work items per class, longest first
    std::map<std::tuple<int, int, int>, std::vector<std::pair<int64_t, BatchItem>>> classes;
    for (int s = 0; s < n_sets; ++s) {
        const SetPlan &p = sp[s];
        if (sets[s].q == 0) continue;
        auto &items = classes[std::make_tuple(p.mi.norm, p.mi.d, p.mi.dm)];
        for (int c = 0; c < p.n_chunks; ++c) {
            const int64_t t0 = (int64_t)c * p.tiles_per_chunk;
            const int64_t nt = std::min<int64_t>(p.tiles_per_chunk, p.n_tiles - t0);
            const int64_t cost = nt * p.tile;
            for (int64_t qb = 0; qb < p.qblocks; ++qb)
                items.push_back({cost, BatchItem{s, c, qb}});
        }
    }
    size_t items_off = off;
    size_t n_items_total = 0;
    for (auto &kv : classes) n_items_total += kv.second.size();
    if (n_items_total > 0xffffffffull) return LIP_E_SHAPE;
    off += align_up(n_items_total * sizeof(BatchItem), 256);
    const size_t args_off = off;
    off += align_up((size_t)std::max(n_sets, 1) * sizeof(FwdArgs), 256);
    const size_t stage_off = off;
    off += align_up((size_t)std::max(n_sets, 1) * sizeof(BatchStage), 256);
    const size_t chunked_off = off;
    off += align_up((size_t)std::max<size_t>(chunked.size(), 1) * sizeof(int32_t), 256);
    const size_t counters_off = off;
    off += align_up(std::max<size_t>(classes.size(), 1) * sizeof(unsigned int), 256);

    lip_plan *p = new lip_plan();
    p->tiles.resize(n_sets);
    for (int s = 0; s < n_sets; ++s)
        p->tiles[s] = lip_tile_cfg{sp[s].tile, sp[s].n_chunks, 4, sp[s].flags};
    if (hipGetDevice(&p->device) != hipSuccess || hipMalloc(&p->mem, off) != hipSuccess) {
        free_plan(p);
        return LIP_E_DEVICE;
    }
    char *base = (char *)p->mem;

    // descriptor tables (host side, then copied)
    std::vector<FwdArgs> args(n_sets);
    std::vector<BatchStage> stg(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        const SetPlan &q = sp[s];
        const lip_batch_desc &d = sets[s];
        FwdArgs a{};
        a.data = (const float *)(base + q.staged_off);
        a.n = d.n;
        a.n_tiles = q.n_tiles;
        a.tile = q.tile;
        a.tiles_per_chunk = q.tiles_per_chunk;
        a.n_chunks = q.n_chunks;
        a.l2_filter = (q.flags & LIP_TILE_L2_FILTER) ? 1 : 0;
        a.xq = d.xq;
        a.q = d.q;
        a.xf = q.mi.xf;
        a.xf.origin = (const float *)(base + q.origin_off);
        a.g = d.g;
        a.h_up = d.h_up;
        a.h_lo = d.h_lo;
        a.arg_up = d.arg_up;
        a.arg_lo = d.arg_lo;
        a.keys = q.n_chunks > 1 ? (unsigned long long *)(base + q.keys_off) : nullptr;
        args[s] = a;
        BatchStage b{};
        b.x = d.x;
        b.y = d.y;
        b.Mk = d.Mk;
        b.M = d.M;
        b.d = q.mi.d;
        b.l1_mon = q.mi.norm == LIP_L1 ? q.mi.dm : 0;
        b.n = d.n;
        b.n_pad = q.n_pad;
        b.xf = a.xf;
        b.origin = (float *)(base + q.origin_off);
        b.out = (float *)(base + q.staged_off);
        stg[s] = b;
    }
    std::vector<BatchItem> flat;
    flat.reserve(n_items_total);
    struct ClassRun {
        BatchLauncher launch;
        size_t first, count;
    };
    std::vector<ClassRun> runs;
    for (auto &kv : classes) {
        auto &v = kv.second;
        std::stable_sort(v.begin(), v.end(),
                         [](const std::pair<int64_t, BatchItem> &a,
                            const std::pair<int64_t, BatchItem> &b) { return a.first > b.first; });
        ClassRun r;
        r.launch = fwd_launchers(std::get<0>(kv.first), std::get<1>(kv.first),
                                 std::get<2>(kv.first)).batched;
        r.first = flat.size();
        r.count = v.size();
        for (auto &e : v) flat.push_back(e.second);
        runs.push_back(r);
    }
    bool ok = true;
    if (n_sets > 0) {
        ok = ok && hipMemcpy(base + args_off, args.data(), sizeof(FwdArgs) * n_sets,
                             hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(base + stage_off, stg.data(), sizeof(BatchStage) * n_sets,
                             hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!flat.empty())
        ok = ok && hipMemcpy(base + items_off, flat.data(), sizeof(BatchItem) * flat.size(),
                             hipMemcpyHostToDevice) == hipSuccess;
    if (!chunked.empty())
        ok = ok && hipMemcpy(base + chunked_off, chunked.data(), sizeof(int32_t) * chunked.size(),
                             hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        free_plan(p);
        return LIP_E_DEVICE;
    }

    // record the graph
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess ||
        hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        free_plan(p);
        return LIP_E_DEVICE;
    }
    hipStream_t cs = p->cap;
    unsigned int *counters = (unsigned int *)(base + counters_off);
    if (!runs.empty())
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, cs, counters, (int)runs.size(),
                           0u);
    if (keys_end > keys_begin) {
        const int64_t nk = (int64_t)((keys_end - keys_begin) / sizeof(unsigned long long));
        const int64_t g = std::min<int64_t>((nk + 255) / 256, 8192);
        hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)g), dim3(256), 0, cs,
                           (unsigned long long *)(base + keys_begin), nk, ~0ull);
    }
    if (n_sets > 0)
        hipLaunchKernelGGL(batched_stage_kernel, dim3((unsigned)std::min(n_sets, 4096)), dim3(256),
                           0, cs, (const BatchStage *)(base + stage_off), n_sets);
    for (size_t r = 0; r < runs.size(); ++r) {
        BatchArgs b{};
        b.sets = (const FwdArgs *)(base + args_off);
        b.items = (const BatchItem *)(base + items_off) + runs[r].first;
        b.n_items = (unsigned int)runs[r].count;
        b.counter = counters + r;
        // persistent: at most 4 workgroups (16 waves) per CU
        const int64_t waves = std::min<int64_t>((int64_t)runs[r].count, 256 * 16);
        runs[r].launch(b, dim3((unsigned)((waves + 3) / 4)), dim3(256), cs);
    }
    if (!chunked.empty())
        hipLaunchKernelGGL(batched_finalize_kernel,
                           dim3((unsigned)std::min<size_t>(chunked.size(), 4096)), dim3(256), 0, cs,
                           (const FwdArgs *)(base + args_off),
                           (const int32_t *)(base + chunked_off), (int)chunked.size());
    const hipError_t launch_err = hipGetLastError();
    if (hipStreamEndCapture(cs, &p->graph) != hipSuccess || launch_err != hipSuccess ||
        hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        free_plan(p);
        return LIP_E_DEVICE;
    }
    *plan = p;
    return LIP_OK;
}

extern "C" lip_status lip_plan_execute(lip_plan *plan, lip_stream stream)
{
    if (!plan || !plan->exec) return LIP_E_ARG;
    return dev_status(hipGraphLaunch(plan->exec, (hipStream_t)stream));
}

extern "C" lip_status lip_plan_tiles(const lip_plan *plan, int32_t set, lip_tile_cfg *cfg)
{
    if (!plan || !cfg) return LIP_E_ARG;
    if (set < 0 || set >= (int32_t)plan->tiles.size()) return LIP_E_SHAPE;
    *cfg = plan->tiles[set];
    return LIP_OK;
}

extern "C" lip_status lip_plan_destroy(lip_plan *plan)
{
    if (!plan) return LIP_OK;
    if (plan->cap) (void)hipStreamSynchronize(plan->cap);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return LIP_OK;
}

// ---- autotuner ------------------------------------------------------------------

namespace lip {

// Seeded synthetic data of the requested shape (uniform coordinates from an
// integer hash, smooth values); only the timing matters.
__global__ void synth_kernel(float *x, float *y, int64_t n, int d, uint32_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int j = 0; j < d; ++j) {
        uint32_t h = (uint32_t)(i * 2654435761u) ^ (uint32_t)(j * 40503u) ^ seed;
        h ^= h >> 16;
        h *= 0x7feb352du;
        h ^= h >> 15;
        h *= 0x846ca68bu;
        h ^= h >> 16;
        const float v = (float)(h >> 8) * (1.0f / 16777216.0f);
        x[i * d + j] = v;
        s += v;
    }
    if (y) y[i] = s * 0.5f;
}

}  // namespace lip

extern "C" lip_status lip_autotune(int32_t d, int32_t n_mon, int32_t norm, int64_t n, int64_t q,
                                   lip_stream stream, lip_tile_cfg *best)
{
    if (!best) return LIP_E_ARG;
    if (d < 1 || d > kMaxDim || n_mon < 0 || n_mon > d) return LIP_E_SHAPE;
    if (norm != LIP_L1 && norm != LIP_L2 && norm != LIP_LINF) return LIP_E_ARG;
    if (n < 1 || q < 1 || n > kMaxIndex - kMaxTile || q > kMaxIndex) return LIP_E_SHAPE;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int8_t> mon(d, 0);
    for (int i = d - n_mon; i < d; ++i) mon[i] = 1;
    lip_metric m{d, norm, nullptr, mon.data()};
    MetricInfo mi;
    lip_status st = parse_metric(&m, &mi);
    if (st != LIP_OK) return st;
    const size_t ws_bytes = lip_workspace_size(n, q, d, 0);
    float *x = nullptr, *y = nullptr, *xq = nullptr, *g = nullptr;
    void *ws = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (x) (void)hipFree(x);
        if (y) (void)hipFree(y);
        if (xq) (void)hipFree(xq);
        if (g) (void)hipFree(g);
        if (ws) (void)hipFree(ws);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&x, sizeof(float) * n * d) != hipSuccess ||
        hipMalloc(&y, sizeof(float) * n) != hipSuccess ||
        hipMalloc(&xq, sizeof(float) * q * d) != hipSuccess ||
        hipMalloc(&g, sizeof(float) * q) != hipSuccess || hipMalloc(&ws, ws_bytes) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return LIP_E_DEVICE;
    }
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, d,
                       1u);
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, xq,
                       (float *)nullptr, q, d, 2u);
    float best_ms = 1e30f;
    lip_tile_cfg best_cfg = tune_lookup(d, n_mon, norm, n, q);
    const int tiles[] = {16, 32, 64, 128};
    const int splits[] = {1, 2, 4, 8, 16, 32};
    const int waves[] = {1, 2, 4, 8};
    // flag sets: none; for l2 with monotone coordinates also the filter, and
    // the filter with the query order
    const int flag_sets[] = {0, LIP_TILE_L2_FILTER, LIP_TILE_L2_FILTER | LIP_TILE_QUERY_ORDER};
    const int n_flags = (norm == LIP_L2 && n_mon > 0) ? 3 : 1;
    for (int fl = 0; fl < n_flags; ++fl)
    for (int t : tiles)
        for (int sp : splits)
            for (int w : waves) {
                if (w > sp) continue;  // the same launch as w = sp
                lip_tile_cfg c{t, sp, w, flag_sets[fl]};
                // warm-up, then the mean of 3 runs
                st = run_bounds(mi, x, y, n, 1.0f, nullptr, xq, q, g, nullptr, nullptr, nullptr,
                                nullptr, ws, ws_bytes, c, s);
                if (st != LIP_OK) {
                    cleanup();
                    return st;
                }
                if (hipEventRecord(e0, s) != hipSuccess) {
                    cleanup();
                    return LIP_E_DEVICE;
                }
                for (int r = 0; r < 3; ++r)
                    (void)run_bounds(mi, x, y, n, 1.0f, nullptr, xq, q, g, nullptr, nullptr,
                                     nullptr, nullptr, ws, ws_bytes, c, s);
                float ms = 0.0f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    cleanup();
                    return LIP_E_DEVICE;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best_cfg = c;
                }
            }
    cleanup();
    st = lip_tune_set(d, n_mon, norm, n, q, &best_cfg);
    if (st != LIP_OK) return st;
    tune_autosave();
    *best = best_cfg;
    return LIP_OK;
}
