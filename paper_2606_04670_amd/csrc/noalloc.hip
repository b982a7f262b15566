// lip_fit_eval_noalloc: the bound path of lip_fit_eval with its scratch
// memory (coordinate origin, staged records, split partials) in a
// file-scope device array instead of a caller workspace, for callers that
// cannot allocate (code under stream capture, tight serving loops).
//
// Each GPU the library runs on holds one copy of `scratch` (kScratchBytes)
// until the process ends.  Its device address is resolved once per device
// with hipGetSymbolAddress, with that device current, and kept; host code
// never passes the array's own name to a kernel (on the host it is only a
// stand-in for the symbol).  The kernels write every scratch byte they read
// in the same call, so nothing needs clearing between calls.  Calls that
// overlap on one GPU (different streams or host threads without ordering)
// share the array and race; calls on one stream are ordered and safe.
#include <mutex>

#include "host_common.hpp"

namespace lip {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of this device's copy of `scratch`.
lip_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LIP_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LIP_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LIP_OK;
}

}  // namespace

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_fit_eval_noalloc(const lip_metric *metric, const float *x,
                                           const float *y, int64_t n, float M, const float *Mk,
                                           const float *xq, int64_t q, float *g, float *h_up,
                                           float *h_lo, int32_t *arg_up, int32_t *arg_lo,
                                           uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = validate_bounds(metric, x, y, n, M, Mk, xq, q, flags, &mi);
    if (st != LIP_OK) return st;
    if (flags != 0 || mi.regional) return LIP_E_UNSUPPORTED;
    // the staged data alone must fit; then the largest data split whose
    // partial results fit as well
    const size_t base = kOriginBytes + staged_bytes(n, mi.d);
    if (base > kScratchBytes) return LIP_E_SHAPE;
    if (q == 0) return LIP_OK;
    lip_tile_cfg cfg = tune_lookup(mi.d, mi.dm, mi.norm, n, q);
    cfg.flags &= ~LIP_TILE_QUERY_ORDER;  // its keys would need scratch of their own
    for (;;) {
        const size_t part = fwd_partial_bytes(make_fwd_plan(mi, n, q, cfg), q);
        if (base + part <= kScratchBytes || cfg.split <= 1) break;
        cfg.split /= 2;
    }
    void *ws = nullptr;
    st = scratch_address(&ws);
    if (st != LIP_OK) return st;
    return run_bounds(mi, x, y, n, M, Mk, xq, q, g, h_up, h_lo, arg_up, arg_lo, ws, kScratchBytes,
                      cfg, (hipStream_t)stream);
}
