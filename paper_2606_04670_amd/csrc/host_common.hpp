// Host-side helpers shared by the entry points: argument validation (no HIP
// call is made before it passes), metric -> coordinate transform, tiling
// choices and workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lipfit.h"
#include "lip_internal.hpp"

namespace lip {

constexpr int kMaxTile = 256;                 // largest argmin tile (records)
constexpr int kMaxChunks = 64;                // largest data split
constexpr int kMaxFwdWaves = 8;               // waves per workgroup of the bound kernel
constexpr int64_t kMaxPartials = 1ll << 23;   // n_chunks * q cap (per bound)
constexpr int64_t kMaxIndex = 2147483647ll;   // indices are int32

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Every path that stages coordinates (bound kernels, k-best, step-function
// forward, smoothing, regional bounds) takes this many bytes off the front
// of its workspace for the coordinate origin (launch_origin).
constexpr size_t kOriginBytes = align_up(kOriginAreaBytes, 256);

// Launches the origin reduction for the data x [n][d] into `area` and
// returns xf with its origin pointer set.
inline lip_status origin_for(const float *x, int64_t n, int d, Xform &xf, void *area,
                             hipStream_t s)
{
    xf.origin = (const float *)area;
    return launch_origin(x, n, d, xf.perm, (float *)area, s) == hipSuccess ? LIP_OK
                                                                            : LIP_E_DEVICE;
}

// Validated metric: transform of the coordinates and monotone count.
struct MetricInfo {
    int d = 0;
    int norm = 0;
    int dm = 0;          // number of monotone coordinates
    Xform xf{};          // free coordinates first, then monotone ones
    double w[kMaxDim];   // weights (for the FP64 passes)
    int8_t mon[kMaxDim]; // original monotonicity (for the FP64 passes)
    // monotonicity on parts of the domain (some kind is a LIP_MON_CASE_*):
    // per coordinate the intervals where f is not decreasing (nd) and not
    // increasing (ni), [s, t] with infinite ends allowed, empty as [+inf, -inf]
    bool regional = false;
    float nd_s[kMaxDim], nd_t[kMaxDim], ni_s[kMaxDim], ni_t[kMaxDim];
};

// Validates the metric; the LIP_MON_CASE_* kinds are accepted only with
// allow_regional (else LIP_E_UNSUPPORTED).
lip_status parse_metric(const lip_metric *m, MetricInfo *out, bool allow_regional = false);

// Resolved tiling for one bound-kernel launch.
struct FwdPlan {
    int R = 0;
    int tile = 64;
    int waves = 4;           // waves per workgroup (d <= 8: chunks merged in LDS)
    int64_t n_pad = 0, n_tiles = 0;
    int tiles_per_chunk = 0;
    int n_chunks = 1;        // chunks launched (a multiple of waves, the last ones may be empty)
    int part_chunks = 1;     // partial results per query the combine kernel reduces (1: none)
    int64_t grid = 0;
};

// Bytes of the query order of the bound path (sorted keys, box scratch and
// the queries in that order).
inline size_t query_order_bytes(int64_t q, int d)
{
    return align_up((size_t)sort_len(q > 0 ? q : 1) * 8, 256) + 256 +
           align_up((size_t)(q > 0 ? q : 1) * (size_t)d * 4, 256);
}

// Bytes of the split partials of a plan (values and indices of both bounds).
inline size_t fwd_partial_bytes(const FwdPlan &p, int64_t q)
{
    if (p.part_chunks <= 1) return 0;
    return 2 * align_up((size_t)p.part_chunks * (size_t)q * 2 * sizeof(float), 256);
}

// Tile parameters (tune.cpp): the tuning table's entry for the shape and
// size class of (n, q), else an entry set for every size, else the default.
lip_tile_cfg default_tile_cfg(int d, int dm, int norm, int64_t n, int64_t q);
lip_tile_cfg tune_lookup(int d, int dm, int norm, int64_t n, int64_t q);
// Writes the table to the file named by LIPFIT_TUNE_CACHE, if set.
void tune_autosave();
FwdPlan make_fwd_plan(const MetricInfo &mi, int64_t n, int64_t q, const lip_tile_cfg &cfg);

// Workspace layout of the bound path.
size_t staged_bytes(int64_t n, int d);
size_t partial_bytes(int64_t q);

FwdLaunchers fwd_launchers(int norm, int d, int dm);

// Runs the bound path (stage -> fused kernel -> optional combine) on a
// validated problem.  ws must hold staged_bytes + partial_bytes.
lip_status run_bounds(const MetricInfo &mi, const float *x, const float *y, int64_t n, float M,
                      const float *Mk, const float *xq, int64_t q, float *g, float *h_up,
                      float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws, size_t ws_bytes,
                      const lip_tile_cfg &cfg, hipStream_t stream);

// Argument checks of lip_bounds / lip_fit_eval (no HIP call).
lip_status validate_bounds(const lip_metric *metric, const float *x, const float *y, int64_t n,
                           float M, const float *Mk, const float *xq, int64_t q, uint32_t flags,
                           MetricInfo *mi);

// BF16-MFMA l2 variant of run_bounds (bf16_l2.hip).
lip_status run_bounds_bf16(const MetricInfo &mi, const float *x, const float *y, int64_t n, float M,
                           const float *Mk, const float *xq, int64_t q, float *g, float *h_up,
                           float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws,
                           size_t ws_bytes, hipStream_t stream);
size_t bf16_extra_bytes(int64_t n, int64_t q, int d);

// Workspace needs of the other passes.
size_t data_side_ws_bytes(int64_t n, int d);
size_t backward_ws_bytes(int64_t n);
size_t local_ws_bytes(int64_t n, int64_t q, int d);
size_t smooth_ws_bytes(int64_t n, int d);
size_t topk_ws_bytes(int64_t n, int64_t q, int d);
size_t reg_ws_bytes(int64_t n, int64_t q, int d);

// Bound path with monotonicity on parts of the domain (bounds_reg.hip).
lip_status run_bounds_reg(const MetricInfo &mi, const float *x, const float *y, int64_t n,
                          float M, const float *Mk, const float *xq, int64_t q, float *g,
                          float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws,
                          size_t ws_bytes, hipStream_t stream);

lip_status check_finite(const float *const *arrays, const int64_t *counts, int n_arrays,
                        void *ws, hipStream_t stream);

inline lip_status dev_status(hipError_t e) { return e == hipSuccess ? LIP_OK : LIP_E_DEVICE; }

}  // namespace lip
