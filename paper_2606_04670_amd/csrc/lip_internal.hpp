// Internal declarations shared by the host library and the kernel
// translation units.  Not part of the public ABI (include/lipfit.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lip_device.hpp"

namespace lip {

// Queries per lane for a dimension: keeps R (D + 7) around 80-100 VGPRs.
constexpr int rows_for_dim(int D) { return D <= 2 ? 12 : (D <= 4 ? 8 : (D <= 6 ? 6 : 4)); }
// Largest dimension whose single-set bound kernel merges the chunks of a
// workgroup in LDS (bounds_fwd.hpp).
constexpr int kFwdMergeMaxDim = 8;
// Waves per workgroup above that dimension (the kernel's launch bound).
constexpr int kFwdPlainMaxWaves = 4;

// Arguments of the fused bound kernel (see bounds_fwd.hpp).
struct FwdArgs {
    const float *data;       // staged records [n_pad][D + 3]
    int64_t n;               // real data count (n <= n_pad)
    int64_t n_tiles;         // n_pad / tile
    int32_t tile;            // records per argmin tile (multiple of 8)
    int32_t tiles_per_chunk;
    int32_t n_chunks;        // chunks launched (d <= 8: a multiple of the waves per workgroup)
    int32_t l2_filter;       // l2 with monotone coordinates: root-free filter (bounds_fwd.hpp)
    const float *xq;         // [q][D] row-major, untransformed
    int64_t q;
    Xform xf;                // query transform (same as the staging one)
    float *g, *h_up, *h_lo;  // outputs (n_chunks == 1), any may be NULL
    int32_t *arg_up, *arg_lo;
    float *part_v;           // [2][parts][q] partial values (parts = n_chunks / waves at
                             // d <= 8, else n_chunks; parts > 1)
    int32_t *part_i;         // [2][parts][q] partial indices
    unsigned long long *keys;  // [2][q] packed keys (batched plans, n_chunks > 1)
    // query order: xq holds the queries permuted, position p being query
    // (uint32)qorder[p] (sorted (Morton code << 32 | index) keys); partials
    // are kept by position, outputs written by query index.  NULL: xq in
    // index order.
    const unsigned long long *qorder;
};

// One work item of a batched plan: one wave's queries of one set against
// one data chunk.
struct BatchItem {
    int32_t set;
    int32_t chunk;
    int64_t qblock;
};

struct BatchArgs {
    const FwdArgs *sets;
    const BatchItem *items;
    unsigned int n_items;
    unsigned int *counter;
};

typedef void (*FwdLauncher)(const FwdArgs &, dim3, dim3, hipStream_t);
typedef void (*BatchLauncher)(const BatchArgs &, dim3, dim3, hipStream_t);

struct FwdLaunchers {
    FwdLauncher plain;
    BatchLauncher batched;
};

// Staging of the data set into bound-kernel records (stage.hip).
struct StageArgs {
    const float *x;   // [n][D] row-major
    const float *y;   // [n]
    const float *Mk;  // [n] or NULL
    float M;          // global constant when Mk == NULL
    int32_t l1_mon;   // number of monotone coordinates when the norm is l1, else 0
    int64_t n, n_pad;
    Xform xf;
    float *out;       // [n_pad][D + 3]
};

// Chunk-partial reduction (stage.hip).
struct CombineArgs {
    const float *part_v;
    const int32_t *part_i;
    int64_t q;
    int32_t n_chunks;
    int32_t pad0;
    float *g, *h_up, *h_lo;
    int32_t *arg_up, *arg_lo;
    const unsigned long long *qorder;  // partial position -> query index, or NULL
};

// Coordinate origin (stage.hip): the area holds origin[kMaxDim] (permuted
// order, perm[j] = original coordinate of staged coordinate j) followed by
// the pass-1 partials; kOriginAreaBytes of device memory.
constexpr int kOriginBlocks = 240;
constexpr size_t kOriginAreaBytes = (size_t)(kMaxDim * 4 + kOriginBlocks * kMaxDim * 2) * 4;
hipError_t launch_origin(const float *x, int64_t n, int d, const int32_t *perm, float *area,
                         hipStream_t s);

hipError_t launch_stage(int d, const StageArgs &a, hipStream_t s);
hipError_t launch_combine(const CombineArgs &a, hipStream_t s);
hipError_t launch_nonfinite(const float *v, int64_t n, int *flag, hipStream_t s);
hipError_t launch_fill_i32(int *p, int64_t n, int v, hipStream_t s);

// Ascending in-place sort of P 64-bit keys, P = sort_len(n) (a power of two
// >= max(n, 1024); the caller pads with ~0) (sort.hip).
int64_t sort_len(int64_t n);
hipError_t launch_sort_u64(unsigned long long *keys, int64_t P, hipStream_t s);
// Morton order of q queries [q][d] into P = sort_len(q) sorted keys; bb is
// 2 kMaxDim words of scratch (stage.hip).
hipError_t launch_query_order(const float *xq, int64_t q, int d, unsigned int *bb,
                              unsigned long long *keys, int64_t P, hipStream_t s);
// out[p] = xq[(uint32)keys[p]] for p < q (rows of d floats).
hipError_t launch_query_gather(const float *xq, int64_t q, int d, const unsigned long long *keys,
                               float *out, hipStream_t s);

FwdLaunchers fwd_launchers_l1(int d, int dm);
FwdLaunchers fwd_launchers_l2(int d, int dm);
FwdLaunchers fwd_launchers_linf(int d, int dm);

}  // namespace lip
