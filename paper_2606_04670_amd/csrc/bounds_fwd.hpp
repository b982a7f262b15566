// Fused all-pairs bound kernel: distance -> bound candidates -> min / max ->
// first attaining index, for Eq. (2)-(3), without materialising the
// query x data matrix.
//
// Work decomposition.  A wave owns 64*R queries (R per lane, held in VGPRs)
// and one chunk of the data (a run of whole tiles).  The data are streamed
// in groups of 4 records through scalar loads (the next group is requested
// before the current one is used); every record is used by all R queries of
// all 64 lanes before it is dropped.  Workgroups are numbered chunk-fastest,
// so with a chunk count that divides 8 or is a multiple of 8, each XCD
// (blockIdx % 8) always reads the same chunks and keeps them in its own L2.
//
// Argmin without per-pair index tracking.  The inner loop keeps only the
// running min/max.  At the end of each tile a lane records the tile id if
// its running value strictly improved during that tile.  The attaining index
// is then the first index in the last improving tile whose candidate equals
// the final value; a re-scan of that one tile per query with the identical
// arithmetic (pair_bounds) finds it.  Ties therefore resolve to the lowest
// index, as in the definition.
//
// Chunks of one query block (d <= 8).  The waves of a workgroup take the
// same 64 R queries and consecutive data chunks, and merge their results as
// packed (value, index) 64-bit keys with LDS atomic minima (lowest index on
// ties); the workgroup writes the final values, or, when the data are split
// into more chunks than it has waves, one partial result per group of
// chunks, which a combine kernel reduces in group order (strict comparisons
// keep the lower index on ties).  More waves per workgroup fill the chip like
// a global split of the same chunk count, but read each query from HBM once
// and write no partials.  At d >= 9 the records of two scalar-load groups
// leave no scalar registers for the merge's state, so there the waves of a
// workgroup take different query blocks of one chunk and every chunk writes
// partials.  Batched plans merge the chunks of a set with global atomics on
// the same keys.

#pragma once

#include <array>
#include <climits>
#include <utility>

#include "lip_device.hpp"
#include "lip_internal.hpp"

namespace lip {

// Records per scalar-load group: two groups (current and next) must fit in
// the SGPR file next to the loop state.  Tiles are multiples of 8 records, so
// a tile always holds an even number of groups.
constexpr int group_for_dim(int D) { return D <= 5 ? 4 : 2; }

template <int D, int DM, int NORM>
struct FwdTraits {
    static constexpr int R = rows_for_dim(D);
    static constexpr bool kQm = (NORM == kNormL1 && DM > 0);
};

template <int D>
__device__ __forceinline__ void load_group(cfloat_ptr p, float (&v)[group_for_dim(D) * Rec<D>::S])
{
#pragma unroll
    for (int i = 0; i < group_for_dim(D) * Rec<D>::S; ++i) v[i] = p[i];
}

template <int D, int DM, int NORM>
__device__ __forceinline__ void eval_group(const float (&v)[group_for_dim(D) * Rec<D>::S],
                                           const float (&q)[D], float qm, float big, float &hu,
                                           float &hl)
{
    constexpr int S = Rec<D>::S;
    constexpr int kGroup = group_for_dim(D);
    float uu[kGroup], ll[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
        float xk[D];
#pragma unroll
        for (int j = 0; j < D; ++j) xk[j] = v[g * S + j];
        pair_bounds<D, DM, NORM>(q, qm, xk, v[g * S + Rec<D>::Y], v[g * S + Rec<D>::M],
                                 v[g * S + Rec<D>::YU], big, uu[g], ll[g]);
    }
#pragma unroll
    for (int g = 0; g < kGroup; g += 2) {
        hu = fminf(fminf(hu, uu[g]), uu[g + 1]);
        hl = fmaxf(fmaxf(hl, ll[g]), ll[g + 1]);
    }
}

// A wave-uniform value computed by the vector unit, read into a scalar
// register.
__device__ __forceinline__ float uniform_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// l2 with monotone coordinates, filtered: the exact candidates need two
// square roots per pair (v_sqrt_f32 issues at a quarter of the VALU rate and
// takes about half of the pair's time), but few records can change a row's
// running bounds.  Each pair first gets root-free bounds of its candidates
// from the largest weighted component of each distance; a record is
// evaluated exactly (pair_bounds) for a row of 64 queries only if some lane
// of the row could improve.  Results are identical to the unfiltered loop:
//   * with c_max the largest component (of the rounded differences the exact
//     path squares), the exact path's rounded sum of squares is at least
//     fl(c_max^2) (every step adds a non-negative term, rounding is
//     monotone), which is >= c_max^2 (1 - 2^-24) when c_max >= 2^-60 (no
//     underflow); v_sqrt_f32 errs by far less than 2^-21 relative (taken as
//     its bound), so the exact root s >= c_max (1 - 2^-20);
//   * per record, Ms = fl(M (1 - 2^-19)) <= M (1 - 2^-19 + 2^-24) and
//     Ms c_max <= M s; with t = max(|y| 2^-23, M 2^-58, 2^-126) (>= ulp(y),
//     so fl(y - t) <= y - 0.49 t <= y - M 2^-60), ylo = fl(y - t) and
//     yhi = fl(y + t): for c_max >= 2^-60, Ms c_max + ylo <= M s + y; for
//     c_max < 2^-60 (s may be 0), Ms c_max + ylo <= M 2^-60 + y - M 2^-60 <= y;
//     fma is monotone, hence fma(Ms, c_max, ylo) <= fma(M, s, y) = u, and
//     fma(-Ms, c'_max, yhi) >= l likewise;
//   * a record is skipped for a row only when every lane's bound is >= its
//     running minimum and <= its running maximum, so its exact candidates
//     could not have changed either (ties included: a tie leaves the running
//     value as it is, and the attaining index comes from the re-scan).
// The per-record values are a few VALU operations shared by all R rows (read
// into scalar registers); per pair the filter is 4 differences, 3 maxima,
// 2 FMA and 2 compares.
// Per-record constants of the filter (wave-uniform, moved to scalar
// registers so that the rows share them without holding vector registers).
struct L2fRec {
    float ms, ylo, yhi;
};
__device__ __forceinline__ L2fRec l2f_record(float yk, float mk)
{
    const float t = fmaxf(fmaxf(fabsf(yk) * 0x1p-23f, mk * 0x1p-58f), 0x1p-126f);
    return L2fRec{uniform_f32(mk * (1.0f - 0x1p-19f)), uniform_f32(yk - t), uniform_f32(yk + t)};
}

// Root-free bounds ulb <= u and lub >= l of one pair (the first DF = D - DM
// coordinates free, the rest increasing).
template <int D, int DM>
__device__ __forceinline__ void l2f_bounds(const float (&q)[D], const float (&xk)[D],
                                           const L2fRec &c, float &ulb, float &lub)
{
    constexpr int DF = D - DM;
    float f = 0.0f;
#pragma unroll
    for (int i = 0; i < DF; ++i) f = fmaxf(f, fabsf(q[i] - xk[i]));
    float su = f, sl = f;
#pragma unroll
    for (int i = DF; i < D; ++i) {
        const float dl = q[i] - xk[i];
        su = fmaxf(su, dl);
        sl = fmaxf(sl, -dl);
    }
    ulb = fmaf(c.ms, su, c.ylo);
    lub = fmaf(-c.ms, sl, c.yhi);
}

template <int D, int DM, int R>
__device__ __forceinline__ void eval_group_l2f(const float (&v)[group_for_dim(D) * Rec<D>::S],
                                               const float (&q)[R][D], float big,
                                               float (&hu)[R], float (&hl)[R])
{
    constexpr int S = Rec<D>::S;
    constexpr int kGroup = group_for_dim(D);
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
        float xk[D];
#pragma unroll
        for (int j = 0; j < D; ++j) xk[j] = v[g * S + j];
        const float yk = v[g * S + Rec<D>::Y], mk = v[g * S + Rec<D>::M];
        const L2fRec c = l2f_record(yk, mk);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float ulb, lub;
            l2f_bounds<D, DM>(q[r], xk, c, ulb, lub);
            if (__builtin_amdgcn_ballot_w64((ulb < hu[r]) | (lub > hl[r]))) {
                float u, l;
                pair_bounds<D, DM, kNormL2>(q[r], 0.0f, xk, yk, mk, yk, big, u, l);
                hu[r] = __builtin_amdgcn_fmed3f(hu[r], u, -big);  // min, no canonicalisation
                hl[r] = __builtin_amdgcn_fmed3f(hl[r], l, big);   // max
            }
        }
    }
}

// One group of records for all R rows of a lane: filtered (l2 with monotone
// coordinates, when the launch asks for it) or plain.  Without monotone
// coordinates the filter is not compiled in: there it was slower than the
// plain loop, and its branch alone cost the plain loop registers.
template <int D, int DM, int NORM, int R>
__device__ __forceinline__ void eval_group_rows(const FwdArgs &a,
                                                const float (&v)[group_for_dim(D) * Rec<D>::S],
                                                const float (&qv)[R][D], const float (&qm)[R],
                                                float big, float (&hu)[R], float (&hl)[R])
{
    if constexpr (NORM == kNormL2 && DM > 0) {
        if (a.l2_filter) {
            eval_group_l2f<D, DM, R>(v, qv, big, hu, hl);
            return;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) eval_group<D, DM, NORM>(v, qv[r], qm[r], big, hu[r], hl[r]);
}

// One lane's scan of its R queries (q0 + 64 r + lane) over data chunk
// `chunk` (non-empty): running min / max and the attaining indices, handed
// to emit(hu, hl, au, al).  The arrays stay local to the scan: passing them
// out by reference cost registers in the main loop at d >= 9.
template <int D, int DM, int NORM, class Emit>
__device__ __forceinline__ void fwd_scan(const FwdArgs &a, int chunk, int64_t q0, Emit &&emit)
{
    constexpr int S = Rec<D>::S;
    constexpr int R = FwdTraits<D, DM, NORM>::R;
    constexpr int kGroup = group_for_dim(D);
    constexpr int GS = kGroup * S;
    const int lane = threadIdx.x & 63;

    const float big = opaque_inf();
    float qv[R][D];
    float qm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t qi = q0 + r * 64 + lane;
        qi = qi < a.q ? qi : a.q - 1;
        const float *src = a.xq + qi * D;
#pragma unroll
        for (int j = 0; j < D; ++j) qv[r][j] = xf_coord(a.xf, src, j);
        qm[r] = query_mon_sum<D, DM>(qv[r]);
    }

    const int64_t t0 = (int64_t)chunk * a.tiles_per_chunk;
    int64_t t1 = t0 + a.tiles_per_chunk;
    t1 = t1 < a.n_tiles ? t1 : a.n_tiles;
    const int tile = a.tile;
    const int gpt = tile / kGroup;  // groups per tile

    float hu[R], hl[R], pu[R], pl[R];
    int tu[R], tl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        hu[r] = __builtin_inff();
        hl[r] = -__builtin_inff();
        pu[r] = hu[r];
        pl[r] = hl[r];
        tu[r] = (int)t0;
        tl[r] = (int)t0;
    }

    // Double-buffered scalar loads: group gi+1 is requested before group gi
    // is evaluated.  A tile holds an even number of groups, so the loop body
    // handles two groups and the tile-end bookkeeping follows the second.
    const cfloat_ptr base = as_const(a.data);
    const int64_t g0 = t0 * gpt, g1 = t1 * gpt;
    float ga[GS], gb[GS];
    if (g0 < g1) load_group<D>(base + g0 * GS, ga);
    int left = gpt / 2;
    int64_t t = t0;
    for (int64_t gi = g0; gi < g1; gi += 2) {
        load_group<D>(base + (gi + 1) * GS, gb);
        eval_group_rows<D, DM, NORM, R>(a, ga, qv, qm, big, hu, hl);
        const int64_t gn = gi + 2 < g1 ? gi + 2 : gi + 1;
        load_group<D>(base + gn * GS, ga);
        eval_group_rows<D, DM, NORM, R>(a, gb, qv, qm, big, hu, hl);
        if (--left == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                tu[r] = hu[r] < pu[r] ? (int)t : tu[r];
                tl[r] = hl[r] > pl[r] ? (int)t : tl[r];
                pu[r] = hu[r];
                pl[r] = hl[r];
            }
            left = gpt / 2;
            ++t;
        }
    }

    // Re-scan the last improving tile of each query for the first index that
    // attains the final value (descending scan: the last hit is the lowest).
    int au[R], al[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t bu = (int64_t)tu[r] * tile, bl = (int64_t)tl[r] * tile;
        int iu = INT_MAX, il = INT_MAX;
#pragma unroll 2
        for (int k = tile - 1; k >= 0; --k) {
            const float *ru = a.data + (bu + k) * S;
            const float *rl = a.data + (bl + k) * S;
            float xu[D], xl[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                xu[j] = ru[j];
                xl[j] = rl[j];
            }
            float u, l, unused;
            pair_bounds<D, DM, NORM>(qv[r], qm[r], xu, ru[Rec<D>::Y], ru[Rec<D>::M], ru[Rec<D>::YU],
                                     big, u, unused);
            pair_bounds<D, DM, NORM>(qv[r], qm[r], xl, rl[Rec<D>::Y], rl[Rec<D>::M], rl[Rec<D>::YU],
                                     big, unused, l);
            iu = (u == hu[r]) ? (int)(bu + k) : iu;
            il = (l == hl[r]) ? (int)(bl + k) : il;
        }
        au[r] = iu;
        al[r] = il;
    }
    emit(hu, hl, au, al);
}

// One wave's work item of a batched plan: queries [64 R qblock, 64 R
// (qblock + 1)) against data chunk `chunk`.  Outputs: final values (one
// chunk) or packed (value, index) keys merged with atomics (a.keys).
template <int D, int DM, int NORM>
__device__ __forceinline__ void fwd_wave(const FwdArgs &a, int chunk, int64_t qblock)
{
    constexpr int R = FwdTraits<D, DM, NORM>::R;
    const int lane = threadIdx.x & 63;
    const int64_t q0 = qblock * (64 * R);
    if (q0 >= a.q) return;  // wave-uniform: no query of this wave exists

    fwd_scan<D, DM, NORM>(a, chunk, q0, [&](const float(&hu)[R], const float(&hl)[R], const int(&au)[R], const int(&al)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t qi = q0 + r * 64 + lane;
            if (qi >= a.q) continue;
            if (a.n_chunks == 1) {
                if (a.g) a.g[qi] = 0.5f * (hu[r] + hl[r]);
                if (a.h_up) a.h_up[qi] = hu[r];
                if (a.h_lo) a.h_lo[qi] = hl[r];
                if (a.arg_up) a.arg_up[qi] = au[r];
                if (a.arg_lo) a.arg_lo[qi] = al[r];
            } else {
                atomicMin(a.keys + qi, up_key(hu[r], au[r]));
                atomicMin(a.keys + a.q + qi, lo_key(hl[r], al[r]));
            }
        }
    });
}

// One workgroup of the single-set kernel, d <= 8: workgroup b takes
// queries [64 R (b / outer), 64 R (b / outer + 1)) and, with outer = n_chunks
// / waves, wave w takes chunk oc waves + w of oc = b % outer (chunks past the
// data are empty); with outer > 1 the merged result is partial number oc of
// the combine kernel.  d >= 9: wave w takes queries [64 R qb, 64 R (qb + 1))
// with qb = (b / n_chunks) waves + w and chunk b % n_chunks, and writes that
// chunk's partials (or the final values with one chunk).
constexpr bool fwd_merges(int D) { return D <= kFwdMergeMaxDim; }

template <int D, int DM, int NORM>
__device__ __forceinline__ void fwd_block_plain(const FwdArgs &a)
{
    constexpr int R = FwdTraits<D, DM, NORM>::R;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int chunk = (int)(blockIdx.x % (unsigned)a.n_chunks);
    const int64_t q0 = ((int64_t)(blockIdx.x / (unsigned)a.n_chunks) * nw + wave) * (64 * R);
    if (q0 >= a.q) return;  // wave-uniform
    fwd_scan<D, DM, NORM>(a, chunk, q0, [&](const float(&hu)[R], const float(&hl)[R], const int(&au)[R], const int(&al)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t qi = q0 + r * 64 + lane;
            if (qi >= a.q) continue;
            if (a.n_chunks == 1) {
                const int64_t qo = a.qorder ? (int64_t)(uint32_t)a.qorder[qi] : qi;
                if (a.g) a.g[qo] = 0.5f * (hu[r] + hl[r]);
                if (a.h_up) a.h_up[qo] = hu[r];
                if (a.h_lo) a.h_lo[qo] = hl[r];
                if (a.arg_up) a.arg_up[qo] = au[r];
                if (a.arg_lo) a.arg_lo[qo] = al[r];
            } else {
                const int64_t o = (int64_t)chunk * a.q + qi;
                const int64_t o2 = ((int64_t)a.n_chunks + chunk) * a.q + qi;
                a.part_v[o] = hu[r];
                a.part_i[o] = au[r];
                a.part_v[o2] = hl[r];
                a.part_i[o2] = al[r];
            }
        }
    });
}

template <int D, int DM, int NORM>
__device__ __forceinline__ void fwd_block_merge(const FwdArgs &a)
{
    constexpr int R = FwdTraits<D, DM, NORM>::R;
    __shared__ unsigned long long mk[2][64 * R];
    // wave index is wave-uniform; readfirstlane lets the compiler keep every
    // loop counter and address derived from it in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int outer = a.n_chunks / nw;
    const int oc = (int)(blockIdx.x % (unsigned)outer);
    const int64_t q0 = (int64_t)(blockIdx.x / (unsigned)outer) * (64 * R);
    if (q0 >= a.q) return;  // workgroup-uniform
    for (int i = threadIdx.x; i < 2 * 64 * R; i += blockDim.x) (&mk[0][0])[i] = ~0ull;
    __syncthreads();
    const int chunk = oc * nw + wave;
    if ((int64_t)chunk * a.tiles_per_chunk < a.n_tiles) {  // wave-uniform
        fwd_scan<D, DM, NORM>(a, chunk, q0, [&](const float(&hu)[R], const float(&hl)[R], const int(&au)[R], const int(&al)[R]) {
            const int lane = threadIdx.x & 63;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                atomicMin(&mk[0][r * 64 + lane], up_key(hu[r], au[r]));
                atomicMin(&mk[1][r * 64 + lane], lo_key(hl[r], al[r]));
            }
        });
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * R; i += blockDim.x) {
        const int64_t qi = q0 + i;
        if (qi >= a.q) break;
        float vu, vl;
        int iu, il;
        decode_keys(mk[0][i], mk[1][i], vu, iu, vl, il);
        if (outer == 1) {
            const int64_t qo = a.qorder ? (int64_t)(uint32_t)a.qorder[qi] : qi;
            if (a.g) a.g[qo] = 0.5f * (vu + vl);
            if (a.h_up) a.h_up[qo] = vu;
            if (a.h_lo) a.h_lo[qo] = vl;
            if (a.arg_up) a.arg_up[qo] = iu;
            if (a.arg_lo) a.arg_lo[qo] = il;
        } else {
            const int64_t o = (int64_t)oc * a.q + qi;
            const int64_t o2 = ((int64_t)outer + oc) * a.q + qi;
            a.part_v[o] = vu;
            a.part_i[o] = iu;
            a.part_v[o2] = vl;
            a.part_i[o2] = il;
        }
    }
}

template <int D, int DM, int NORM>
__device__ __forceinline__ void fwd_block(const FwdArgs &a)
{
    if constexpr (fwd_merges(D))
        fwd_block_merge<D, DM, NORM>(a);
    else
        fwd_block_plain<D, DM, NORM>(a);
}

// Workgroups of up to 8 waves where chunks merge, else up to 4.
constexpr int fwd_max_threads(int D) { return fwd_merges(D) ? 512 : 64 * kFwdPlainMaxWaves; }

template <int D, int DM, int NORM>
__global__ void __launch_bounds__(fwd_max_threads(D)) bounds_fwd_kernel(FwdArgs a)
{
    fwd_block<D, DM, NORM>(a);
}

// The same kernel held to 128 VGPRs (4 waves per SIMD) for the norms and
// dimensions where that costs no spills (l2 and linf, d = 3..8; the l1 form
// with its extra per-query sum spills): more waves to hide the latency of
// the square roots and of the scalar loads.
template <int D, int DM, int NORM>
__global__ void __launch_bounds__(fwd_max_threads(D)) __attribute__((amdgpu_waves_per_eu(4)))
bounds_fwd_kernel_o4(FwdArgs a)
{
    fwd_block<D, DM, NORM>(a);
}

constexpr bool fwd_use_o4(int D, int NORM) { return NORM != kNormL1 && D >= 3 && D <= 8; }

// d >= 9 (4 rows per lane) held to 168 VGPRs, 3 waves per SIMD: the
// unconstrained allocation takes a few registers more than that at some
// dimensions (d = 15 keeps it: under the cap it spills to scratch).
template <int D, int DM, int NORM>
__global__ void __launch_bounds__(fwd_max_threads(D)) __attribute__((amdgpu_waves_per_eu(3)))
bounds_fwd_kernel_o3(FwdArgs a)
{
    fwd_block<D, DM, NORM>(a);
}

constexpr bool fwd_use_o3(int D) { return D >= 9 && D != 15; }

// Persistent kernel for many independent data sets of one shape class
// (d, monotone count, norm): every wave repeatedly takes the next work item
// (set, query block, data chunk) from a counter; the items are ordered
// longest first.  Each item runs the same wave body as bounds_fwd_kernel, so
// the results are identical to per-set launches.
template <int D, int DM, int NORM>
__global__ void __launch_bounds__(256) batched_fwd_kernel(BatchArgs b)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned int id = 0;
        if (lane == 0) id = atomicAdd(b.counter, 1u);
        id = __builtin_amdgcn_readfirstlane(id);
        if (id >= b.n_items) break;
        const BatchItem it = b.items[id];
        const FwdArgs a = b.sets[it.set];
        fwd_wave<D, DM, NORM>(a, it.chunk, it.qblock);
    }
}

template <int NORM, int D, int DM>
void launch_fwd(const FwdArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    if constexpr (fwd_use_o4(D, NORM))
        hipLaunchKernelGGL((bounds_fwd_kernel_o4<D, DM, NORM>), grid, block, 0, s, a);
    else if constexpr (fwd_use_o3(D))
        hipLaunchKernelGGL((bounds_fwd_kernel_o3<D, DM, NORM>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((bounds_fwd_kernel<D, DM, NORM>), grid, block, 0, s, a);
}

template <int NORM, int D, int DM>
void launch_batched(const BatchArgs &b, dim3 grid, dim3 block, hipStream_t s)
{
    hipLaunchKernelGGL((batched_fwd_kernel<D, DM, NORM>), grid, block, 0, s, b);
}

template <int NORM, int D, int... DMs>
constexpr std::array<FwdLaunchers, D + 1> fwd_row(std::integer_sequence<int, DMs...>)
{
    return {{FwdLaunchers{&launch_fwd<NORM, D, DMs>, &launch_batched<NORM, D, DMs>}...}};
}

template <int NORM, int D>
FwdLaunchers fwd_pick(int dm)
{
    constexpr auto row = fwd_row<NORM, D>(std::make_integer_sequence<int, D + 1>{});
    return row[dm];
}

template <int NORM>
FwdLaunchers fwd_table(int d, int dm)
{
    if (dm < 0 || dm > d) return FwdLaunchers{nullptr, nullptr};
    switch (d) {
    case 1: return fwd_pick<NORM, 1>(dm);
    case 2: return fwd_pick<NORM, 2>(dm);
    case 3: return fwd_pick<NORM, 3>(dm);
    case 4: return fwd_pick<NORM, 4>(dm);
    case 5: return fwd_pick<NORM, 5>(dm);
    case 6: return fwd_pick<NORM, 6>(dm);
    case 7: return fwd_pick<NORM, 7>(dm);
    case 8: return fwd_pick<NORM, 8>(dm);
    case 9: return fwd_pick<NORM, 9>(dm);
    case 10: return fwd_pick<NORM, 10>(dm);
    case 11: return fwd_pick<NORM, 11>(dm);
    case 12: return fwd_pick<NORM, 12>(dm);
    case 13: return fwd_pick<NORM, 13>(dm);
    case 14: return fwd_pick<NORM, 14>(dm);
    case 15: return fwd_pick<NORM, 15>(dm);
    case 16: return fwd_pick<NORM, 16>(dm);
    default: return FwdLaunchers{nullptr, nullptr};
    }
}

}  // namespace lip
