// l2 bounds with a BF16 matrix-core cross term and exact FP32 re-scoring
// (lip_fit_eval / lip_bounds with LIP_FLAG_BF16; Euclidean distance without
// monotone coordinates).  The results (values and indices) are those of the
// FP32 path bit for bit: the matrix cores only decide which (query, datum)
// pairs can attain the min / max of Eq. (2); every such pair is evaluated
// with the FP32 path's own pair formula on the same staged record.
//
// Filter.  With a = w.q and b = w.x (the FP32 values the FP32 path uses) the
// squared distance is S = |a|^2 + |b|^2 - 2 a.b.  One MFMA dot product over
// the augmented vectors
//     datum row:    [-2 bf16(b_0) .. -2 bf16(b_{d-1}) | n1 n2 n3 | 1 1 1 | 0..]
//     query column: [   bf16(a_0) ..    bf16(a_{d-1}) | 1  1  1  | m1 m2 m3 | 0..]
// with n1 + n2 + n3 = (1 - cE)|b|^2 and m1 + m2 + m3 = (1 - cE)|a|^2 (three
// BF16 pieces each) gives L, a lower bound of S:
//   * the cross term errs by at most (2^-7 + 2^-16) * 2 sum|a_i b_i|
//     <= (2^-7 + 2^-16) (|a|^2 + |b|^2) (BF16 rounding of each factor);
//   * FP32 accumulation of at most 33 terms of total magnitude
//     <= 2.01 (|a|^2 + |b|^2) errs by at most 33 * 2^-23 of that (a bound
//     that holds for any summation order, even without round-to-nearest);
//   * the norms (FP32 sums of squares, three-piece split) err by ~1e-6
//     relative;
// so cE = 2^-7 + 2^-11 covers all three with a 2^-11 margin.  Products or
// sums that underflow add at most ~2^-120 absolute, covered by the test's
// absolute slack 2^-100.
//
// If u_k = fl(y_k + M_k s_k) <= T (s_k = v_sqrt_f32 of the FP32 sum S32_k),
// then M_k s_k <= T' - y_k with T' = T + 2^-21|T| + 2^-126 (one rounding of
// the fma), s_k >= (1 - 2^-21) sqrt(S32_k) (v_sqrt_f32 is within one ulp;
// four are allowed) and S32_k >= (1 - 2^-24)^(d+2) S_k (every step rounds a
// non-negative sum), so S_k <= r_k^2 (1 + 2.1e-6) with
// r_k = (T' - y_k) / M_k.  Symmetrically for the lower bound with
// T'_lo = T_lo - 2^-21|T_lo| - 2^-126.  Per tile of 64 data the kernel uses
//     r = max(T'_up - ymin, ymax - T'_lo) * (1 + 2^-16) / Mmin,
// which dominates every r_k of the tile with a 1.5e-5 relative margin (more
// than the 2.1e-6 plus the rounding of the four operations), and a pair is a
// candidate unless  fma(r, -|r|, L) > 2^-100.  The running thresholds T are
// the exact FP32 values of candidates re-scored so far, so the attaining
// pair and every pair tied with it always pass.  Non-finite or huge norms
// (> 2^100), non-positive M_k or NaN make every pair of the query / tile a
// candidate.
//
// Order of the data.  The data are sorted by y (sort of packed (y, index)
// keys) and cut into tiles of 64, so a tile's y range is narrow
// and the tile-level radius is close to the per-datum one.  Each data chunk
// takes every C-th tile of the sorted order and visits them from both ends
// alternately (lowest y, highest y, second lowest, ...), so that both
// thresholds tighten within the first tiles.
//
// Work decomposition.  A wave owns 4 blocks of 32 queries (B operands, in
// VGPRs for the whole scan) and one data chunk; per tile of 64 data it issues
// 8 (d <= 10) or 16 v_mfma_f32_32x32x16_bf16.  Lane l holds column l % 32 (one
// query) and 32 rows (data) of each block's two 32 x 32 results, so the tile
// test is a min over 32 accumulators, the radius (4 instructions), one fma
// and one compare per lane and block.  Candidates go
// to a per-wave queue in LDS; when it holds 64 entries the whole wave
// re-scores 64 pairs at once (one per lane) with the FP32 pair formula and
// merges them into per-query packed (value, index) keys in LDS with 64-bit
// atomic min, which keeps the lowest index on ties; the thresholds are then
// refreshed from those keys.
#include <array>
#include <climits>
#include <utility>

#include "host_common.hpp"

namespace lip {
namespace {

constexpr int kBTile = 64;   // data per tile (two 32-row MFMA blocks, one y range)
constexpr int kRB = kBTile / 32;
constexpr int kBQB = 4;      // 32-query blocks per wave
constexpr int kBWaves = 4;   // waves per workgroup
constexpr int kBCap = 256;   // re-scoring queue entries per wave
constexpr float kCE = 0x1p-7f + 0x1p-11f;
constexpr float kHuge = 0x1p100f;
constexpr float kTiny = 0x1p-100f;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int ksteps(int d) { return d + 6 <= 16 ? 1 : 2; }

// BF16 round-to-nearest-even of a finite float (bits of the result).
__device__ __forceinline__ uint32_t bf16_bits(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// Three BF16 pieces whose sum is v to ~2^-24 relative.
__device__ __forceinline__ void split3(float v, uint32_t (&p)[3])
{
    p[0] = bf16_bits(v);
    const float r1 = v - bf16_value(p[0]);
    p[1] = bf16_bits(r1);
    const float r2 = r1 - bf16_value(p[1]);
    p[2] = bf16_bits(r2);
}

__device__ __forceinline__ uint4 pack8(const uint32_t (&e)[8])
{
    return make_uint4(e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16),
                      e[6] | (e[7] << 16));
}

__device__ __forceinline__ float key_value(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// NaN-propagating minimum (v_minimum3_f32 on gfx950; no operand
// canonicalisation is needed, unlike fminf).
__device__ __forceinline__ float fmin_nan(float a, float b) { return __builtin_elementwise_minimum(a, b); }

// ---- sort of (y, index) keys ------------------------------------------------

__global__ void sort_init_kernel(const float *y, int64_t n, int64_t P, unsigned long long *keys)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += stride)
        keys[i] = i < n ? (((unsigned long long)f32_order_key(y[i]) << 32) | (uint32_t)i)
                        : ~0ull;
}

// ---- staging ------------------------------------------------------------------

struct Bf16Stage {
    const float *x, *y, *Mk;
    float M;
    int32_t C;
    int64_t n, n_pad, per, rem;
    Xform xf;
    const unsigned long long *sorted;
    float *rec;       // [n_pad][D + 3] FP32 records in scan order
    int32_t *idx;     // [n_pad] original index of each scan position
    uint4 *A;         // [nt][KS][64] MFMA A operands
    float4 *stats;    // [nt] (ymin, ymax, (1 + 2^-16) / Mmin, 0)
};

// Scan position p (tile j = p / 32, row p % 32) -> chunk c, local tile i ->
// sorted tile c + C * (i even ? i / 2 : cnt - 1 - i / 2).
__device__ __forceinline__ int64_t scan_to_sorted(int64_t p, int64_t C, int64_t per, int64_t rem)
{
    const int64_t j = p / kBTile;
    const int64_t big = rem * (per + 1);
    int64_t c, base, cnt;
    if (j < big) {
        c = j / (per + 1);
        base = c * (per + 1);
        cnt = per + 1;
    } else {
        c = rem + (j - big) / per;
        base = big + (c - rem) * per;
        cnt = per;
    }
    const int64_t i = j - base;
    const int64_t tl = (i & 1) ? cnt - 1 - (i >> 1) : (i >> 1);
    return (c + C * tl) * kBTile + p % kBTile;
}

template <int D>
__global__ void __launch_bounds__(256) bf16_stage_kernel(Bf16Stage a)
{
    constexpr int S = Rec<D>::S;
    constexpr int KS = ksteps(D);
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n_pad) return;  // whole tiles (n_pad is a multiple of 64)
    const int within = (int)(p % kBTile);
    const int rb = within / 32, row = within % 32;
    const int64_t j = p / kBTile;
    int64_t s = scan_to_sorted(p, a.C, a.per, a.rem);
    if (s >= a.n) s = a.n - 1;  // padding repeats the largest-y datum
    const int64_t orig = (int64_t)(uint32_t)(a.sorted[s] & 0xFFFFFFFFull);

    // FP32 record: the same expressions as the FP32 path's staging
    const float *xs = a.x + orig * D;
    float xv[D];
#pragma unroll
    for (int jj = 0; jj < D; ++jj) xv[jj] = xf_coord(a.xf, xs, jj);
    const float y = a.y[orig];
    const float m = a.Mk ? a.Mk[orig] : a.M;
    float *o = a.rec + p * S;
#pragma unroll
    for (int jj = 0; jj < D; ++jj) o[jj] = xv[jj];
    o[Rec<D>::Y] = y;
    o[Rec<D>::M] = m;
    o[Rec<D>::YU] = y;
    a.idx[p] = (int32_t)orig;

    // MFMA row: [-2 bf16(b) | norm pieces | 1 1 1 | 0 ..]
    float nx = xv[0] * xv[0];
#pragma unroll
    for (int jj = 1; jj < D; ++jj) nx = fmaf(xv[jj], xv[jj], nx);
    const bool flag = !(nx <= kHuge);
    uint32_t np[3];
    split3(flag ? 0.0f : nx * (1.0f - kCE), np);
    uint32_t row_e[16 * KS];
#pragma unroll
    for (int k = 0; k < 16 * KS; ++k) {
        uint32_t e = 0;
        if (k < D) e = flag ? 0u : bf16_bits(-2.0f * bf16_value(bf16_bits(xv[k < D ? k : 0])));
        else if (k < D + 3) e = np[k < D + 3 ? k - D : 0];
        else if (k < D + 6) e = 0x3F80u;  // 1.0
        row_e[k] = e;
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            uint32_t e8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) e8[e] = row_e[16 * ks + 8 * g + e];
            a.A[((j * kRB + rb) * KS + ks) * 64 + 32 * g + row] = pack8(e8);
        }
    }

    // tile statistics over the 64 lanes (one wave) of this tile
    float ymin = y, ymax = flag ? __builtin_inff() : y, mmin = m;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ymin = fminf(ymin, __shfl_xor(ymin, off));
        ymax = fmaxf(ymax, __shfl_xor(ymax, off));
        mmin = fminf(mmin, __shfl_xor(mmin, off));
    }
    if (within == 0) {
        const float inv = mmin > 0.0f ? (1.0f / mmin) * (1.0f + 0x1p-16f) : __builtin_nanf("");
        a.stats[j] = make_float4(ymin, ymax, inv, 0.0f);
    }
}

// ---- bound kernel ---------------------------------------------------------------

struct Bf16Args {
    const uint4 *A;
    const float4 *stats;
    const float *rec;
    const int32_t *idx;
    const float *xq;
    int64_t q;
    Xform xf;
    int64_t per, rem;
    int32_t C;
    int32_t pad0;
    float *g, *h_up, *h_lo;
    int32_t *arg_up, *arg_lo;
    unsigned long long *keys;  // [2][q] packed keys when C > 1
};

__device__ __forceinline__ float pad_up(float t) { return fmaf(fabsf(t), 0x1p-21f, t) + 0x1p-126f; }
__device__ __forceinline__ float pad_lo(float t) { return fmaf(-fabsf(t), 0x1p-21f, t) - 0x1p-126f; }

template <int D>
__global__ void __launch_bounds__(256) bf16_bounds_kernel(Bf16Args a)
{
    constexpr int S = Rec<D>::S;
    constexpr int KS = ksteps(D);
    constexpr int QB = kBQB;
    __shared__ uint2 queue[kBWaves][kBCap];
    __shared__ unsigned long long kup[kBWaves][32 * QB];
    __shared__ unsigned long long klo[kBWaves][32 * QB];
    __shared__ uint32_t evm[kBWaves][QB][64];  // candidate rows of the last tile, per block and lane

    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int col = lane & 31, grp = lane >> 5;
    const int chunk = blockIdx.x % a.C;
    const int64_t q0 = ((int64_t)(blockIdx.x / a.C) * kBWaves + w) * (32 * QB);
    if (q0 >= a.q) return;  // wave-uniform

    // query columns (B operands) and thresholds
    uint4 bop[QB][KS];
    bool qflag[QB];
    float tu[QB], tl[QB];
#pragma unroll
    for (int b = 0; b < QB; ++b) {
        int64_t row = q0 + 32 * b + col;
        row = row < a.q ? row : a.q - 1;
        const float *src = a.xq + row * D;
        float av[D];
#pragma unroll
        for (int jj = 0; jj < D; ++jj) av[jj] = xf_coord(a.xf, src, jj);
        float nq = av[0] * av[0];
#pragma unroll
        for (int jj = 1; jj < D; ++jj) nq = fmaf(av[jj], av[jj], nq);
        const bool flag = !(nq <= kHuge);
        uint32_t mp[3];
        split3(flag ? 0.0f : nq * (1.0f - kCE), mp);
        uint32_t ce[16 * KS];
#pragma unroll
        for (int k = 0; k < 16 * KS; ++k) {
            uint32_t e = 0;
            if (k < D) e = flag ? 0u : bf16_bits(av[k < D ? k : 0]);
            else if (k < D + 3) e = 0x3F80u;
            else if (k < D + 6) e = mp[k >= D + 3 && k < D + 6 ? k - D - 3 : 0];
            ce[k] = e;
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            uint32_t e0[8], e1[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                e0[e] = ce[16 * ks + e];
                e1[e] = ce[16 * ks + 8 + e];
            }
            const uint4 v0 = pack8(e0), v1 = pack8(e1);
            bop[b][ks] = make_uint4(grp ? v1.x : v0.x, grp ? v1.y : v0.y, grp ? v1.z : v0.z,
                                    grp ? v1.w : v0.w);
        }
        qflag[b] = flag;
        tu[b] = __builtin_inff();
        tl[b] = -__builtin_inff();
        kup[w][32 * b + col] = ~0ull;
        klo[w][32 * b + col] = ~0ull;
    }

    // this chunk's run of scan tiles
    const int64_t big = a.rem * (a.per + 1);
    const int64_t jb = chunk < a.rem ? chunk * (a.per + 1) : big + (chunk - a.rem) * a.per;
    const int64_t cnt = chunk < a.rem ? a.per + 1 : a.per;

    const float big_inf = opaque_inf();
    int qcount = 0;

    // Re-score the queued pairs with the FP32 pair formula (one per lane),
    // merge them into the per-query keys, refresh the thresholds.
    auto drain = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        for (int base = 0; base < qcount; base += 64) {
            if (base + lane < qcount) {
                const uint2 e = queue[w][base + lane];
                const int64_t p = e.x;
                const int qs = (int)e.y;
                int64_t row = q0 + qs;
                row = row < a.q ? row : a.q - 1;
                const float *src = a.xq + row * D;
                float qv[D], xk[D];
#pragma unroll
                for (int jj = 0; jj < D; ++jj) qv[jj] = xf_coord(a.xf, src, jj);
                const float *rp = a.rec + p * S;
#pragma unroll
                for (int jj = 0; jj < D; ++jj) xk[jj] = rp[jj];
                float u, l;
                pair_bounds<D, 0, kNormL2>(qv, 0.0f, xk, rp[Rec<D>::Y], rp[Rec<D>::M],
                                           rp[Rec<D>::YU], big_inf, u, l);
                const uint32_t id = (uint32_t)a.idx[p];
                // +0.0f folds -0 into +0: equal values get equal keys
                const unsigned long long ku = ((unsigned long long)f32_order_key(u + 0.0f) << 32) | id;
                const unsigned long long kl =
                    ((unsigned long long)f32_order_key(l + 0.0f) << 32) | (uint32_t)~id;
                atomicMin(&kup[w][qs], ku);
                atomicMin(&klo[w][qs], ~kl);
            }
        }
        qcount = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const unsigned long long ku = kup[w][32 * b + col];
            const unsigned long long kl = klo[w][32 * b + col];
            const float vu = ku == ~0ull ? __builtin_inff() : pad_up(key_value((uint32_t)(ku >> 32)));
            const float vl = kl == ~0ull ? -__builtin_inff()
                                         : pad_lo(key_value((uint32_t)(~kl >> 32)));
            tu[b] = qflag[b] ? __builtin_inff() : vu;
            tl[b] = qflag[b] ? -__builtin_inff() : vl;
        }
    };

    // Queue every candidate bit of pm (block b, tile j): bit 16 rb + i is
    // accumulator i of row block rb.
    auto append = [&](uint32_t pm, int b, int64_t j) {
        for (;;) {
            const bool has = pm != 0;
            const uint64_t mask = __builtin_amdgcn_ballot_w64(has);
            if (mask == 0) break;
            if (qcount > kBCap - 64) drain();
            const int bit = has ? __builtin_ctz(pm) : 0;
            pm &= pm - 1;
            const int pos = qcount + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            if (has) {
                const int rb = bit >> 4, i = bit & 15;
                // row of accumulator i in lane l of a 32x32 MFMA result
                const int rrow = 32 * rb + 8 * (i >> 2) + 4 * grp + (i & 3);
                queue[w][pos] = make_uint2((uint32_t)(j * kBTile + rrow), (uint32_t)(32 * b + col));
            }
            qcount += __builtin_popcountll(mask);
        }
    };

    const cfloat_ptr stc = as_const((const float *)a.stats);
    // Tile test for all blocks.  The MFMAs of block b + 1 are issued before
    // the test of block b reads its accumulators.
    struct Acc2 {
        f32x16 v[kRB];
    };
    auto mma = [&](const uint4 (&av)[kRB][KS], int b) -> Acc2 {
        Acc2 acc;
#pragma unroll
        for (int rb = 0; rb < kRB; ++rb) {
            acc.v[rb] = f32x16{};
            acc.v[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[rb][0]),
                                                                __builtin_bit_cast(bf16x8, bop[b][0]),
                                                                acc.v[rb], 0, 0, 0);
        }
        if constexpr (KS == 2) {
#pragma unroll
            for (int rb = 0; rb < kRB; ++rb)
                acc.v[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, av[rb][1]), __builtin_bit_cast(bf16x8, bop[b][1]),
                    acc.v[rb], 0, 0, 0);
        }
        return acc;
    };
    // Returns a wave-uniform mask of the blocks with candidates; their per-lane
    // row bits are left in evm (LDS), so the common path carries no masks.
    auto tile_test = [&](const uint4 (&av)[kRB][KS], float symin, float symax,
                         float sinv) -> uint32_t {
        uint32_t ev = 0;
        Acc2 acc[2];
        acc[0] = mma(av, 0);
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            if (b + 1 < QB) acc[(b + 1) & 1] = mma(av, b + 1);
            const Acc2 &c = acc[b & 1];
            const float r = fmaxf(tu[b] - symin, symax - tl[b]) * sinv;
            float lm = fmin_nan(fmin_nan(c.v[0][0], c.v[0][1]), c.v[0][2]);
#pragma unroll
            for (int i = 3; i < 15; i += 2) lm = fmin_nan(fmin_nan(lm, c.v[0][i]), c.v[0][i + 1]);
            lm = fmin_nan(fmin_nan(lm, c.v[0][15]), c.v[1][0]);
#pragma unroll
            for (int i = 1; i < 15; i += 2) lm = fmin_nan(fmin_nan(lm, c.v[1][i]), c.v[1][i + 1]);
            lm = fmin_nan(lm, c.v[1][15]);
            const bool pass = !(fmaf(r, -fabsf(r), lm) > kTiny);
            // interleave the next block's MFMAs with this block's test so that
            // the matrix and vector pipes work at the same time
            if (b + 1 < QB) {
#pragma unroll
                for (int k = 0; k < kRB * KS; ++k) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
                }
            }
            if (__builtin_amdgcn_ballot_w64(pass) != 0) {
                // bit 16 rb + i, shifted in from the top bit down (no mask
                // constants held in registers)
                uint32_t m = 0;
#pragma unroll
                for (int rb = kRB - 1; rb >= 0; --rb)
#pragma unroll
                    for (int i = 15; i >= 0; --i)
                        m = (m << 1) | (uint32_t)!(fmaf(r, -fabsf(r), c.v[rb][i]) > kTiny);
                evm[w][b][lane] = m;
                ev |= 1u << b;
            }
        }
        return ev;
    };
    auto handle = [&](uint32_t ev, int64_t j) {
        if (ev == 0) return;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
        for (int b = 0; b < QB; ++b)
            if ((ev >> b) & 1u) append(evm[w][b][lane], b, j);
        if (qcount >= 64) drain();
    };

    // A operands and tile statistics are loaded one tile ahead
    constexpr int TS = kRB * KS * 64;  // uint4 per tile
    const uint4 *Ab = a.A + jb * TS + lane;
    auto load_a = [&](const uint4 *ptr, uint4 (&av)[kRB][KS]) {
#pragma unroll
        for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) av[rb][ks] = ptr[(rb * KS + ks) * 64];
    };
    uint4 ba[kRB][KS], bb[kRB][KS];

    // Warm start: in the chunk's first two tiles (lowest and highest y), each
    // lane re-scores, per block, the datum with the smallest L (y is nearly
    // constant inside a tile, so that is about the tile's best pair for both
    // bounds).  The thresholds then start close to their final values; the
    // two tiles are tested again in full below.
#pragma unroll 1
    for (int64_t t0 = 0; t0 < (cnt < 2 ? cnt : 2); ++t0) {
        load_a(Ab + t0 * TS, ba);
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const Acc2 c = mma(ba, b);
            float best = c.v[0][0];
            int bi = 0;
#pragma unroll
            for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const bool lt = c.v[rb][i] < best;
                    best = lt ? c.v[rb][i] : best;
                    bi = lt ? 16 * rb + i : bi;
                }
            const int rb = bi >> 4, i = bi & 15;
            const int rrow = 32 * rb + 8 * (i >> 2) + 4 * grp + (i & 3);
            queue[w][qcount + lane] =
                make_uint2((uint32_t)((jb + t0) * kBTile + rrow), (uint32_t)(32 * b + col));
            qcount += 64;
        }
        drain();
    }

    load_a(Ab, ba);
    float sa0 = stc[4 * jb], sa1 = stc[4 * jb + 1], sa2 = stc[4 * jb + 2];
    int64_t t = 0;
    for (; t + 1 < cnt; t += 2) {
        const int64_t j = jb + t;
        load_a(Ab + (t + 1) * TS, bb);
        const float sb0 = stc[4 * (j + 1)], sb1 = stc[4 * (j + 1) + 1], sb2 = stc[4 * (j + 1) + 2];
        handle(tile_test(ba, sa0, sa1, sa2), j);
        const int64_t tn = t + 2 < cnt ? t + 2 : t + 1;
        load_a(Ab + tn * TS, ba);
        sa0 = stc[4 * (jb + tn)];
        sa1 = stc[4 * (jb + tn) + 1];
        sa2 = stc[4 * (jb + tn) + 2];
        handle(tile_test(bb, sb0, sb1, sb2), j + 1);
    }
    if (t < cnt) handle(tile_test(ba, sa0, sa1, sa2), jb + t);
    if (qcount > 0) drain();

    if (grp == 0) {
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const int64_t qi = q0 + 32 * b + col;
            if (qi >= a.q) continue;
            const unsigned long long ku = kup[w][32 * b + col];
            const unsigned long long kl = klo[w][32 * b + col];
            if (a.C > 1) {
                atomicMin(a.keys + qi, ku);
                atomicMin(a.keys + a.q + qi, kl);
            } else {
                const float hu = key_value((uint32_t)(ku >> 32));
                const float hl = key_value((uint32_t)(~kl >> 32));
                if (a.g) a.g[qi] = 0.5f * (hu + hl);
                if (a.h_up) a.h_up[qi] = hu;
                if (a.h_lo) a.h_lo[qi] = hl;
                if (a.arg_up) a.arg_up[qi] = (int32_t)(uint32_t)ku;
                if (a.arg_lo) a.arg_lo[qi] = (int32_t)(uint32_t)kl;
            }
        }
    }
}

__global__ void bf16_fill_kernel(unsigned long long *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = ~0ull;
}

// Keys of split chunks -> outputs.  The lower-bound key is stored
// complemented: ~(key(l) << 32 | ~index), so its low word is the index.
__global__ void bf16_finalize_kernel(const unsigned long long *keys, int64_t q, float *g,
                                     float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q; i += stride) {
        const unsigned long long ku = keys[i], kl = keys[q + i];
        const float hu = key_value((uint32_t)(ku >> 32));
        const float hl = key_value((uint32_t)(~kl >> 32));
        if (g) g[i] = 0.5f * (hu + hl);
        if (h_up) h_up[i] = hu;
        if (h_lo) h_lo[i] = hl;
        if (arg_up) arg_up[i] = (int32_t)(uint32_t)ku;
        if (arg_lo) arg_lo[i] = (int32_t)(uint32_t)kl;
    }
}

// ---- host side --------------------------------------------------------------------

typedef void (*Bf16StageFn)(const Bf16Stage &, dim3, hipStream_t);
typedef void (*Bf16BoundsFn)(const Bf16Args &, dim3, hipStream_t);

template <int D>
void stage_launch(const Bf16Stage &a, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((bf16_stage_kernel<D>), grid, dim3(256), 0, s, a);
}

template <int D>
void bounds_launch(const Bf16Args &a, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((bf16_bounds_kernel<D>), grid, dim3(64 * kBWaves), 0, s, a);
}

template <int... Ds>
constexpr std::array<std::pair<Bf16StageFn, Bf16BoundsFn>, sizeof...(Ds)> bf16_fns(
    std::integer_sequence<int, Ds...>)
{
    return {{std::make_pair(&stage_launch<Ds + 1>, &bounds_launch<Ds + 1>)...}};
}

constexpr auto kBf16Fns = bf16_fns(std::make_integer_sequence<int, kMaxDim>{});

struct Bf16Layout {
    int64_t nt = 0, n_pad = 0, P = 0;
    size_t sort = 0, rec = 0, idx = 0, A = 0, stats = 0, keys = 0, total = 0;
};

Bf16Layout bf16_layout(int64_t n, int64_t q, int d)
{
    Bf16Layout L;
    L.nt = (n + kBTile - 1) / kBTile;
    L.n_pad = L.nt * kBTile;
    L.P = sort_len(n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes, 256);
        return o;
    };
    L.sort = take((size_t)L.P * 8);
    L.rec = take((size_t)L.n_pad * (d + 3) * 4);
    L.idx = take((size_t)L.n_pad * 4);
    L.A = take((size_t)L.nt * kRB * ksteps(d) * 64 * 16);
    L.stats = take((size_t)L.nt * 16);
    L.keys = take((size_t)(q > 0 ? q : 1) * 2 * 8);
    L.total = off;
    return L;
}

int64_t grid_for(int64_t work, int64_t block)
{
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return g;
}

}  // namespace

size_t bf16_extra_bytes(int64_t n, int64_t q, int d) { return bf16_layout(n, q, d).total; }

lip_status run_bounds_bf16(const MetricInfo &mi, const float *x, const float *y, int64_t n, float M,
                           const float *Mk, const float *xq, int64_t q, float *g, float *h_up,
                           float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws,
                           size_t ws_bytes, hipStream_t stream)
{
    if (mi.norm != LIP_L2 || mi.dm != 0) return LIP_E_UNSUPPORTED;
    const int d = mi.d;
    const Bf16Layout L = bf16_layout(n, q, d);
    if (ws_bytes < kOriginBytes + L.total) return LIP_E_WORKSPACE;
    Xform xf = mi.xf;
    const lip_status st = origin_for(x, n, d, xf, ws, stream);
    if (st != LIP_OK) return st;
    char *base = (char *)ws + kOriginBytes;
    unsigned long long *sorted = (unsigned long long *)(base + L.sort);

    // sort (y, index) keys
    hipLaunchKernelGGL(sort_init_kernel, dim3((unsigned)grid_for(L.P, 256)), dim3(256), 0, stream,
                       y, n, L.P, sorted);
    if (launch_sort_u64(sorted, L.P, stream) != hipSuccess) return LIP_E_DEVICE;

    // data chunks: enough waves to fill the chip, at least 8 tiles a chunk
    const int64_t qwaves = (q + 32 * kBQB - 1) / (32 * kBQB);
    int C = 1;
    while (C < kMaxChunks && qwaves * C < 4096 && L.nt >= 8ll * C) C *= 2;
    const int64_t per = L.nt / C, rem = L.nt % C;

    Bf16Stage sa{};
    sa.x = x;
    sa.y = y;
    sa.Mk = Mk;
    sa.M = M;
    sa.C = C;
    sa.n = n;
    sa.n_pad = L.n_pad;
    sa.per = per;
    sa.rem = rem;
    sa.xf = xf;
    sa.sorted = sorted;
    sa.rec = (float *)(base + L.rec);
    sa.idx = (int32_t *)(base + L.idx);
    sa.A = (uint4 *)(base + L.A);
    sa.stats = (float4 *)(base + L.stats);
    kBf16Fns[d - 1].first(sa, dim3((unsigned)((L.n_pad + 255) / 256)), stream);

    Bf16Args ba{};
    ba.A = sa.A;
    ba.stats = sa.stats;
    ba.rec = sa.rec;
    ba.idx = sa.idx;
    ba.xq = xq;
    ba.q = q;
    ba.xf = xf;
    ba.per = per;
    ba.rem = rem;
    ba.C = C;
    ba.g = g;
    ba.h_up = h_up;
    ba.h_lo = h_lo;
    ba.arg_up = arg_up;
    ba.arg_lo = arg_lo;
    ba.keys = (unsigned long long *)(base + L.keys);
    if (C > 1)
        hipLaunchKernelGGL(bf16_fill_kernel, dim3((unsigned)grid_for(2 * q, 256)), dim3(256), 0,
                           stream, ba.keys, 2 * q);
    const int64_t wgs = (qwaves + kBWaves - 1) / kBWaves;
    kBf16Fns[d - 1].second(ba, dim3((unsigned)(wgs * C)), stream);
    if (C > 1)
        hipLaunchKernelGGL(bf16_finalize_kernel, dim3((unsigned)grid_for(q, 256)), dim3(256), 0,
                           stream, ba.keys, q, g, h_up, h_lo, arg_up, arg_lo);
    return hipGetLastError() == hipSuccess ? LIP_OK : LIP_E_DEVICE;
}

}  // namespace lip
