// Host entry point of the k-best weighted bounds (lip_fit_eval_k) and the
// merge of split partial lists; the kernel is in bounds_topk.hpp,
// instantiated per norm in bounds_topk_{l1,l2,linf}.hip.
#include "bounds_topk.hpp"
#include "host_common.hpp"

namespace lip {

namespace {

// Merge of the chunks' sorted lists: the KL smallest upper and largest
// lower values over all chunks, then the weighted sums.
template <int KL>
__global__ void topk_merge_kernel(TopkArgs A)
{
    const FwdArgs &a = A.f;
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= a.q) return;
    float U[KL], L[KL];
#pragma unroll
    for (int j = 0; j < KL; ++j) {
        U[j] = __builtin_inff();
        L[j] = -__builtin_inff();
    }
    for (int c = 0; c < a.n_chunks; ++c) {
        const float *pu = A.part + (((int64_t)c * a.q + qi) * KL);
        const float *pl = A.part + ((((int64_t)a.n_chunks + c) * a.q + qi) * KL);
#pragma unroll
        for (int j = 0; j < KL; ++j) {
            topk_insert_up<KL>(U, pu[j]);
            topk_insert_lo<KL>(L, pl[j]);
        }
    }
    float hu = 0.0f, hl = 0.0f;
#pragma unroll
    for (int j = 0; j < KL; ++j) {
        if (j < A.k) {
            hu = fmaf(A.wk[j], U[j], hu);
            hl = fmaf(A.wk[j], L[j], hl);
        }
    }
    if (a.g) a.g[qi] = 0.5f * (hu + hl);
    if (a.h_up) a.h_up[qi] = hu;
    if (a.h_lo) a.h_lo[qi] = hl;
}

TopkLaunch get_topk(int norm, int d, int dm, int kl)
{
    switch (norm) {
    case LIP_L1: return topk_l1(d, dm, kl);
    case LIP_L2: return topk_l2(d, dm, kl);
    case LIP_LINF: return topk_linf(d, dm, kl);
    default: return nullptr;
    }
}

void launch_topk_merge(int kl, const TopkArgs &A, hipStream_t s)
{
    const dim3 g((unsigned)((A.f.q + 255) / 256)), b(256);
    switch (kl) {
    case 4: hipLaunchKernelGGL(topk_merge_kernel<4>, g, b, 0, s, A); break;
    case 8: hipLaunchKernelGGL(topk_merge_kernel<8>, g, b, 0, s, A); break;
    case 16: hipLaunchKernelGGL(topk_merge_kernel<16>, g, b, 0, s, A); break;
    default: hipLaunchKernelGGL(topk_merge_kernel<32>, g, b, 0, s, A); break;
    }
}

// Data chunks x list length of the split partials: 16 chunks of 4-lists,
// fewer chunks of longer lists (which also hold fewer queries per lane, so
// the queries alone fill more of the chip).
constexpr int kTopkMaxPartial = 64;

}  // namespace

size_t topk_ws_bytes(int64_t n, int64_t q, int d)
{
    return kOriginBytes + staged_bytes(n, d) +
           align_up((size_t)2 * kTopkMaxPartial * (size_t)q * 4, 256) + 256;
}

}  // namespace lip

using namespace lip;

extern "C" lip_status lip_fit_eval_k(const lip_metric *metric, const float *x, const float *y,
                                     int64_t n, float M, const float *Mk, int32_t k,
                                     const float *wk, const float *xq, int64_t q, float *g,
                                     float *h_up, float *h_lo, void *ws, size_t ws_bytes,
                                     uint32_t flags, lip_stream stream)
{
    MetricInfo mi;
    lip_status st = parse_metric(metric, &mi);
    if (st != LIP_OK) return st;
    if (flags & LIP_FLAG_BF16) return LIP_E_UNSUPPORTED;
    if (flags & ~LIP_FLAG_CHECK_FINITE) return LIP_E_ARG;
    if (n <= 0 || q < 0 || n > kMaxIndex - kMaxTile || q > kMaxIndex) return LIP_E_SHAPE;
    if (k < 1 || k > kTopKMax || k > n) return LIP_E_SHAPE;
    if (!x || !y || !wk || (q > 0 && !xq)) return LIP_E_ARG;
    if (!Mk && (!(M >= 0.0f) || !__builtin_isfinite(M))) return LIP_E_VALUE;
    for (int j = 0; j < k; ++j)
        if (!(wk[j] >= 0.0f) || !__builtin_isfinite(wk[j])) return LIP_E_VALUE;
    if (!ws || ws_bytes < topk_ws_bytes(n, q, mi.d)) return LIP_E_WORKSPACE;
    if (q == 0) return LIP_OK;
    hipStream_t s = (hipStream_t)stream;
    if (flags & LIP_FLAG_CHECK_FINITE) {
        const float *arr[4] = {x, y, Mk, xq};
        const int64_t cnt[4] = {n * mi.d, n, Mk ? n : 0, q * mi.d};
        st = check_finite(arr, cnt, 4, ws, s);
        if (st != LIP_OK) return st;
    }
    const int kl = topk_list_len(k);
    TopkLaunch launch = get_topk(mi.norm, mi.d, mi.dm, kl);
    if (!launch) return LIP_E_UNSUPPORTED;
    const int64_t n_pad = (n + 7) / 8 * 8;
    Xform xf = mi.xf;
    st = origin_for(x, n, mi.d, xf, ws, s);
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
    sa.n_pad = n_pad;
    sa.xf = xf;
    sa.out = staged;
    if (launch_stage(mi.d, sa, s) != hipSuccess) return LIP_E_DEVICE;
    TopkArgs A{};
    A.f.data = staged;
    A.f.n = n;
    A.f.xq = xq;
    A.f.q = q;
    A.f.xf = xf;
    A.f.g = g;
    A.f.h_up = h_up;
    A.f.h_lo = h_lo;
    A.k = k;
    for (int j = 0; j < kTopKMax; ++j) A.wk[j] = j < k ? wk[j] : 0.0f;
    // data split when the queries alone do not fill the chip
    const int R = topk_rows(mi.d, kl);
    const int64_t qwaves = (q + 64 * R - 1) / (64 * R);
    int nc = 1;
    const int nc_max = kTopkMaxPartial / kl;
    while (nc < nc_max && qwaves * nc < 16384 && n >= (int64_t)nc * 2 * 64) nc *= 2;
    int64_t recs = (n + nc - 1) / nc;
    recs = (recs + 7) / 8 * 8;
    A.chunk_recs = recs;
    A.f.n_chunks = (int)((n + recs - 1) / recs);
    A.part = (float *)((char *)ws + staged_bytes(n, mi.d));
    const unsigned grid = (unsigned)(((qwaves + 3) / 4) * A.f.n_chunks);
    launch(A, dim3(grid), dim3(256), s);
    if (hipGetLastError() != hipSuccess) return LIP_E_DEVICE;
    if (A.f.n_chunks > 1) launch_topk_merge(kl, A, s);
    return dev_status(hipGetLastError());
}
