// Host side of the bounds with monotonicity on parts of the domain
// (Sec. 4.2): staging of the clamped records, chunking, launch and combine.
// The pair kernel is in bounds_reg.hpp.
#include "bounds_reg.hpp"

namespace lip {

namespace {

// Records [w (x_free - o).. | c_ND, c_NI per restricted coordinate | y | M_k]
// in the kernel's coordinate order (A.perm); padded records are zero.
__global__ void reg_stage_kernel(const float *x, const float *y, const float *Mk, float M, int d,
                                 int df, int64_t n, int64_t npad, RegArgs A, float *rec)
{
    const int S = 2 * d - df + 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad; k += stride) {
        float *o = rec + k * S;
        const bool in = k < n;
        for (int i = 0; i < df; ++i) o[i] = in ? A.w[i] * (x[k * d + A.perm[i]] - A.origin[i]) : 0.0f;
        for (int i = df; i < d; ++i) {
            const float v = in ? x[k * d + A.perm[i]] : 0.0f;
            o[df + 2 * (i - df)] = reg_clamp(v, A.nd_s[i], A.nd_t[i], A.w[i], A.origin[i]);
            o[df + 2 * (i - df) + 1] = reg_clamp(v, A.ni_s[i], A.ni_t[i], A.w[i], A.origin[i]);
        }
        o[S - 2] = in ? y[k] : 0.0f;
        o[S - 1] = in ? (Mk ? Mk[k] : M) : 0.0f;
    }
}

constexpr int kRegMaxChunks = 16;

int64_t reg_npad(int64_t n) { return (n + 63) / 64 * 64; }

}  // namespace

size_t reg_ws_bytes(int64_t n, int64_t q, int d)
{
    return kOriginBytes + align_up((size_t)reg_npad(n) * (size_t)(2 * d + 2) * 4, 256) +
           partial_bytes(q) + 256;
}

lip_status run_bounds_reg(const MetricInfo &mi, const float *x, const float *y, int64_t n,
                          float M, const float *Mk, const float *xq, int64_t q, float *g,
                          float *h_up, float *h_lo, int32_t *arg_up, int32_t *arg_lo, void *ws,
                          size_t ws_bytes, hipStream_t s)
{
    if (ws_bytes < reg_ws_bytes(n, q, mi.d)) return LIP_E_WORKSPACE;
    RegArgs A{};
    A.n = n;
    A.npad = reg_npad(n);
    // free coordinates (both intervals unbounded) first, then the restricted
    // ones, each in index order
    const float inf = __builtin_inff();
    int order[kMaxDim], df = 0;
    for (int i = 0; i < mi.d; ++i)
        if (mi.nd_s[i] == -inf && mi.nd_t[i] == inf && mi.ni_s[i] == -inf && mi.ni_t[i] == inf)
            order[df++] = i;
    int k = df;
    for (int i = 0; i < mi.d; ++i)
        if (!(mi.nd_s[i] == -inf && mi.nd_t[i] == inf && mi.ni_s[i] == -inf && mi.ni_t[i] == inf))
            order[k++] = i;
    for (int p = 0; p < kMaxDim; ++p) {
        const bool in = p < mi.d;
        const int i = in ? order[p] : 0;
        float nds = in ? mi.nd_s[i] : 0.0f, ndt = in ? mi.nd_t[i] : 0.0f;
        float nis = in ? mi.ni_s[i] : 0.0f, nit = in ? mi.ni_t[i] : 0.0f;
        // an empty region clamps everything to one point: zero length
        if (!(nds <= ndt)) nds = ndt = 0.0f;
        if (!(nis <= nit)) nis = nit = 0.0f;
        A.perm[p] = i;
        A.nd_s[p] = nds;
        A.nd_t[p] = ndt;
        A.ni_s[p] = nis;
        A.ni_t[p] = nit;
        A.w[p] = in ? (float)mi.w[i] : 1.0f;
    }
    RegLaunch launch = mi.norm == LIP_L1   ? reg_l1(mi.d, df)
                       : mi.norm == LIP_L2 ? reg_l2(mi.d, df)
                                           : reg_linf(mi.d, df);
    if (!launch) return LIP_E_UNSUPPORTED;
    if (launch_origin(x, n, mi.d, A.perm, (float *)ws, s) != hipSuccess) return LIP_E_DEVICE;
    A.origin = (const float *)ws;
    ws = (char *)ws + kOriginBytes;
    float *rec = (float *)ws;
    char *p = (char *)ws + align_up((size_t)A.npad * (size_t)(2 * mi.d + 2) * 4, 256);
    A.rec = rec;
    A.xq = xq;
    A.q = q;
    A.g = g;
    A.h_up = h_up;
    A.h_lo = h_lo;
    A.arg_up = arg_up;
    A.arg_lo = arg_lo;
    const int R = reg_rows(mi.d);
    const int64_t qwaves = (q + 64 * R - 1) / (64 * R);
    int nc = 1;
    while (nc < kRegMaxChunks && qwaves * nc < 16384 && n >= (int64_t)nc * 2 * 64 &&
           (int64_t)nc * 2 * q <= kMaxPartials)
        nc *= 2;
    int64_t cols = (n + nc - 1) / nc;
    cols = (cols + kRegTile - 1) / kRegTile * kRegTile;
    A.chunk_cols = cols;
    A.n_chunks = (int)((n + cols - 1) / cols);
    if (A.n_chunks > 1) {
        const int64_t entries = (int64_t)A.n_chunks * q;
        A.part_v = (float *)p;
        A.part_i = (int32_t *)(p + align_up((size_t)entries * 2 * sizeof(float), 256));
    }
    int64_t gs = (A.npad + 255) / 256;
    if (gs > 65536) gs = 65536;
    hipLaunchKernelGGL(reg_stage_kernel, dim3((unsigned)gs), dim3(256), 0, s, x, y, Mk, M, mi.d,
                       df, n, A.npad, A, rec);
    const unsigned grid = (unsigned)(((qwaves + 3) / 4) * A.n_chunks);
    launch(A, dim3(grid), dim3(256), s);
    if (hipGetLastError() != hipSuccess) return LIP_E_DEVICE;
    if (A.n_chunks > 1) {
        CombineArgs c{};
        c.part_v = A.part_v;
        c.part_i = A.part_i;
        c.q = q;
        c.n_chunks = A.n_chunks;
        c.g = g;
        c.h_up = h_up;
        c.h_lo = h_lo;
        c.arg_up = arg_up;
        c.arg_lo = arg_lo;
        if (launch_combine(c, s) != hipSuccess) return LIP_E_DEVICE;
    }
    return dev_status(hipGetLastError());
}

}  // namespace lip
