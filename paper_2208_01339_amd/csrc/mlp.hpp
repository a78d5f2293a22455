// Learned spectral bounds: operator features (FP64) and a small multilayer
// perceptron (FP32) with hand-written forward, backward and Adam kernels.
//
// The MLP is tiny (16 -> 128 -> 128 -> 128 -> 3, ~35k parameters, batches of
// at most 1024), so every kernel computes one output element per thread with
// a fixed-order loop: results are deterministic and no atomics are used.
#pragma once
#include "kernels.hpp"

namespace ppm {

using ppk::BLOCK;
using ppk::WAVE;
using ppk::WPB;

// C[M][N] = opA(A) opB(B) (+ bias[N]).
//   opA(A)(i,k) = TA ? A[k*lda + i] : A[i*lda + k]
//   opB(B)(k,j) = TB ? B[j*ldb + k] : B[k*ldb + j]
// mode 0: store C;  mode 1: C = Z and H = relu(Z);  mode 2: C *= (zmask > 0)
template <bool TA, bool TB>
__global__ __launch_bounds__(BLOCK) void km_mm(int M, int N, int K, const float *__restrict__ A, int lda,
                                               const float *__restrict__ B, int ldb, const float *__restrict__ bias,
                                               float *__restrict__ C, int ldc, int mode, const float *__restrict__ zmask,
                                               float *__restrict__ H)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= M * N) return;
    const int i = idx / N, j = idx % N;
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) {
        const float a = TA ? A[(size_t)k * lda + i] : A[(size_t)i * lda + k];
        const float b = TB ? B[(size_t)j * ldb + k] : B[(size_t)k * ldb + j];
        acc = fmaf(a, b, acc);
    }
    if (bias) acc += bias[j];
    if (mode == 2) acc = zmask[(size_t)i * ldc + j] > 0.0f ? acc : 0.0f;
    C[(size_t)i * ldc + j] = acc;
    if (mode == 1) H[(size_t)i * ldc + j] = acc > 0.0f ? acc : 0.0f;
}

// db[j] = sum_i dZ[i][j]  (rows in order)
static __global__ __launch_bounds__(BLOCK) void km_colsum(int M, int N, const float *__restrict__ dZ,
                                                          float *__restrict__ db)
{
    const int j = blockIdx.x * BLOCK + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += dZ[(size_t)i * N + j];
    db[j] = s;
}

// loss = mean (Y - T)^2 (one workgroup, fixed order), dY = 2 (Y - T) / (M N)
static __global__ __launch_bounds__(BLOCK) void km_loss(int M, int N, const float *__restrict__ Y,
                                                        const float *__restrict__ T, float *__restrict__ dY,
                                                        double *__restrict__ loss)
{
    __shared__ double lds[WPB];
    const int total = M * N;
    const float scale = 2.0f / (float)total;
    double part = 0.0;
    for (int i = threadIdx.x; i < total; i += BLOCK) {
        const float d = Y[i] - T[i];
        if (dY) dY[i] = scale * d;
        part += (double)d * (double)d;
    }
    const double s = ppk::block_sum(part, lds);
    if (threadIdx.x == 0) *loss = s / (double)total;
}

// Adam: m = b1 m + (1-b1) g ; v = b2 v + (1-b2) g^2 ; p -= lr mhat / (sqrt(vhat) + eps)
static __global__ __launch_bounds__(BLOCK) void km_adam(int64_t count, float *__restrict__ p,
                                                        const float *__restrict__ g, float *__restrict__ m,
                                                        float *__restrict__ v, float lr, float b1, float b2, float eps,
                                                        float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// operator features (FP64)
// ---------------------------------------------------------------------------

constexpr int NSTAT = 9;  // per-workgroup partials of k_feat_rows

// Row statistics of the (scaled) operator in the slice layout.
// d_i: the unscaled diagonal (1/dis_i^2 under Jacobi, else the stored a_ii).
// rowabs_i: sum_j |a_ij| over the A part plus, for the trace columns,
//           sum_t |c_ti| ts_t (ts_t = sum_j |(M^-1 C)_tj|): an upper bound of
//           the row sum of |S|.
// Partials: [sum ld, sum ld^2, min ld, max ld, max rowabs, sum (rowabs - a_ii),
//            min (a_ii - sum_{j!=i} |a_ij|) over the A part, max len, min len]
// with ld = log10 d_i and len the number of nonzero stored entries.
static __global__ __launch_bounds__(BLOCK) void k_feat_rows(ppk::SellView A, const double *__restrict__ dis,
                                                            const double *__restrict__ ts,
                                                            double *__restrict__ part)
{
    __shared__ double red[NSTAT][WPB];
    const int G = (int)gridDim.x;
    const int L = ppk::xcd_remap((int)blockIdx.x, G);
    double s_ld = 0, s_ld2 = 0, mn_ld = INFINITY, mx_ld = -INFINITY, mx_abs = 0, s_off = 0, mn_gl = INFINITY,
           mx_len = 0, mn_len = INFINITY;
    ppk::for_my_slices(A.nslices, L, G, [&](int64_t row, int64_t s, int lane) {
        if (row >= A.n) return;
        double aii = 0, offa = 0, tr = 0, len = 0;
        if (A.nd > 0) {  // symmetric diagonal part: a_{i,i+o} at [d][i], a_{i,i-o} at [d][i-o]
            const double *dv = (const double *)A.dv;
            aii = dv[row];
            if (aii != 0.0) len += 1;
            for (int d = 1; d < A.nd; ++d) {
                const int64_t o = A.doff[d];
                const double u = dv[(int64_t)d * A.dstride + row];
                const double l = row >= o ? dv[(int64_t)d * A.dstride + row - o] : 0.0;
                offa += fabs(u) + fabs(l);
                len += (u != 0.0) + (l != 0.0);
            }
        }
        int64_t base = 0;
        int width = 0;
        if (A.sell) ppk::slice_span(A, s, base, width);
        const double *v = (const double *)A.val;
        for (int j = 0; j < width; ++j) {
            const int64_t o = base + (int64_t)j * WAVE + lane;
            const int c = A.col[o];
            const double a = v[o];
            if (a != 0.0) len += 1;
            if (c == row) aii += a;
            else if (c < A.nx) offa += fabs(a);
            else tr += fabs(a) * ts[c - A.nx];
        }
        const double d = dis ? 1.0 / (dis[row] * dis[row]) : aii;
        const double ld = log10(d > 0 ? d : 1e-300);
        const double rowabs = fabs(aii) + offa + tr;
        s_ld += ld;
        s_ld2 += ld * ld;
        mn_ld = fmin(mn_ld, ld);
        mx_ld = fmax(mx_ld, ld);
        mx_abs = fmax(mx_abs, rowabs);
        s_off += rowabs - aii;
        mn_gl = fmin(mn_gl, aii - offa);
        mx_len = fmax(mx_len, len);
        mn_len = fmin(mn_len, len);
    });
    double vals[NSTAT] = {s_ld, s_ld2, mn_ld, mx_ld, mx_abs, s_off, mn_gl, mx_len, mn_len};
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) {
        double x = vals[q];
        const bool is_sum = (q == 0 || q == 1 || q == 5);
        const bool is_min = (q == 2 || q == 6 || q == 8);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_down(x, off, WAVE);
            x = is_sum ? x + y : (is_min ? fmin(x, y) : fmax(x, y));
        }
        if (lane == 0) red[q][w] = x;
    }
    __syncthreads();
    if (threadIdx.x < NSTAT) {
        const int q = threadIdx.x;
        const bool is_sum = (q == 0 || q == 1 || q == 5);
        const bool is_min = (q == 2 || q == 6 || q == 8);
        double x = red[q][0];
        for (int i = 1; i < WPB; ++i) x = is_sum ? x + red[q][i] : (is_min ? fmin(x, red[q][i]) : fmax(x, red[q][i]));
        part[(size_t)L * NSTAT + q] = x;
    }
}

// combine the G x NSTAT partials in workgroup order -> out[NSTAT]
static __global__ __launch_bounds__(64) void k_feat_fin(const double *__restrict__ part, int G, double *__restrict__ out)
{
    const int q = threadIdx.x;
    if (q >= NSTAT) return;
    const bool is_sum = (q == 0 || q == 1 || q == 5);
    const bool is_min = (q == 2 || q == 6 || q == 8);
    double x = part[q];
    for (int b = 1; b < G; ++b) {
        const double y = part[(size_t)b * NSTAT + q];
        x = is_sum ? x + y : (is_min ? fmin(x, y) : fmax(x, y));
    }
    out[q] = x;
}

// ts_t = sum_j |cm_tj| (Schur trace rows)
static __global__ __launch_bounds__(BLOCK) void k_trace_abs(ppk::CsrView Cm, double *__restrict__ ts)
{
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= Cm.rows) return;
    const double *v = (const double *)Cm.val;
    double s = 0;
    for (int64_t p = Cm.rp[t]; p < Cm.rp[t + 1]; ++p) s += fabs(v[p]);
    ts[t] = s;
}

// power step on (shift I - A) when shifted, else A:  w = shift ? c v - y : y
// (y = A v given); partials [v.w, v.v] per workgroup
static __global__ __launch_bounds__(BLOCK) void k_pow_dots(int64_t n, const double *__restrict__ v,
                                                           const double *__restrict__ y, double *__restrict__ w,
                                                           const double *__restrict__ cptr, int shifted,
                                                           double *__restrict__ part)
{
    __shared__ double lds[WPB];
    const int G = (int)gridDim.x;
    const int L = ppk::xcd_remap((int)blockIdx.x, G);
    const double c = shifted ? *cptr : 0.0;
    double vw = 0, vv = 0;
    ppk::for_my_elems(n, L, G, [&](int64_t i) {
        const double vi = v[i];
        const double wi = shifted ? c * vi - y[i] : y[i];
        w[i] = wi;
        vw += vi * wi;
        vv += vi * vi;
    });
    const double a = ppk::block_sum(vw, lds);
    const double b = ppk::block_sum(vv, lds);
    if (threadIdx.x == 0) {
        part[(size_t)L * 2] = a;
        part[(size_t)L * 2 + 1] = b;
    }
}

// out = (sum v.w) / (sum v.v) in workgroup order
static __global__ __launch_bounds__(64) void k_pow_fin(const double *__restrict__ part, int G, double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double a = 0, b = 0;
    for (int i = 0; i < G; ++i) {
        a += part[2 * (size_t)i];
        b += part[2 * (size_t)i + 1];
    }
    *out = a / b;
}

}  // namespace ppm
