// Spectral low-rank correction of the polynomial preconditioner (section 3.1):
//   P = p_k(A) + V (V^T A V)^{-1} V^T,   V = n x p (p <= LR_MAX), column-major.
//
// In CG the corrected z never exists as a vector: with c = V^T r and
// y = Hinv c (Hinv = (V^T A V)^{-1}),
//   r.z = r.p_k(A)r + c.y      (the fused last Chebyshev step gives the first
//                               term, the finaliser adds the second),
//   p   = p_k(A)r + V y + beta p   (one pass, k_p_lr),
// and c is reduced in the same pass that updates r (k_xr_lr).  So the
// correction costs two reads of V and p extra dot products per iteration
// (the rank-one rows of Table tab11: four dot products per iteration).
#pragma once
#include "kernels.hpp"

namespace ppk {

// partials[L * p + j] = sum over my rows of V_j[i] * s_i * r_i   (s = scale or 1)
static __global__ __launch_bounds__(BLOCK) void k_lr_dots(int64_t n, int p, const double *__restrict__ V,
                                                          int64_t ldv, const double *__restrict__ r,
                                                          const double *__restrict__ scale, double *partials,
                                                          const State *st)
{
    PPK_PROLOGUE(st)
    double acc[LR_MAX];
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) acc[j] = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const double ri = scale ? r[i] * scale[i] : r[i];
#pragma unroll
        for (int j = 0; j < LR_MAX; ++j)
            if (j < p) acc[j] += V[(int64_t)j * ldv + i] * ri;
    });
    __shared__ double lds[WPB];
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) {
        if (j < p) {
            const double s = block_sum(acc[j], lds);
            if (threadIdx.x == 0) partials[(int64_t)L * p + j] = s;
        }
    }
}

// x += alpha p ; r -= alpha q ; partials[L * (1 + p)] = r.r, then V_j^T r
static __global__ __launch_bounds__(BLOCK) void k_xr_lr(int64_t n, int p, const double *__restrict__ V,
                                                        int64_t ldv, const double *__restrict__ pv,
                                                        const double *__restrict__ q, double *__restrict__ x,
                                                        double *__restrict__ r, double *partials, State *st)
{
    PPK_PROLOGUE(st)
    const double alpha = st->alpha;
    double rr = 0.0, acc[LR_MAX];
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) acc[j] = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        x[i] = x[i] + alpha * pv[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rr += ri * ri;
#pragma unroll
        for (int j = 0; j < LR_MAX; ++j)
            if (j < p) acc[j] += V[(int64_t)j * ldv + i] * ri;
    });
    __shared__ double lds[WPB];
    const double s0 = block_sum(rr, lds);
    if (threadIdx.x == 0) partials[(int64_t)L * (1 + p)] = s0;
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) {
        if (j < p) {
            const double s = block_sum(acc[j], lds);
            if (threadIdx.x == 0) partials[(int64_t)L * (1 + p) + 1 + j] = s;
        }
    }
}

enum LrFin : int {
    LR_FIN_C = 0,   // c = sums[0..p)
    LR_FIN_RR = 1   // rr = sums[0] (convergence logic of FIN_RR), c = sums[1..p]
};

// Sum the G rows of `width` partials column by column in index order; then
// c, y = Hinv c into the CG state (and the residual logic for LR_FIN_RR).
static __global__ __launch_bounds__(BLOCK) void k_fin_lr(const double *__restrict__ partials, int G, int width,
                                                         State *st, int mode, int p,
                                                         const double *__restrict__ hinv)
{
    if (st->done) return;
    __shared__ double lds[WPB];
    __shared__ double sums[1 + LR_MAX];
    for (int col = 0; col < width; ++col) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < G; i += BLOCK) acc += partials[(int64_t)i * width + col];
        const double tot = block_sum(acc, lds);
        if (threadIdx.x == 0) sums[col] = tot;
    }
    if (threadIdx.x == 0) {
        const int o = mode == LR_FIN_RR ? 1 : 0;
        if (mode == LR_FIN_RR) finalize(st, FIN_RR, 0, sums[0]);
        for (int j = 0; j < p; ++j) st->lr_c[j] = sums[o + j];
        for (int i = 0; i < p; ++i) {
            double y = 0.0;
            for (int j = 0; j < p; ++j) y += hinv[i * p + j] * sums[o + j];
            st->lr_y[i] = y;
        }
        st->lr_p = p;
    }
}

// out[col] = sum over the G rows of `width` partials (index order); one workgroup
static __global__ __launch_bounds__(BLOCK) void k_colsum(const double *__restrict__ partials, int G, int width,
                                                         double *__restrict__ out)
{
    __shared__ double lds[WPB];
    for (int col = 0; col < width; ++col) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < G; i += BLOCK) acc += partials[(int64_t)i * width + col];
        const double tot = block_sum(acc, lds);
        if (threadIdx.x == 0) out[col] = tot;
    }
}

// p = z + V y + beta p   (first: p = z + V y)
static __global__ __launch_bounds__(BLOCK) void k_p_lr(int64_t n, int p, const double *__restrict__ V, int64_t ldv,
                                                       const double *__restrict__ z, double *__restrict__ pv,
                                                       const State *st, int first)
{
    PPK_PROLOGUE(st)
    const double beta = first ? 0.0 : st->beta;
    double y[LR_MAX];
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) y[j] = j < p ? st->lr_y[j] : 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        double zi = z[i];
#pragma unroll
        for (int j = 0; j < LR_MAX; ++j)
            if (j < p) zi += V[(int64_t)j * ldv + i] * y[j];
        pv[i] = first ? zi : zi + beta * pv[i];
    });
}

// z += s .* (V y)   (s = scale or 1; pp_apply with the correction)
static __global__ __launch_bounds__(BLOCK) void k_lr_axpy(int64_t n, int p, const double *__restrict__ V, int64_t ldv,
                                                          const double *__restrict__ scale, double *__restrict__ z,
                                                          const State *st)
{
    PPK_PROLOGUE(st)
    double y[LR_MAX];
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) y[j] = j < p ? st->lr_y[j] : 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < LR_MAX; ++j)
            if (j < p) a += V[(int64_t)j * ldv + i] * y[j];
        z[i] = z[i] + (scale ? scale[i] : 1.0) * a;
    });
}

// V[:, c] = sum_j Q[:, j] S[j, c]   (Ritz vectors from the Lanczos basis; S: m x p row-major)
static __global__ __launch_bounds__(BLOCK) void k_lr_combine(int64_t n, int m, int p, const double *__restrict__ Q,
                                                             const double *__restrict__ S, double *__restrict__ V)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) {
        double acc[LR_MAX];
#pragma unroll
        for (int c = 0; c < LR_MAX; ++c) acc[c] = 0.0;
        for (int j = 0; j < m; ++j) {
            const double q = Q[(int64_t)j * n + i];
#pragma unroll
            for (int c = 0; c < LR_MAX; ++c)
                if (c < p) acc[c] += q * S[j * p + c];
        }
#pragma unroll
        for (int c = 0; c < LR_MAX; ++c)
            if (c < p) V[(int64_t)c * n + i] = acc[c];
    });
}

// partials[L] = sum over my rows of (y_i - a x_i)^2
static __global__ __launch_bounds__(BLOCK) void k_resid_norm2(int64_t n, double a, const double *__restrict__ x,
                                                              const double *__restrict__ y, double *partials)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const double d = y[i] - a * x[i];
        part += d * d;
    });
    store_partial(part, partials, L);
}

// w -= sum_j Q_j coef[j]   (j < p <= LR_MAX; coef on the device)
static __global__ __launch_bounds__(BLOCK) void k_lr_sub(int64_t n, int p, const double *__restrict__ Q, int64_t ldq,
                                                         const double *__restrict__ coef, double *__restrict__ w)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    double c[LR_MAX];
#pragma unroll
    for (int j = 0; j < LR_MAX; ++j) c[j] = j < p ? coef[j] : 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < LR_MAX; ++j)
            if (j < p) a += Q[(int64_t)j * ldq + i] * c[j];
        w[i] = w[i] - a;
    });
}

// Lanczos step on another operator whose product w = B v is already formed:
// w -= beta_{j-1} vprev ; reduce v.w -> lz_alpha[j]
static __global__ __launch_bounds__(BLOCK) void k_lz_wsub(int64_t n, const double *__restrict__ v,
                                                          const double *__restrict__ vprev, double *__restrict__ w,
                                                          double *partials, State *st, int j)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const double bp = (j > 0) ? st->lz_beta[j - 1] : 0.0;
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const double wi = w[i] - bp * vprev[i];
        w[i] = wi;
        part += v[i] * wi;
    });
    store_partial(part, partials, L);
}

}  // namespace ppk
