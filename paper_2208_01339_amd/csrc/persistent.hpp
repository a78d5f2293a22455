// Persistent PCG driver: the whole solve in one cooperative launch.
//
// Every phase of the stream-driven path (kernels.hpp) runs here in the same
// order, separated by grid-wide barriers.  A reduction writes one partial per
// workgroup, crosses a barrier, and then EVERY workgroup sums the G partials
// in index order: all workgroups hold bitwise-identical scalars, take the
// same branches (convergence, breakdown, maxit) and therefore execute the
// same sequence of barriers -- no workgroup can leave the loop alone.  The
// partial buffer alternates between two halves so that a fast workgroup
// writing the next reduction never overwrites a partial a slow workgroup is
// still reading (a barrier always separates reuse of the same half).
// The launch is cooperative, so the runtime refuses a grid that cannot be
// co-resident instead of letting a barrier wait forever.
#pragma once
#include <hip/hip_cooperative_groups.h>

#include "kernels.hpp"

namespace ppk {

struct PersistArgs {
    SellView A;      // FP64 values
    SellView A32;    // FP32 values (mixed)
    CsrView Cm;      // trace operator, FP64
    CsrView Cm32;    // trace operator, FP32
    const double *b;
    double *x;
    const double *dis;
    double *bh, *xh, *r, *p, *q, *z, *sA, *sB, *tw;
    float *r32, *sA32, *sB32, *tw32;
    const double *coef;  // [k][4]: cx, cold, cr, cA of step j = 1..k
    double *partials;    // 2 * G doubles
    State *st;
    double theta_inv;    // 1 / theta-bar (degree 0)
    double tol;
    int k;
    int maxit;
};

namespace pcgp {

struct Ctx {
    int L, G, pbuf;
    double *partials;
    double *lds;
    double *red;
};

// grid-wide sum of per-workgroup partials; the value is returned to every thread
__device__ __forceinline__ double grid_sum(cooperative_groups::grid_group &grid, Ctx &c, double part)
{
    const double s = block_sum(part, c.lds);
    double *P = c.partials + (size_t)c.pbuf * c.G;
    c.pbuf ^= 1;
    if (threadIdx.x == 0) __hip_atomic_store(&P[c.L], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    grid.sync();
    double acc = 0.0;
    for (int i = threadIdx.x; i < c.G; i += BLOCK)
        acc += __hip_atomic_load(&P[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double tot = block_sum(acc, c.lds);
    if (threadIdx.x == 0) *c.red = tot;
    __syncthreads();
    const double v = *c.red;
    __syncthreads();
    return v;
}

// z = p_k(A-hat) r and the grid-wide r.z
template <bool SCHUR, bool MIXED>
__device__ __forceinline__ double poly(cooperative_groups::grid_group &grid, Ctx &c, const PersistArgs &a)
{
    const int L = c.L, G = c.G, k = a.k;
    const int64_t n = a.A.n;
    if (k == 0) {
        const double part = ph_scale<double, double, true>(n, a.r, a.theta_inv, a.z, L, G);
        return grid_sum(grid, c, part);
    }
    if (!MIXED) {
        for (int j = 1; j <= k; ++j) {
            const double *cf = a.coef + 4 * (j - 1);
            const bool last = (j == k);
            const double *gsrc = (j == 1) ? a.r : ((j % 2 == 0) ? a.sA : a.sB);
            const double *old = (j % 2 == 0) ? a.sB : a.sA;
            double *out = last ? a.z : ((j % 2 == 1) ? a.sA : a.sB);
            if (SCHUR) {
                ph_trace<double, double>(a.Cm, gsrc, a.tw, L, G);
                grid.sync();
            }
            double part;
            if (j == 1)
                part = ph_cheb<double, double, double, double, 1, SCHUR, true, false, true>(
                    a.A, gsrc, a.tw, a.r, (const double *)nullptr, out, cf[0], cf[1], cf[2], cf[3], nullptr, L, G);
            else if (j == 2)
                part = ph_cheb<double, double, double, double, 2, SCHUR, true, false, true>(
                    a.A, gsrc, a.tw, a.r, (const double *)nullptr, out, cf[0], cf[1], cf[2], cf[3], nullptr, L, G);
            else
                part = ph_cheb<double, double, double, double, 3, SCHUR, true, false, true>(
                    a.A, gsrc, a.tw, a.r, old, out, cf[0], cf[1], cf[2], cf[3], nullptr, L, G);
            if (last) return grid_sum(grid, c, part);
            grid.sync();
        }
        return 0.0;
    }
    // FP32 recurrence; the last step reads r in FP64 and writes z in FP64
    ph_scale<double, float, false>(n, a.r, 1.0, a.r32, L, G);
    grid.sync();
    for (int j = 1; j <= k; ++j) {
        const double *cf = a.coef + 4 * (j - 1);
        const float fx = (float)cf[0], fo = (float)cf[1], fr = (float)cf[2], fa = (float)cf[3];
        const bool last = (j == k);
        const float *gsrc = (j == 1) ? a.r32 : ((j % 2 == 0) ? a.sA32 : a.sB32);
        const float *old = (j % 2 == 0) ? a.sB32 : a.sA32;
        float *out32 = (j % 2 == 1) ? a.sA32 : a.sB32;
        if (SCHUR) {
            ph_trace<float, float>(a.Cm32, gsrc, a.tw32, L, G);
            grid.sync();
        }
        if (!last) {
            if (j == 1)
                ph_cheb<float, float, float, float, 1, SCHUR, false, false, true>(
                    a.A32, gsrc, a.tw32, a.r32, (const float *)nullptr, out32, fx, fo, fr, fa, nullptr, L, G);
            else if (j == 2)
                ph_cheb<float, float, float, float, 2, SCHUR, false, false, true>(
                    a.A32, gsrc, a.tw32, a.r32, (const float *)nullptr, out32, fx, fo, fr, fa, nullptr, L, G);
            else
                ph_cheb<float, float, float, float, 3, SCHUR, false, false, true>(
                    a.A32, gsrc, a.tw32, a.r32, old, out32, fx, fo, fr, fa, nullptr, L, G);
            grid.sync();
        } else {
            double part;
            if (j == 1)
                part = ph_cheb<float, float, double, double, 1, SCHUR, true, false, true>(
                    a.A32, gsrc, a.tw32, a.r, (const float *)nullptr, a.z, fx, fo, fr, fa, nullptr, L, G);
            else if (j == 2)
                part = ph_cheb<float, float, double, double, 2, SCHUR, true, false, true>(
                    a.A32, gsrc, a.tw32, a.r, (const float *)nullptr, a.z, fx, fo, fr, fa, nullptr, L, G);
            else
                part = ph_cheb<float, float, double, double, 3, SCHUR, true, false, true>(
                    a.A32, gsrc, a.tw32, a.r, old, a.z, fx, fo, fr, fa, nullptr, L, G);
            return grid_sum(grid, c, part);
        }
    }
    return 0.0;
}

}  // namespace pcgp

template <bool SCHUR, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_pcg_persistent(PersistArgs a)
{
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ double lds[WPB];
    __shared__ double red;
    pcgp::Ctx c;
    c.G = (int)gridDim.x;
    c.L = xcd_remap((int)blockIdx.x, c.G);
    c.pbuf = 0;
    c.partials = a.partials;
    c.lds = lds;
    c.red = &red;
    const int L = c.L, G = c.G;
    const int64_t n = a.A.n;

    int it = 0, status = 1, zero_b = 0;
    double rho = 0.0, rr = 0.0;

    const double bn2 = pcgp::grid_sum(grid, c, ph_init_scale(n, a.b, a.x, a.dis, a.bh, a.xh, L, G));
    const double tol2 = a.tol * a.tol * bn2;
    if (!(bn2 < INFINITY)) {
        status = 2;
    } else if (bn2 == 0.0) {
        status = 0;
        zero_b = 1;
    } else {
        if (SCHUR) {
            ph_trace<double, double>(a.Cm, a.xh, a.tw, L, G);
            grid.sync();
        }
        rr = pcgp::grid_sum(grid, c, ph_init_resid<SCHUR>(a.A, a.xh, a.tw, a.bh, a.r, L, G));
        bool go = true;
        if (!(rr < INFINITY)) { status = 2; go = false; }
        else if (rr <= tol2) { status = 0; go = false; }
        else if (a.maxit <= 0) { status = 1; go = false; }
        if (go) {
            rho = pcgp::poly<SCHUR, MIXED>(grid, c, a);
            if (!finite_pos(rho)) { status = 2; go = false; }
        }
        if (go) {
            ph_p(n, a.z, a.p, 0.0, true, L, G);
            grid.sync();
            while (true) {
                if (SCHUR) {
                    ph_trace<double, double>(a.Cm, a.p, a.tw, L, G);
                    grid.sync();
                }
                const double gamma = pcgp::grid_sum(grid, c, ph_pq<SCHUR, true>(a.A, a.p, a.tw, a.q, L, G));
                if (!finite_pos(gamma)) { status = 2; break; }
                const double alpha = rho / gamma;
                rr = pcgp::grid_sum(grid, c, ph_xr(n, a.p, a.q, a.xh, a.r, alpha, L, G));
                it += 1;
                if (!(rr < INFINITY)) { status = 2; break; }
                if (rr <= tol2) { status = 0; break; }
                if (it >= a.maxit) { status = 1; break; }
                const double rho_new = pcgp::poly<SCHUR, MIXED>(grid, c, a);
                if (!finite_pos(rho_new)) { status = 2; break; }
                const double beta = rho_new / rho;
                rho = rho_new;
                ph_p(n, a.z, a.p, beta, false, L, G);
                grid.sync();
            }
        }
    }
    ph_final_x(n, a.xh, a.dis, a.x, zero_b != 0, L, G);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.st->it = it;
        a.st->status = status;
        a.st->rr = rr;
        a.st->bnorm2 = bn2;
        a.st->rho = rho;
        a.st->zero_b = zero_b;
        a.st->done = 1;
    }
}

}  // namespace ppk
