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
//
// Grid barriers.  The runtime's cooperative barrier costs about 0.1 us per
// workgroup (measured in a cooperative launch: 5.1 us at 32 workgroups, 104
// us at 1024).  Two hand-written barriers replace it (the runtime's stays
// selectable, mode 0):
//   flat (mode 1): every workgroup writes back the L2 (agent-scope release),
//     arrives on one counter and polls it until all G have arrived, then
//     acquires (invalidates L2 and L1);
//   two-level (mode 2): each XCD's workgroups arrive on a counter of their
//     own.  The last to arrive writes back that XCD's L2 once -- it holds the
//     other workgroups' stores, which each made complete at the L2 before
//     arriving -- and arrives on the global counter among the XCD leaders;
//     when all leaders are in, each invalidates its L2 and raises its XCD's
//     flag, which the other workgroups poll before invalidating their L1
//     (and L2) themselves.  Workgroups find their XCD from the hardware's
//     XCC_ID register and count themselves once per launch.
// Every counter only grows (barrier g completes at g times the arrivals),
// so nothing is reset between barriers; the host zeroes the words before
// each launch.  Every wait is bounded: after `spin` polls it raises a
// sticky abort word that all waiting workgroups also poll, every workgroup
// leaves the solve, and the launch reports PP_ERR_TIMEOUT.
#pragma once
#include <hip/hip_cooperative_groups.h>

#include "../../include/pp.h"
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
    unsigned long long *bw;  // barrier words, GB_LINES lines of GB_LINE, zeroed before the launch
    int bar_mode;            // 0 runtime barrier, 1 flat, 2 two-level
    unsigned int spin;       // polls before a barrier wait gives up
};

// barrier words: one 128-byte line each
constexpr int GB_LINE = 16;  // uint64 per line
constexpr int GB_GLOBAL = 0, GB_ABORT = 1, GB_CENSUS = 2, GB_XCD = 18, GB_FLAG = 34, GB_LINES = 50;

// zero n words (one workgroup, queued before each persistent launch)
static __global__ __launch_bounds__(BLOCK) void k_zero_u64(unsigned long long *p, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += BLOCK) p[i] = 0ull;
}

namespace pcgp {

struct Ctx {
    int L, G, pbuf;
    double *partials;
    double *lds;
    double *red;
    int *flag;                // LDS word: the barrier's outcome for the workgroup
    unsigned long long *bw;   // barrier words
    unsigned long long g;     // barriers passed
    int mode, xcd, xn, nx;    // barrier mode; XCD, its workgroups, XCDs in use
    unsigned int spin;
    int abort;                // a barrier wait timed out: leave the solve
};

using u64 = unsigned long long;

__device__ __forceinline__ u64 bw_load(u64 *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ u64 bw_add(u64 *p) { return __hip_atomic_fetch_add(p, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void bw_store(u64 *p, u64 v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// one thread: wait until *p >= target; false after c.spin polls (raising the
// abort word) or once another workgroup has raised it
__device__ bool bw_wait(Ctx &c, u64 *p, u64 target)
{
    u64 *ab = c.bw + GB_ABORT * GB_LINE;
    unsigned int n = 0;
    while (bw_load(p) < target) {
        if (++n > c.spin) {
            bw_store(ab, 1ull);
            return false;
        }
        if ((n & 63u) == 0u && bw_load(ab) != 0ull) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Barrier set-up: with the two-level barrier, count the workgroups of each
// XCD (one pass of the runtime's barrier).
__device__ void gbar_init(cooperative_groups::grid_group &grid, Ctx &c)
{
    c.g = 0;
    c.abort = 0;
    c.xcd = 0;
    c.xn = c.G;
    c.nx = 1;
    if (c.mode != 2) return;
    c.xcd = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15);  // HW_REG_XCC_ID, bits 3:0
    if (threadIdx.x == 0) bw_add(c.bw + (GB_CENSUS + c.xcd) * GB_LINE);
    grid.sync();
    c.xn = (int)bw_load(c.bw + (GB_CENSUS + c.xcd) * GB_LINE);
    c.nx = 0;
    for (int i = 0; i < 16; ++i) c.nx += bw_load(c.bw + (GB_CENSUS + i) * GB_LINE) != 0ull ? 1 : 0;
}

// Grid barrier.  Every workgroup reaches it in the same order (the scalars
// that steer the solve are identical everywhere); after an abort it returns
// at once and the caller leaves the solve.
__device__ void gbar(cooperative_groups::grid_group &grid, Ctx &c)
{
    if (c.mode == 0) {
        grid.sync();
        return;
    }
    if (c.abort) return;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        c.g += 1;
        bool ok;
        u64 *gc = c.bw + GB_GLOBAL * GB_LINE;
        if (c.mode == 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            bw_add(gc);
            ok = bw_wait(c, gc, c.g * (u64)c.G);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        } else {
            u64 *flag = c.bw + (GB_FLAG + c.xcd) * GB_LINE;
            if (bw_add(c.bw + (GB_XCD + c.xcd) * GB_LINE) + 1ull == c.g * (u64)c.xn) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                bw_add(gc);
                ok = bw_wait(c, gc, c.g * (u64)c.nx);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                bw_store(flag, c.g);
            } else {
                ok = bw_wait(c, flag, c.g);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        *c.flag = ok ? 0 : 1;
    }
    __syncthreads();
    if (*c.flag) c.abort = 1;
    __syncthreads();
}

// grid-wide sum of per-workgroup partials; the value is returned to every
// thread (NaN once a barrier has timed out, which ends the solve)
__device__ __forceinline__ double grid_sum(cooperative_groups::grid_group &grid, Ctx &c, double part)
{
    const double s = block_sum(part, c.lds);
    double *P = c.partials + (size_t)c.pbuf * c.G;
    c.pbuf ^= 1;
    if (threadIdx.x == 0) __hip_atomic_store(&P[c.L], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    gbar(grid, c);
    if (c.abort) return __builtin_nan("");
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
                gbar(grid, c);
                if (c.abort) return 0.0;
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
            gbar(grid, c);
            if (c.abort) return 0.0;
        }
        return 0.0;
    }
    // FP32 recurrence; the last step reads r in FP64 and writes z in FP64
    ph_scale<double, float, false>(n, a.r, 1.0, a.r32, L, G);
    gbar(grid, c);
    if (c.abort) return 0.0;
    for (int j = 1; j <= k; ++j) {
        const double *cf = a.coef + 4 * (j - 1);
        const float fx = (float)cf[0], fo = (float)cf[1], fr = (float)cf[2], fa = (float)cf[3];
        const bool last = (j == k);
        const float *gsrc = (j == 1) ? a.r32 : ((j % 2 == 0) ? a.sA32 : a.sB32);
        const float *old = (j % 2 == 0) ? a.sB32 : a.sA32;
        float *out32 = (j % 2 == 1) ? a.sA32 : a.sB32;
        if (SCHUR) {
            ph_trace<float, float>(a.Cm32, gsrc, a.tw32, L, G);
            gbar(grid, c);
            if (c.abort) return 0.0;
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
            gbar(grid, c);
            if (c.abort) return 0.0;
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
    __shared__ int bflag;
    pcgp::Ctx c;
    c.G = (int)gridDim.x;
    c.L = xcd_remap((int)blockIdx.x, c.G);
    c.pbuf = 0;
    c.partials = a.partials;
    c.lds = lds;
    c.red = &red;
    c.flag = &bflag;
    c.bw = a.bw;
    c.mode = a.bar_mode;
    c.spin = a.spin;
    pcgp::gbar_init(grid, c);
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
            pcgp::gbar(grid, c);
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
            pcgp::gbar(grid, c);
            while (!c.abort) {
                if (SCHUR) {
                    ph_trace<double, double>(a.Cm, a.p, a.tw, L, G);
                    pcgp::gbar(grid, c);
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
                pcgp::gbar(grid, c);
            }
        }
    }
    if (c.abort) status = (int)PP_ERR_TIMEOUT;
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
