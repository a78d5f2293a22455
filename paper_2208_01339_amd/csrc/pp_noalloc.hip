// pcg_solve_csr_noalloc: polynomial-preconditioned CG on a plain CSR matrix
// that allocates nothing.  Every work vector, the per-workgroup partial sums
// and the CG state live in one file-scope device array (`scratch`) of fixed
// size; the entry point only queues kernels, copies a few bytes of state to
// the host and synchronises.  It serves callers that cannot allocate device
// memory (code between graph captures, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The method is the one pcg_solve runs (standard PCG with P = p_k(A) on
// [lambda_min, lambda_max] and the centre moved by xi, section 2.2 and
// eq. thetamod of section 2.4; Algorithm 2 for P r; optional Jacobi scaling,
// the diagonal seed of section 3), on the caller's CSR arrays as they are:
// one kernel per polynomial step reads the CSR rows with eight lanes per row
// and applies the three-term update in the same pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace {

using ppc::fail;
using ppc::HipError;
using ppk::BLOCK;
using ppk::State;
using ppk::xcd_remap;

constexpr int64_t NA_NMAX = int64_t(1) << 20;  // rows
constexpr int NA_GMAX = 2048;                  // workgroups per launch
constexpr int NA_NVEC = 9;                     // dis, bh, xh, r, p, q, z, two step buffers
constexpr int NA_KMAX = 1024;                  // polynomial degree
constexpr int NA_LPR = 8;                      // lanes per CSR row
constexpr size_t NA_STATE_BYTES = (sizeof(State) + 255) / 256 * 256;
constexpr size_t NA_PART_OFF = NA_STATE_BYTES;
constexpr size_t NA_VEC_OFF = NA_PART_OFF + (size_t)NA_GMAX * sizeof(double);
constexpr size_t NA_SCRATCH_BYTES = NA_VEC_OFF + (size_t)NA_NVEC * (size_t)NA_NMAX * sizeof(double);

}  // namespace

// The scratch memory of pcg_solve_csr_noalloc (about 72 MiB; one copy per
// device, held until the process ends).  Host code never passes this name to
// a kernel: it is a host-side stand-in, and the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

namespace {

// ---------------------------------------------------------------------------
// kernels on the caller's CSR arrays
// ---------------------------------------------------------------------------

enum : int { NA_RESID = 0, NA_PQ = 1, NA_STEP = 2 };

// One CSR row per group of NA_LPR lanes (32 rows per pass of a workgroup over
// its contiguous row range).  y_i = (A-hat x)_i with A-hat = D^{-1/2} A D^{-1/2}
// when dis is given, then per mode:
//   NA_RESID: out_i = r_i - y_i                  partial sum of out_i^2
//   NA_PQ:    out_i = y_i                        partial sum of x_i out_i
//   NA_STEP:  out_i = cx x_i + cold sold_i + cr r_i + cA y_i,
//                                                partial sum of r_i out_i when DOT
// sold may be out itself (a step overwrites s_{j-2}): each element is read
// before it is written, by the same lane.
template <int MODE, bool JAC, bool DOT>
__global__ __launch_bounds__(BLOCK) void k_na_csr(int64_t n, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  const double *__restrict__ dis, const double *__restrict__ x,
                                                  const double *__restrict__ r, const double *sold, double *out,
                                                  double cx, double cold, double cr, double cA, double *partials,
                                                  State *st)
{
    PPK_PROLOGUE(st)
    int64_t r0, r1;
    ppk::block_range(n, L, G, r0, r1);
    const int sub = (int)threadIdx.x % NA_LPR;
    const int grp = (int)threadIdx.x / NA_LPR;
    constexpr int RPP = BLOCK / NA_LPR;  // rows per pass
    double part = 0.0;
    for (int64_t base = r0; base < r1; base += RPP) {
        const int64_t i = base + grp;
        const bool live = i < r1;
        double s = 0.0;
        if (live) {
            const int64_t p0 = rp[i], p1 = rp[i + 1];
            for (int64_t p = p0 + sub; p < p1; p += NA_LPR) {
                const int32_t c = col[p];
                const double xv = JAC ? dis[c] * x[c] : x[c];
                s += val[p] * xv;
            }
        }
        // fixed-order tree over the row's lanes
#pragma unroll
        for (int off = NA_LPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, NA_LPR);
        if (live && sub == 0) {
            const double y = JAC ? dis[i] * s : s;
            if (MODE == NA_RESID) {
                const double o = r[i] - y;
                out[i] = o;
                part += o * o;
            } else if (MODE == NA_PQ) {
                out[i] = y;
                part += x[i] * y;
            } else {
                const double so = cold != 0.0 ? sold[i] : 0.0;
                const double o = cx * x[i] + cold * so + cr * r[i] + cA * y;
                out[i] = o;
                if (DOT) part += r[i] * o;
            }
        }
    }
    if (MODE != NA_STEP || DOT) ppk::store_partial(part, partials, L);
}

// dis_i = 1 / sqrt(a_ii) (sum of the row's entries in column i); a row
// without a positive diagonal ends the solve with PP_ERR_ARG.
__global__ __launch_bounds__(BLOCK) void k_na_dis(int64_t n, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const double *__restrict__ val, double *__restrict__ dis,
                                                  State *st)
{
    const int G = (int)gridDim.x;
    const int L = ppk::xcd_remap((int)blockIdx.x, G);
    ppk::for_my_elems(n, L, G, [&](int64_t i) {
        double d = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (col[p] == i) d += val[p];
        if (d > 0.0 && d < INFINITY) {
            dis[i] = 1.0 / sqrt(d);
        } else {
            dis[i] = 0.0;
            st->status = (int32_t)PP_ERR_ARG;  // every such row writes the same values
            st->done = 1;
        }
    });
}

// z = c r (degree 0), partial sum of r_i z_i
__global__ __launch_bounds__(BLOCK) void k_na_deg0(int64_t n, const double *__restrict__ r, double c,
                                                   double *__restrict__ z, double *partials, State *st)
{
    PPK_PROLOGUE(st)
    double part = 0.0;
    ppk::for_my_elems(n, L, G, [&](int64_t i) {
        const double zi = c * r[i];
        z[i] = zi;
        part += r[i] * zi;
    });
    ppk::store_partial(part, partials, L);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

constexpr int NA_MAXDEV = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[NA_MAXDEV] = {};
int g_na_grid[NA_MAXDEV] = {};

// Device address of `scratch` on the current device, looked up once per device.
pp_status na_scratch(unsigned char **ptr, int *grid)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAXDEV) {
        (void)hipGetLastError();
        return fail(PP_ERR_HIP, "pcg_solve_csr_noalloc: no current device");
    }
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return fail(PP_ERR_HIP, std::string("pcg_solve_csr_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                                        hipGetErrorString(e));
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
            (void)hipGetLastError();
            cus = 256;
        }
        g_na_grid[dev] = std::min(NA_GMAX, 8 * cus);
        g_na_ptr[dev] = (unsigned char *)p;
    }
    *ptr = g_na_ptr[dev];
    *grid = g_na_grid[dev];
    return PP_OK;
}

struct NaStep {
    double cx, cold, cr, cA;
};

// Coefficients of Algorithm 2's steps in the form
// out = cx x + cold s_{j-2} + cr r + cA (A x), x = s_{j-1}:
//   step 1 (x = r): (2 rho_1 / delta)(2 r - A r / theta)
//   step j >= 2:    rho_j (2 sigma x - rho_{j-1} s_{j-2} + (2 / delta)(r - A x))
// with theta the centre theta-bar = (lmax + lmin)/2 (1 + xi).  s_0 = r / theta
// is never stored: step 2's s_{j-2} term is folded into its r coefficient.
std::vector<NaStep> na_steps(int k, double lmin, double lmax, double xi, double *theta)
{
    const double th = (lmax + lmin) / 2.0 * (1.0 + xi);
    const double de = (lmax - lmin) / 2.0;
    const double si = th / de;
    std::vector<double> rho((size_t)k + 1);
    rho[0] = 1.0 / si;
    for (int j = 1; j <= k; ++j) rho[j] = 1.0 / (2.0 * si - rho[j - 1]);
    std::vector<NaStep> c((size_t)k);
    for (int j = 1; j <= k; ++j) {
        NaStep s;
        if (j == 1) {
            s = {0.0, 0.0, 4.0 * rho[1] / de, -2.0 * rho[1] / (de * th)};
        } else {
            s = {2.0 * si * rho[j], -rho[j] * rho[j - 1], 2.0 * rho[j] / de, -2.0 * rho[j] / de};
            if (j == 2) {
                s.cr += s.cold / th;
                s.cold = 0.0;
            }
        }
        c[(size_t)j - 1] = s;
    }
    *theta = th;
    return c;
}

struct NaCtx {
    int64_t n;
    const int64_t *rp;
    const int32_t *col;
    const double *val;
    const double *dis;  // null without Jacobi
    int G;
    double *partials;
    State *st;
    hipStream_t s;
};

void na_fin(const NaCtx &c, int fin)
{
    hipLaunchKernelGGL(ppk::k_fin, dim3(1), dim3(BLOCK), 0, c.s, (const double *)c.partials, c.G, c.st, fin, 0);
}

template <int MODE, bool DOT>
void na_csr(const NaCtx &c, const double *x, const double *r, const double *sold, double *out, const NaStep &k)
{
    if (c.dis)
        hipLaunchKernelGGL((k_na_csr<MODE, true, DOT>), dim3(c.G), dim3(BLOCK), 0, c.s, c.n, c.rp, c.col, c.val,
                           c.dis, x, r, sold, out, k.cx, k.cold, k.cr, k.cA, c.partials, c.st);
    else
        hipLaunchKernelGGL((k_na_csr<MODE, false, DOT>), dim3(c.G), dim3(BLOCK), 0, c.s, c.n, c.rp, c.col, c.val,
                           c.dis, x, r, sold, out, k.cx, k.cold, k.cr, k.cA, c.partials, c.st);
}

// z = p_k(A-hat) r, and r.z into the state by `fin` (FIN_RHO0 / FIN_RHO)
void na_poly(const NaCtx &c, const std::vector<NaStep> &steps, double theta, const double *r, double *z,
             double *sa, double *sb, int fin)
{
    const int k = (int)steps.size();
    if (k == 0) {
        hipLaunchKernelGGL(k_na_deg0, dim3(c.G), dim3(BLOCK), 0, c.s, c.n, r, 1.0 / theta, z, c.partials, c.st);
        na_fin(c, fin);
        return;
    }
    // s_{j-1} in x, s_{j-2} in old; the last step writes z
    const double *x = r;
    double *old = sb, *cur = sa;
    for (int j = 1; j <= k; ++j) {
        double *out = j == k ? z : (j == 1 ? sa : old);
        if (j == k)
            na_csr<NA_STEP, true>(c, x, r, old, out, steps[(size_t)j - 1]);
        else
            na_csr<NA_STEP, false>(c, x, r, old, out, steps[(size_t)j - 1]);
        if (j == 1) {
            x = sa;
            old = sb;
            cur = sa;
        } else {
            old = cur;
            cur = out;
            x = out;
        }
    }
    na_fin(c, fin);
}

}  // namespace

extern "C" {

pp_status pcg_solve_csr_noalloc(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *colind,
                                const double *val, unsigned flags, int k, double lambda_min, double lambda_max,
                                double scaling, const double *b, double *x, double tol, int maxit, int *iters,
                                double *relres, void *stream)
{
    if (n <= 0 || nnz < 0) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: n must be > 0 and nnz >= 0");
    if (n > NA_NMAX)
        return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: n exceeds the scratch capacity of 1048576 rows "
                                "(use pp_create_csr and pcg_solve)");
    if (nnz > INT64_C(1) << 31) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: nnz must fit 31 bits");
    if (!rowptr || !colind || !val || !b || !x) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: NULL argument");
    if (b == x) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: b and x must not alias");
    if ((flags & ~(unsigned)PP_JACOBI) != 0)
        return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: flags may only hold PP_JACOBI");
    if (k < 0 || k > NA_KMAX) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: k must be in [0, 1024]");
    if (!std::isfinite(lambda_min) || !std::isfinite(lambda_max) || !(lambda_min > 0.0) ||
        !(lambda_max > lambda_min))
        return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: need finite 0 < lambda_min < lambda_max");
    if (!std::isfinite(scaling) || scaling < 0.0) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: xi must be >= 0");
    if (!std::isfinite(tol) || tol < 0.0) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: tol must be >= 0");
    if (maxit < 0) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: maxit must be >= 0");
    unsigned char *base = nullptr;
    int gdev = 0;
    pp_status ps = na_scratch(&base, &gdev);
    if (ps != PP_OK) return ps;
    try {
        NaCtx c;
        c.n = n;
        c.rp = rowptr;
        c.col = colind;
        c.val = val;
        c.G = (int)std::max<int64_t>(1, std::min<int64_t>(gdev, (n + BLOCK - 1) / BLOCK));
        c.st = (State *)base;
        c.partials = (double *)(base + NA_PART_OFF);
        c.s = (hipStream_t)stream;
        double *vec = (double *)(base + NA_VEC_OFF);
        double *dis = vec, *bh = vec + n, *xh = vec + 2 * n, *r = vec + 3 * n, *p = vec + 4 * n, *q = vec + 5 * n,
               *z = vec + 6 * n, *sa = vec + 7 * n, *sb = vec + 8 * n;
        c.dis = (flags & PP_JACOBI) ? dis : nullptr;
        double theta = 0.0;
        const std::vector<NaStep> steps = na_steps(k, lambda_min, lambda_max, scaling, &theta);
        const NaStep none{0.0, 0.0, 0.0, 0.0};
        const int ge = c.G;

        // the state and every vector are written before they are read
        hipLaunchKernelGGL(ppk::k_state_init, dim3(1), dim3(64), 0, c.s, c.st, tol, maxit);
        if (c.dis) {
            hipLaunchKernelGGL(k_na_dis, dim3(ge), dim3(BLOCK), 0, c.s, n, rowptr, colind, val, dis, c.st);
            int32_t bad = 0;
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(&bad, &c.st->done, sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
            HIPCHK(hipStreamSynchronize(c.s));
            if (bad) return fail(PP_ERR_ARG, "pcg_solve_csr_noalloc: a diagonal entry is not positive");
        }
        hipLaunchKernelGGL(ppk::k_init_scale, dim3(ge), dim3(BLOCK), 0, c.s, n, b, (const double *)x,
                           (const double *)c.dis, bh, xh, c.partials, c.st, (const int32_t *)nullptr);
        na_fin(c, ppk::FIN_BNORM);
        na_csr<NA_RESID, true>(c, xh, bh, nullptr, r, none);
        na_fin(c, ppk::FIN_RR0);
        na_poly(c, steps, theta, r, z, sa, sb, ppk::FIN_RHO0);
        hipLaunchKernelGGL(ppk::k_p, dim3(ge), dim3(BLOCK), 0, c.s, n, (const double *)z, p, (const State *)c.st, 1);
        HIPCHK(hipGetLastError());
        // chunks of iterations; the done flag (set on the device by the
        // convergence test) is read back after each chunk, synchronously
        const int chunk = n >= (1 << 16) ? 4 : 8;
        int32_t done = 0;
        for (int enq = 0; enq < maxit && !done;) {
            const int m = std::min(chunk, maxit - enq);
            for (int i = 0; i < m; ++i) {
                na_csr<NA_PQ, true>(c, p, nullptr, nullptr, q, none);
                na_fin(c, ppk::FIN_GAMMA);
                hipLaunchKernelGGL(ppk::k_xr, dim3(ge), dim3(BLOCK), 0, c.s, n, (const double *)p, (const double *)q,
                                   xh, r, c.partials, c.st, (float *)nullptr);
                na_fin(c, ppk::FIN_RR);
                na_poly(c, steps, theta, r, z, sa, sb, ppk::FIN_RHO);
                hipLaunchKernelGGL(ppk::k_p, dim3(ge), dim3(BLOCK), 0, c.s, n, (const double *)z, p,
                                   (const State *)c.st, 0);
            }
            HIPCHK(hipGetLastError());
            enq += m;
            HIPCHK(hipMemcpyAsync(&done, &c.st->done, sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
            HIPCHK(hipStreamSynchronize(c.s));
        }
        hipLaunchKernelGGL(ppk::k_final_x, dim3(ge), dim3(BLOCK), 0, c.s, n, (const double *)xh,
                           (const double *)c.dis, x, (const State *)c.st, (const int32_t *)nullptr);
        HIPCHK(hipGetLastError());
        State hs;
        HIPCHK(hipMemcpyAsync(&hs, c.st, sizeof(State), hipMemcpyDeviceToHost, c.s));
        HIPCHK(hipStreamSynchronize(c.s));
        pp_status ret = (pp_status)hs.status;
        double rel = hs.bnorm2 > 0 ? std::sqrt(hs.rr / hs.bnorm2) : 0.0;
        if (hs.zero_b) {
            ret = PP_OK;
            rel = 0.0;
        }
        if (iters) *iters = hs.it;
        if (relres) *relres = rel;
        return ret;
    } catch (HipError &e) {
        return ppc::hip_fail(e);
    }
}

}  // extern "C"
