// The DFN Schur complement of section 4.1,
//   S_u = G^u - a B^T A^{-1} C - a C^T A^{-1} B + C^T A^{-1} G^h A^{-1} C,
// applied by Algorithm 3 with the exact Cholesky factor of the block-diagonal A.
//
// A's blocks are 2-D grids of G x G cells numbered by lines, so every entry lies
// within distance G of the diagonal and the factor L of a block is banded with
// the same half-width.  The factor is held by diagonals, Lb[k * n_h + i] =
// L(i, i-k), k = 0..G (zero where i-k leaves the block).
//
// One wavefront owns one fracture.  A triangular sweep runs over the G grid
// lines of the block: lane l owns row l of the current line; the coupling to
// the previous (forward) or next (backward) line is a dense product, and the
// line's own lower (upper) triangle is solved in G steps, each finishing one
// row and broadcasting its value from that lane.  All vectors of the block
// live in LDS during the three solves of Algorithm 3.
#pragma once
#include "kernels.hpp"

namespace ppk {

constexpr int DFN_GMAX = 64;  // grid side (band half-width) of a fracture block
constexpr int DFN_WAVE = 64;

struct CsrD {
    const int64_t *rp;
    const int32_t *col;
    const double *val;
};

struct DfnView {
    int64_t F, G, nf, nh, nu;
    const double *Lb;       // band factor by diagonals, (G + 1) x nh
    CsrD c, b, gh;          // rows of the fracture cells (b holds a B)
    CsrD ct, bt, gu;        // rows of the unknowns (bt holds a B^T)
};

// LDS row stride of a staged line of the factor (even, >= G + 1)
__host__ __device__ constexpr int dfn_stride(int G) { return (G + 2) & ~1; }

__device__ __forceinline__ double dfn_rdlane(double v, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------

// Lower band of A into Lb (zeroed before): Lb[(i - j) nh + i] = a_ij, j <= i.
// bad = 1 for an entry outside its fracture block or farther than G from the
// diagonal.
static __global__ __launch_bounds__(BLOCK) void k_dfn_band(int64_t nh, int64_t nf, int64_t G, CsrD a,
                                                           double *__restrict__ Lb, int *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nh; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t f0 = i / nf * nf;
        for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            const int64_t j = a.col[e];
            if (j < f0 || j >= f0 + nf || j > i + G || j < i - G) {
                atomicOr(bad, 1);
                continue;
            }
            if (j <= i) Lb[(i - j) * nh + i] += a.val[e];
        }
    }
}

// bad |= 2 for an entry of a (n x n) without an equal mirrored entry, or for
// a row whose columns are not strictly ascending; bad |= 1 for an entry of a
// fracture-local matrix outside its block or band (nf > 0)
static __global__ __launch_bounds__(BLOCK) void k_dfn_sym(int64_t n, CsrD a, int64_t nf, int64_t G, int *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            const int64_t j = a.col[e];
            if (e > a.rp[i] && a.col[e - 1] >= j) atomicOr(bad, 2);
            if (nf > 0) {
                const int64_t f0 = i / nf * nf;
                if (j < f0 || j >= f0 + nf || j > i + G || j < i - G) atomicOr(bad, 1);
            }
            bool found = false;
            for (int64_t p = a.rp[j]; p < a.rp[j + 1]; ++p)
                if (a.col[p] == i) {
                    found = a.val[p] == a.val[e];
                    break;
                }
            if (!found) atomicOr(bad, 2);
        }
    }
}

// Exact Cholesky factor of every block, in place in Lb (which holds A's lower
// band on entry).  One wavefront per fracture, row by row:
//   L(i, j) = (a_ij - sum_{m<j} L(i, m) L(j, m)) / L(j, j)   for the G columns j < i,
//   L(i, i) = sqrt(a_ii - sum_{m<i} L(i, m)^2).
// Lane l holds column j = i - G + l; the G columns are finished in order, the
// last G rows of L kept in an LDS ring.  bad = 4 when a pivot is not positive.
static __global__ __launch_bounds__(DFN_WAVE) void k_dfn_chol(int64_t nh, int64_t nf, int G, double *__restrict__ Lb,
                                                              int *bad)
{
    __shared__ double ring[DFN_GMAX * (DFN_GMAX + 2)];
    __shared__ double rinv[DFN_GMAX];
    const int lane = threadIdx.x;
    const int SP = dfn_stride(G);
    const int64_t f0 = (int64_t)blockIdx.x * nf;
    for (int64_t il = 0; il < nf; ++il) {
        const int64_t i = f0 + il;
        const int64_t jl = il - G + lane;  // local column of this lane
        const bool act = lane < G && jl >= 0;
        double s = act ? Lb[(int64_t)(G - lane) * nh + i] : 0.0;
        for (int q = 0; q < G; ++q) {
            const int64_t jq = il - G + q;
            if (jq < 0) continue;  // uniform
            const double yq = dfn_rdlane(s * rinv[jq % G], q);
            if (lane == q) s = yq;
            else if (act && lane > q) s -= ring[(jl % G) * SP + (lane - q)] * yq;
        }
        double sq = act ? s * s : 0.0;
        for (int o = DFN_WAVE / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
        const double d = Lb[i] - sq;
        const bool ok = d > 0.0;
        const double lii = ok ? sqrt(d) : 1.0;
        if (!ok && lane == 0) atomicOr(bad, 4);
        __syncthreads();
        const int slot = (int)(il % G);
        if (lane < G) {
            const double v = act ? s : 0.0;
            ring[slot * SP + (G - lane)] = v;
            Lb[(int64_t)(G - lane) * nh + i] = v;
        }
        if (lane == 0) {
            ring[slot * SP] = lii;
            rinv[slot] = 1.0 / lii;
            Lb[i] = lii;
        }
        __syncthreads();
    }
}

// Transpose of a CSR matrix (rows x cols) into CSR by columns, scaled by `scale`:
// count, exclusive scan, fill, then sort every transposed row by its column so
// the result does not depend on the order of the atomic fill.
static __global__ __launch_bounds__(BLOCK) void k_t_count(int64_t rows, CsrD a, int64_t *__restrict__ cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < rows; i += (int64_t)gridDim.x * BLOCK)
        for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e)
            atomicAdd((unsigned long long *)&cnt[a.col[e]], 1ull);
}

static __global__ __launch_bounds__(1024) void k_scan_i64(int64_t n, const int64_t *__restrict__ cnt,
                                                          int64_t *__restrict__ off)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = (int64_t)t * chunk, hi = lo + chunk < n ? lo + chunk : n;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        off[i] = acc;
        acc += cnt[i];
    }
    if (t == 1023) off[n] = acc;
}

static __global__ __launch_bounds__(BLOCK) void k_t_fill(int64_t rows, CsrD a, double scale,
                                                         const int64_t *__restrict__ trp, int64_t *__restrict__ fillc,
                                                         int32_t *__restrict__ tcol, double *__restrict__ tval)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < rows; i += (int64_t)gridDim.x * BLOCK)
        for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            const int64_t c = a.col[e];
            const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&fillc[c], 1ull);
            tcol[trp[c] + pos] = (int32_t)i;
            tval[trp[c] + pos] = scale * a.val[e];
        }
}

static __global__ __launch_bounds__(BLOCK) void k_t_sort(int64_t rows, const int64_t *__restrict__ trp,
                                                         int32_t *__restrict__ tcol, double *__restrict__ tval)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < rows; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t lo = trp[i], hi = trp[i + 1];
        for (int64_t p = lo + 1; p < hi; ++p) {
            const int32_t c = tcol[p];
            const double v = tval[p];
            int64_t q = p - 1;
            while (q >= lo && tcol[q] > c) {
                tcol[q + 1] = tcol[q];
                tval[q + 1] = tval[q];
                --q;
            }
            tcol[q + 1] = c;
            tval[q + 1] = v;
        }
    }
}

// bad |= 8 when an entry of column j of C (row j of C^T) lies outside the block
// of the fracture that owns unknown j
static __global__ __launch_bounds__(BLOCK) void k_dfn_owner(int64_t nu, int64_t nf, CsrD ct,
                                                            const int32_t *__restrict__ owner, int *bad)
{
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < nu; j += (int64_t)gridDim.x * BLOCK)
        for (int64_t e = ct.rp[j]; e < ct.rp[j + 1]; ++e)
            if (ct.col[e] / nf != owner[j]) atomicOr(bad, 8);
}

// diag(S_u) by Algorithm 4:  z_j = A^{-1} c_j (c_j: column j of C, inside the
// owner's block), (D_S)_j = (G^u)_jj + z_j^T (G^h z_j) - 2 z_j^T (a b_j).
// One lane per unknown j, 64 unknowns of one fracture per workgroup
// (wg_frac / wg_first give the fracture and the first unknown).  The forward
// sweep keeps its last G values in an LDS ring and writes all of them to y
// (nf x 64 per workgroup); the backward sweep accumulates z^T G^h z from the
// ring (G^h couples within distance G) and z^T (a b_j) from the entries of B^T.
// dis[j] = D^{-1/2}; bad |= 16 for a non-positive D.
static __global__ __launch_bounds__(DFN_WAVE) void k_dfn_diag(DfnView g, const int32_t *__restrict__ wg_frac,
                                                              const int64_t *__restrict__ wg_first,
                                                              const int64_t *__restrict__ u_end,
                                                              double *__restrict__ yscr, double *__restrict__ dsv,
                                                              double *__restrict__ dis, int *bad)
{
    __shared__ double ring[DFN_GMAX * DFN_WAVE];
    const int lane = threadIdx.x;
    const int f = wg_frac[blockIdx.x];
    const int64_t j = wg_first[blockIdx.x] + lane;
    const bool act = j < u_end[f];
    const int64_t nf = g.nf, nh = g.nh, f0 = (int64_t)f * nf;
    const int G = (int)g.G;
    double *y = yscr + (int64_t)blockIdx.x * nf * DFN_WAVE;
    int64_t pc = act ? g.ct.rp[j] : 0, pce = act ? g.ct.rp[j + 1] : 0;
    for (int64_t r = 0; r < nf; ++r) {
        const int64_t gr = f0 + r;
        double acc = 0.0;
        if (pc < pce && g.ct.col[pc] == gr) acc = g.ct.val[pc++];
        const int kmax = r < G ? (int)r : G;
        for (int k = kmax; k >= 1; --k) acc -= g.Lb[(int64_t)k * nh + gr] * ring[((r - k) & (DFN_GMAX - 1)) * DFN_WAVE + lane];
        const double v = acc / g.Lb[gr];
        ring[(r & (DFN_GMAX - 1)) * DFN_WAVE + lane] = v;
        y[r * DFN_WAVE + lane] = v;
    }
    double zgz = 0.0, zb = 0.0;
    int64_t pb = act ? g.bt.rp[j + 1] - 1 : -1;
    const int64_t pbe = act ? g.bt.rp[j] : 0;
    while (pb >= pbe && g.bt.col[pb] >= f0 + nf) --pb;
    for (int64_t r = nf - 1; r >= 0; --r) {
        const int64_t gr = f0 + r;
        double acc = y[r * DFN_WAVE + lane];
        const int kmax = nf - 1 - r < G ? (int)(nf - 1 - r) : G;
        for (int k = kmax; k >= 1; --k)
            acc -= g.Lb[(int64_t)k * nh + gr + k] * ring[((r + k) & (DFN_GMAX - 1)) * DFN_WAVE + lane];
        const double z = acc / g.Lb[gr];
        double gz = 0.0;
        for (int64_t e = g.gh.rp[gr]; e < g.gh.rp[gr + 1]; ++e) {
            const int64_t c = g.gh.col[e];
            if (c == gr) gz += g.gh.val[e] * z;
            else if (c > gr) gz += 2.0 * g.gh.val[e] * ring[((c - f0) & (DFN_GMAX - 1)) * DFN_WAVE + lane];
        }
        zgz += z * gz;
        ring[(r & (DFN_GMAX - 1)) * DFN_WAVE + lane] = z;
        if (pb >= pbe && g.bt.col[pb] == gr) zb += z * g.bt.val[pb--];
    }
    if (act) {
        double gjj = 0.0;
        for (int64_t e = g.gu.rp[j]; e < g.gu.rp[j + 1]; ++e)
            if (g.gu.col[e] == j) gjj += g.gu.val[e];
        const double d = gjj + zgz - 2.0 * zb;
        dsv[j] = d;
        if (d > 0.0 && d < INFINITY) dis[j] = 1.0 / sqrt(d);
        else atomicOr(bad, 16);
    }
}

// ---------------------------------------------------------------------------
// application (Algorithm 3), right-hand side and recovery
// ---------------------------------------------------------------------------

// L x = b for NR right-hand sides held in LDS (in place), one wavefront.
template <int NR>
__device__ __forceinline__ void dfn_fwd(const DfnView &g, int64_t f0, double *const (&X)[NR], double *LS)
{
    const int lane = threadIdx.x, G = (int)g.G, SP = dfn_stride(G);
    const int64_t nh = g.nh;
    const bool act = lane < G;
    for (int K = 0; K < G; ++K) {
        const int il = K * G + lane;
        double Lr[DFN_GMAX + 1];
#pragma unroll
        for (int k = 0; k <= DFN_GMAX; ++k) Lr[k] = (act && k <= G) ? g.Lb[(int64_t)k * nh + f0 + il] : 0.0;
        if (act) {
#pragma unroll
            for (int k = 0; k <= DFN_GMAX; ++k)
                if (k <= G) LS[lane * SP + k] = Lr[k];
        }
        double s[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] = act ? X[r][il] : 0.0;
        if (K > 0) {
#pragma unroll
            for (int k = 1; k <= DFN_GMAX; ++k)
                if (act && k <= G && k > lane) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) s[r] -= Lr[k] * X[r][il - k];
                }
        }
        __syncthreads();
        const double inv = act ? 1.0 / Lr[0] : 0.0;
        for (int q = 0; q < G; ++q) {
            double xq[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) xq[r] = dfn_rdlane(s[r] * inv, q);
            if (lane == q) {
#pragma unroll
                for (int r = 0; r < NR; ++r) s[r] = xq[r];
            } else if (act && lane > q) {
                const double l = LS[lane * SP + (lane - q)];
#pragma unroll
                for (int r = 0; r < NR; ++r) s[r] -= l * xq[r];
            }
        }
        if (act) {
#pragma unroll
            for (int r = 0; r < NR; ++r) X[r][il] = s[r];
        }
        __syncthreads();
    }
}

// L^T x = b for NR right-hand sides in LDS (in place); LSa, LSb: two staged lines.
template <int NR>
__device__ __forceinline__ void dfn_bwd(const DfnView &g, int64_t f0, double *const (&X)[NR], double *LSa, double *LSb)
{
    const int lane = threadIdx.x, G = (int)g.G, SP = dfn_stride(G);
    const int64_t nh = g.nh;
    const bool act = lane < G;
    double *cur = LSa, *nxt = LSb;
    for (int K = G - 1; K >= 0; --K) {
        const int il = K * G + lane;
        if (act)
            for (int k = 0; k <= G; ++k) cur[lane * SP + k] = g.Lb[(int64_t)k * nh + f0 + il];
        __syncthreads();
        double s[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] = act ? X[r][il] : 0.0;
        if (K < G - 1 && act) {
            // rows (K+1) G + m of the next line couple at distance G + m - lane <= G
            for (int m = 0; m <= lane; ++m) {
                const double l = nxt[m * SP + (G + m - lane)];
#pragma unroll
                for (int r = 0; r < NR; ++r) s[r] -= l * X[r][(K + 1) * G + m];
            }
        }
        const double inv = act ? 1.0 / cur[lane * SP] : 0.0;
        for (int q = G - 1; q >= 0; --q) {
            double xq[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) xq[r] = dfn_rdlane(s[r] * inv, q);
            if (lane == q) {
#pragma unroll
                for (int r = 0; r < NR; ++r) s[r] = xq[r];
            } else if (act && lane < q) {
                const double l = cur[q * SP + (q - lane)];
#pragma unroll
                for (int r = 0; r < NR; ++r) s[r] -= l * xq[r];
            }
        }
        if (act) {
#pragma unroll
            for (int r = 0; r < NR; ++r) X[r][il] = s[r];
        }
        __syncthreads();
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
}

// One fracture per wavefront (fracture = blockIdx.x):
//   v = q + C (s.x),  z = a B (s.x)      (q, x, s may be NULL: zero / 1)
//   t = A^{-1} v,  w = A^{-1} z,  w2 = A^{-1} (G^h t),  d = w - w2
// and t, d to HBM.  For Algorithm 3 (q = 0) these are the t of its step 4 and
// the w of step 6 minus the w of step 10; with x = 0 they give the reduced
// right-hand side (t = A^{-1} q, d = -A^{-1} G^h A^{-1} q); with x = u they are
// the recovered h and p.  Dynamic LDS: 2 nf + 2 G SP doubles.
static __global__ __launch_bounds__(DFN_WAVE) void k_dfn_frac(DfnView g, const double *__restrict__ x,
                                                              const double *__restrict__ s,
                                                              const double *__restrict__ q, double *__restrict__ out_t,
                                                              double *__restrict__ out_d, const State *st)
{
    if (st != nullptr && st->done) return;
    extern __shared__ __align__(16) unsigned char dfn_lds[];
    const int lane = threadIdx.x;
    const int G = (int)g.G, SP = dfn_stride(G);
    const int64_t nf = g.nf, f0 = (int64_t)blockIdx.x * nf;
    double *X1 = (double *)dfn_lds, *X2 = X1 + nf, *LSa = X2 + nf, *LSb = LSa + (int64_t)G * SP;
    for (int64_t il = lane; il < nf; il += DFN_WAVE) {
        const int64_t gi = f0 + il;
        double v = q ? q[gi] : 0.0, z = 0.0;
        if (x) {
            for (int64_t e = g.c.rp[gi]; e < g.c.rp[gi + 1]; ++e) {
                const int64_t c = g.c.col[e];
                v += g.c.val[e] * (s ? s[c] * x[c] : x[c]);
            }
            for (int64_t e = g.b.rp[gi]; e < g.b.rp[gi + 1]; ++e) {
                const int64_t c = g.b.col[e];
                z += g.b.val[e] * (s ? s[c] * x[c] : x[c]);
            }
        }
        X1[il] = v;
        X2[il] = z;
    }
    __syncthreads();
    {
        double *const XX[2] = {X1, X2};
        dfn_fwd<2>(g, f0, XX, LSa);
        dfn_bwd<2>(g, f0, XX, LSa, LSb);
    }
    for (int64_t il = lane; il < nf; il += DFN_WAVE) {
        out_t[f0 + il] = X1[il];
        out_d[f0 + il] = X2[il];
    }
    __syncthreads();
    for (int64_t il = lane; il < nf; il += DFN_WAVE) {
        const int64_t gi = f0 + il;
        double v = 0.0;
        for (int64_t e = g.gh.rp[gi]; e < g.gh.rp[gi + 1]; ++e) v += g.gh.val[e] * X1[g.gh.col[e] - f0];
        X2[il] = v;
    }
    __syncthreads();
    {
        double *const XX[1] = {X2};
        dfn_fwd<1>(g, f0, XX, LSa);
        dfn_bwd<1>(g, f0, XX, LSa, LSb);
    }
    for (int64_t il = lane; il < nf; il += DFN_WAVE) out_d[f0 + il] = out_d[f0 + il] - X2[il];
}

// Rows of the unknowns:  y = s .* (cg G^u (s.x) + cb (a B^T) t + cc C^T d)
// (s may be NULL: 1; x may be NULL when cg = 0).  Algorithm 3: cg = 1,
// cb = cc = -1 gives G^u r - a B^T t - C^T (w - w2) = its y.  Right-hand side:
// cg = 0, cb = cc = 1.
static __global__ __launch_bounds__(BLOCK) void k_dfn_urow(DfnView g, const double *__restrict__ x,
                                                           const double *__restrict__ s,
                                                           const double *__restrict__ t,
                                                           const double *__restrict__ d, double cg, double cb,
                                                           double cc, double *__restrict__ y, const State *st)
{
    if (st != nullptr && st->done) return;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < g.nu; j += (int64_t)gridDim.x * BLOCK) {
        double a = 0.0, b = 0.0, c = 0.0;
        if (cg != 0.0)
            for (int64_t e = g.gu.rp[j]; e < g.gu.rp[j + 1]; ++e) {
                const int64_t k = g.gu.col[e];
                a += g.gu.val[e] * (s ? s[k] * x[k] : x[k]);
            }
        for (int64_t e = g.bt.rp[j]; e < g.bt.rp[j + 1]; ++e) b += g.bt.val[e] * t[g.bt.col[e]];
        for (int64_t e = g.ct.rp[j]; e < g.ct.rp[j + 1]; ++e) c += g.ct.val[e] * d[g.ct.col[e]];
        const double v = cg * a + cb * b + cc * c;
        y[j] = s ? s[j] * v : v;
    }
}

static __global__ __launch_bounds__(BLOCK) void k_dfn_axv(int64_t n, double a, const double *__restrict__ x,
                                                          double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) y[i] = a * x[i];
}

// Slice layout with one unit entry per row at column n + i: the fused kernels'
// trace-column path then reads (A x)_i from the vector Algorithm 3 wrote.
static __global__ __launch_bounds__(BLOCK) void k_dfn_unit(int64_t n, int64_t nslices, int64_t *__restrict__ sp,
                                                           int32_t *__restrict__ scol, double *__restrict__ sval)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nslices * WAVE; i += (int64_t)gridDim.x * BLOCK) {
        scol[i] = i < n ? (int32_t)(n + i) : 0;
        sval[i] = i < n ? 1.0 : 0.0;
        if (i % WAVE == 0) sp[i / WAVE] = i;
        if (i == 0) sp[nslices] = nslices * WAVE;
    }
}

}  // namespace ppk
