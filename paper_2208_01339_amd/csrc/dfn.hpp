// The DFN Schur complement of section 4.2,
//   S_u = G^u - a B^T A^{-1} C - a C^T A^{-1} B + C^T A^{-1} G^h A^{-1} C,
// applied by Algorithm 3 with the exact Cholesky factor of the block-diagonal A.
//
// A's blocks are 2-D grids of G x G cells numbered by lines, so every entry lies
// within distance G of the diagonal and the factor L of a block is banded with
// the same half-width.  The factor is held by rows with its columns scaled by
// their diagonal, L~ = L D^{-1} (D = diag L): Lb[i * SP] = 1 / L(i, i) and
// Lb[i * SP + k] = L(i, i-k) / L(i-k, i-k), k = 1..G (zero where i-k leaves the
// block), SP = dfn_stride(G) >= G + 1 even, so a row loads as 16-byte vectors
// from one address.  With L~ the forward sweep gives y = D x for L x = b and
// the backward sweep takes x / L(i, i) = y / L(i, i)^2: every step of a sweep
// subtracts a coupling times an unscaled, broadcast value, with no division
// or product by a diagonal on the dependent chain.
//
// One wavefront owns one fracture.  The sweeps of the application read the
// factor rearranged by sweep step (k_dfn_qcoef): a sweep is a chain of nf
// steps, each finishing one row and broadcasting its value from the lane that
// holds it, while every lane takes that value's coupling off its own row.  All
// vectors of the block live in LDS during the solves of Algorithm 3.
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
    const double *Lb;       // band factor by rows, nh x dfn_stride(G) (+ DFN_GMAX + 2 padding); create only
    const double *Qf, *Qb;  // the factor by sweep steps, nh x G each (+ DFN_WAVE padding)
    const double *di2;      // 1 / L(i, i)^2, nh
    const int32_t *ghc;     // G^h by entry slots: entry j of row i at j nh + i (W = ghw slots,
    const double *ghv;      // padded with column i and value 0); ghw = 0: use the CSR gh
    int ghw;
    CsrD c, b, gh;          // rows of the fracture cells (b holds a B)
    CsrD ct, bt, gu;        // rows of the unknowns (bt holds a B^T)
};

// row stride of the factor in HBM (even, >= G + 1: rows load as 16-byte vectors)
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

// Lower band of A into Lb (zeroed before): Lb[i SP + (i - j)] = a_ij, j <= i.
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
            if (j <= i) Lb[i * dfn_stride((int)G) + (i - j)] += a.val[e];
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
// band on entry; L~ and 1 / L(i, i) on exit).  One wavefront per fracture, row by row:
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
        double s = act ? Lb[i * SP + (G - lane)] : 0.0;
        for (int q = 0; q < G; ++q) {
            const int64_t jq = il - G + q;
            if (jq < 0) continue;  // uniform
            const double yq = dfn_rdlane(s * rinv[jq % G], q);
            if (lane == q) s = yq;
            else if (act && lane > q) s -= ring[(jl % G) * SP + (lane - q)] * yq;
        }
        double sq = act ? s * s : 0.0;
        for (int o = DFN_WAVE / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
        const double d = Lb[i * SP] - sq;
        const bool ok = d > 0.0;
        const double lii = ok ? sqrt(d) : 1.0;
        if (!ok && lane == 0) atomicOr(bad, 4);
        __syncthreads();
        const int slot = (int)(il % G);
        // the ring keeps L itself (the recurrence needs it), Lb gets L~
        const double v = act ? s : 0.0;
        const double vs = act ? s * rinv[jl % G] : 0.0;
        __syncthreads();
        if (lane < G) {
            ring[slot * SP + (G - lane)] = v;
            Lb[i * SP + (G - lane)] = vs;
        }
        if (lane == 0) {
            ring[slot * SP] = lii;
            rinv[slot] = 1.0 / lii;
            Lb[i * SP] = 1.0 / lii;
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
    const int64_t nf = g.nf, f0 = (int64_t)f * nf;
    const int G = (int)g.G, SP = dfn_stride(G);
    double *y = yscr + (int64_t)blockIdx.x * nf * DFN_WAVE;
    int64_t pc = act ? g.ct.rp[j] : 0, pce = act ? g.ct.rp[j + 1] : 0;
    for (int64_t r = 0; r < nf; ++r) {
        const int64_t gr = f0 + r;
        double acc = 0.0;
        if (pc < pce && g.ct.col[pc] == gr) acc = g.ct.val[pc++];
        const int kmax = r < G ? (int)r : G;
        for (int k = kmax; k >= 1; --k) acc -= g.Lb[gr * SP + k] * ring[((r - k) & (DFN_GMAX - 1)) * DFN_WAVE + lane];
        ring[(r & (DFN_GMAX - 1)) * DFN_WAVE + lane] = acc;  // y = D (L^{-1} c)
        y[r * DFN_WAVE + lane] = acc;
    }
    double zgz = 0.0, zb = 0.0;
    int64_t pb = act ? g.bt.rp[j + 1] - 1 : -1;
    const int64_t pbe = act ? g.bt.rp[j] : 0;
    while (pb >= pbe && g.bt.col[pb] >= f0 + nf) --pb;
    for (int64_t r = nf - 1; r >= 0; --r) {
        const int64_t gr = f0 + r;
        const double iv = g.Lb[gr * SP];
        double acc = y[r * DFN_WAVE + lane] * iv * iv;
        const int kmax = nf - 1 - r < G ? (int)(nf - 1 - r) : G;
        for (int k = kmax; k >= 1; --k)
            acc -= g.Lb[(gr + k) * SP + k] * ring[((r + k) & (DFN_GMAX - 1)) * DFN_WAVE + lane];
        const double z = acc;
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

// Sweep layout of the factor.  Either triangular sweep of a block is one
// recurrence over its rows in sweep order (rows 0, 1, ... for L~; rows nf-1,
// nf-2, ... for L~^T), and sweep position p sits in lane p mod G: one grid line
// of G rows across the lanes.  At step p the value of position p is final.  Its
// lane broadcasts it, and every lane subtracts its row's coupling to that
// value; a lane's row is the next position of its residue class after p, at
// distance k = ((l - p - 1) mod G) + 1 in 1..G.  The broadcasting lane moves on
// to position p + G, and its coefficient carries an extra 1: the FMA clears
// the finished value and leaves only the new row's coupling to it.  Step p's
// coefficients for lanes 0..G-1 are stored together:
//   forward   Qf[p][l] = L~(p + k, p)
//   backward  Qb[p][l] = L~(nf-1-p, nf-1-p-k)
// plus 1 where l = p mod G, and 0 where the coupled row leaves the block (the
// forward sweep reads a column of L~ per step, the backward one a row).  Both
// arrays carry DFN_WAVE doubles of padding.  di2[i] = 1 / L(i, i)^2.
static __global__ __launch_bounds__(BLOCK) void k_dfn_qcoef(int64_t nh, int64_t nf, int G,
                                                            const double *__restrict__ Lb, double *__restrict__ Qf,
                                                            double *__restrict__ Qb, double *__restrict__ di2)
{
    const int SP = dfn_stride(G);
    const int64_t tot = nh * G;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < tot; e += (int64_t)gridDim.x * BLOCK) {
        const int64_t gp = e / G;
        const int l = (int)(e - gp * G);
        const int64_t f0 = gp / nf * nf, p = gp - f0;
        const int s = (int)(p % G);
        const int k = (l - s - 1 + 2 * G) % G + 1;
        const double one = l == s ? 1.0 : 0.0;
        const int64_t rf = p + k;  // forward: row p + k couples to row p
        Qf[e] = (rf < nf ? Lb[(f0 + rf) * SP + k] : 0.0) + one;
        const int64_t t = nf - 1 - p;  // backward: row t couples to row t - k
        Qb[e] = (t - k >= 0 ? Lb[(f0 + t) * SP + k] : 0.0) + one;
        if (l == 0) {
            const double v = Lb[gp * SP];
            di2[gp] = v * v;
        }
    }
}

// v_writelane through its LLVM intrinsic (clang exposes no builtin for it)
__device__ int dfn_writelane_i32(int v, int lane, int old) __asm("llvm.amdgcn.writelane");

// old with lane l replaced by the (uniform) value v
__device__ __forceinline__ double dfn_wrlane(double v, double old, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned long long o = (unsigned long long)__double_as_longlong(old);
    const int lo = dfn_writelane_i32((int)(unsigned)(u & 0xffffffffull), l, (int)(unsigned)(o & 0xffffffffull));
    const int hi = dfn_writelane_i32((int)(unsigned)(u >> 32), l, (int)(unsigned)(o >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The fracture kernels run one wavefront per workgroup, so LDS traffic between
// lanes needs only wavefront-scope ordering.
__device__ __forceinline__ void dfn_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One triangular sweep of a block, in place on its nf values X (LDS):
//   forward  (REV = false): X = D^{-2} L~^{-1} X   (di2: the block's 1/L(i,i)^2)
//   backward (REV = true):  X = L~^{-T} X
// so forward then backward gives A^{-1} X (A = L~ D^2 L~^T).  Q: the block's
// Qf or Qb.  A line of GM steps is unrolled (GM >= G; EX: GM == G) with the
// lane's coefficients in registers, two buffers used by alternate lines, so
// the loads of the lines ahead are in flight while this line runs.  Lanes
// G..63 hold no row and their values are never stored.
template <int GM, bool EX, bool REV>
__device__ __forceinline__ void dfn_sweep(const double *__restrict__ Q, const double *__restrict__ di2, int G,
                                          double *X)
{
    const int lane = threadIdx.x;
    const bool act = lane < G;
    const int64_t nf = (int64_t)G * G;
    const double *qp = Q + (act ? lane : 0);  // the lane's coefficient of step p: qp[p * G]
    auto row = [&](int K) -> int64_t {       // the row of line K in this lane
        const int64_t p = (int64_t)K * G + lane;
        return REV ? nf - 1 - p : p;
    };
    // coefficient q of the line starting at step nl.  Narrower blocks (not EX)
    // run all GM steps of a line: steps q >= G get coefficient 0 on every lane
    // and lanes >= G get 0 on every step, so those lanes stay 0 and those steps
    // change nothing (the loops stay fully unrolled, the buffers in registers).
    auto coef = [&](int64_t nl, int q) -> double {
        if (EX) return qp[(nl + q) * G];
        const double c = qp[(nl + (q < G ? q : 0)) * G];
        return (q < G && act) ? c : 0.0;
    };
    double ca[GM], cb[GM];
    double acc = act ? X[row(0)] : 0.0, fin = 0.0;
    // line K with coefficients cur; the next line's (the last line: its own again) into nxt
    // steps q0..q1-1 of the current line
    auto steps = [&](const double (&cur)[GM], int q0, int q1) {
#pragma unroll
        for (int q = 0; q < GM; ++q) {
            if (q < q0 || q >= q1) continue;
            const double v = dfn_rdlane(acc, q);
            fin = dfn_wrlane(v, fin, q);
            acc -= cur[q] * v;
        }
    };
    // HALF (lines of at most 48 steps): the first half of line K+2 is loaded
    // into the half of cur just used, the second half of line K+1 into nxt at
    // the start of line K, so every coefficient is requested 1.5 lines ahead.
    // Otherwise all of line K+1 into nxt at the start of line K (one line
    // ahead: the wider buffers would not fit the registers).
    constexpr bool HALF = GM <= 48;
    constexpr int H = HALF ? GM / 2 : 0;
    auto line = [&](int K, double (&cur)[GM], double (&nxt)[GM]) {
        const int64_t n1 = (int64_t)(K + 1 < G ? K + 1 : K) * G;
        const int64_t n2 = (int64_t)(K + 2 < G ? K + 2 : K) * G;
        const double sc = (!REV && act) ? di2[row(K)] : 1.0;
#pragma unroll
        for (int q = H; q < GM; ++q) nxt[q] = coef(n1, q);
        if constexpr (HALF) {
            steps(cur, 0, H);
#pragma unroll
            for (int q = 0; q < H; ++q) cur[q] = coef(n2, q);
            steps(cur, H, GM);
        } else {
            steps(cur, 0, GM);
        }
        if (act) X[row(K)] = REV ? fin : fin * sc;
        if (K + 1 < G && act) acc += X[row(K + 1)];
    };
#pragma unroll
    for (int q = 0; q < GM; ++q) ca[q] = coef(0, q);
#pragma unroll
    for (int q = 0; q < H; ++q) cb[q] = coef(1 < G ? G : 0, q);
    for (int K = 0; K < G; K += 2) {
        line(K, ca, cb);
        if (K + 1 < G) line(K + 1, cb, ca);
    }
}

// The fracture kernel's right-hand sides, one thread per cell (all fractures):
//   v = q + C (s.x),  z = a B (s.x)      (q, x, s may be NULL: zero / 1)
static __global__ __launch_bounds__(BLOCK) void k_dfn_cb(DfnView g, const double *__restrict__ x,
                                                         const double *__restrict__ s, const double *__restrict__ q,
                                                         double *__restrict__ vo, double *__restrict__ zo,
                                                         const State *st)
{
    if (st != nullptr && st->done) return;
    for (int64_t gi = (int64_t)blockIdx.x * BLOCK + threadIdx.x; gi < g.nh; gi += (int64_t)gridDim.x * BLOCK) {
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
        vo[gi] = v;
        zo[gi] = z;
    }
}

// G^h entry-slot layout from its CSR rows (one thread per row).
static __global__ __launch_bounds__(BLOCK) void k_dfn_ghell(int64_t nh, CsrD gh, int W, int32_t *__restrict__ ghc,
                                                            double *__restrict__ ghv)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nh; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t b = gh.rp[i], n = gh.rp[i + 1] - b;
        for (int j = 0; j < W; ++j) {
            ghc[j * nh + i] = j < n ? gh.col[b + j] : (int32_t)i;
            ghv[j * nh + i] = j < n ? gh.val[b + j] : 0.0;
        }
    }
}

// The longest row of a CSR matrix (atomicMax into *w).
static __global__ __launch_bounds__(BLOCK) void k_dfn_maxrow(int64_t n, const int64_t *__restrict__ rp, int *w)
{
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        m = max(m, (int)min<int64_t>(rp[i + 1] - rp[i], 1 << 30));
    if (m > 0) atomicMax(w, m);
}

constexpr int DFN_ELL_MAX = 16;  // widest G^h row kept in the entry-slot layout
constexpr int DFN_GH_ROWS = 36;  // rows per lane whose G^h loads are in flight together

// One fracture per wavefront (fracture = blockIdx.x), after k_dfn_cb wrote v
// to t and z to d:
//   t = A^{-1} v,  d = A^{-1} (z - G^h t)
// in place.  Algorithm 3 (q = 0) solves with A three times, for its t, its w
// and the w of its step 10; d is that w minus the latter, obtained with one
// solve since A^{-1} is linear.  With x = 0 they give the reduced right-hand
// side (t = A^{-1} q, d = -A^{-1} G^h A^{-1} q); with x = u they are the
// recovered h and p.  Dynamic LDS: 2 nf doubles.
template <int GM, bool EX>
static __global__ __launch_bounds__(DFN_WAVE) void k_dfn_frac(DfnView g, double *__restrict__ io_t,
                                                              double *__restrict__ io_d, const State *st)
{
    if (st != nullptr && st->done) return;
    extern __shared__ __align__(16) unsigned char dfn_lds[];
    const int lane = threadIdx.x;
    const int G = EX ? GM : (int)g.G;
    const int64_t nf = (int64_t)G * G, f0 = (int64_t)blockIdx.x * nf;
    double *X1 = (double *)dfn_lds, *X2 = X1 + nf;
#pragma unroll 18
    for (int64_t il = lane; il < nf; il += DFN_WAVE) {
        X1[il] = io_t[f0 + il];
        X2[il] = io_d[f0 + il];
    }
    const double *Qf = g.Qf + f0 * G, *Qb = g.Qb + f0 * G, *di2 = g.di2 + f0;
    dfn_wave_sync();
    dfn_sweep<GM, EX, false>(Qf, di2, G, X1);
    dfn_wave_sync();
    dfn_sweep<GM, EX, true>(Qb, di2, G, X1);
    dfn_wave_sync();
    if (g.ghw > 0) {
        // z - G^h t: the loads of DFN_GH_ROWS rows per lane go out together, slot by slot
        const int64_t nh = g.nh;
        for (int64_t b0 = lane; b0 < nf; b0 += (int64_t)DFN_GH_ROWS * DFN_WAVE) {
            double v[DFN_GH_ROWS];
#pragma unroll
            for (int m = 0; m < DFN_GH_ROWS; ++m) v[m] = 0.0;
            for (int j = 0; j < g.ghw; ++j) {
                const int32_t *cj = g.ghc + j * nh + f0;
                const double *vj = g.ghv + j * nh + f0;
#pragma unroll
                for (int m = 0; m < DFN_GH_ROWS; ++m) {
                    const int64_t il = b0 + (int64_t)m * DFN_WAVE;
                    if (il < nf) v[m] += vj[il] * X1[cj[il] - f0];
                }
            }
#pragma unroll
            for (int m = 0; m < DFN_GH_ROWS; ++m) {
                const int64_t il = b0 + (int64_t)m * DFN_WAVE;
                if (il < nf) {
                    io_t[f0 + il] = X1[il];
                    X2[il] -= v[m];
                }
            }
        }
    } else {
        for (int64_t il = lane; il < nf; il += DFN_WAVE) {
            const int64_t gi = f0 + il;
            double v = 0.0;
            for (int64_t e = g.gh.rp[gi]; e < g.gh.rp[gi + 1]; ++e) v += g.gh.val[e] * X1[g.gh.col[e] - f0];
            io_t[gi] = X1[il];
            X2[il] -= v;
        }
    }
    dfn_wave_sync();
    dfn_sweep<GM, EX, false>(Qf, di2, G, X2);
    dfn_wave_sync();
    dfn_sweep<GM, EX, true>(Qb, di2, G, X2);
    dfn_wave_sync();
    for (int64_t il = lane; il < nf; il += DFN_WAVE) io_d[f0 + il] = X2[il];
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
