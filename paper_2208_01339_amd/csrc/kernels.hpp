// Device code for polynomial-preconditioned CG on gfx950 (CDNA4).
//
// Layout.  Rows are grouped in slices of 64 (one wavefront, one lane per
// row).  The operator has up to two parts:
//  * symmetric stored diagonals: for each densely populated column offset
//    o >= 0 one array of a_{i,i+o}; the mirrored entry a_{i,i-o} = a_{i-o,i}
//    is the same array read o places back (a cache hit: rows i - o were
//    streamed moments before by a workgroup of the same XCD), so a symmetric
//    stencil is read at half its CSR value bytes and with no column indices;
//  * a wavefront-row-group ("sliced ELLPACK") part for everything else: inside
//    a slice the j-th stored entry of all 64 rows is contiguous, so every
//    load of values and column indices is a fully coalesced 512 B (FP64) or
//    256 B (int32 / FP32) wave access; a slice is padded to its longest row
//    with (col = own row, val = 0).  For the Schur shape the trace term C^T w
//    is appended to the rows as extra columns n + t that index the trace
//    vector w.
//
// Scheduling.  Every streaming kernel runs a fixed grid of G workgroups of
// 256 threads.  Workgroup b runs on XCD b % 8; it is remapped so that the G/8
// workgroups of one XCD cover one contiguous eighth of the rows, and each
// workgroup owns a contiguous range of slices (its four waves interleave over
// it).  Neighbouring rows of a stencil-like operator are then gathered from
// the same XCD's L2.
//
// Reductions are deterministic: a fixed-order wave shuffle tree, a fixed
// order over the waves of a workgroup, one partial per workgroup, and a
// one-workgroup kernel that sums the G partials in index order and applies
// the CG scalar logic on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ppk {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int WPB = BLOCK / WAVE;  // waves per workgroup
constexpr int LZ_MAX = 64;         // max Lanczos steps
constexpr int LR_MAX = 8;          // max rank of the low-rank correction

// Device-resident solver state: CG scalars live here, never on the host.
struct State {
    double rho;      // r.z of the current iteration
    double alpha;    // rho / p.q
    double beta;     // rho' / rho
    double gamma;    // p.q
    double rr;       // r.r after the update
    double bnorm2;   // b_hat.b_hat
    double tol2;     // tol^2 * bnorm2, set once bnorm2 is known
    double tol;      // requested relative tolerance
    double lz_alpha[LZ_MAX];
    double lz_beta[LZ_MAX];
    double scratch[4];
    double lr_c[LR_MAX];  // low-rank correction: V^T r of the current residual
    double lr_y[LR_MAX];  // (V^T A V)^{-1} lr_c; r.z gains lr_c . lr_y
    int32_t lr_p;         // rank in use for this solve (0 = no correction)
    int32_t lr_pad;
    int32_t it;      // iterations done
    int32_t maxit;
    int32_t done;    // 1 once converged / failed / maxit: later kernels return at entry
    int32_t status;  // pp_status
    int32_t zero_b;  // b_hat == 0 -> x = 0
    int32_t pad;
    uint32_t ticket; // unused
    uint32_t pad2;
};

enum Fin : int {
    FIN_NONE = 0,
    FIN_BNORM,       // bnorm2 = sum; zero b -> done
    FIN_RR0,         // initial residual check
    FIN_RHO0,        // rho = r.z (before the first iteration)
    FIN_GAMMA,       // gamma = p.q, alpha = rho/gamma
    FIN_RR,          // rr = r.r, it++, convergence / maxit
    FIN_RHO,         // rho' = r.z, beta = rho'/rho, rho = rho'
    FIN_LZ_NORM0,    // scratch[0] = sqrt(sum) (start vector norm)
    FIN_LZ_ALPHA,    // lz_alpha[idx] = sum
    FIN_LZ_BETA      // lz_beta[idx] = sqrt(sum)
};

constexpr int DMAX = 16;  // stored diagonals of the symmetric diagonal storage

// The operator: an optional symmetric diagonal part plus an optional slice
// part.  Diagonal part: stored diagonal d (0 <= d < nd) holds a_{i, i + doff[d]}
// at dv[d * dstride + i] (doff[0] = 0 < doff[1] < ...); the mirrored entry
// a_{i, i - doff[d]} of a symmetric matrix is the same value, read from index
// i - doff[d].  Entries outside the covered offsets (and the trace columns of
// the Schur shape) live in the slice part.
struct SellView {
    const int64_t *sp = nullptr;   // [nslices + 1] element offset of each slice (multiple of 64)
    const int32_t *col = nullptr;  // [sp[nslices]]
    const void *val = nullptr;     // [sp[nslices]] double or float
    int64_t n = 0;                 // rows
    int64_t nslices = 0;
    int64_t nx = 0;                // columns < nx index x; columns >= nx index w[col - nx]
    int sell = 1;                  // 0: the slice part is empty and is skipped
    int nd = 0;                    // stored diagonals, 0 = no diagonal part
    const void *dv = nullptr;      // [nd][dstride] double or float
    int64_t dstride = 0;
    int64_t doff[DMAX] = {};
};

struct CsrView {         // plain CSR (trace operator M^{-1} C)
    const int64_t *rp;
    const int32_t *col;
    const void *val;
    int64_t rows;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ void block_range(int64_t total, int L, int G, int64_t &lo, int64_t &hi)
{
    lo = total * (int64_t)L / G;
    hi = total * (int64_t)(L + 1) / G;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, WAVE);
    return v;
}

// Sum over the workgroup; result valid in thread 0.  Fixed order.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < WPB; ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < INFINITY; }

// CG scalar logic, run by thread 0 of the last workgroup of a reduction.
__device__ inline void finalize(State *st, int fin, int idx, double s)
{
    switch (fin) {
    case FIN_BNORM:
        st->bnorm2 = s;
        st->tol2 = st->tol * st->tol * s;
        if (!(s < INFINITY)) { st->done = 1; st->status = 2; }
        else if (s == 0.0) { st->done = 1; st->status = 0; st->zero_b = 1; }
        break;
    case FIN_RR0:
        st->rr = s;
        if (!(s < INFINITY)) { st->done = 1; st->status = 2; }
        else if (s <= st->tol2) { st->done = 1; st->status = 0; }
        else if (st->maxit <= 0) { st->done = 1; st->status = 1; }
        break;
    case FIN_RHO0:
        for (int j = 0; j < st->lr_p; ++j) s += st->lr_c[j] * st->lr_y[j];
        st->rho = s;
        if (!finite_pos(s)) { st->done = 1; st->status = 2; }
        break;
    case FIN_GAMMA:
        st->gamma = s;
        if (!finite_pos(s)) { st->done = 1; st->status = 2; }
        else st->alpha = st->rho / s;
        break;
    case FIN_RR:
        st->rr = s;
        st->it += 1;
        if (!(s < INFINITY)) { st->done = 1; st->status = 2; }
        else if (s <= st->tol2) { st->done = 1; st->status = 0; }
        else if (st->it >= st->maxit) { st->done = 1; st->status = 1; }
        break;
    case FIN_RHO: {
        for (int j = 0; j < st->lr_p; ++j) s += st->lr_c[j] * st->lr_y[j];
        if (!finite_pos(s)) { st->done = 1; st->status = 2; break; }
        st->beta = s / st->rho;
        st->rho = s;
        break;
    }
    case FIN_LZ_NORM0: st->scratch[0] = sqrt(s); break;
    case FIN_LZ_ALPHA: st->lz_alpha[idx] = s; break;
    case FIN_LZ_BETA: st->lz_beta[idx] = sqrt(s); break;
    default: break;
    }
}

// Publish this workgroup's partial (one double per workgroup, plain store).
// The reduction over workgroups is a separate one-workgroup kernel (k_fin):
// the kernel boundary orders the stores before it, so no workgroup has to
// flush its L2 with an agent-scope release before retiring.
__device__ __forceinline__ void store_partial(double part, double *partials, int L)
{
    __shared__ double lds[WPB];
    const double s = block_sum(part, lds);
    if (threadIdx.x == 0) partials[L] = s;
}

template <bool NT, typename T>
__device__ __forceinline__ T ldm(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// (A x)_row for one lane of a slice whose entries start at `base` (width
// entries per row).  Entries are taken in chunks of U: all U column indices
// and values are loaded before any gather is issued, so one chunk costs two
// dependent memory round trips whatever its length; indices past the row's
// width are clamped to the last entry (an L1 hit) and their product dropped.
// Columns >= nx read the trace vector w.
template <int U, typename T, typename XT, bool SCHUR, bool NT>
__device__ __forceinline__ T sell_row_u(const SellView &A, const XT *__restrict__ x,
                                        const T *__restrict__ w, int64_t base, int width, int lane)
{
    const int32_t *c = A.col + base + lane;
    const T *v = (const T *)A.val + base + lane;
    T acc = (T)0;
    for (int j0 = 0; j0 < width; j0 += U) {
        int cj[U];
        T vj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = (j0 + u < width) ? j0 + u : width - 1;
            cj[u] = ldm<NT>(c + (int64_t)j * WAVE);
            vj[u] = ldm<NT>(v + (int64_t)j * WAVE);
        }
        T xj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (SCHUR) xj[u] = (cj[u] < A.nx) ? (T)x[cj[u]] : w[cj[u] - A.nx];
            else xj[u] = (T)x[cj[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < width) acc += vj[u] * xj[u];
    }
    return acc;
}

// Slices of at most two entries per row (the trace columns left beside a
// diagonal part) take chunks of two, so they issue no clamped loads.
template <typename T, typename XT, bool SCHUR, bool NT = false>
__device__ __forceinline__ T sell_row(const SellView &A, const XT *__restrict__ x,
                                      const T *__restrict__ w, int64_t base, int width, int lane)
{
    if (width <= 2) return sell_row_u<2, T, XT, SCHUR, NT>(A, x, w, base, width, lane);
    return sell_row_u<8, T, XT, SCHUR, NT>(A, x, w, base, width, lane);
}

__device__ __forceinline__ void slice_span(const SellView &A, int64_t s, int64_t &base, int &width)
{
    base = A.sp[s];
    width = (int)((A.sp[s + 1] - base) >> 6);
}

// (A x)_i over the diagonal part.  The diagonal first, then the off-diagonal
// offsets in chunks of U: the upper value a_{i,i+o} streams from HBM, the
// mirrored value a_{i,i-o} = a_{i-o,i} is the same array U o entries back and
// is read from cache (rows i - o were streamed by this or a neighbouring
// workgroup of the same XCD moments before).  All loads of a chunk are issued
// before any product; offsets past nd are clamped to the last one and their
// products dropped.  Column indices past either end of the matrix are
// redirected to row i (their value is zero).
template <typename T, typename XT, int U>
__device__ __forceinline__ T dia_chunk(const SellView &A, const XT *__restrict__ x, int64_t i, int d0)
{
    const T *dv = (const T *)A.dv;
    const int64_t n = A.n, ds = A.dstride;
    const int nd = A.nd;
    T vl[U], vu[U], xl[U], xu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int d = d0 + u < nd ? d0 + u : nd - 1;
        const int64_t o = A.doff[d];
        const int64_t il = i >= o ? i - o : i;
        const int64_t iu = i + o < n ? i + o : i;
        vu[u] = dv[(int64_t)d * ds + i];
        vl[u] = dv[(int64_t)d * ds + il];
        xu[u] = (T)x[iu];
        xl[u] = (T)x[il];
    }
    T acc = (T)0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (d0 + u < nd) {
            if (i >= A.doff[d0 + u]) acc += vl[u] * xl[u];
            acc += vu[u] * xu[u];
        }
    }
    return acc;
}

template <typename T, typename XT>
__device__ __forceinline__ T dia_row(const SellView &A, const XT *__restrict__ x, int64_t i)
{
    const T *dv = (const T *)A.dv;
    T acc = dv[i] * (T)x[i];
    if (A.nd <= 3) {  // 5-point (and narrower) stencils: one chunk, nothing wasted
        if (A.nd > 1) acc += dia_chunk<T, XT, 2>(A, x, i, 1);
    } else if (A.nd == 4) {  // 7-point stencils
        acc += dia_chunk<T, XT, 3>(A, x, i, 1);
    } else {
        for (int d0 = 1; d0 < A.nd; d0 += 4) acc += dia_chunk<T, XT, 4>(A, x, i, d0);
    }
    return acc;
}

// (A x)_row for lane `lane` of slice s: diagonal part plus slice part.  The
// slice span is read first so that its load overlaps the diagonal part.
template <typename T, typename XT, bool SCHUR, bool NT = false>
__device__ __forceinline__ T op_row(const SellView &A, const XT *__restrict__ x, const T *__restrict__ w,
                                    int64_t row, int64_t s, int lane)
{
    int64_t base = 0;
    int width = 0;
    if (A.sell) slice_span(A, s, base, width);
    T acc = (T)0;
    if (A.nd > 0) acc = dia_row<T, XT>(A, x, row < A.n ? row : A.n - 1);
    if (A.sell) acc += sell_row<T, XT, SCHUR, NT>(A, x, w, base, width, lane);
    return acc;
}

// The same with the storage fixed at compile time, for the hot loops: DK
// off-diagonal offsets in one straight-line chunk (DK = 0: no diagonal part,
// DK < 0: the runtime form above), SP: slice part present.  With no branch
// between them, every load of the row is issued before the first product.
// UNITD: the stored main diagonal is exactly 1 (Jacobi-scaled CSR operator)
// and is not read (1 * x_i = x_i, so the sum is the same bit for bit).
template <int DK, bool SP, typename T, typename XT, bool SCHUR, bool NT, bool UNITD = false>
__device__ __forceinline__ T op_row_fixed(const SellView &A, const XT *__restrict__ x, const T *__restrict__ w,
                                          int64_t row, int64_t s, int lane)
{
    if constexpr (DK < 0) {
        return op_row<T, XT, SCHUR, NT>(A, x, w, row, s, lane);
    } else {
        int64_t base = 0;
        int width = 0;
        if constexpr (SP) slice_span(A, s, base, width);
        T acc = (T)0;
        if constexpr (DK > 0) {
            const int64_t i = row < A.n ? row : A.n - 1;
            if constexpr (UNITD) acc = dia_chunk<T, XT, DK>(A, x, i, 1) + (T)x[i];
            else acc = dia_chunk<T, XT, DK>(A, x, i, 1) + ((const T *)A.dv)[i] * (T)x[i];
        } else if constexpr (!SP) {
            // diagonal only (nd == 1)
            const int64_t i = row < A.n ? row : A.n - 1;
            acc = ((const T *)A.dv)[i] * (T)x[i];
        }
        if constexpr (SP) acc += sell_row<T, XT, SCHUR, NT>(A, x, w, base, width, lane);
        return acc;
    }
}

// Call f(integral_constant<int, DK>, bool_constant<SP>) with the storage of A.
template <typename F>
__device__ __forceinline__ void with_storage(const SellView &A, F f)
{
    using std::integral_constant;
    if (A.nd == 0) f(integral_constant<int, 0>{}, std::true_type{});
    else if (A.nd == 4 && !A.sell) f(integral_constant<int, 3>{}, std::false_type{});
    else if (A.nd == 4) f(integral_constant<int, 3>{}, std::true_type{});
    else if (A.nd == 3 && A.sell) f(integral_constant<int, 2>{}, std::true_type{});
    else if (A.nd == 3) f(integral_constant<int, 2>{}, std::false_type{});
    else f(integral_constant<int, -1>{}, std::true_type{});
}

// Iterate the rows owned by logical workgroup L: fn(row, slice, lane).
template <typename F>
__device__ __forceinline__ void for_my_slices(int64_t nslices, int L, int G, F fn)
{
    int64_t s0, s1;
    block_range(nslices, L, G, s0, s1);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int lane = threadIdx.x & (WAVE - 1);
    for (int64_t s = s0 + w; s < s1; s += WPB) fn(s * WAVE + lane, s, lane);
}

template <typename F>
__device__ __forceinline__ void for_my_elems(int64_t n, int L, int G, F fn)
{
    int64_t e0, e1;
    block_range(n, L, G, e0, e1);
    for (int64_t i = e0 + threadIdx.x; i < e1; i += BLOCK) fn(i);
}

#define PPK_PROLOGUE(st)                                  \
    if (st != nullptr && st->done) return;                \
    const int G = (int)gridDim.x;                         \
    const int L = xcd_remap((int)blockIdx.x, G);

// ---------------------------------------------------------------------------
// operator kernels
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// phases: the body of each step of the solve for the rows owned by logical
// workgroup L of G.  The stream-driven kernels below wrap one phase each; the
// persistent driver chains them with grid-wide barriers.
// ---------------------------------------------------------------------------

// w_t = sum_p cm_tp x[col_p]  (trace phase of the Schur operator: M^{-1} C x,
// with 1/m_t and the Jacobi column scaling folded into cm).  One thread per
// trace row; rows are short (two entries).
template <typename T, typename XT>
__device__ __forceinline__ void ph_trace(const CsrView &Cm, const XT *__restrict__ x, T *__restrict__ w,
                                         int L, int G)
{
    for_my_elems(Cm.rows, L, G, [&](int64_t t) {
        T acc = (T)0;
        const T *v = (const T *)Cm.val;
        for (int64_t p = Cm.rp[t]; p < Cm.rp[t + 1]; ++p) acc += v[p] * (T)x[Cm.col[p]];
        w[t] = acc;
    });
}

// One step of Algorithm 2, fused with the operator application:
//   out = ax * x_i + aold * sold_i + ar * r_i + aA * (A x)_i
// MODE 1 (first step):  x = r gathered, coefficients (0, 0, 4 rho1/delta, -2 rho1/(delta theta))
// MODE 2 (second step): x = s_1, s_0 = r/theta folded into ar
// MODE 3 (j >= 3):      x = s_{j-1}, sold = s_{j-2}
// DOT: return this workgroup's share of r.out (r read as RT, double products).
// SCALE: out *= dis_i (pp_apply with Jacobi returns D^{-1/2} s_k).
// out may alias sold (each thread reads sold_i before writing out_i).
template <typename T, typename XT, typename RT, typename OT, int MODE, bool SCHUR, bool DOT, bool SCALE,
          bool NT, bool UNITD = false>
__device__ __forceinline__ double ph_cheb(const SellView &A, const XT *__restrict__ xg,
                                          const T *__restrict__ w, const RT *__restrict__ r,
                                          const T *sold, OT *out, T ax, T aold, T ar, T aA,
                                          const double *__restrict__ dis, int L, int G)
{
    double part = 0.0;
    with_storage(A, [&](auto dk, auto sp) {
        constexpr int DK = decltype(dk)::value;
        constexpr bool SP = decltype(sp)::value;
        // With a diagonal part, r, s_{j-2} and the output are pure streams:
        // non-temporal accesses (NT: operators much larger than the caches)
        // keep them from evicting the gathered x and the mirrored diagonal
        // values that the neighbouring rows re-read.  (With the slice layout
        // only, the matrix stream is the non-temporal one and the vectors do
        // better cached.)
        constexpr bool NTV = DK != 0 && NT;
        for_my_slices(A.nslices, L, G, [&](int64_t row, int64_t s, int lane) {
            // row-level operands first, so they are in flight with the matrix stream
            const int64_t rc = row < A.n ? row : A.n - 1;
            const RT ri = ldm<NTV>(r + rc);
            const T xs = (MODE >= 2) ? (T)xg[rc] : (T)0;
            const T so = (MODE == 3) ? ldm<NTV>(sold + rc) : (T)0;
            const double ds = SCALE ? dis[rc] : 1.0;
            T a = op_row_fixed<DK, SP, T, XT, SCHUR, NT, UNITD>(A, xg, w, row, s, lane);
            if (row < A.n) {
                T o = aA * a + ar * (T)ri;
                if (MODE >= 2) o += ax * xs;
                if (MODE == 3) o += aold * so;
                OT ov = (OT)o;
                if (SCALE) ov = (OT)((double)ov * ds);
                if constexpr (NTV) __builtin_nontemporal_store(ov, out + row);
                else out[row] = ov;
                if (DOT) part += (double)ri * (double)ov;
            }
        });
    });
    return part;
}

// bh = dis .* b, xh = x ./ dis; returns the share of bh.bh
// perm (new -> old numbering, or null): the operator was renumbered at create
// and b, x are in the caller's numbering.
__device__ __forceinline__ double ph_init_scale(int64_t n, const double *__restrict__ b,
                                                const double *__restrict__ x,
                                                const double *__restrict__ dis, double *__restrict__ bh,
                                                double *__restrict__ xh, int L, int G,
                                                const int32_t *__restrict__ perm = nullptr)
{
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const int64_t o = perm ? (int64_t)perm[i] : i;
        const double d = dis ? dis[i] : 1.0;
        const double bi = d * b[o];
        bh[i] = bi;
        xh[i] = x[o] / d;
        part += bi * bi;
    });
    return part;
}

// r = bh - A xh; returns the share of r.r
template <bool SCHUR>
__device__ __forceinline__ double ph_init_resid(const SellView &A, const double *__restrict__ xh,
                                                const double *__restrict__ w, const double *__restrict__ bh,
                                                double *__restrict__ r, int L, int G)
{
    double part = 0.0;
    for_my_slices(A.nslices, L, G, [&](int64_t row, int64_t s, int lane) {
        double a = op_row<double, double, SCHUR>(A, xh, w, row, s, lane);
        if (row < A.n) {
            const double ri = bh[row] - a;
            r[row] = ri;
            part += ri * ri;
        }
    });
    return part;
}

// q = A p; returns the share of p.q
template <bool SCHUR, bool NT, bool UNITD = false>
__device__ __forceinline__ double ph_pq(const SellView &A, const double *__restrict__ p,
                                        const double *__restrict__ w, double *__restrict__ q, int L, int G)
{
    double part = 0.0;
    with_storage(A, [&](auto dk, auto sp) {
        constexpr int DK = decltype(dk)::value;
        constexpr bool SP = decltype(sp)::value;
        for_my_slices(A.nslices, L, G, [&](int64_t row, int64_t s, int lane) {
            const int64_t rc = row < A.n ? row : A.n - 1;
            const double pi = p[rc];
            double a = op_row_fixed<DK, SP, double, double, SCHUR, NT, UNITD>(A, p, w, row, s, lane);
            if (row < A.n) {
                q[row] = a;
                part += pi * a;
            }
        });
    });
    return part;
}

// x += alpha p; r -= alpha q; returns the share of r.r.  r32 (mixed mode, or
// NULL): the FP32 copy of the new r the polynomial reads.
__device__ __forceinline__ double ph_xr(int64_t n, const double *__restrict__ p, const double *__restrict__ q,
                                        double *__restrict__ x, double *__restrict__ r, double alpha, int L,
                                        int G, float *__restrict__ r32 = nullptr)
{
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
        part += ri * ri;
    });
    return part;
}

// p = z + beta p   (first: p = z)
__device__ __forceinline__ void ph_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                     double beta, bool first, int L, int G)
{
    for_my_elems(n, L, G, [&](int64_t i) { p[i] = first ? z[i] : z[i] + beta * p[i]; });
}

// x = dis .* xh (or 0 when b_hat == 0); with perm, x in the caller's numbering
__device__ __forceinline__ void ph_final_x(int64_t n, const double *__restrict__ xh,
                                           const double *__restrict__ dis, double *__restrict__ x, bool zb,
                                           int L, int G, const int32_t *__restrict__ perm = nullptr)
{
    for_my_elems(n, L, G, [&](int64_t i) {
        x[perm ? (int64_t)perm[i] : i] = zb ? 0.0 : (dis ? dis[i] : 1.0) * xh[i];
    });
}

// y = c x (converting type); returns the share of x.y when DOT
template <typename XT, typename YT, bool DOT>
__device__ __forceinline__ double ph_scale(int64_t n, const XT *__restrict__ x, double c, YT *__restrict__ y,
                                           int L, int G)
{
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const double xi = (double)x[i];
        const YT yi = (YT)(xi * c);
        y[i] = yi;
        if (DOT) part += xi * (double)yi;
    });
    return part;
}

// ---------------------------------------------------------------------------
// stream-driven kernels: one phase per launch
// ---------------------------------------------------------------------------

template <typename T, typename XT>
__global__ __launch_bounds__(BLOCK) void k_trace(CsrView Cm, const XT *__restrict__ x,
                                                 T *__restrict__ w, const State *st)
{
    PPK_PROLOGUE(st)
    ph_trace<T, XT>(Cm, x, w, L, G);
}

// y = A x (plain SpMV in the slice layout).
template <typename T, bool SCHUR>
__global__ __launch_bounds__(BLOCK) void k_spmv(SellView A, const T *__restrict__ x,
                                                const T *__restrict__ w, T *__restrict__ y, int nt)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_slices(A.nslices, L, G, [&](int64_t row, int64_t s, int lane) {
        T a = op_row<T, T, SCHUR>(A, x, w, row, s, lane);
        if (row < A.n) y[row] = a;
    });
}

template <typename T, typename XT, typename RT, typename OT, int MODE, bool SCHUR, bool DOT, bool SCALE,
          bool NT, bool UNITD = false>
static __global__ __launch_bounds__(BLOCK) void k_cheb(SellView A, const XT *__restrict__ xg,
                                                const T *__restrict__ w, const RT *__restrict__ r,
                                                const T *sold, OT *out, double cx, double cold,
                                                double cr, double cA, const double *__restrict__ dis,
                                                double *partials, State *st, int fin, int nt)
{
    PPK_PROLOGUE(st)
    const double part = ph_cheb<T, XT, RT, OT, MODE, SCHUR, DOT, SCALE, NT, UNITD>(
        A, xg, w, r, sold, out, (T)cx, (T)cold, (T)cr, (T)cA, dis, L, G);
    if (DOT) store_partial(part, partials, L);
}

static __global__ __launch_bounds__(BLOCK) void k_state_init(State *st, double tol, int maxit)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho = st->alpha = st->beta = st->gamma = st->rr = st->bnorm2 = st->tol2 = 0.0;
        st->tol = tol;
        st->it = 0;
        st->maxit = maxit;
        st->done = 0;
        st->status = 1;
        st->zero_b = 0;
        st->ticket = 0u;
        st->lr_p = 0;
    }
}

static __global__ __launch_bounds__(BLOCK) void k_init_scale(int64_t n, const double *__restrict__ b,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ dis,
                                                      double *__restrict__ bh, double *__restrict__ xh,
                                                      double *partials, State *st,
                                                      const int32_t *__restrict__ perm)
{
    PPK_PROLOGUE(st)
    const double part = ph_init_scale(n, b, x, dis, bh, xh, L, G, perm);
    store_partial(part, partials, L);
}

template <bool SCHUR>
__global__ __launch_bounds__(BLOCK) void k_init_resid(SellView A, const double *__restrict__ xh,
                                                      const double *__restrict__ w,
                                                      const double *__restrict__ bh,
                                                      double *__restrict__ r, double *partials,
                                                      State *st, int nt)
{
    PPK_PROLOGUE(st)
    const double part = ph_init_resid<SCHUR>(A, xh, w, bh, r, L, G);
    store_partial(part, partials, L);
}

// q = A-hat p and this workgroup's share of p.q.  UNITD: unit main diagonal, not read.
template <bool SCHUR, bool UNITD = false>
__global__ __launch_bounds__(BLOCK) void k_pq(SellView A, const double *__restrict__ p,
                                              const double *__restrict__ w, double *__restrict__ q,
                                              double *partials, State *st, int nt)
{
    PPK_PROLOGUE(st)
    const double part = nt ? ph_pq<SCHUR, true, UNITD>(A, p, w, q, L, G)
                           : ph_pq<SCHUR, false, UNITD>(A, p, w, q, L, G);
    store_partial(part, partials, L);
}

static __global__ __launch_bounds__(BLOCK) void k_xr(int64_t n, const double *__restrict__ p,
                                              const double *__restrict__ q, double *__restrict__ x,
                                              double *__restrict__ r, double *partials, State *st,
                                              float *__restrict__ r32)
{
    PPK_PROLOGUE(st)
    const double part = ph_xr(n, p, q, x, r, st->alpha, L, G, r32);
    store_partial(part, partials, L);
}

static __global__ __launch_bounds__(BLOCK) void k_p(int64_t n, const double *__restrict__ z,
                                             double *__restrict__ p, const State *st, int first)
{
    PPK_PROLOGUE(st)
    ph_p(n, z, p, first ? 0.0 : st->beta, first != 0, L, G);
}

// runs even when done is set
static __global__ __launch_bounds__(BLOCK) void k_final_x(int64_t n, const double *__restrict__ xh,
                                                   const double *__restrict__ dis,
                                                   double *__restrict__ x, const State *st,
                                                   const int32_t *__restrict__ perm)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    ph_final_x(n, xh, dis, x, st->zero_b != 0, L, G, perm);
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------

// y = s .* x (s may be null = 1), converting type
template <typename XT, typename YT>
__global__ __launch_bounds__(BLOCK) void k_scale(int64_t n, const XT *__restrict__ x,
                                                 const double *__restrict__ s, double c,
                                                 YT *__restrict__ y)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) {
        double v = (double)x[i] * c;
        if (s) v *= s[i];
        y[i] = (YT)v;
    });
}

// out = a x + b y   (y may be null when b == 0; out may alias x or y)
static __global__ __launch_bounds__(BLOCK) void k_lin2(int64_t n, double a, const double *x, double b,
                                                       const double *y, double *out)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) { out[i] = a * x[i] + (y ? b * y[i] : 0.0); });
}

// y = s .* s .* x * c   (k = 0 preconditioner with Jacobi)
static __global__ __launch_bounds__(BLOCK) void k_scale2(int64_t n, const double *__restrict__ x,
                                                  const double *__restrict__ s, double c,
                                                  double *__restrict__ y)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) {
        const double d = s ? s[i] : 1.0;
        y[i] = d * (d * (x[i] * c));
    });
}

// Sum the G workgroup partials in index order and run the scalar logic.  Skips
// when the solve is already done (the producer kernel then wrote nothing).
static __global__ __launch_bounds__(BLOCK) void k_fin(const double *__restrict__ partials, int G, State *st,
                                                      int fin, int idx)
{
    if (st->done) return;
    __shared__ double lds[WPB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < G; i += BLOCK) acc += partials[i];
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) finalize(st, fin, idx, tot);
}

// r.z into the CG state (degree-0 preconditioner: no operator step to fuse into)
static __global__ __launch_bounds__(BLOCK) void k_dot_fin(int64_t n, const double *__restrict__ x,
                                                   const double *__restrict__ y, double *partials,
                                                   State *st, int fin)
{
    PPK_PROLOGUE(st)
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) { part += x[i] * y[i]; });
    store_partial(part, partials, L);
}

// y = x ./ d
static __global__ __launch_bounds__(BLOCK) void k_div(int64_t n, const double *__restrict__ x,
                                               const double *__restrict__ d, double *__restrict__ y)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) { y[i] = x[i] / d[i]; });
}

// ---------------------------------------------------------------------------
// Lanczos
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// v_i = fmix32(i) / 2^32 - 0.5 ; reduce v.v -> FIN_LZ_NORM0.  i is the row in the
// caller's numbering (perm[i] when the operator was renumbered).
static __global__ __launch_bounds__(BLOCK) void k_lz_start(int64_t n, double *__restrict__ v,
                                                    double *partials, State *st,
                                                    const int32_t *__restrict__ perm)
{
    PPK_PROLOGUE(st)
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const uint32_t g = perm ? (uint32_t)perm[i] : (uint32_t)i;
        const double x = (double)fmix32(g) / 4294967296.0 - 0.5;
        v[i] = x;
        part += x * x;
    });
    store_partial(part, partials, L);
}

// v /= scratch[0]
static __global__ __launch_bounds__(BLOCK) void k_lz_norm(int64_t n, double *__restrict__ v, const State *st)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const double nv = st->scratch[0];
    for_my_elems(n, L, G, [&](int64_t i) { v[i] = v[i] / nv; });
}

// w = A v - beta_{j-1} vprev ; reduce v.w -> lz_alpha[j]
template <bool SCHUR>
__global__ __launch_bounds__(BLOCK) void k_lz_apply(SellView A, const double *__restrict__ v,
                                                    const double *__restrict__ tw,
                                                    const double *__restrict__ vprev,
                                                    double *__restrict__ wout, double *partials,
                                                    State *st, int j, int nt)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const double bp = (j > 0) ? st->lz_beta[j - 1] : 0.0;
    double part = 0.0;
    for_my_slices(A.nslices, L, G, [&](int64_t row, int64_t s, int lane) {
        double a = op_row<double, double, SCHUR>(A, v, tw, row, s, lane);
        if (row < A.n) {
            const double wi = a - bp * vprev[row];
            wout[row] = wi;
            part += v[row] * wi;
        }
    });
    store_partial(part, partials, L);
}

// w -= alpha_j v ; reduce w.w -> lz_beta[j]
static __global__ __launch_bounds__(BLOCK) void k_lz_orth(int64_t n, const double *__restrict__ v,
                                                   double *__restrict__ w, double *partials,
                                                   State *st, int j)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const double a = st->lz_alpha[j];
    double part = 0.0;
    for_my_elems(n, L, G, [&](int64_t i) {
        const double wi = w[i] - a * v[i];
        w[i] = wi;
        part += wi * wi;
    });
    store_partial(part, partials, L);
}

// vprev = v ; v = w / beta_j
static __global__ __launch_bounds__(BLOCK) void k_lz_next(int64_t n, double *__restrict__ vprev,
                                                   double *__restrict__ v,
                                                   const double *__restrict__ w, const State *st,
                                                   int j)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const double b = st->lz_beta[j];
    for_my_elems(n, L, G, [&](int64_t i) {
        vprev[i] = v[i];
        v[i] = w[i] / b;
    });
}

// y[i] = c s[i] x[perm[i]]  (s may be null = 1): a vector of the caller's numbering
// into the operator's
static __global__ __launch_bounds__(BLOCK) void k_gather_scale(int64_t n, const double *__restrict__ x,
                                                               const int32_t *__restrict__ perm,
                                                               const double *__restrict__ s, double c,
                                                               double *__restrict__ y)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) { y[i] = c * (s ? s[i] : 1.0) * x[perm[i]]; });
}

// dst[perm[i]] = src[i]: back to the caller's numbering
static __global__ __launch_bounds__(BLOCK) void k_scatter(int64_t n, const double *__restrict__ src,
                                                          const int32_t *__restrict__ perm,
                                                          double *__restrict__ dst)
{
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    for_my_elems(n, L, G, [&](int64_t i) { dst[perm[i]] = src[i]; });
}

// Renumbered CSR: new row i is old row perm[i], its columns mapped by iperm
// and sorted (insertion sort: rows are short, the host refuses long ones).
static __global__ __launch_bounds__(BLOCK) void k_perm_csr(int64_t n, const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           const double *__restrict__ val,
                                                           const int32_t *__restrict__ perm,
                                                           const int32_t *__restrict__ iperm,
                                                           const int64_t *__restrict__ nrp, int32_t *__restrict__ ncol,
                                                           double *__restrict__ nval)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i], p0 = rp[o], len = rp[o + 1] - p0, q0 = nrp[i];
    for (int64_t t = 0; t < len; ++t) {
        const int32_t c = iperm[col[p0 + t]];
        const double v = val[p0 + t];
        int64_t u = t;
        while (u > 0 && ncol[q0 + u - 1] > c) {
            ncol[q0 + u] = ncol[q0 + u - 1];
            nval[q0 + u] = nval[q0 + u - 1];
            --u;
        }
        ncol[q0 + u] = c;
        nval[q0 + u] = v;
    }
}

// ---------------------------------------------------------------------------
// setup kernels: diagonal, Jacobi scaling, slice layout
// ---------------------------------------------------------------------------

// Offsets covered by the diagonal part: an entry (i, j) is covered when
// |j - i| is one of off[0..nd).
struct DiaSet {
    int nd = 0;
    int64_t off[DMAX] = {};
};

__device__ __forceinline__ int dia_index(const DiaSet &D, int64_t a)
{
    for (int d = 0; d < D.nd; ++d)
        if (D.off[d] == a) return d;
    return -1;
}

// d_i = a_ii + sum over appended trace entries (c_ti^2 / m_t); flag non-positive.
static __global__ __launch_bounds__(BLOCK) void k_diag(int64_t n, const int64_t *__restrict__ rp,
                                                const int32_t *__restrict__ col,
                                                const double *__restrict__ val,
                                                const int64_t *__restrict__ ctp,
                                                const int32_t *__restrict__ ctt,
                                                const double *__restrict__ ctv,
                                                const double *__restrict__ m,
                                                double *__restrict__ d, double *__restrict__ dis,
                                                int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
        if (col[p] == i) s += val[p];
    if (ctp) {
        for (int64_t p = ctp[i]; p < ctp[i + 1]; ++p) s += ctv[p] * ctv[p] / m[ctt[p]];
    }
    d[i] = s;
    if (!(s > 0.0) || !(s < INFINITY)) {
        atomicOr(bad, 1);
        dis[i] = 1.0;
    } else {
        dis[i] = 1.0 / sqrt(s);
    }
}

// width of each slice = max over its rows of (row length + appended trace entries)
// (entries covered by the diagonal part D are not counted)
static __global__ __launch_bounds__(BLOCK) void k_slice_width(int64_t n, int64_t nslices,
                                                       const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, DiaSet D,
                                                       const int64_t *__restrict__ ctp,
                                                       int64_t *__restrict__ width)
{
    const int64_t s = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (s >= nslices) return;
    const int64_t row = s * WAVE + lane;
    int64_t len = 0;
    if (row < n) {
        if (D.nd == 0) {
            len = rp[row + 1] - rp[row];
        } else {
            for (int64_t p = rp[row]; p < rp[row + 1]; ++p) {
                const int64_t o = (int64_t)col[p] - row;
                if (dia_index(D, o < 0 ? -o : o) < 0) ++len;
            }
        }
        if (ctp) len += ctp[row + 1] - ctp[row];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        int64_t o = __shfl_down(len, off, WAVE);
        len = o > len ? o : len;
    }
    if (lane == 0) width[s] = len;
}

// exclusive scan of width*64 into sp[0..nslices]; one workgroup, fixed order
static __global__ __launch_bounds__(1024) void k_scan_slices(int64_t nslices, const int64_t *__restrict__ width,
                                                      int64_t *__restrict__ sp)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (nslices + 1023) / 1024;
    const int64_t lo = (int64_t)t * chunk;
    const int64_t hi = lo + chunk < nslices ? lo + chunk : nslices;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += width[i] * WAVE;
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < 1024; ++i) {
            int64_t v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        sp[i] = acc;
        acc += width[i] * WAVE;
    }
    if (hi == nslices && lo < hi) sp[nslices] = acc;
    if (nslices == 0 && t == 0) sp[0] = 0;
}

// Fill the slice layout: scaled values a_ij dis_i dis_j, appended trace
// entries (column nx + t, value c_ti dis_i), padding (own row, 0).
static __global__ __launch_bounds__(BLOCK) void k_slice_fill(int64_t n, int64_t nslices, int64_t nx,
                                                      const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val, DiaSet D,
                                                      const int64_t *__restrict__ ctp,
                                                      const int32_t *__restrict__ ctt,
                                                      const double *__restrict__ ctv,
                                                      const double *__restrict__ dis,
                                                      const int64_t *__restrict__ sp,
                                                      int32_t *__restrict__ scol,
                                                      double *__restrict__ sval,
                                                      float *__restrict__ sval32)
{
    const int64_t s = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (s >= nslices) return;
    const int64_t row = s * WAVE + lane;
    const int64_t base = sp[s];
    const int width = (int)((sp[s + 1] - base) / WAVE);
    int j = 0;
    const int32_t self = (int32_t)(row < n ? row : 0);
    if (row < n) {
        const double di = dis ? dis[row] : 1.0;
        for (int64_t p = rp[row]; p < rp[row + 1]; ++p) {
            const int32_t c = col[p];
            if (D.nd > 0) {
                const int64_t o = (int64_t)c - row;
                if (dia_index(D, o < 0 ? -o : o) >= 0) continue;
            }
            const double v = dis ? val[p] * di * dis[c] : val[p];
            const int64_t o = base + (int64_t)j * WAVE + lane;
            scol[o] = c;
            sval[o] = v;
            if (sval32) sval32[o] = (float)v;
            ++j;
        }
        if (ctp) {
            for (int64_t p = ctp[row]; p < ctp[row + 1]; ++p, ++j) {
                const double v = ctv[p] * di;
                const int64_t o = base + (int64_t)j * WAVE + lane;
                scol[o] = (int32_t)(nx + ctt[p]);
                sval[o] = v;
                if (sval32) sval32[o] = (float)v;
            }
        }
    }
    for (; j < width; ++j) {
        const int64_t o = base + (int64_t)j * WAVE + lane;
        scol[o] = self;
        sval[o] = 0.0;
        if (sval32) sval32[o] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// symmetric diagonal storage: setup
// ---------------------------------------------------------------------------

constexpr int OFF_SLOTS = 128;  // distinct column offsets tracked (power of two)
constexpr unsigned long long OFF_EMPTY = 0x8000000000000000ull;

// Count one occurrence of offset o in an open-addressing table; false when full.
__device__ __forceinline__ bool off_insert(unsigned long long *key, unsigned long long *cnt, int64_t o,
                                           unsigned long long add)
{
    const unsigned long long k = (unsigned long long)o;
    unsigned h = (unsigned)((k * 0x9E3779B97F4A7C15ull) >> 57) & (OFF_SLOTS - 1);
    for (int probe = 0; probe < OFF_SLOTS; ++probe, h = (h + 1) & (OFF_SLOTS - 1)) {
        const unsigned long long cur = atomicCAS(&key[h], OFF_EMPTY, k);
        if (cur == OFF_EMPTY || cur == k) {
            atomicAdd(&cnt[h], add);
            return true;
        }
    }
    return false;
}

// Histogram of the column offsets col - row over the nonzero entries (at
// most OFF_SLOTS distinct ones; *overflow is set when there are more).  A
// table per workgroup in LDS, merged into the global table at the end.
// Rows are i = 0..n-1 of rp; their global index (that col refers to) is i + row_base.
static __global__ __launch_bounds__(BLOCK) void k_offsets(int64_t n, int64_t row_base,
                                                          const int64_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ val,
                                                          unsigned long long *gkey, unsigned long long *gcnt,
                                                          int *overflow)
{
    __shared__ unsigned long long key[OFF_SLOTS], cnt[OFF_SLOTS];
    __shared__ int full;
    for (int t = threadIdx.x; t < OFF_SLOTS; t += BLOCK) {
        key[t] = OFF_EMPTY;
        cnt[t] = 0;
    }
    if (threadIdx.x == 0) full = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (val[p] != 0.0 && !off_insert(key, cnt, (int64_t)col[p] - (i + row_base), 1)) {
                full = 1;
                break;
            }
        if (full) break;
    }
    __syncthreads();
    if (full) {
        if (threadIdx.x == 0) atomicOr(overflow, 1);
        return;
    }
    for (int t = threadIdx.x; t < OFF_SLOTS; t += BLOCK)
        if (key[t] != OFF_EMPTY && !off_insert(gkey, gcnt, (int64_t)key[t], cnt[t])) atomicOr(overflow, 1);
}

// Raw values of the covered entries with offset >= 0 into dv[d][i] (dv zeroed
// beforehand).  cnt[0] / cnt[1] count the nonzero covered entries above / below
// the diagonal; a covered offset seen twice in one row (a duplicate entry)
// sets bad |= 16.  Row i of rp has global index i + row_base.
static __global__ __launch_bounds__(BLOCK) void k_dia_fill(int64_t n, int64_t row_base, const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           const double *__restrict__ val, DiaSet D,
                                                           double *__restrict__ dv, int64_t ds,
                                                           unsigned long long *cnt, int *bad)
{
    __shared__ unsigned long long c[2];
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long cu = 0, cl = 0;
    int b = 0;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) {
        uint32_t seen_u = 0, seen_l = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t o = (int64_t)col[p] - (i + row_base);
            const int d = dia_index(D, o < 0 ? -o : o);
            if (d < 0) continue;
            const double v = val[p];
            if (o >= 0) {
                if ((seen_u >> d) & 1u) b |= 16;
                seen_u |= 1u << d;
                dv[(int64_t)d * ds + i] = v;
                if (o > 0 && v != 0.0) ++cu;
            } else {
                if ((seen_l >> d) & 1u) b |= 16;
                seen_l |= 1u << d;
                if (v != 0.0) ++cl;
            }
        }
    }
    if (b) atomicOr(bad, b);
    if (cu) atomicAdd(&c[0], cu);
    if (cl) atomicAdd(&c[1], cl);
    __syncthreads();
    if (threadIdx.x < 2 && c[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], c[threadIdx.x]);
}

// Every covered entry below the diagonal must equal the stored value of its
// mirror: a_{i, i-o} == a_{i-o, i} (else bad |= 32).  With no duplicates and
// equal counts of nonzero entries above and below, the covered part is then
// exactly symmetric and the mirrored reads reproduce it.
static __global__ __launch_bounds__(BLOCK) void k_dia_check(int64_t n, int64_t row_base,
                                                            const int64_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val, DiaSet D,
                                                            const double *__restrict__ dv, int64_t ds,
                                                            int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
        const int64_t j = (int64_t)col[p] - row_base;
        if (j >= i) continue;
        const int d = dia_index(D, i - j);
        if (d >= 0 && !(dv[(int64_t)d * ds + j] == val[p])) {
            atomicOr(bad, 32);
            return;
        }
    }
}

// Scale the stored diagonals to the Jacobi-scaled operator:
// dv[d][i] = (a_{i,i+o} dis_i) dis_{i+o}, and write the FP32 copy.  unit_d0:
// the stored diagonals hold the whole diagonal of the operator (a CSR
// matrix), so the scaled diagonal is one by definition and is stored as
// exactly 1 (the product above rounds to within two ulps of it).
static __global__ __launch_bounds__(BLOCK) void k_dia_scale(int64_t n, DiaSet D, const double *__restrict__ dis,
                                                            double *__restrict__ dv, float *__restrict__ dv32,
                                                            int64_t ds, int unit_d0)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < D.nd; ++d) {
        const int64_t j = i + D.off[d];
        double v = dv[(int64_t)d * ds + i];
        if (dis) v = j < n ? v * dis[i] * dis[j] : 0.0;
        if (dis && unit_d0 && D.off[d] == 0) v = 1.0;
        dv[(int64_t)d * ds + i] = v;
        if (dv32) dv32[(int64_t)d * ds + i] = (float)v;
    }
}

// Trace operator values: cm_tp = c_tp dis_{col} / m_t (and an FP32 copy).
static __global__ __launch_bounds__(BLOCK) void k_trace_fill(int64_t nt, const int64_t *__restrict__ crp,
                                                      const int32_t *__restrict__ ccol,
                                                      const double *__restrict__ cval,
                                                      const double *__restrict__ m,
                                                      const double *__restrict__ dis,
                                                      double *__restrict__ cm,
                                                      float *__restrict__ cm32)
{
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= nt) return;
    for (int64_t p = crp[t]; p < crp[t + 1]; ++p) {
        const double v = cval[p] * (dis ? dis[ccol[p]] : 1.0) / m[t];
        cm[p] = v;
        if (cm32) cm32[p] = (float)v;
    }
}

// validate CSR structure: monotone row pointers, columns in range
static __global__ __launch_bounds__(BLOCK) void k_check_csr(int64_t rows, int64_t ncols, int64_t nnz,
                                                     const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col, int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= rows) return;
    const int64_t a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || b > nnz || (i == 0 && a != 0) || (i == rows - 1 && b != nnz)) {
        atomicOr(bad, 2);
        return;
    }
    for (int64_t p = a; p < b; ++p) {
        const int32_t c = col[p];
        if (c < 0 || (int64_t)c >= ncols) {
            atomicOr(bad, 4);
            return;
        }
    }
}

}  // namespace ppk
