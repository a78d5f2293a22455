// Batched polynomial-preconditioned CG: many independent systems (segments)
// and/or a block of right-hand sides solved together.
//
// Layout.  The systems are stacked block-diagonally; every system is padded to
// whole 64-row slices, so a slice never mixes two systems.  Vectors are
// row-major blocks [rows][NB] (NB = internal block width >= nrhs, a power of
// two).  The matrix is read once per step for all NB columns.
//
// Work split.  Every workgroup belongs to exactly one segment and owns a
// contiguous slice range inside it.  Inside a wavefront, W lanes share a row
// (64/W rows per pass) and each lane handles CPL = NB/W contiguous columns;
// matrix entries are loaded once per row group (same address across the W
// lanes) and the gathers of X[col][c0 .. c0+CPL) are contiguous.
//
// Reductions.  Per-(segment, column) dot products: each workgroup writes NB
// partials, and a finalising kernel with one workgroup per segment sums them
// in workgroup order and runs the CG scalar logic for that segment's columns.  A column that finished keeps its iterate frozen; a segment whose
// columns all finished is skipped by every later kernel.
#pragma once
#include "kernels.hpp"

namespace ppb {

using ppk::BLOCK;
using ppk::WAVE;
using ppk::WPB;

constexpr int NB_MAX = 32;

struct Batch {
    // workgroup -> segment map
    const int32_t *blk_seg;   // [G]
    const int64_t *blk_s0;    // [G] first slice
    const int64_t *blk_s1;    // [G] end slice
    const int32_t *seg_blk0;  // [S + 1] workgroups of segment s: [seg_blk0[s], seg_blk0[s+1])
    const int64_t *seg_row0;  // [S + 1] internal first row of segment s (multiple of 64)
    const int64_t *seg_n;     // [S] real rows of segment s
    const int64_t *ext_row0;  // [S + 1] caller's first row of segment s
    int32_t S;
    int32_t NB;               // internal block width
    int32_t nrhs;             // caller's block width
    int32_t k;                // polynomial degree
    // symmetric stored diagonals per system (see ppk::SellView): system s has
    // seg_nd[s] of them (0: all its entries in the slice layout) with offsets
    // seg_off[s * DMAX + d], values dv[d * dstride + internal row]
    const int32_t *seg_nd;    // [S]
    const int32_t *seg_sell;  // [S] 1 when system s also has entries in the slice layout
    const int64_t *seg_off;   // [S * DMAX]
    const double *dv64;
    const float *dv32;
    int64_t dstride;
    int32_t unit_d0;          // 1: the stored main diagonals are exactly 1 (Jacobi), not read
};

// Per-(segment, column) CG state, arrays of S * NB (index s * NB + c).
struct BState {
    double *rho, *alpha, *beta, *rr, *bn2, *tol2, *lz;  // lz: Lanczos scratch [S][2 * LZ_MAX + 2]
    int32_t *it, *status, *done, *zero_b;
    int32_t *seg_ndone;   // [S] columns finished
    int32_t *seg_done;    // [S] 1 when all NB columns finished
    uint32_t *ticket;     // [S]
    int32_t *ndone;       // [1] total (segment, column) pairs finished
    double tol;
    int32_t maxit;
};

enum BFin : int { BF_NONE = 0, BF_BNORM, BF_RR0, BF_RHO0, BF_GAMMA, BF_RR, BF_RHO, BF_LZN, BF_LZA, BF_LZB };

__device__ __forceinline__ void mark_done(const Batch &bt, BState &st, int s, int c, int status)
{
    const int i = s * bt.NB + c;
    st.done[i] = 1;
    st.status[i] = status;
    atomicAdd(st.ndone, 1);  // several segments finalise at once
    st.seg_ndone[s] += 1;    // only segment s's finalising workgroup writes its own entries
    if (st.seg_ndone[s] >= bt.NB) st.seg_done[s] = 1;
}

// CG scalar logic for column c of segment s (run by one thread).
__device__ inline void bfinalize(const Batch &bt, BState &st, int fin, int s, int c, double v, int idx)
{
    const int i = s * bt.NB + c;
    if (fin >= BF_LZN) {
        double *lz = st.lz + (size_t)s * (2 * ppk::LZ_MAX + 2);
        if (fin == BF_LZN) lz[2 * ppk::LZ_MAX] = sqrt(v);
        else if (fin == BF_LZA) lz[idx] = v;
        else lz[ppk::LZ_MAX + idx] = sqrt(v);
        return;
    }
    if (st.done[i]) return;
    switch (fin) {
    case BF_BNORM:
        st.bn2[i] = v;
        st.tol2[i] = st.tol * st.tol * v;
        if (!(v < INFINITY)) mark_done(bt, st, s, c, 2);
        else if (v == 0.0) { st.zero_b[i] = 1; mark_done(bt, st, s, c, 0); }
        break;
    case BF_RR0:
        st.rr[i] = v;
        if (!(v < INFINITY)) mark_done(bt, st, s, c, 2);
        else if (v <= st.tol2[i]) mark_done(bt, st, s, c, 0);
        else if (st.maxit <= 0) mark_done(bt, st, s, c, 1);
        break;
    case BF_RHO0:
        st.rho[i] = v;
        if (!ppk::finite_pos(v)) mark_done(bt, st, s, c, 2);
        break;
    case BF_GAMMA:
        if (!ppk::finite_pos(v)) mark_done(bt, st, s, c, 2);
        else st.alpha[i] = st.rho[i] / v;
        break;
    case BF_RR:
        st.rr[i] = v;
        st.it[i] += 1;
        if (!(v < INFINITY)) mark_done(bt, st, s, c, 2);
        else if (v <= st.tol2[i]) mark_done(bt, st, s, c, 0);
        else if (st.it[i] >= st.maxit) mark_done(bt, st, s, c, 1);
        break;
    case BF_RHO:
        if (!ppk::finite_pos(v)) { mark_done(bt, st, s, c, 2); break; }
        st.beta[i] = v / st.rho[i];
        st.rho[i] = v;
        break;
    default: break;
    }
}

// logical workgroup: consecutive logical workgroups (one system's slices) run on
// the same XCD, so stencil neighbours are gathered from that XCD's L2
__device__ __forceinline__ int logical_block() { return ppk::xcd_remap((int)blockIdx.x, (int)gridDim.x); }

// Publish this workgroup's NB column partials (plain stores); kb_fin reduces them.
template <int NB>
__device__ __forceinline__ void store_seg(double *partials, const double *mine, int b)
{
    if (threadIdx.x < NB) partials[(size_t)b * NB + threadIdx.x] = mine[threadIdx.x];
}

template <int NB>
__device__ __forceinline__ void store_seg(double *partials, const double *mine)
{
    store_seg<NB>(partials, mine, logical_block());
}

// One workgroup per segment: sum the segment's workgroup partials per column
// in workgroup order and run the scalar logic for its columns.
template <int NB>
__device__ __forceinline__ void kbd_fin(int s, Batch bt, BState st, const double *__restrict__ partials, int fin,
                                        int idx)
{
    if (fin < BF_LZN && st.seg_done[s]) return;
    __shared__ double lds[BLOCK + NB_MAX];
    constexpr int M = BLOCK / NB;
    const int c = threadIdx.x % NB, m = threadIdx.x / NB;
    const int b0 = bt.seg_blk0[s], b1 = bt.seg_blk0[s + 1];
    double acc = 0.0;
    for (int q = b0 + m; q < b1; q += M) acc += partials[(size_t)q * NB + c];
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < NB) {
        double tot = 0.0;
        for (int q = 0; q < M; ++q) tot += lds[q * NB + threadIdx.x];
        lds[BLOCK + threadIdx.x] = tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int cc = 0; cc < NB; ++cc)
            if (fin >= BF_LZN || cc < bt.nrhs) bfinalize(bt, st, fin, s, cc, lds[BLOCK + cc], idx);
    }
}

template <int NB>
__global__ __launch_bounds__(BLOCK) void kb_fin(Batch bt, BState st, const double *__restrict__ partials, int fin,
                                                int idx)
{
    kbd_fin<NB>(blockIdx.x, bt, st, partials, fin, idx);
}

// Workgroup sum of per-thread column partials: part[q] belongs to column
// c0 + q of this lane; lanes sharing a column are those with equal lane % W.
// Result: out[c] for c < NB, in lds-backed array visible to thread 0.
template <int W, int CPL>
__device__ __forceinline__ void block_colsum(const double (&part)[CPL], double *lds, double *out)
{
    constexpr int NB = W * CPL;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        double v = part[q];
        // reduce across the 64/W row groups of the wave (lanes lane, lane+W, ...)
#pragma unroll
        for (int off = 32; off >= W; off >>= 1) v += __shfl_down(v, off, WAVE);
        if (lane < W) lds[w * NB + lane * CPL + q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < WPB; ++i) t += lds[i * NB + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

struct BlockRange {
    int seg;
    int64_t s0, s1, row_end;  // slice range and end of the segment's real rows
};

__device__ __forceinline__ BlockRange my_range(const Batch &bt, int b)
{
    BlockRange r;
    r.seg = bt.blk_seg[b];
    r.s0 = bt.blk_s0[b];
    r.s1 = bt.blk_s1[b];
    r.row_end = bt.seg_row0[r.seg] + bt.seg_n[r.seg];
    return r;
}

__device__ __forceinline__ BlockRange my_range(const Batch &bt) { return my_range(bt, logical_block()); }

template <typename T, int CPL>
struct Vec {
    T v[CPL];
};

template <typename T, int CPL, bool NT = false>
__device__ __forceinline__ Vec<T, CPL> ldv(const T *p)
{
    Vec<T, CPL> r;
#pragma unroll
    for (int q = 0; q < CPL; ++q) r.v[q] = ppk::ldm<NT>(p + q);
    return r;
}

// Y = A X for one row (W lanes per row, CPL columns per lane), chunked like sell_row.
template <typename T, int W, int CPL, bool NT>
__device__ __forceinline__ void spmm_row(const ppk::SellView &A, const T *__restrict__ X, int NB, int64_t base,
                                         int width, int rin, int c0, T (&acc)[CPL])
{
    constexpr int U = 8;
    const int32_t *cp = A.col + base + rin;
    const T *vp = (const T *)A.val + base + rin;
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[q] = (T)0;
    for (int j0 = 0; j0 < width; j0 += U) {
        int cj[U];
        T vj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = (j0 + u < width) ? j0 + u : width - 1;
            cj[u] = ppk::ldm<NT>(cp + (int64_t)j * WAVE);
            vj[u] = ppk::ldm<NT>(vp + (int64_t)j * WAVE);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const Vec<T, CPL> xv = ldv<T, CPL>(X + (int64_t)cj[u] * NB + c0);
            if (j0 + u < width) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) acc[q] += vj[u] * xv.v[q];
            }
        }
    }
}

// Iterate the rows of this workgroup: fn(row, rin (row within slice), base,
// width); base and width (the slice's entries in the slice layout) are read
// only when SP.
template <int W, bool SP = true, typename F>
__device__ __forceinline__ void for_rows(const ppk::SellView &A, const BlockRange &br, F fn)
{
    constexpr int R = WAVE / W;  // rows per pass of a wave
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = lane / W;
    for (int64_t s = br.s0 + w; s < br.s1; s += WPB) {
        int64_t base = 0;
        int width = 0;
        if constexpr (SP) {
            base = A.sp[s];
            width = (int)((A.sp[s + 1] - base) >> 6);
        }
        for (int r0 = 0; r0 < WAVE; r0 += R) {
            const int rin = r0 + g;
            fn(s * WAVE + rin, rin, base, width);
        }
    }
}

// The stored diagonals of one system, read once per workgroup.
template <int DK>
struct SegDia {
    int64_t row0, row_end;  // internal rows of the system: [row0, row_end) are real
    int64_t off[DK + 1];
};

template <int DK>
__device__ __forceinline__ SegDia<DK> seg_dia(const Batch &bt, int seg)
{
    SegDia<DK> g;
    g.row0 = bt.seg_row0[seg];
    g.row_end = g.row0 + bt.seg_n[seg];
#pragma unroll
    for (int d = 0; d <= DK; ++d) g.off[d] = bt.seg_off[(int64_t)seg * ppk::DMAX + d];
    return g;
}

template <typename T>
__device__ __forceinline__ const T *dv_of(const Batch &bt)
{
    if constexpr (sizeof(T) == 8) return (const T *)bt.dv64;
    else return (const T *)bt.dv32;
}

// Y = A X for one row over the system's stored diagonals (W lanes per row, CPL
// columns per lane): the diagonal, then DK offset pairs, every load issued
// before the first product.  Neighbours outside the system's real rows have a
// zero value; their indices are redirected to the row itself.
template <typename T, int CPL, int DK>
__device__ __forceinline__ void spmm_dia(const T *__restrict__ dv, int64_t ds, const SegDia<DK> &g,
                                         const T *__restrict__ X, int NB, int64_t row, int c0, T (&acc)[CPL],
                                         bool unit)
{
    const Vec<T, CPL> x0 = ldv<T, CPL>(X + row * NB + c0);
    T v0 = (T)1;  // a unit main diagonal (Jacobi-scaled) is not read
    if (!unit) v0 = dv[row];
    T vu[DK], vl[DK];
    Vec<T, CPL> xu[DK], xl[DK];
#pragma unroll
    for (int u = 0; u < DK; ++u) {
        const int64_t o = g.off[u + 1];
        const int64_t iu = row + o < g.row_end ? row + o : row;
        const bool lok = row - o >= g.row0;
        const int64_t il = lok ? row - o : row;
        vu[u] = dv[(int64_t)(u + 1) * ds + row];
        const T l = dv[(int64_t)(u + 1) * ds + il];
        vl[u] = lok ? l : (T)0;
        xu[u] = ldv<T, CPL>(X + iu * NB + c0);
        xl[u] = ldv<T, CPL>(X + il * NB + c0);
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        T a = v0 * x0.v[q];
#pragma unroll
        for (int u = 0; u < DK; ++u) a += vl[u] * xl[u].v[q] + vu[u] * xu[u].v[q];
        acc[q] = a;
    }
}

// Call f(integral_constant<int, DK>, bool_constant<SP>) with the storage of
// system seg: DK stored off-diagonal offsets (0: slice layout only), SP: the
// system has entries in the slice layout.
template <typename F>
__device__ __forceinline__ void with_seg_storage(const Batch &bt, int seg, F f)
{
    using std::integral_constant;
    const int nd = bt.seg_nd[seg];
    const bool sp = bt.seg_sell[seg] != 0;
    if (nd == 4 && !sp) f(integral_constant<int, 3>{}, std::false_type{});
    else if (nd == 4) f(integral_constant<int, 3>{}, std::true_type{});
    else if (nd == 3 && !sp) f(integral_constant<int, 2>{}, std::false_type{});
    else if (nd == 3) f(integral_constant<int, 2>{}, std::true_type{});
    else f(integral_constant<int, 0>{}, std::true_type{});
}

// Y = A X for one row in the system's storage.
template <typename T, int W, int CPL, int DK, bool SP, bool NT>
__device__ __forceinline__ void spmm_any(const ppk::SellView &A, const Batch &bt, const SegDia<DK> &g,
                                         const T *__restrict__ X, int NB, int64_t row, int64_t base, int width,
                                         int rin, int c0, T (&acc)[CPL])
{
    if constexpr (DK > 0) {
        spmm_dia<T, CPL, DK>(dv_of<T>(bt), bt.dstride, g, X, NB, row, c0, acc, bt.unit_d0 != 0);
        if constexpr (SP) {
            T more[CPL];
            spmm_row<T, W, CPL, NT>(A, X, NB, base, width, rin, c0, more);
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[q] += more[q];
        }
    } else {
        spmm_row<T, W, CPL, NT>(A, X, NB, base, width, rin, c0, acc);
    }
}

#define PPB_PROLOGUE_B(b)                               \
    const BlockRange br = my_range(bt, b);              \
    if (st.seg_done[br.seg]) return;                    \
    const int lane = threadIdx.x & (WAVE - 1);          \
    const int c0 = (lane % W) * CPL;                    \
    (void)c0;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Bh = dis .* B (caller layout [n_ext][nrhs] -> internal [rows][NB]), Xh = X ./ dis;
// column sums of Bh.Bh -> BF_BNORM.  Padding rows and columns >= nrhs are zero.
template <int W, int CPL>
__device__ __forceinline__ void kbd_init_scale(int b, Batch bt, BState st, ppk::SellView A,
                                               const double *__restrict__ B, const double *__restrict__ X,
                                               const double *__restrict__ dis, double *__restrict__ Bh,
                                               double *__restrict__ Xh, double *partials)
{
    constexpr int NB = W * CPL;
    __shared__ double lds[BLOCK + NB_MAX * 2 + NB * WPB];
    PPB_PROLOGUE_B(b)
    double part[CPL] = {};
    const int64_t ext0 = bt.ext_row0[br.seg], row0 = bt.seg_row0[br.seg];
    for_rows<W, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
        const bool real = row < br.row_end;
        const int64_t er = ext0 + (row - row0);
        const double d = real && dis ? dis[row] : 1.0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int c = c0 + q;
            const bool on = real && c < bt.nrhs;
            const double bi = on ? d * B[er * bt.nrhs + c] : 0.0;
            const double xi = on ? X[er * bt.nrhs + c] / d : 0.0;
            Bh[row * NB + c] = bi;
            Xh[row * NB + c] = xi;
            part[q] += bi * bi;
        }
    });
    block_colsum<W, CPL>(part, lds, lds + BLOCK + NB_MAX);
    store_seg<NB>(partials, lds + BLOCK + NB_MAX, b);
}

template <int W, int CPL>
__global__ __launch_bounds__(BLOCK) void kb_init_scale(Batch bt, BState st, ppk::SellView A,
                                                       const double *__restrict__ B, const double *__restrict__ X,
                                                       const double *__restrict__ dis, double *__restrict__ Bh,
                                                       double *__restrict__ Xh, double *partials)
{
    kbd_init_scale<W, CPL>(logical_block(), bt, st, A, B, X, dis, Bh, Xh, partials);
}

// R = Bh - A Xh -> BF_RR0 ; Q = A P -> BF_GAMMA (p.q) ; both FP64
template <int W, int CPL, int WHICH, bool NT>
__device__ __forceinline__ void kbd_apply64(int b, Batch bt, BState st, ppk::SellView A,
                                            const double *__restrict__ X, const double *__restrict__ Bh,
                                            double *__restrict__ Y, double *partials)
{
    constexpr int NB = W * CPL;
    __shared__ double lds[BLOCK + NB_MAX * 2 + NB * WPB];
    PPB_PROLOGUE_B(b)
    double part[CPL] = {};
    with_seg_storage(bt, br.seg, [&](auto dk, auto spc) {
        constexpr int DK = decltype(dk)::value;
        constexpr bool SP = decltype(spc)::value;
        const SegDia<DK> g = seg_dia<DK>(bt, br.seg);
        for_rows<W, SP>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
            double acc[CPL];
            spmm_any<double, W, CPL, DK, SP, NT>(A, bt, g, X, NB, row, base, width, rin, c0, acc);
            if (row < br.row_end) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int64_t o = row * NB + c0 + q;
                    if (WHICH == 0) {
                        const double ri = Bh[o] - acc[q];
                        Y[o] = ri;
                        part[q] += ri * ri;
                    } else {
                        Y[o] = acc[q];
                        part[q] += X[o] * acc[q];
                    }
                }
            }
        });
    });
    block_colsum<W, CPL>(part, lds, lds + BLOCK + NB_MAX);
    store_seg<NB>(partials, lds + BLOCK + NB_MAX, b);
}

template <int W, int CPL, int WHICH, bool NT>
__global__ __launch_bounds__(BLOCK) void kb_apply64(Batch bt, BState st, ppk::SellView A,
                                                    const double *__restrict__ X, const double *__restrict__ Bh,
                                                    double *__restrict__ Y, double *partials)
{
    kbd_apply64<W, CPL, WHICH, NT>(logical_block(), bt, st, A, X, Bh, Y, partials);
}

// One Chebyshev step on all columns (coefficients of the row's segment):
//   OUT = cx X + cold SOLD + cr R + cA (A X).  LAST: R read in FP64, OUT FP64,
//   column sums of R.OUT -> fin.  OUT may alias SOLD.
template <typename T, typename RT, typename OT, int W, int CPL, int MODE, bool LAST, bool NT>
__device__ __forceinline__ void kbd_cheb(int b, Batch bt, BState st, ppk::SellView A, const T *__restrict__ X,
                                         const RT *__restrict__ Rv, const T *SOLD, OT *OUT,
                                         const double *__restrict__ coef, int j, double *partials, int fin)
{
    constexpr int NB = W * CPL;
    __shared__ double lds[BLOCK + NB_MAX * 2 + NB * WPB];
    PPB_PROLOGUE_B(b)
    const double *cf = coef + ((size_t)br.seg * bt.k + (j - 1)) * 4;
    const T ax = (T)cf[0], aold = (T)cf[1], ar = (T)cf[2], aA = (T)cf[3];
    double part[CPL] = {};
    with_seg_storage(bt, br.seg, [&](auto dk, auto spc) {
        constexpr int DK = decltype(dk)::value;
        constexpr bool SP = decltype(spc)::value;
        const SegDia<DK> g = seg_dia<DK>(bt, br.seg);
        // stored diagonals: R, SOLD and OUT are pure streams (see ph_cheb)
        constexpr bool NTV = DK > 0;
        for_rows<W, SP>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
            const int64_t o = row * NB + c0;
            Vec<RT, CPL> rv = ldv<RT, CPL, NTV>(Rv + o);
            Vec<T, CPL> xs, so;
            if (MODE >= 2) xs = ldv<T, CPL>(X + o);
            if (MODE == 3) so = ldv<T, CPL, NTV>(SOLD + o);
            T acc[CPL];
            spmm_any<T, W, CPL, DK, SP, NT>(A, bt, g, X, NB, row, base, width, rin, c0, acc);
            if (row < br.row_end) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    T v = aA * acc[q] + ar * (T)rv.v[q];
                    if (MODE >= 2) v += ax * xs.v[q];
                    if (MODE == 3) v += aold * so.v[q];
                    if constexpr (NTV) __builtin_nontemporal_store((OT)v, OUT + o + q);
                    else OUT[o + q] = (OT)v;
                    if (LAST) part[q] += (double)rv.v[q] * (double)(OT)v;
                }
            }
        });
    });
    if (LAST) {
        block_colsum<W, CPL>(part, lds, lds + BLOCK + NB_MAX);
        store_seg<NB>(partials, lds + BLOCK + NB_MAX, b);
    }
}

template <typename T, typename RT, typename OT, int W, int CPL, int MODE, bool LAST, bool NT>
__global__ __launch_bounds__(BLOCK) void kb_cheb(Batch bt, BState st, ppk::SellView A, const T *__restrict__ X,
                                                 const RT *__restrict__ Rv, const T *SOLD, OT *OUT,
                                                 const double *__restrict__ coef, int j, double *partials, int fin)
{
    kbd_cheb<T, RT, OT, W, CPL, MODE, LAST, NT>(logical_block(), bt, st, A, X, Rv, SOLD, OUT, coef, j, partials, fin);
}

// Z = theta^-1 R (degree 0) with column sums of R.Z -> fin
template <int W, int CPL>
__device__ __forceinline__ void kbd_deg0(int b, Batch bt, BState st, ppk::SellView A, const double *__restrict__ Rv,
                                         double *__restrict__ Z, const double *__restrict__ thinv,
                                         double *partials, int fin)
{
    constexpr int NB = W * CPL;
    __shared__ double lds[BLOCK + NB_MAX * 2 + NB * WPB];
    PPB_PROLOGUE_B(b)
    const double ti = thinv[br.seg];
    double part[CPL] = {};
    for_rows<W, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int64_t o = row * NB + c0 + q;
            const double z = Rv[o] * ti;
            Z[o] = z;
            part[q] += Rv[o] * z;
        }
    });
    block_colsum<W, CPL>(part, lds, lds + BLOCK + NB_MAX);
    store_seg<NB>(partials, lds + BLOCK + NB_MAX, b);
}

template <int W, int CPL>
__global__ __launch_bounds__(BLOCK) void kb_deg0(Batch bt, BState st, ppk::SellView A, const double *__restrict__ Rv,
                                                 double *__restrict__ Z, const double *__restrict__ thinv,
                                                 double *partials, int fin)
{
    kbd_deg0<W, CPL>(logical_block(), bt, st, A, Rv, Z, thinv, partials, fin);
}

// Xh += alpha P ; R -= alpha Q (frozen columns keep their values) -> BF_RR
template <int W, int CPL>
__device__ __forceinline__ void kbd_xr(int b, Batch bt, BState st, ppk::SellView A, const double *__restrict__ P,
                                       const double *__restrict__ Q, double *__restrict__ Xh,
                                       double *__restrict__ Rv, double *partials)
{
    constexpr int NB = W * CPL;
    __shared__ double lds[BLOCK + NB_MAX * 2 + NB * WPB];
    PPB_PROLOGUE_B(b)
    double al[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int i = br.seg * NB + c0 + q;
        al[q] = st.done[i] ? 0.0 : st.alpha[i];
    }
    double part[CPL] = {};
    for_rows<W, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int64_t o = row * NB + c0 + q;
            Xh[o] = Xh[o] + al[q] * P[o];
            const double r = Rv[o] - al[q] * Q[o];
            Rv[o] = r;
            part[q] += r * r;
        }
    });
    block_colsum<W, CPL>(part, lds, lds + BLOCK + NB_MAX);
    store_seg<NB>(partials, lds + BLOCK + NB_MAX, b);
}

template <int W, int CPL>
__global__ __launch_bounds__(BLOCK) void kb_xr(Batch bt, BState st, ppk::SellView A, const double *__restrict__ P,
                                               const double *__restrict__ Q, double *__restrict__ Xh,
                                               double *__restrict__ Rv, double *partials)
{
    kbd_xr<W, CPL>(logical_block(), bt, st, A, P, Q, Xh, Rv, partials);
}

// P = Z + beta P (first: P = Z); frozen columns keep P
template <int W, int CPL>
__device__ __forceinline__ void kbd_p(int b, Batch bt, BState st, ppk::SellView A, const double *__restrict__ Z,
                                      double *__restrict__ P, int first)
{
    constexpr int NB = W * CPL;
    PPB_PROLOGUE_B(b)
    double be[CPL];
    bool fr[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int i = br.seg * NB + c0 + q;
        fr[q] = st.done[i] != 0;
        be[q] = first ? 0.0 : st.beta[i];
    }
    for_rows<W, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int64_t o = row * NB + c0 + q;
            if (!fr[q]) P[o] = first ? Z[o] : Z[o] + be[q] * P[o];
        }
    });
}

template <int W, int CPL>
__global__ __launch_bounds__(BLOCK) void kb_p(Batch bt, BState st, ppk::SellView A, const double *__restrict__ Z,
                                              double *__restrict__ P, int first)
{
    kbd_p<W, CPL>(logical_block(), bt, st, A, Z, P, first);
}

// R32 = (float) R
template <int W, int CPL>
__device__ __forceinline__ void kbd_conv(int b, Batch bt, BState st, ppk::SellView A, const double *__restrict__ Rv,
                                         float *__restrict__ R32)
{
    PPB_PROLOGUE_B(b)
    constexpr int NB = W * CPL;
    for_rows<W, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) R32[row * NB + c0 + q] = (float)Rv[row * NB + c0 + q];
    });
}

template <int W, int CPL>
__global__ __launch_bounds__(BLOCK) void kb_conv(Batch bt, BState st, ppk::SellView A, const double *__restrict__ Rv,
                                                 float *__restrict__ R32)
{
    kbd_conv<W, CPL>(logical_block(), bt, st, A, Rv, R32);
}

// X (caller layout) = dis .* Xh (zero where b_hat == 0); runs for every segment
template <int W, int CPL>
__device__ __forceinline__ void kbd_final(int b, Batch bt, BState st, ppk::SellView A, const double *__restrict__ Xh,
                                          const double *__restrict__ dis, double *__restrict__ X)
{
    constexpr int NB = W * CPL;
    const BlockRange br = my_range(bt, b);
    const int lane = threadIdx.x & (WAVE - 1);
    const int c0 = (lane % W) * CPL;
    const int64_t ext0 = bt.ext_row0[br.seg], row0 = bt.seg_row0[br.seg];
    for_rows<W, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
        if (row >= br.row_end) return;
        const int64_t er = ext0 + (row - row0);
        const double d = dis ? dis[row] : 1.0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int c = c0 + q;
            if (c < bt.nrhs) X[er * bt.nrhs + c] = st.zero_b[br.seg * NB + c] ? 0.0 : d * Xh[row * NB + c];
        }
    });
}

template <int W, int CPL>
__global__ __launch_bounds__(BLOCK) void kb_final(Batch bt, BState st, ppk::SellView A, const double *__restrict__ Xh,
                                                  const double *__restrict__ dis, double *__restrict__ X)
{
    kbd_final<W, CPL>(logical_block(), bt, st, A, Xh, dis, X);
}

// reset the per-(segment, column) state before a solve or a Lanczos run
static __global__ __launch_bounds__(BLOCK) void kb_state_init(BState st, int S, int NB)
{
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < S * NB) {
        st.rho[i] = st.alpha[i] = st.beta[i] = st.rr[i] = st.bn2[i] = st.tol2[i] = 0.0;
        st.it[i] = 0;
        st.status[i] = 1;
        st.done[i] = 0;
        st.zero_b[i] = 0;
    }
    if (i < S) {
        st.seg_ndone[i] = 0;
        st.seg_done[i] = 0;
        st.ticket[i] = 0u;
    }
    if (i == 0) st.ndone[0] = 0;
}

// columns nrhs..NB-1 of every segment are padding: mark them finished
static __global__ __launch_bounds__(BLOCK) void kb_pad_cols(BState st, int S, int NB, int nrhs)
{
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= S || nrhs >= NB) return;
    for (int c = nrhs; c < NB; ++c) {
        st.done[s * NB + c] = 1;
        st.status[s * NB + c] = 0;
        st.zero_b[s * NB + c] = 1;
    }
    st.seg_ndone[s] = NB - nrhs;
    atomicAdd(st.ndone, NB - nrhs);
}

// ---------------------------------------------------------------------------
// batched Lanczos (one start vector per segment, vectors [rows], NB = 1 layout)
// ---------------------------------------------------------------------------

static __global__ __launch_bounds__(BLOCK) void kb_lz_start(Batch bt, BState st, ppk::SellView A, double *__restrict__ v,
                                                     double *partials)
{
    __shared__ double lds[BLOCK + NB_MAX * 2 + WPB];
    const BlockRange br = my_range(bt);
    const int64_t row0 = bt.seg_row0[br.seg];
    double part[1] = {0.0};
    for_rows<1, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
        double x = 0.0;
        if (row < br.row_end) x = (double)ppk::fmix32((uint32_t)(row - row0)) / 4294967296.0 - 0.5;
        v[row] = x;
        part[0] += x * x;
    });
    block_colsum<1, 1>(part, lds, lds + BLOCK + NB_MAX);
    store_seg<1>(partials, lds + BLOCK + NB_MAX);
}

// mode 0: v /= ||v|| and vprev = 0 ; mode 1: vprev = v, v = w / beta_j
static __global__ __launch_bounds__(BLOCK) void kb_lz_vec(Batch bt, BState st, ppk::SellView A, double *__restrict__ v,
                                                   double *__restrict__ vprev, const double *__restrict__ w,
                                                   int mode, int j)
{
    const BlockRange br = my_range(bt);
    const double *lz = st.lz + (size_t)br.seg * (2 * ppk::LZ_MAX + 2);
    const double d = mode == 0 ? lz[2 * ppk::LZ_MAX] : lz[ppk::LZ_MAX + j];
    for_rows<1, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
        if (mode == 0) {
            v[row] = v[row] / d;
            vprev[row] = 0.0;
        } else {
            vprev[row] = v[row];
            v[row] = row < br.row_end ? w[row] / d : 0.0;
        }
    });
}

// w = A v - beta_{j-1} vprev ; alpha_j = v.w   (which = 0)
// w -= alpha_j v ; beta_j = ||w||             (which = 1)
template <int WHICH>
__global__ __launch_bounds__(BLOCK) void kb_lz_step(Batch bt, BState st, ppk::SellView A, const double *__restrict__ v,
                                                    const double *__restrict__ vprev, double *__restrict__ w,
                                                    double *partials, int j)
{
    __shared__ double lds[BLOCK + NB_MAX * 2 + WPB];
    const BlockRange br = my_range(bt);
    const double *lz = st.lz + (size_t)br.seg * (2 * ppk::LZ_MAX + 2);
    double part[1] = {0.0};
    if (WHICH == 0) {
        const double bp = j > 0 ? lz[ppk::LZ_MAX + j - 1] : 0.0;
        with_seg_storage(bt, br.seg, [&](auto dk, auto spc) {
            constexpr int DK = decltype(dk)::value;
            constexpr bool SP = decltype(spc)::value;
            const SegDia<DK> g = seg_dia<DK>(bt, br.seg);
            for_rows<1, SP>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
                double acc[1];
                spmm_any<double, 1, 1, DK, SP, false>(A, bt, g, v, 1, row, base, width, rin, 0, acc);
                const double wi = row < br.row_end ? acc[0] - bp * vprev[row] : 0.0;
                w[row] = wi;
                part[0] += v[row] * wi;
            });
        });
    } else {
        const double a = lz[j];
        for_rows<1, false>(A, br, [&](int64_t row, int rin, int64_t base, int width) {
            const double wi = w[row] - a * v[row];
            w[row] = wi;
            part[0] += wi * wi;
        });
    }
    block_colsum<1, 1>(part, lds, lds + BLOCK + NB_MAX);
    store_seg<1>(partials, lds + BLOCK + NB_MAX);
}

// ---------------------------------------------------------------------------
// setup: slice widths / fill for the padded block-diagonal layout
// ---------------------------------------------------------------------------

// internal row -> caller row (or -1 for padding), via the slice's segment
__device__ __forceinline__ int64_t ext_of(const int32_t *slice_seg, const int64_t *seg_row0, const int64_t *seg_n,
                                          const int64_t *ext_row0, int64_t row)
{
    const int s = slice_seg[row / WAVE];
    const int64_t off = row - seg_row0[s];
    return off < seg_n[s] ? ext_row0[s] + off : -1;
}

// Is entry (e, c) (caller rows) covered by system g's stored diagonals?
__device__ __forceinline__ bool seg_covered(const int32_t *seg_nd, const int64_t *seg_off, int g, int64_t e,
                                            int64_t c)
{
    const int nd = seg_nd[g];
    const int64_t a = c >= e ? c - e : e - c;
    for (int d = 0; d < nd; ++d)
        if (seg_off[(int64_t)g * ppk::DMAX + d] == a) return true;
    return false;
}

// entries per slice that are not covered by their system's stored diagonals
static __global__ __launch_bounds__(BLOCK) void kb_slice_width(int64_t nslices, const int32_t *slice_seg,
                                                        const int64_t *seg_row0, const int64_t *seg_n,
                                                        const int64_t *ext_row0, const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, const int32_t *seg_nd,
                                                        const int64_t *seg_off, int64_t *__restrict__ width)
{
    const int64_t s = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (s >= nslices) return;
    const int g = slice_seg[s];
    const int64_t e = ext_of(slice_seg, seg_row0, seg_n, ext_row0, s * WAVE + lane);
    int64_t len = 0;
    if (e >= 0) {
        if (seg_nd[g] == 0) {
            len = rp[e + 1] - rp[e];
        } else {
            for (int64_t p = rp[e]; p < rp[e + 1]; ++p)
                if (!seg_covered(seg_nd, seg_off, g, e, col[p])) ++len;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_down(len, off, WAVE);
        len = o > len ? o : len;
    }
    if (lane == 0) width[s] = len;
}

// diag (for Jacobi) per internal row; bad flag if not positive or a column leaves its system
static __global__ __launch_bounds__(BLOCK) void kb_diag(int64_t nslices, const int32_t *slice_seg, const int64_t *seg_row0,
                                                 const int64_t *seg_n, const int64_t *ext_row0,
                                                 const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, double *__restrict__ dis, int jacobi,
                                                 int *bad)
{
    const int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (row >= nslices * WAVE) return;
    const int s = slice_seg[row / WAVE];
    const int64_t e = ext_of(slice_seg, seg_row0, seg_n, ext_row0, row);
    if (e < 0) {
        dis[row] = 1.0;
        return;
    }
    double d = 0.0;
    for (int64_t p = rp[e]; p < rp[e + 1]; ++p) {
        const int64_t c = col[p];
        if (c < ext_row0[s] || c >= ext_row0[s] + seg_n[s]) atomicOr(bad, 8);
        if (c == e) d += val[p];
    }
    if (jacobi) {
        if (!(d > 0.0) || !(d < INFINITY)) {
            atomicOr(bad, 1);
            dis[row] = 1.0;
        } else {
            dis[row] = 1.0 / sqrt(d);
        }
    } else {
        dis[row] = 1.0;
    }
}

static __global__ __launch_bounds__(BLOCK) void kb_slice_fill(int64_t nslices, const int32_t *slice_seg,
                                                       const int64_t *seg_row0, const int64_t *seg_n,
                                                       const int64_t *ext_row0, const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const double *__restrict__ val,
                                                       const int32_t *seg_nd, const int64_t *seg_off,
                                                       const double *__restrict__ dis, const int64_t *__restrict__ sp,
                                                       int32_t *__restrict__ scol, double *__restrict__ sval,
                                                       float *__restrict__ sval32, int jacobi)
{
    const int64_t s = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (s >= nslices) return;
    const int64_t row = s * WAVE + lane;
    const int g = slice_seg[s];
    const int64_t e = ext_of(slice_seg, seg_row0, seg_n, ext_row0, row);
    const int64_t base = sp[s];
    const int width = (int)((sp[s + 1] - base) / WAVE);
    int j = 0;
    if (e >= 0) {
        const double di = dis[row];
        for (int64_t p = rp[e]; p < rp[e + 1]; ++p) {
            if (seg_nd[g] > 0 && seg_covered(seg_nd, seg_off, g, e, col[p])) continue;
            const int64_t ci = (int64_t)col[p] - ext_row0[g] + seg_row0[g];  // internal column
            const double v = jacobi ? val[p] * di * dis[ci] : val[p];
            const int64_t o = base + (int64_t)j * WAVE + lane;
            scol[o] = (int32_t)ci;
            sval[o] = v;
            if (sval32) sval32[o] = (float)v;
            ++j;
        }
    }
    for (; j < width; ++j) {
        const int64_t o = base + (int64_t)j * WAVE + lane;
        scol[o] = (int32_t)row;
        sval[o] = 0.0;
        if (sval32) sval32[o] = 0.0f;
    }
}

}  // namespace ppb
