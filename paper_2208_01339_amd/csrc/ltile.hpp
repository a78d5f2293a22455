// LDS-staged x tiles for operators held in 64-row slices only.
//
// The rows are cut into tiles of LT_TS slices (1024 rows).  At create the
// columns that a tile's entries gather are merged into a few column segments
// (gaps up to LT_GAP columns are bridged), and every stored slot gets, next to
// its int32 column, a 16-bit index into the concatenation of its tile's
// segments.  The fused Chebyshev step then stages each tile's segments of x
// into LDS with coalesced loads (one read of every x value per tile) and
// gathers from LDS, reading 10 bytes per stored entry (value + LDS index)
// instead of 12.  Stencil-like and bandwidth-limited numberings (natural
// order, reverse Cuthill-McKee) touch a few segments of about the tile's
// length around each neighbour offset, which is what makes this pay; a
// tile that would stage more than LT_CAP values gathers from memory instead
// (and an operator with too many such tiles keeps the plain kernel).  The
// sums run over the entries in the same order as the plain slice kernel, so
// both give the same result bit for bit.
#pragma once
#include "kernels.hpp"

namespace ppk {

constexpr int LT_TS = 16;      // slices per tile
constexpr int LT_CAP = 6144;   // staged values per tile (48 KB of LDS)
constexpr int LT_GAP = 32;     // columns bridged between two touched columns

struct LtView {
    int64_t ntiles = 0;
    int cap = 0;                       // largest staged size of any tile (values)
    const int32_t *seg_ptr = nullptr;  // [ntiles + 1] segments of tile t: seg_ptr[t] .. seg_ptr[t+1]-1
    const int32_t *staged = nullptr;   // [ntiles] 1: the tile stages x in LDS, 0: it gathers from memory
    const int32_t *seg_col = nullptr;  // first column of each segment
    const int32_t *seg_lds = nullptr;  // its offset in the tile's staging buffer
    const int32_t *seg_len = nullptr;  // its length
    const uint16_t *lcol = nullptr;    // [stored slots] index into the staging buffer
};

// One fused Chebyshev step (the contract of ph_cheb, FP64, slices only):
//   out = ax x_i + aold sold_i + ar r_i + aA (A x)_i   (MODE 1/2/3 as ph_cheb)
// DOT: partials[L] = this workgroup's share of r.out; SCALE: out *= dis_i.
// out may alias sold.
template <int MODE, bool DOT, bool SCALE>
static __global__ __launch_bounds__(BLOCK) void k_cheb_lt(SellView A, LtView T, const double *__restrict__ xg,
                                                          const double *__restrict__ r, const double *sold,
                                                          double *out, double ax, double aold, double ar, double aA,
                                                          const double *__restrict__ dis, double *partials,
                                                          State *st)
{
    PPK_PROLOGUE(st)
    extern __shared__ double lt_x[];
    int64_t t0, t1;
    block_range(T.ntiles, L, G, t0, t1);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int lane = threadIdx.x & (WAVE - 1);
    const double *val = (const double *)A.val;
    double part = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const bool staged = T.staged[t] != 0;
        const int k0 = T.seg_ptr[t], k1 = T.seg_ptr[t + 1];
        for (int k = k0; k < k1; ++k) {
            const int64_t c0 = T.seg_col[k];
            const int lo = T.seg_lds[k], len = T.seg_len[k];
            for (int e = threadIdx.x; e < len; e += BLOCK) lt_x[lo + e] = xg[c0 + e];
        }
        __syncthreads();
        const int64_t s0 = t * LT_TS, s1 = s0 + LT_TS < A.nslices ? s0 + LT_TS : A.nslices;
        for (int64_t s = s0 + w; s < s1; s += WPB) {
            const int64_t row = s * WAVE + lane;
            const int64_t rc = row < A.n ? row : A.n - 1;
            const double ri = r[rc];
            const double xi = (MODE >= 2) ? xg[rc] : 0.0;
            const double so = (MODE == 3) ? sold[rc] : 0.0;
            const double ds = SCALE ? dis[rc] : 1.0;
            const int64_t base = A.sp[s];
            const int width = (int)((A.sp[s + 1] - base) >> 6);
            const double *v = val + base + lane;
            double acc = 0.0;
            if (staged) {
                const uint16_t *lc = T.lcol + base + lane;
                for (int j0 = 0; j0 < width; j0 += 8) {
                    int cj[8];
                    double vj[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int j = (j0 + u < width) ? j0 + u : width - 1;
                        cj[u] = lc[(int64_t)j * WAVE];
                        vj[u] = v[(int64_t)j * WAVE];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (j0 + u < width) acc += vj[u] * lt_x[cj[u]];
                }
            } else {
                const int32_t *gc = A.col + base + lane;
                for (int j0 = 0; j0 < width; j0 += 8) {
                    int cj[8];
                    double vj[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int j = (j0 + u < width) ? j0 + u : width - 1;
                        cj[u] = gc[(int64_t)j * WAVE];
                        vj[u] = v[(int64_t)j * WAVE];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (j0 + u < width) acc += vj[u] * xg[cj[u]];
                }
            }
            if (row < A.n) {
                double o = aA * acc + ar * ri;
                if (MODE >= 2) o += ax * xi;
                if (MODE == 3) o += aold * so;
                if (SCALE) o = o * ds;
                out[row] = o;
                if (DOT) part += ri * o;
            }
        }
        __syncthreads();
    }
    if (DOT) store_partial(part, partials, L);
}

}  // namespace ppk
