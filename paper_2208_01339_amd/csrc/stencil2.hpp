// Two Chebyshev steps per pass for 3-D 7-point operators held as symmetric
// stored diagonals with offsets {0, 1, N, N*N} (rows i = x + N (y + N z),
// n = N * N * NZ, no coupling across the x- and y-faces of the box).
//
//   s_j     = c1x s_{j-1} + c1o s_{j-2} + c1r r + c1A (A s_{j-1})
//   s_{j+1} = c2x s_j     + c2o s_{j-1} + c2r r + c2A (A s_j)
//
// Each workgroup owns S2_TY whole x-lines (contiguous rows of N cells, so the
// HBM streams stay long) over a range of z-planes and marches up z.  For
// every plane it computes s_j on its lines plus one halo line each side (from
// s_{j-1} in HBM / cache) into an LDS ring of three planes, and from that
// ring s_{j+1} one plane behind.  The operator, r and s_{j-1} are
// thus read once for both steps; the ring cells and the planes just outside
// the z-range are computed twice (by the neighbouring tiles too), with the
// same arithmetic, so both copies are identical.  s_j and s_{j+1} go to two
// fresh buffers: no input may be overwritten while neighbours still read it.
#pragma once
#include "kernels.hpp"

namespace ppk {

constexpr int S2_TY = 8;              // y-rows per tile (full x-lines, one halo row each side)
constexpr int S2_RY = S2_TY + 2;
constexpr int S2_ZC = 16;             // z-planes per workgroup
constexpr int64_t S2_NMAX = 256;      // widest x-line: the ring (3 x 10 x N doubles) stays within 64 KB

struct Stencil2 {
    int64_t N, NZ, n;
    int nty, nzc;   // y-tiles and z-chunks
};

// (A v)_i over the stored diagonals with the neighbour coordinates checked:
// the same terms, in the same order, as the one-step kernels (the couplings
// a face-crossing index would reach are zero).
template <typename T>
__device__ __forceinline__ T s2_apply(const T *__restrict__ dv, int64_t ds, const Stencil2 &g,
                                      const T *__restrict__ v, int64_t i, int64_t x, int64_t y, int64_t z)
{
    const int64_t N = g.N, N2 = g.N * g.N;
    const bool xl = x > 0, xu = x + 1 < N, yl = y > 0, yu = y + 1 < N, zl = z > 0, zu = z + 1 < g.NZ;
    // loads first (indices of absent neighbours redirected to i, values zeroed)
    const T v0 = dv[i];
    const T u1 = dv[ds + i], u2 = dv[2 * ds + i], u3 = dv[3 * ds + i];
    const T l1 = dv[ds + (xl ? i - 1 : i)], l2 = dv[2 * ds + (yl ? i - N : i)], l3 = dv[3 * ds + (zl ? i - N2 : i)];
    const T xc = v[i];
    const T x1m = v[xl ? i - 1 : i], x1p = v[xu ? i + 1 : i];
    const T x2m = v[yl ? i - N : i], x2p = v[yu ? i + N : i];
    const T x3m = v[zl ? i - N2 : i], x3p = v[zu ? i + N2 : i];
    T acc = (T)0;
    if (xl) acc += l1 * x1m;
    acc += (xu ? u1 : (T)0) * x1p;
    if (yl) acc += l2 * x2m;
    acc += (yu ? u2 : (T)0) * x2p;
    if (zl) acc += l3 * x3m;
    acc += (zu ? u3 : (T)0) * x3p;
    return acc + v0 * xc;
}

// Dynamic LDS: 3 planes of S2_RY x N values (the ring of s_j).
template <typename T, bool NT>
static __global__ __launch_bounds__(BLOCK) void k_cheb2_stencil(Stencil2 g, const T *__restrict__ dv, int64_t ds,
                                                                const T *__restrict__ sm1, const T *__restrict__ sm2,
                                                                const T *__restrict__ r, T *__restrict__ out1,
                                                                T *__restrict__ out2, double c1x, double c1o,
                                                                double c1r, double c1A, double c2x, double c2o,
                                                                double c2r, double c2A, const State *st)
{
    if (st != nullptr && st->done) return;
    extern __shared__ __align__(16) unsigned char s2_lds[];
    T *ring = (T *)s2_lds;
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const int ty = L % g.nty, tz = L / g.nty;
    const int64_t N = g.N, N2 = N * N;
    const int64_t y0 = (int64_t)ty * S2_TY - 1;  // region row 0
    const int64_t z0 = (int64_t)tz * S2_ZC, z1 = z0 + S2_ZC < g.NZ ? z0 + S2_ZC : g.NZ;
    const int64_t plane_cells = (int64_t)S2_RY * N;
    const T a1x = (T)c1x, a1o = (T)c1o, a1r = (T)c1r, a1A = (T)c1A;
    const T a2x = (T)c2x, a2o = (T)c2o, a2r = (T)c2r, a2A = (T)c2A;
    for (int64_t zz = z0 - 1; zz <= z1; ++zz) {
        // s_j on plane zz over the tile's rows plus one halo row each side
        T *plane = ring + ((zz + 3) % 3) * plane_cells;
        for (int64_t c = threadIdx.x; c < plane_cells; c += BLOCK) {
            const int64_t ly = c / N, x = c - ly * N, y = y0 + ly;
            const bool valid = y >= 0 && y < N && zz >= 0 && zz < g.NZ;
            T sj = (T)0;
            if (valid) {
                const int64_t i = x + N * (y + N * zz);
                const T ri = r[i];  // cached: the s_{j+1} pass re-reads it one plane later
                const T xs = sm1[i];
                const T so = ldm<NT>(sm2 + i);
                const T a = s2_apply<T>(dv, ds, g, sm1, i, x, y, zz);
                T o = a1A * a + a1r * ri;
                o += a1x * xs;
                o += a1o * so;
                sj = o;
                if (ly >= 1 && ly <= S2_TY && zz >= z0 && zz < z1) {
                    if constexpr (NT) __builtin_nontemporal_store(sj, out1 + i);
                    else out1[i] = sj;
                }
            }
            plane[c] = sj;
        }
        __syncthreads();
        // s_{j+1} on plane zz - 1 (tile rows only), from the ring
        const int64_t zm = zz - 1;
        if (zm >= z0 && zm < z1) {
            const T *pc = ring + ((zm + 3) % 3) * plane_cells;
            const T *pl = ring + ((zm + 2) % 3) * plane_cells;
            const T *pu = ring + ((zm + 4) % 3) * plane_cells;
            for (int64_t c = N + threadIdx.x; c < (int64_t)(S2_TY + 1) * N; c += BLOCK) {
                const int64_t ly = c / N, x = c - ly * N, y = y0 + ly;
                if (y >= N) continue;
                const int64_t i = x + N * (y + N * zm);
                const bool xl = x > 0, xu = x + 1 < N, yl = y > 0, yu = y + 1 < N, zl = zm > 0, zu = zm + 1 < g.NZ;
                const T v0 = dv[i];
                const T u1 = dv[ds + i], u2 = dv[2 * ds + i], u3 = dv[3 * ds + i];
                const T l1 = dv[ds + (xl ? i - 1 : i)], l2 = dv[2 * ds + (yl ? i - N : i)],
                        l3 = dv[3 * ds + (zl ? i - N2 : i)];
                const T ri = r[i];
                const T so = sm1[i];
                const T xc = pc[c];
                T acc = (T)0;
                if (xl) acc += l1 * pc[c - 1];
                acc += (xu ? u1 : (T)0) * pc[xu ? c + 1 : c];
                if (yl) acc += l2 * pc[c - N];
                acc += (yu ? u2 : (T)0) * pc[c + N];
                if (zl) acc += l3 * pl[c];
                acc += (zu ? u3 : (T)0) * pu[c];
                const T a = acc + v0 * xc;
                T o = a2A * a + a2r * ri;
                o += a2x * xc;
                o += a2o * so;
                if constexpr (NT) __builtin_nontemporal_store(o, out2 + i);
                else out2[i] = o;
            }
        }
        __syncthreads();
    }
}

// Flag couplings across the x- or y-faces of the box (bad = 1): the two-step
// kernel leaves them out, so it may run only when they are all zero.
static __global__ __launch_bounds__(BLOCK) void k_s2_check(int64_t n, int64_t N, const double *__restrict__ dv,
                                                           int64_t ds, int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int64_t x = i % N, y = (i / N) % N;
    if ((x == N - 1 && dv[ds + i] != 0.0) || (y == N - 1 && dv[2 * ds + i] != 0.0)) atomicOr(bad, 1);
}

}  // namespace ppk
