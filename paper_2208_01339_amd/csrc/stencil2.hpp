// Two Chebyshev steps per pass for 3-D 7-point operators held as symmetric
// stored diagonals with offsets {0, 1, N, N*N} (rows i = x + N (y + N z),
// n = N * N * NZ, no coupling across the x- and y-faces of the box).
//
//   s_j     = c1x s_{j-1} + c1o s_{j-2} + c1r r + c1A (A s_{j-1})
//   s_{j+1} = c2x s_j     + c2o s_{j-1} + c2r r + c2A (A s_j)
//
// Each workgroup owns S2_TY whole x-lines (contiguous rows of N cells, so the
// HBM streams stay long) over zc z-planes and marches up z.  For every
// plane it computes s_j on its lines plus one halo line each side, and s_{j+1}
// one plane behind.  The operator, r and s_{j-1} are read once for both steps;
// the halo lines and the planes just outside the z-range are computed twice
// (by the neighbouring tiles too), with the same arithmetic, so both copies
// are identical.  s_j and s_{j+1} go to two fresh buffers: no input may be
// overwritten while neighbours still read it.
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace ppk {

constexpr int S2_TY = 8;              // y-rows per tile (full x-lines, one halo row each side)
constexpr int S2_RY = S2_TY + 2;
constexpr int S2_ZC_MAX = 32;         // z-planes per workgroup: 32, else 16 (enough workgroups)
constexpr int64_t S2_NMAX = 256;      // widest x-line (sizes the per-thread register arrays)
constexpr int S2_BS = 512;            // threads per workgroup
constexpr bool S2_SL = true;          // in-plane neighbours of s_{j-1} from LDS

struct Stencil2 {
    int64_t N, NZ, n;
    int nty, nzc;   // y-tiles and z-chunks
    int zc;         // z-planes per chunk
};

template <int BS>
constexpr int s2_cells_per_thread() { return (S2_RY * (int)S2_NMAX + BS - 1) / BS; }

// Thread t owns the cells c = t + BS m of the tile's plane (S2_RY x N) on
// every plane.  While it computes s_j on plane z it holds row z of the
// operator in registers, so once s_j(z) is in LDS it forms the part of
// (A s_j) on plane z that needs only planes z-1 and z (the x-, y- and -z
// terms, in the order of the one-step kernels) and adds the +z term and the
// diagonal term one plane later, when s_j(z+1) exists.  s_{j-1} on planes z-1
// and z and the coupling to plane z-1 travel in registers from plane to
// plane, so nothing is read twice apart from the in-plane neighbours of
// s_{j-1} (cache hits).  LDS: two planes of s_j (double buffer, one barrier
// per plane).  DOT: the pair ends the polynomial; partials[L] receives this
// workgroup's part of r . s_{j+1} (the dot product of the CG step).  Absent neighbours enter as zero couplings times a clamped
// (in-range) value.  UNITD: the main diagonal is 1 (Jacobi-scaled operators) and is not read.
// O2 = double with T = float: the last pair of the mixed-precision polynomial,
// whose second step writes z in FP64 and reduces r . z with r in FP64 (r64);
// it computes in FP32 with r rounded to FP32, as the single FP32 step does.
template <typename T, bool NT, int BS, bool SL, bool DOT, bool UNITD, typename O2 = T>
static __global__ __launch_bounds__(BS) void k_cheb2_stencil(Stencil2 g, const T *__restrict__ dv, int64_t ds,
                                                         const T *__restrict__ sm1, const T *__restrict__ sm2,
                                                         const T *__restrict__ r, const double *__restrict__ r64,
                                                         T *__restrict__ out1, O2 *__restrict__ out2, double c1x,
                                                         double c1o, double c1r, double c1A, double c2x, double c2o,
                                                         double c2r, double c2A, const State *st, double *partials)
{
    constexpr bool R64 = !std::is_same_v<O2, T>;
    if (st != nullptr && st->done) return;
    double dotp = 0.0;  // r . s_{j+1} over this workgroup (DOT)
    constexpr int MM = s2_cells_per_thread<BS>();
    extern __shared__ __align__(16) unsigned char s2_lds[];
    const int G = (int)gridDim.x;
    const int L = xcd_remap((int)blockIdx.x, G);
    const int ty = L % g.nty, tz = L / g.nty;
    const int64_t N = g.N, N2 = N * N, NZ = g.NZ;
    const int64_t y0 = (int64_t)ty * S2_TY - 1;
    const int64_t z0 = (int64_t)tz * g.zc, z1 = z0 + g.zc < NZ ? z0 + g.zc : NZ;
    const int64_t cells = (int64_t)S2_RY * N;
    const T a1x = (T)c1x, a1o = (T)c1o, a1r = (T)c1r, a1A = (T)c1A;
    const T a2x = (T)c2x, a2o = (T)c2o, a2r = (T)c2r, a2A = (T)c2A;
    // carried per owned cell
    T s_c[MM], s_m[MM];  // s_{j-1} on planes z and z-1
    T u3p[MM];           // coupling of plane z-1 to plane z (= the -z coupling of plane z)
    T v0p[MM], rp[MM], sjp[MM], part[MM];  // plane z-1: diagonal, r, s_j, partial (A s_j)
    double rp64[R64 ? MM : 1];             // plane z-1: r in FP64 (R64)
    // Every global load of a plane is issued before the first use of any of
    // them: indices are clamped to a valid row (0) where a cell is absent and
    // the values are masked where they are used, so the loads form one
    // branch-free block and are in flight together.
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int64_t c = threadIdx.x + (int64_t)BS * m;
        const int64_t ly = c / N, x = c - ly * N, y = y0 + ly;
        const bool rowok = c < cells && y >= 0 && y < N;
        const int64_t za = z0 - 1, zb = z0 - 2;
        const int64_t ia = rowok && za >= 0 ? x + N * (y + N * za) : 0;
        const int64_t ib = rowok && zb >= 0 ? x + N * (y + N * zb) : 0;
        s_c[m] = sm1[ia];
        s_m[m] = sm1[ib];
        u3p[m] = dv[3 * ds + ib];
    }
    // s_{j-1} planes in LDS (SL): rows -1 .. S2_RY of the tile, two buffers
    T *const sl0 = (T *)s2_lds + 2 * cells;
    const int64_t scells = cells + 2 * N;
    static_assert(2 * S2_NMAX <= BS, "one halo cell per thread");
    T hx0 = (T)0;
    if constexpr (SL) {
        const int64_t e = threadIdx.x, row = e < N ? -1 : S2_RY, x = e < N ? e : e - N, y = y0 + row;
        const int64_t za = z0 - 1;
        hx0 = sm1[e < 2 * N && y >= 0 && y < N && za >= 0 ? x + N * (y + N * za) : 0];
    }
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int64_t c = threadIdx.x + (int64_t)BS * m;
        const int64_t ly = c / N, y = y0 + ly;
        const bool rowok = c < cells && y >= 0 && y < N;
        s_c[m] = rowok && z0 - 1 >= 0 ? s_c[m] : (T)0;
        s_m[m] = rowok && z0 - 2 >= 0 ? s_m[m] : (T)0;
        u3p[m] = rowok && z0 - 2 >= 0 ? u3p[m] : (T)0;
        v0p[m] = rp[m] = sjp[m] = part[m] = (T)0;
        if constexpr (R64) rp64[m] = 0.0;
        if constexpr (SL)
            if (c < cells) sl0[c + N] = s_c[m];
    }
    if constexpr (SL) {
        const int64_t e = threadIdx.x, row = e < N ? -1 : S2_RY, x = e < N ? e : e - N, y = y0 + row;
        if (e < 2 * N) sl0[(row + 1) * N + x] = y >= 0 && y < N && z0 - 1 >= 0 ? hx0 : (T)0;
        __syncthreads();
    }
    int buf = 0;
    for (int64_t zz = z0 - 1; zz <= z1; ++zz) {
        const bool zin = zz >= 0 && zz < NZ;
        const bool fin2 = zz - 1 >= z0 && zz - 1 < z1;  // finish s_{j+1} on plane zz-1
        const bool part_now = zz >= z0 && zz < z1;      // partial sums for plane zz
        const bool zu = zz + 1 < NZ;
        T *pl = (T *)s2_lds + buf * cells;
        // the plane's global loads: operator row, r, s_{j-2} on plane zz, s_{j-1} on plane zz+1
        T v0[MM], u1[MM], u2[MM], u3[MM], l1[MM], l2[MM], ri[MM], so[MM], xp[MM];
        double r64v[R64 ? MM : 1];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const int64_t c = threadIdx.x + (int64_t)BS * m;
            const int64_t ly = c / N, x = c - ly * N, y = y0 + ly;
            const bool rowok = c < cells && y >= 0 && y < N;
            const bool ok = rowok && zin;
            const int64_t i = ok ? x + N * (y + N * zz) : 0;
            if constexpr (UNITD) v0[m] = (T)1;  // unit diagonal (Jacobi-scaled): not stored data to read
            else v0[m] = dv[i];
            u1[m] = dv[ds + i];
            u2[m] = dv[2 * ds + i];
            u3[m] = dv[3 * ds + i];
            // the mirrored couplings a_{i,i-1} and a_{i,i-N}; at the box's x- and
            // y-faces they read a stored zero of the face row (the pair kernel
            // runs only on operators without couplings across those faces)
            l1[m] = dv[ds + (ok ? (i > 0 ? i - 1 : N - 1) : 0)];
            l2[m] = dv[2 * ds + (ok ? (i >= N ? i - N : i + (N - 1) * N) : 0)];
            ri[m] = r[i];
            if constexpr (R64) r64v[m] = r64[i];
            so[m] = ldm<NT>(sm2 + i);
            xp[m] = sm1[rowok && zu ? x + N * (y + N * (zz + 1)) : 0];
        }
        T hx = (T)0;  // s_{j-1} on the halo rows -1 and S2_RY of plane zz+1 (SL)
        if constexpr (SL) {
            const int64_t e = threadIdx.x, row = e < N ? -1 : S2_RY, x = e < N ? e : e - N, y = y0 + row;
            hx = sm1[e < 2 * N && y >= 0 && y < N && zu ? x + N * (y + N * (zz + 1)) : 0];
        }
        // s_j on plane zz for every owned cell (branch-free, so that the LDS
        // reads of all cells are in flight together; absent cells give 0)
        T cur[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const int64_t c = threadIdx.x + (int64_t)BS * m;
            const int64_t ly = c / N, x = c - ly * N, y = y0 + ly;
            const bool rowok = c < cells && y >= 0 && y < N;
            const bool ok = rowok && zin;
            const int64_t i = ok ? x + N * (y + N * zz) : 0;
            // Neighbour values: a neighbour outside the box has a zero coupling
            // (stored zeros at the faces; 0 above the last plane and below the
            // first), so its value only has to be finite, read at a valid index.
            T x1m, x1p, x2m, x2p;
            if constexpr (SL) {
                const T *sp = sl0 + buf * scells + (ok ? c : 0) + N;
                x1m = sp[-1];
                x1p = sp[1];
                x2m = sp[-N];
                x2p = sp[N];
            } else {
                const bool xl = x > 0, xu = x + 1 < N, yl = y > 0, yu = y + 1 < N;
                x1m = sm1[ok && xl ? i - 1 : i];
                x1p = sm1[ok && xu ? i + 1 : i];
                x2m = sm1[ok && yl ? i - N : i];
                x2p = sm1[ok && yu ? i + N : i];
            }
            const T xs = s_c[m];
            const T xpm = rowok && zu ? xp[m] : (T)0;
            T acc = (T)0;
            acc += l1[m] * x1m;
            acc += u1[m] * x1p;
            acc += l2[m] * x2m;
            acc += u2[m] * x2p;
            acc += u3p[m] * s_m[m];
            acc += u3[m] * xpm;
            const T a = acc + v0[m] * xs;
            T o = a1A * a + a1r * ri[m];
            o += a1x * xs;
            o += a1o * so[m];
            cur[m] = ok ? o : (T)0;
        }
        // stores of s_j (plane zz) and s_{j+1} (plane zz-1); LDS copies for the next phase
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const int64_t c = threadIdx.x + (int64_t)BS * m;
            const int64_t ly = c / N, x = c - ly * N, y = y0 + ly;
            const bool rowok = c < cells && y >= 0 && y < N;
            const bool interior = ly >= 1 && ly <= S2_TY && rowok;
            const T sj = cur[m];
            if (interior && zz >= z0 && zz < z1) {
                const int64_t i = x + N * (y + N * zz);
                if constexpr (NT) __builtin_nontemporal_store(sj, out1 + i);
                else out1[i] = sj;
            }
            if (fin2 && interior) {
                const int64_t i2 = x + N * (y + N * (zz - 1));
                const T acc2 = part[m] + u3p[m] * sj;
                const T a2 = acc2 + v0p[m] * sjp[m];
                T o2 = a2A * a2 + a2r * rp[m];
                o2 += a2x * sjp[m];
                o2 += a2o * s_m[m];
                const O2 ov = (O2)o2;
                if constexpr (NT) __builtin_nontemporal_store(ov, out2 + i2);
                else out2[i2] = ov;
                if constexpr (DOT) {
                    if constexpr (R64) dotp += rp64[m] * (double)ov;
                    else dotp += (double)rp[m] * (double)ov;
                }
            }
            if (c < cells) pl[c] = sj;
            if constexpr (SL)
                if (c < cells) sl0[(buf ^ 1) * scells + c + N] = rowok && zu ? xp[m] : (T)0;
        }
        if constexpr (SL) {
            const int64_t e = threadIdx.x, row = e < N ? -1 : S2_RY, x = e < N ? e : e - N, y = y0 + row;
            if (e < 2 * N) sl0[(buf ^ 1) * scells + (row + 1) * N + x] = y >= 0 && y < N && zu ? hx : (T)0;
        }
        __syncthreads();
        // partial sums of (A s_j) on plane zz (branch-free; cells outside give 0)
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const int64_t c = threadIdx.x + (int64_t)BS * m;
            const int64_t ly = c / N, y = y0 + ly;
            const bool rowok = c < cells && y >= 0 && y < N;
            const bool ok = rowok && zin;
            const bool pc = part_now && ly >= 1 && ly <= S2_TY && c < cells && y < N;
            const int64_t cc = pc ? c : N;  // rows 1 .. S2_TY: c +- 1 and c +- N stay inside the plane
            T pn = (T)0;
            pn += l1[m] * pl[cc - 1];
            pn += u1[m] * pl[cc + 1];
            pn += l2[m] * pl[cc - N];
            pn += u2[m] * pl[cc + N];
            pn += u3p[m] * sjp[m];
            part[m] = pc ? pn : (T)0;
            v0p[m] = ok ? v0[m] : (T)0;
            rp[m] = ok ? ri[m] : (T)0;
            if constexpr (R64) rp64[m] = ok ? r64v[m] : 0.0;
            sjp[m] = cur[m];
            u3p[m] = ok ? u3[m] : (T)0;
            s_m[m] = s_c[m];
            s_c[m] = rowok && zu ? xp[m] : (T)0;
        }
        buf ^= 1;
    }
    if constexpr (DOT) {
        // this workgroup's part of r . s_{j+1}, summed in a fixed order
        __shared__ double red[BS / WAVE];
        dotp = wave_sum(dotp);
        if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = dotp;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < BS / WAVE; ++w) tot += red[w];
            partials[L] = tot;
        }
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
