// Persistent batched PCG: the whole batched solve in one cooperative launch.
//
// The phases of the graph-driven solve run here in the same order, each
// followed by a grid barrier (ppk::pcgp::gbar, the single-system driver's
// barriers with bounded waits).  Every workgroup sweeps the same workgroup
// map as the graph path: the launch has G <= nblk workgroups and workgroup L
// runs the map's entries b = L, L + G, ...  So every partial sum, its
// per-segment total (summed in map order by the segment's finalising phase,
// run by workgroup s mod G) and therefore every iterate equal those of the
// graph path when that path does not redistribute workgroups.  The loop ends
// once every (segment, column) pair has finished: the count is read right
// after a barrier, and nobody changes it before the next barrier, so all
// workgroups see the same value and leave together.  No host round trip
// happens between the first phase and the last.
#pragma once
#include "batch.hpp"
#include "persistent.hpp"

namespace ppb {

struct BPArgs {
    Batch bt;
    BState st;
    ppk::SellView A;    // FP64 values
    ppk::SellView A32;  // FP32 values (mixed)
    const double *B;    // caller layout [n_ext][nrhs]
    double *X;          // caller layout: initial guess in, solution out
    const double *dis;
    double *Bh, *Xh, *R, *P, *Q, *Z, *SA64, *SB64;
    float *R32, *SA, *SB;
    double *partials;
    const double *coef;   // [S][k][4]
    const double *thinv;  // [S]
    int nblk;             // entries of the workgroup map
    int k;
    int maxit;
    int total;            // S * NB (segment, column) pairs
    unsigned long long *bw;
    int bar_mode;
    unsigned int spin;
};

template <int W, int CPL, bool MIXED>
__global__ __launch_bounds__(BLOCK) void kbp_solve(BPArgs a)
{
    constexpr int NB = W * CPL;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ int bflag;
    ppk::pcgp::Ctx c;
    c.G = (int)gridDim.x;
    c.L = ppk::xcd_remap((int)blockIdx.x, c.G);
    c.pbuf = 0;
    c.partials = nullptr;
    c.lds = nullptr;
    c.red = nullptr;
    c.flag = &bflag;
    c.bw = a.bw;
    c.mode = a.bar_mode;
    c.spin = a.spin;
    ppk::pcgp::gbar_init(grid, c);
    const Batch bt = a.bt;
    const BState st = a.st;
    // one phase over the map, then a barrier
    auto blocks = [&](auto f) {
        for (int b = c.L; b < a.nblk; b += c.G) f(b);
        ppk::pcgp::gbar(grid, c);
    };
    // the segments' finalising phase (partials -> CG scalars), then a barrier
    auto fin = [&](int f) {
        for (int s = c.L; s < bt.S; s += c.G) kbd_fin<NB>(s, bt, st, a.partials, f, 0);
        ppk::pcgp::gbar(grid, c);
    };
    auto all_done = [&]() {
        return __hip_atomic_load(st.ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= a.total;
    };
    // Z = p_k(A-hat) R for every column, then R.Z reduced under `f`
    auto poly = [&](int f) {
        if (a.k == 0) {
            blocks([&](int b) { kbd_deg0<W, CPL>(b, bt, st, a.A, a.R, a.Z, a.thinv, a.partials, f); });
            fin(f);
            return;
        }
        if constexpr (!MIXED) {
            for (int j = 1; j <= a.k && !c.abort; ++j) {
                const bool last = (j == a.k);
                const double *X = j == 1 ? a.R : ((j % 2 == 0) ? a.SA64 : a.SB64);
                const double *old = (j % 2 == 0) ? a.SB64 : a.SA64;
                double *out = last ? a.Z : ((j % 2 == 1) ? a.SA64 : a.SB64);
                const int mode = j == 1 ? 1 : (j == 2 ? 2 : 3);
                blocks([&](int b) {
#define KBP64(M, LAST)                                                                                            \
    kbd_cheb<double, double, double, W, CPL, M, LAST, false>(b, bt, st, a.A, X, a.R, old, out, a.coef, j, a.partials, \
                                                             f)
                    if (last) {
                        if (mode == 1) KBP64(1, true);
                        else if (mode == 2) KBP64(2, true);
                        else KBP64(3, true);
                    } else {
                        if (mode == 1) KBP64(1, false);
                        else if (mode == 2) KBP64(2, false);
                        else KBP64(3, false);
                    }
#undef KBP64
                });
                if (last) fin(f);
            }
        } else {
            blocks([&](int b) { kbd_conv<W, CPL>(b, bt, st, a.A32, a.R, a.R32); });
            for (int j = 1; j <= a.k && !c.abort; ++j) {
                const bool last = (j == a.k);
                const float *X = j == 1 ? a.R32 : ((j % 2 == 0) ? a.SA : a.SB);
                const float *old = (j % 2 == 0) ? a.SB : a.SA;
                float *out = (j % 2 == 1) ? a.SA : a.SB;
                const int mode = j == 1 ? 1 : (j == 2 ? 2 : 3);
                blocks([&](int b) {
#define KBP32(M)                                                                                                       \
    kbd_cheb<float, float, float, W, CPL, M, false, false>(b, bt, st, a.A32, X, a.R32, old, out, a.coef, j, a.partials, \
                                                           f)
#define KBP32L(M)                                                                                                      \
    kbd_cheb<float, double, double, W, CPL, M, true, false>(b, bt, st, a.A32, X, a.R, old, a.Z, a.coef, j, a.partials, \
                                                            f)
                    if (last) {
                        if (mode == 1) KBP32L(1);
                        else if (mode == 2) KBP32L(2);
                        else KBP32L(3);
                    } else {
                        if (mode == 1) KBP32(1);
                        else if (mode == 2) KBP32(2);
                        else KBP32(3);
                    }
#undef KBP32
#undef KBP32L
                });
                if (last) fin(f);
            }
        }
    };

    blocks([&](int b) { kbd_init_scale<W, CPL>(b, bt, st, a.A, a.B, a.X, a.dis, a.Bh, a.Xh, a.partials); });
    fin(BF_BNORM);
    blocks([&](int b) { kbd_apply64<W, CPL, 0, false>(b, bt, st, a.A, a.Xh, a.Bh, a.R, a.partials); });
    fin(BF_RR0);
    if (!c.abort && !all_done()) {
        poly(BF_RHO0);
        blocks([&](int b) { kbd_p<W, CPL>(b, bt, st, a.A, a.Z, a.P, 1); });
        for (int it = 0; it < a.maxit && !c.abort; ++it) {
            blocks([&](int b) {
                kbd_apply64<W, CPL, 1, false>(b, bt, st, a.A, a.P, (const double *)nullptr, a.Q, a.partials);
            });
            fin(BF_GAMMA);
            blocks([&](int b) { kbd_xr<W, CPL>(b, bt, st, a.A, a.P, a.Q, a.Xh, a.R, a.partials); });
            fin(BF_RR);
            if (c.abort || all_done()) break;
            poly(BF_RHO);
            blocks([&](int b) { kbd_p<W, CPL>(b, bt, st, a.A, a.Z, a.P, 0); });
        }
    }
    for (int b = c.L; b < a.nblk; b += c.G) kbd_final<W, CPL>(b, bt, st, a.A, a.Xh, a.dis, a.X);
}

}  // namespace ppb
