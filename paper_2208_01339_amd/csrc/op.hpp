// The single-operator handle, shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "dfn.hpp"
#include "kernels.hpp"
#include "ltile.hpp"

constexpr int PP_GRID_DEFAULT = 2048;

struct pp_op_s {
    int kind = 0;  // 0 CSR, 1 Schur, 2 DFN S_u (its A x read from tw, filled by Algorithm 3)
    int64_t n = 0, nt = 0, nnz_c = 0, nnz_given = 0;
    unsigned flags = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    // slice layout of A-hat (and appended trace columns)
    int64_t nslices = 0, nstored = 0;
    int64_t *sp = nullptr;
    int32_t *scol = nullptr;
    double *sval = nullptr;
    float *sval32 = nullptr;
    int sell = 1;  // slice part non-empty
    // symmetric diagonal part: nd diagonals of dstride values each
    int nd = 0;
    int64_t doff[ppk::DMAX] = {};
    int64_t dstride = 0;
    double *dval = nullptr;
    float *dval32 = nullptr;
    // trace operator M^{-1} C-hat (Schur)
    int64_t *crp = nullptr;
    int32_t *ccol = nullptr;
    double *cm = nullptr;
    float *cm32 = nullptr;
    double *tw = nullptr;
    float *tw32 = nullptr;
    // DFN S_u (kind 2): band factor, copies of C, a B, G^h (fracture rows) and
    // of C^T, a B^T, G^u (unknown rows), two fracture-row work vectors
    int64_t dfn_F = 0, dfn_G = 0, dfn_nh = 0;
    double *dfn_Lb = nullptr;
    double *dfn_Q = nullptr;  // Qf, Qb (nh G + DFN_WAVE each), di2 (nh)
    int32_t *dfn_ghc = nullptr;  // G^h by entry slots (dfn_ghw > 0)
    double *dfn_ghv = nullptr;
    int dfn_ghw = 0;
    int64_t *dfn_rp[6] = {};
    int32_t *dfn_col[6] = {};
    double *dfn_val[6] = {};
    double *dfn_t = nullptr, *dfn_d = nullptr;
    // Jacobi
    double *dis = nullptr;
    // renumbering chosen at create (reverse Cuthill-McKee), new -> old row; null = none
    int32_t *perm = nullptr;
    double spread[2] = {0.0, 0.0};  // gather spread of the slices before / after renumbering
    // LDS-staged x tiles (ltile.hpp): slices-only FP64 operators whose tiles fit
    int lt_on = 0;       // planned at create
    int lt_use = 1;      // PP_OPT_LDS_TILES
    int64_t lt_ntiles = 0;
    int lt_cap = 0;
    int32_t *lt_seg = nullptr;  // seg_ptr [ntiles+1], staged [ntiles], then seg_col, seg_lds, seg_len [nseg each]
    uint16_t *lt_lcol = nullptr;
    int64_t lt_nseg = 0;
    // work vectors
    double *xh = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *bh = nullptr;
    double *sA = nullptr, *sB = nullptr;
    float *r32 = nullptr, *sA32 = nullptr, *sB32 = nullptr;
    // two Chebyshev steps per pass (3-D 7-point operators): box N x N x s2NZ,
    // two more step buffers
    bool s2 = false;
    int two_step = 1;  // 0 off, 1 when the box fills the device, 2 for any box
    int cus = 256;     // compute units of the device (pair launches want one workgroup per CU)
    int64_t s2N = 0, s2NZ = 0;
    double *sC = nullptr, *sD = nullptr;
    float *sC32 = nullptr, *sD32 = nullptr;  // the same in mixed mode
    double *partials = nullptr;  // (1 + LR_MAX) * 8192 doubles
    // spectral low-rank correction: V (n x lr_p, column-major), (V^T A V)^{-1}
    int lr_p = 0;
    double *lr_v = nullptr;
    double *lr_hinv = nullptr;
    double *coef_d = nullptr;  // [k][4] step coefficients for the persistent driver
    int coef_k = -1;           // degree the device coefficients were uploaded for
    std::vector<double> coef_h;
    int persist_occ[4] = {0, 0, 0, 0};
    ppk::State *st = nullptr;
    ppk::State *hst = nullptr;  // pinned
    int32_t *hflag = nullptr;   // pinned, 2 slots
    hipEvent_t flag_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> tev;  // timing events (pairs)
    std::vector<hipEvent_t> pev;  // timing events around the fused-pair launches
    size_t pev_i = 0;             // pev used in the current solve
    int pairs_per_poly = 0;       // fused-pair launches in one polynomial application
    bool time_pairs = false;      // record pev (a timed solve is being enqueued)
    hipEvent_t solve_ev[2] = {nullptr, nullptr};
    // polynomial
    bool setup_done = false;
    int k = 0;
    double lmin = 0, lmax = 0, xi = 0, theta = 0, delta = 0, sigma = 0;
    std::vector<double> rho;
    // Newton form (Algorithm 1): form = 1, degree 2^nlev - 1, scalings zeta_0..nlev,
    // two work vectors per level
    int form = 0;
    int nlev = 0;
    std::vector<double> zeta;
    double *nbuf = nullptr;
    int nbuf_levels = 0;
    // options
    int grid_max = PP_GRID_DEFAULT;
    int grid_auto = PP_GRID_DEFAULT;  // resident workgroups of the fused step (CUs x occupancy)
    int chunk = 0;  // 0 = auto
    int timing = 0;
    int driver = -1;  // -1 auto, 0 stream-driven, 1 persistent
    int bar_mode = -1;           // persistent grid barrier: -1 auto, 0 runtime, 1 flat, 2 two-level
    unsigned int spin = 1u << 21;  // polls before a barrier wait gives up
    unsigned long long *bw = nullptr;  // barrier words of the persistent driver
    int ritz_poly = 0;  // pp_lowrank_ritz: 0 Lanczos on A-hat, 1 on p_k(A-hat) with full reorthogonalisation
    std::vector<double> lr_theta, lr_res;  // v^T A-hat v and ||A-hat v - theta v|| of the installed V
    int verify = -1;  // true-residual check at convergence: -1 auto (mixed mode), 0 off, 1 on
    int pass_maxit = 0;  // iteration budget of the current pass of pcg_solve
    int ntload = 1;   // set at create from the operator's size
    pp_stats stats{};

    // kinds whose fused kernels read trace columns from tw
    bool schur() const { return kind == 1 || kind == 2; }
    bool dfn() const { return kind == 2; }
    ppk::DfnView dview() const
    {
        ppk::DfnView v;
        v.F = dfn_F;
        v.G = dfn_G;
        v.nf = dfn_G * dfn_G;
        v.nh = dfn_nh;
        v.nu = n;
        v.Lb = dfn_Lb;
        const size_t qn = (size_t)dfn_nh * dfn_G + ppk::DFN_WAVE;
        v.Qf = dfn_Q;
        v.Qb = dfn_Q ? dfn_Q + qn : nullptr;
        v.di2 = dfn_Q ? dfn_Q + 2 * qn : nullptr;
        v.ghc = dfn_ghc;
        v.ghv = dfn_ghv;
        v.ghw = dfn_ghw;
        ppk::CsrD *m[6] = {&v.c, &v.b, &v.gh, &v.ct, &v.bt, &v.gu};
        for (int i = 0; i < 6; ++i) {
            m[i]->rp = dfn_rp[i];
            m[i]->col = dfn_col[i];
            m[i]->val = dfn_val[i];
        }
        return v;
    }
    bool mixed() const { return (flags & PP_MIXED) != 0; }

    int grid_slices() const
    {
        int64_t g = (nslices + ppk::WPB - 1) / ppk::WPB;
        return (int)std::max<int64_t>(1, std::min<int64_t>(g, grid_max));
    }
    int grid_elems(int64_t cnt) const
    {
        int64_t g = (cnt + ppk::BLOCK - 1) / ppk::BLOCK;
        return (int)std::max<int64_t>(1, std::min<int64_t>(g, grid_max));
    }
    ppk::SellView view(bool f32) const
    {
        ppk::SellView v;
        v.sp = sp;
        v.col = scol;
        v.val = f32 ? (const void *)sval32 : (const void *)sval;
        v.n = n;
        v.nslices = nslices;
        v.nx = n;
        v.sell = sell;
        v.nd = nd;
        v.dv = f32 ? (const void *)dval32 : (const void *)dval;
        v.dstride = dstride;
        for (int d = 0; d < ppk::DMAX; ++d) v.doff[d] = doff[d];
        return v;
    }
    ppk::LtView ltview() const
    {
        ppk::LtView v;
        v.ntiles = lt_ntiles;
        v.cap = lt_cap;
        v.seg_ptr = lt_seg;
        v.staged = lt_seg + lt_ntiles + 1;
        v.seg_col = v.staged + lt_ntiles;
        v.seg_lds = v.seg_col + lt_nseg;
        v.seg_len = v.seg_lds + lt_nseg;
        v.lcol = lt_lcol;
        return v;
    }
    ppk::CsrView cview(bool f32) const
    {
        ppk::CsrView v;
        v.rp = crp;
        v.col = ccol;
        v.val = f32 ? (const void *)cm32 : (const void *)cm;
        v.rows = nt;
        return v;
    }

    void release()
    {
        ppc::dfree(sp); ppc::dfree(scol); ppc::dfree(sval); ppc::dfree(sval32);
        ppc::dfree(dval); ppc::dfree(dval32);
        ppc::dfree(crp); ppc::dfree(ccol); ppc::dfree(cm); ppc::dfree(cm32); ppc::dfree(tw); ppc::dfree(tw32);
        ppc::dfree(dis); ppc::dfree(perm); ppc::dfree(lt_seg); ppc::dfree(lt_lcol);
        ppc::dfree(dfn_Lb); ppc::dfree(dfn_Q); ppc::dfree(dfn_ghc); ppc::dfree(dfn_ghv); ppc::dfree(dfn_t); ppc::dfree(dfn_d);
        for (int i = 0; i < 6; ++i) { ppc::dfree(dfn_rp[i]); ppc::dfree(dfn_col[i]); ppc::dfree(dfn_val[i]); }
        ppc::dfree(xh); ppc::dfree(r); ppc::dfree(p); ppc::dfree(q); ppc::dfree(z); ppc::dfree(bh); ppc::dfree(sA); ppc::dfree(sB);
        ppc::dfree(r32); ppc::dfree(sA32); ppc::dfree(sB32);
        ppc::dfree(sC); ppc::dfree(sD);
        ppc::dfree(sC32); ppc::dfree(sD32);
        ppc::dfree(partials); ppc::dfree(coef_d); ppc::dfree(bw); ppc::dfree(st);
        ppc::dfree(lr_v); ppc::dfree(lr_hinv); ppc::dfree(nbuf);
        if (hst) (void)hipHostFree(hst);
        if (hflag) (void)hipHostFree(hflag);
        hst = nullptr;
        hflag = nullptr;
        for (auto &e : flag_ev) if (e) { (void)hipEventDestroy(e); e = nullptr; }
        for (auto &e : solve_ev) if (e) { (void)hipEventDestroy(e); e = nullptr; }
        for (auto &e : tev) (void)hipEventDestroy(e);
        tev.clear();
        for (auto &e : pev) (void)hipEventDestroy(e);
        pev.clear();
    }
};
