// C-ABI implementation of the batch entry points of include/pp.h: many
// independent systems and/or a block of right-hand sides per system.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "batch.hpp"
#include "batch_persist.hpp"
#include "common.hpp"
#include "dia_plan.hpp"
#include "sym_eig.hpp"

using ppc::dalloc;
using ppc::dfree;
using ppc::fail;
using ppc::hip_fail;
using ppc::HipError;
using ppk::BLOCK;
using ppk::WAVE;
using ppk::WPB;

struct pp_batch_s {
    int S = 0, NB = 1, nrhs = 1, W = 1, CPL = 1;
    unsigned flags = 0;
    hipStream_t ustream = nullptr;  // caller's stream
    hipStream_t stream = nullptr;   // internal stream (capturable)
    int device = 0;
    int64_t n_ext = 0, nnz = 0, nslices = 0, n_int = 0, nstored = 0;
    int G = 0;
    std::vector<int64_t> sys_ptr, seg_row0_h, seg_n_h;
    // workgroup map at create (restored after every solve) and the map in use
    std::vector<int32_t> blk_seg_h, seg_blk0_h, map_seg, map_blk0;
    std::vector<int64_t> blk_s0_h, blk_s1_h, map_s0, map_s1;
    std::vector<int32_t> seg_done_h;
    bool remapped = false;
    // maps
    int32_t *blk_seg = nullptr, *seg_blk0 = nullptr, *slice_seg = nullptr;
    int64_t *blk_s0 = nullptr, *blk_s1 = nullptr, *seg_row0 = nullptr, *seg_n = nullptr, *ext_row0 = nullptr;
    // operator
    int64_t *sp = nullptr;
    int32_t *scol = nullptr;
    double *sval = nullptr;
    float *sval32 = nullptr;
    double *dis = nullptr;
    // symmetric stored diagonals per system
    int32_t *seg_nd = nullptr, *seg_sell = nullptr;
    int64_t *seg_off = nullptr;
    double *dv64 = nullptr;
    float *dv32 = nullptr;
    int diag_systems = 0;
    // vectors [n_int][NB]
    double *Xh = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *Z = nullptr, *Bh = nullptr;
    double *SA64 = nullptr, *SB64 = nullptr;
    float *R32 = nullptr, *SA = nullptr, *SB = nullptr;
    double *partials = nullptr;
    double *coef_d = nullptr, *thinv_d = nullptr;
    // state
    double *d_rho = nullptr, *d_alpha = nullptr, *d_beta = nullptr, *d_rr = nullptr, *d_bn2 = nullptr,
           *d_tol2 = nullptr, *d_lz = nullptr;
    int32_t *d_it = nullptr, *d_status = nullptr, *d_done = nullptr, *d_zero_b = nullptr, *d_seg_ndone = nullptr,
            *d_seg_done = nullptr, *d_ndone = nullptr;
    uint32_t *d_ticket = nullptr;
    int32_t *h_ndone = nullptr;  // pinned [2]
    int32_t *h_segdone = nullptr;  // pinned [2][S]
    hipEvent_t flag_ev[2] = {nullptr, nullptr};
    hipEvent_t sync_ev = nullptr, solve_ev[2] = {nullptr, nullptr};
    // polynomial
    bool setup_done = false;
    int k = 0;
    double xi = 0;
    std::vector<double> lmin, lmax;
    // options
    int chunk = 0, ntload = 1, use_graph = 1;
    int driver = 0;                    // 0: captured iteration chunks, host one chunk behind; 1: one persistent launch
    int pgrid = 0;                     // workgroups of the persistent launch, 0 = all resident ones
    int bar_mode = -1;                 // grid barrier of the persistent launch (PP_OPT_BARRIER)
    unsigned int spin = 1u << 21;      // polls before a barrier wait gives up
    unsigned long long *bw = nullptr;  // barrier words
    unsigned long long h_abort = 0;
    bool timed_out = false;
    int verify = -1;  // true-residual check at convergence: -1 auto (mixed mode), 0 off, 1 on
    // captured iteration chunk
    hipGraphExec_t gexec = nullptr;
    int g_k = -1, g_chunk = -1, g_maxit = -1, g_W = -1;
    double g_tol = -1.0;
    pp_batch_stats stats{};

    bool mixed() const { return (flags & PP_MIXED) != 0; }

    ppb::Batch bt() const
    {
        ppb::Batch b;
        b.blk_seg = blk_seg;
        b.blk_s0 = blk_s0;
        b.blk_s1 = blk_s1;
        b.seg_blk0 = seg_blk0;
        b.seg_row0 = seg_row0;
        b.seg_n = seg_n;
        b.ext_row0 = ext_row0;
        b.S = S;
        b.NB = NB;
        b.nrhs = nrhs;
        b.k = k;
        b.seg_nd = seg_nd;
        b.seg_sell = seg_sell;
        b.seg_off = seg_off;
        b.dv64 = dv64;
        b.dv32 = dv32;
        b.dstride = n_int;
        b.unit_d0 = (flags & PP_JACOBI) != 0 ? 1 : 0;
        return b;
    }
    ppb::BState bst(double tol, int maxit) const
    {
        ppb::BState s;
        s.rho = d_rho; s.alpha = d_alpha; s.beta = d_beta; s.rr = d_rr; s.bn2 = d_bn2; s.tol2 = d_tol2;
        s.lz = d_lz;
        s.it = d_it; s.status = d_status; s.done = d_done; s.zero_b = d_zero_b;
        s.seg_ndone = d_seg_ndone; s.seg_done = d_seg_done; s.ticket = d_ticket; s.ndone = d_ndone;
        s.tol = tol;
        s.maxit = maxit;
        return s;
    }
    ppk::SellView view(bool f32) const
    {
        ppk::SellView v;
        v.sp = sp;
        v.col = scol;
        v.val = f32 ? (const void *)sval32 : (const void *)sval;
        v.n = n_int;
        v.nslices = nslices;
        v.nx = n_int;
        return v;
    }

    void release()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        dfree(blk_seg); dfree(seg_blk0); dfree(slice_seg); dfree(blk_s0); dfree(blk_s1); dfree(seg_row0);
        dfree(seg_n); dfree(ext_row0);
        dfree(sp); dfree(scol); dfree(sval); dfree(sval32); dfree(dis);
        dfree(seg_nd); dfree(seg_sell); dfree(seg_off); dfree(dv64); dfree(dv32);
        dfree(Xh); dfree(R); dfree(P); dfree(Q); dfree(Z); dfree(Bh); dfree(SA64); dfree(SB64);
        dfree(R32); dfree(SA); dfree(SB); dfree(partials); dfree(coef_d); dfree(thinv_d); dfree(bw);
        dfree(d_rho); dfree(d_alpha); dfree(d_beta); dfree(d_rr); dfree(d_bn2); dfree(d_tol2); dfree(d_lz);
        dfree(d_it); dfree(d_status); dfree(d_done); dfree(d_zero_b); dfree(d_seg_ndone); dfree(d_seg_done);
        dfree(d_ndone); dfree(d_ticket);
        if (h_ndone) (void)hipHostFree(h_ndone);
        h_ndone = nullptr;
        if (h_segdone) (void)hipHostFree(h_segdone);
        h_segdone = nullptr;
        for (auto &e : flag_ev) if (e) { (void)hipEventDestroy(e); e = nullptr; }
        for (auto &e : solve_ev) if (e) { (void)hipEventDestroy(e); e = nullptr; }
        if (sync_ev) (void)hipEventDestroy(sync_ev);
        sync_ev = nullptr;
        if (stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};

namespace {

template <int V>
using IC = std::integral_constant<int, V>;

// supported (W, CPL) layouts per internal block width NB
bool layout_ok(int NB, int W)
{
    if (NB == 1) return W == 1;
    if (NB == 8) return W == 8 || W == 4 || W == 2 || W == 1;
    if (NB == 32) return W == 32 || W == 16 || W == 8 || W == 4;
    return false;
}

template <class F>
void with_layout(int W, int CPL, F &&f)
{
    if (W == 1 && CPL == 1) f(IC<1>{}, IC<1>{});
    else if (W == 8 && CPL == 1) f(IC<8>{}, IC<1>{});
    else if (W == 4 && CPL == 2) f(IC<4>{}, IC<2>{});
    else if (W == 2 && CPL == 4) f(IC<2>{}, IC<4>{});
    else if (W == 32 && CPL == 1) f(IC<32>{}, IC<1>{});
    else if (W == 16 && CPL == 2) f(IC<16>{}, IC<2>{});
    else if (W == 8 && CPL == 4) f(IC<8>{}, IC<4>{});
    else if (W == 1 && CPL == 8) f(IC<1>{}, IC<8>{});
    else if (W == 4 && CPL == 8) f(IC<4>{}, IC<8>{});
}

// caller stream -> internal stream ordering
void begin_call(pp_batch_s *op)
{
    HIPCHK(hipEventRecord(op->sync_ev, op->ustream));
    HIPCHK(hipStreamWaitEvent(op->stream, op->sync_ev, 0));
}

void end_call(pp_batch_s *op)
{
    HIPCHK(hipEventRecord(op->sync_ev, op->stream));
    HIPCHK(hipStreamWaitEvent(op->ustream, op->sync_ev, 0));
}

// Symmetric stored diagonals per system, chosen as for a single operator
// (choose_diagonals) on the system's own offset histogram.  The batch kernels
// take 5-point (3 diagonals) and 7-point (4) shapes; any other choice, a
// duplicate entry or an asymmetric value leaves the system in the slice
// layout.  Values live at dv[d * n_int + internal row], Jacobi-scaled.
void build_diagonals(pp_batch_s *op, const int64_t *rowptr, const int32_t *colind, const double *val)
{
    using ppk::OFF_SLOTS;
    typedef unsigned long long u64;
    const int S = op->S;
    std::vector<int32_t> nd(S, 0);
    std::vector<int64_t> off((size_t)S * ppk::DMAX, 0);
    struct Tmp {
        u64 *key = nullptr, *cnt = nullptr;
        int *flag = nullptr;
        ~Tmp() { dfree(key); dfree(cnt); dfree(flag); }
    } t;
    if (!(op->flags & PP_SLICED)) {
        t.key = dalloc<u64>((size_t)S * OFF_SLOTS);
        t.cnt = dalloc<u64>((size_t)S * OFF_SLOTS);
        t.flag = dalloc<int>(S);
        std::vector<u64> hk((size_t)S * OFF_SLOTS, ppk::OFF_EMPTY), hc((size_t)S * OFF_SLOTS, 0);
        std::vector<int> hf(S, 0);
        HIPCHK(hipMemcpyAsync(t.key, hk.data(), sizeof(u64) * hk.size(), hipMemcpyHostToDevice, op->stream));
        HIPCHK(hipMemsetAsync(t.cnt, 0, sizeof(u64) * hc.size(), op->stream));
        HIPCHK(hipMemsetAsync(t.flag, 0, sizeof(int) * S, op->stream));
        for (int s = 0; s < S; ++s) {
            const int64_t n = op->seg_n_h[s], e0 = op->sys_ptr[s];
            const unsigned g = (unsigned)std::min<int64_t>(2048, (n + BLOCK - 1) / BLOCK);
            hipLaunchKernelGGL(ppk::k_offsets, dim3(g), dim3(BLOCK), 0, op->stream, n, e0, rowptr + e0, colind, val,
                               t.key + (size_t)s * OFF_SLOTS, t.cnt + (size_t)s * OFF_SLOTS, t.flag + s);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hk.data(), t.key, sizeof(u64) * hk.size(), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipMemcpyAsync(hc.data(), t.cnt, sizeof(u64) * hc.size(), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipMemcpyAsync(hf.data(), t.flag, sizeof(int) * S, hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        int ndmax = 0;
        std::vector<ppk::DiaSet> D(S);
        for (int s = 0; s < S; ++s) {
            if (hf[s]) continue;
            D[s] = choose_diagonals(hk.data() + (size_t)s * OFF_SLOTS, hc.data() + (size_t)s * OFF_SLOTS,
                                    op->seg_n_h[s]);
            if (D[s].nd != 3 && D[s].nd != 4) D[s] = ppk::DiaSet{};
            ndmax = std::max(ndmax, D[s].nd);
        }
        if (ndmax > 0) {
            const int64_t ds = op->n_int;
            op->dv64 = dalloc<double>((size_t)ndmax * ds);
            HIPCHK(hipMemsetAsync(op->dv64, 0, sizeof(double) * ndmax * ds, op->stream));
            HIPCHK(hipMemsetAsync(t.cnt, 0, sizeof(u64) * 2 * S, op->stream));
            HIPCHK(hipMemsetAsync(t.flag, 0, sizeof(int) * S, op->stream));
            for (int s = 0; s < S; ++s) {
                if (D[s].nd == 0) continue;
                const int64_t n = op->seg_n_h[s], e0 = op->sys_ptr[s], r0 = op->seg_row0_h[s];
                const unsigned gr = (unsigned)((n + BLOCK - 1) / BLOCK);
                hipLaunchKernelGGL(ppk::k_dia_fill, dim3(gr), dim3(BLOCK), 0, op->stream, n, e0, rowptr + e0, colind,
                                   val, D[s], op->dv64 + r0, ds, t.cnt + 2 * s, t.flag + s);
                hipLaunchKernelGGL(ppk::k_dia_check, dim3(gr), dim3(BLOCK), 0, op->stream, n, e0, rowptr + e0,
                                   colind, val, D[s], (const double *)op->dv64 + r0, ds, t.flag + s);
            }
            HIPCHK(hipGetLastError());
            std::vector<u64> ul(2 * S);
            HIPCHK(hipMemcpyAsync(ul.data(), t.cnt, sizeof(u64) * 2 * S, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipMemcpyAsync(hf.data(), t.flag, sizeof(int) * S, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            if (op->mixed()) {
                op->dv32 = dalloc<float>((size_t)ndmax * ds);
                HIPCHK(hipMemsetAsync(op->dv32, 0, sizeof(float) * ndmax * ds, op->stream));
            }
            const bool jac = (op->flags & PP_JACOBI) != 0;
            for (int s = 0; s < S; ++s) {
                if (D[s].nd == 0) continue;
                if (hf[s] || ul[2 * s] != ul[2 * s + 1]) {
                    D[s] = ppk::DiaSet{};
                    continue;
                }
                const int64_t n = op->seg_n_h[s], r0 = op->seg_row0_h[s];
                hipLaunchKernelGGL(ppk::k_dia_scale, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                                   op->stream, n, D[s], jac ? (const double *)op->dis + r0 : (const double *)nullptr,
                                   op->dv64 + r0, op->dv32 ? op->dv32 + r0 : (float *)nullptr, ds, jac ? 1 : 0);
                nd[s] = D[s].nd;
                for (int d = 0; d < ppk::DMAX; ++d) off[(size_t)s * ppk::DMAX + d] = D[s].off[d];
            }
            HIPCHK(hipGetLastError());
        }
    }
    op->diag_systems = (int)std::count_if(nd.begin(), nd.end(), [](int v) { return v > 0; });
    op->seg_nd = dalloc<int32_t>(S);
    op->seg_off = dalloc<int64_t>((size_t)S * ppk::DMAX);
    HIPCHK(hipMemcpyAsync(op->seg_nd, nd.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(op->seg_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));  // host vectors go out of scope
}

pp_status build(pp_batch_s *op, const int64_t *rowptr, const int32_t *colind, const double *val)
{
    const int S = op->S;
    int *flag_d = nullptr;
    int64_t *width = nullptr;
    auto cleanup = [&]() { dfree(flag_d); dfree(width); };
    try {
        HIPCHK(hipStreamCreateWithFlags(&op->stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&op->sync_ev, hipEventDisableTiming));
        for (auto &e : op->flag_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : op->solve_ev) HIPCHK(hipEventCreate(&e));
        begin_call(op);
        // structure check of the whole CSR
        flag_d = dalloc<int>(1);
        HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
        hipLaunchKernelGGL(ppk::k_check_csr, dim3((unsigned)((op->n_ext + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                           op->stream, op->n_ext, op->n_ext, op->nnz, rowptr, colind, flag_d);
        HIPCHK(hipGetLastError());
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, flag_d, sizeof(int), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        if (h) { cleanup(); return fail(PP_ERR_ARG, "invalid CSR structure"); }

        // segment layout: every system padded to whole slices
        op->seg_row0_h.assign(S + 1, 0);
        op->seg_n_h.assign(S, 0);
        std::vector<int64_t> seg_sl0(S + 1, 0);
        for (int s = 0; s < S; ++s) {
            op->seg_n_h[s] = op->sys_ptr[s + 1] - op->sys_ptr[s];
            const int64_t sl = (op->seg_n_h[s] + WAVE - 1) / WAVE;
            seg_sl0[s + 1] = seg_sl0[s] + sl;
            op->seg_row0_h[s + 1] = seg_sl0[s + 1] * WAVE;
        }
        op->nslices = seg_sl0[S];
        op->n_int = op->nslices * WAVE;
        if (op->n_int > (int64_t)INT32_MAX - 1) { cleanup(); return fail(PP_ERR_ARG, "padded rows exceed 2^31"); }
        std::vector<int32_t> slice_seg(op->nslices);
        for (int s = 0; s < S; ++s)
            for (int64_t q = seg_sl0[s]; q < seg_sl0[s + 1]; ++q) slice_seg[q] = s;
        // workgroups: proportional to slices, at least one per system, never two systems in one
        int cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, op->device);
        // many systems: 4x more workgroups, so that the systems still running
        // after the small ones finish keep the device busy
        const int64_t target = (int64_t)cus * (S > 1 ? 32 : 8);
        std::vector<int32_t> blk_seg, seg_blk0(S + 1, 0);
        std::vector<int64_t> blk_s0, blk_s1;
        for (int s = 0; s < S; ++s) {
            const int64_t sl = seg_sl0[s + 1] - seg_sl0[s];
            int64_t nb = (int64_t)std::llround((double)target * (double)sl / (double)op->nslices);
            nb = std::max<int64_t>(1, std::min<int64_t>(nb, (sl + WPB - 1) / WPB));
            for (int64_t i = 0; i < nb; ++i) {
                blk_seg.push_back(s);
                blk_s0.push_back(seg_sl0[s] + sl * i / nb);
                blk_s1.push_back(seg_sl0[s] + sl * (i + 1) / nb);
            }
            seg_blk0[s + 1] = (int32_t)blk_seg.size();
        }
        op->G = (int)blk_seg.size();
        op->blk_seg_h = blk_seg;
        op->blk_s0_h = blk_s0;
        op->blk_s1_h = blk_s1;
        op->seg_blk0_h = seg_blk0;
        auto upload = [&](auto *&dst, const auto &src) {
            using T = typename std::remove_reference<decltype(src[0])>::type;
            dst = dalloc<typename std::remove_const<T>::type>(src.size());
            HIPCHK(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, op->stream));
        };
        upload(op->blk_seg, blk_seg);
        upload(op->blk_s0, blk_s0);
        upload(op->blk_s1, blk_s1);
        upload(op->seg_blk0, seg_blk0);
        upload(op->seg_row0, op->seg_row0_h);
        upload(op->seg_n, op->seg_n_h);
        upload(op->ext_row0, op->sys_ptr);
        upload(op->slice_seg, slice_seg);
        HIPCHK(hipStreamSynchronize(op->stream));  // host vectors may go out of scope

        // diagonal / Jacobi and block-diagonal check
        op->dis = dalloc<double>(op->n_int);
        HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
        hipLaunchKernelGGL(ppb::kb_diag, dim3((unsigned)((op->n_int + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, op->stream,
                           op->nslices, (const int32_t *)op->slice_seg, (const int64_t *)op->seg_row0,
                           (const int64_t *)op->seg_n, (const int64_t *)op->ext_row0, rowptr, colind, val, op->dis,
                           (int)((op->flags & PP_JACOBI) != 0), flag_d);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&h, flag_d, sizeof(int), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        if (h & 8) { cleanup(); return fail(PP_ERR_ARG, "an entry couples two systems (matrix not block diagonal)"); }
        if (h & 1) { cleanup(); return fail(PP_ERR_ARG, "Jacobi scaling needs a positive finite diagonal"); }

        // symmetric stored diagonals, chosen per system
        build_diagonals(op, rowptr, colind, val);

        // slice layout: the entries the stored diagonals do not cover
        width = dalloc<int64_t>(op->nslices);
        op->sp = dalloc<int64_t>(op->nslices + 1);
        const unsigned gs = (unsigned)((op->nslices + WPB - 1) / WPB);
        hipLaunchKernelGGL(ppb::kb_slice_width, dim3(gs), dim3(BLOCK), 0, op->stream, op->nslices,
                           (const int32_t *)op->slice_seg, (const int64_t *)op->seg_row0, (const int64_t *)op->seg_n,
                           (const int64_t *)op->ext_row0, rowptr, colind, (const int32_t *)op->seg_nd,
                           (const int64_t *)op->seg_off, width);
        hipLaunchKernelGGL(ppk::k_scan_slices, dim3(1), dim3(1024), 0, op->stream, op->nslices, (const int64_t *)width,
                           op->sp);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&op->nstored, op->sp + op->nslices, sizeof(int64_t), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        op->scol = dalloc<int32_t>(op->nstored);
        op->sval = dalloc<double>(op->nstored);
        if (op->mixed()) op->sval32 = dalloc<float>(op->nstored);
        hipLaunchKernelGGL(ppb::kb_slice_fill, dim3(gs), dim3(BLOCK), 0, op->stream, op->nslices,
                           (const int32_t *)op->slice_seg, (const int64_t *)op->seg_row0, (const int64_t *)op->seg_n,
                           (const int64_t *)op->ext_row0, rowptr, colind, val, (const int32_t *)op->seg_nd,
                           (const int64_t *)op->seg_off, (const double *)op->dis, (const int64_t *)op->sp, op->scol,
                           op->sval, op->sval32, (int)((op->flags & PP_JACOBI) != 0));
        HIPCHK(hipGetLastError());
        // systems with entries in the slice layout
        {
            std::vector<int64_t> spb(S + 1);
            for (int s = 0; s <= S; ++s)
                HIPCHK(hipMemcpyAsync(&spb[s], op->sp + op->seg_row0_h[s] / WAVE, sizeof(int64_t),
                                      hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            std::vector<int32_t> sell(S);
            for (int s = 0; s < S; ++s) sell[s] = spb[s + 1] > spb[s] ? 1 : 0;
            op->seg_sell = dalloc<int32_t>(S);
            HIPCHK(hipMemcpyAsync(op->seg_sell, sell.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
        }

        // vectors (zeroed: padding rows and columns stay zero for good)
        const size_t nv = (size_t)op->n_int * op->NB;
        auto zalloc64 = [&](double *&p) {
            p = dalloc<double>(nv);
            HIPCHK(hipMemsetAsync(p, 0, nv * sizeof(double), op->stream));
        };
        auto zalloc32 = [&](float *&p) {
            p = dalloc<float>(nv);
            HIPCHK(hipMemsetAsync(p, 0, nv * sizeof(float), op->stream));
        };
        zalloc64(op->Xh); zalloc64(op->R); zalloc64(op->P); zalloc64(op->Q); zalloc64(op->Z); zalloc64(op->Bh);
        if (op->mixed()) { zalloc32(op->R32); zalloc32(op->SA); zalloc32(op->SB); }
        else { zalloc64(op->SA64); zalloc64(op->SB64); }
        op->partials = dalloc<double>((size_t)op->G * op->NB);
        const size_t sn = (size_t)S * op->NB;
        op->d_rho = dalloc<double>(sn); op->d_alpha = dalloc<double>(sn); op->d_beta = dalloc<double>(sn);
        op->d_rr = dalloc<double>(sn); op->d_bn2 = dalloc<double>(sn); op->d_tol2 = dalloc<double>(sn);
        op->d_lz = dalloc<double>((size_t)S * (2 * ppk::LZ_MAX + 2));
        op->d_it = dalloc<int32_t>(sn); op->d_status = dalloc<int32_t>(sn); op->d_done = dalloc<int32_t>(sn);
        op->d_zero_b = dalloc<int32_t>(sn);
        op->d_seg_ndone = dalloc<int32_t>(S); op->d_seg_done = dalloc<int32_t>(S);
        op->d_ticket = dalloc<uint32_t>(S);
        op->d_ndone = dalloc<int32_t>(1);
        HIPCHK(hipMemsetAsync(op->d_ticket, 0, sizeof(uint32_t) * S, op->stream));
        HIPCHK(hipHostMalloc((void **)&op->h_ndone, 2 * sizeof(int32_t), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&op->h_segdone, 2 * sizeof(int32_t) * S, hipHostMallocDefault));
        HIPCHK(hipStreamSynchronize(op->stream));
        end_call(op);
    } catch (std::bad_alloc &) {
        cleanup();
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        cleanup();
        return hip_fail(e);
    }
    cleanup();
    return PP_OK;
}

// ---------------------------------------------------------------------------
// load balance: once systems finish, their workgroups would idle for the rest
// of the solve; the same G workgroups are redistributed over the systems
// still running, in proportion to their slices (blocks past the work get an
// empty range).  Only the map's contents change, so captured graphs stay valid.
// ---------------------------------------------------------------------------

void upload_map(pp_batch_s *op, const std::vector<int32_t> &seg, const std::vector<int64_t> &s0,
                const std::vector<int64_t> &s1, const std::vector<int32_t> &blk0)
{
    const int G = op->G, S = op->S;
    HIPCHK(hipMemcpyAsync(op->blk_seg, seg.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(op->blk_s0, s0.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(op->blk_s1, s1.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(op->seg_blk0, blk0.data(), sizeof(int32_t) * (S + 1), hipMemcpyHostToDevice, op->stream));
}

// New map over the systems with seg_done == 0; false when none is left.
bool rebalance(pp_batch_s *op, const std::vector<int32_t> &seg_done)
{
    const int G = op->G, S = op->S;
    std::vector<int64_t> sl(S, 0);
    int64_t total = 0;
    for (int s = 0; s < S; ++s)
        if (!seg_done[s]) {
            sl[s] = (op->seg_row0_h[s + 1] - op->seg_row0_h[s]) / WAVE;
            total += sl[s];
        }
    if (total == 0) return false;
    std::vector<int64_t> nb(S, 0);
    int64_t used = 0;
    for (int s = 0; s < S; ++s)
        if (sl[s] > 0) {
            nb[s] = std::max<int64_t>(1, std::min<int64_t>((int64_t)((double)G * sl[s] / total),
                                                           (sl[s] + WPB - 1) / WPB));
            used += nb[s];
        }
    while (used > G) {  // more systems than workgroups cannot happen (G >= S), trim the largest
        int big = 0;
        for (int s = 1; s < S; ++s)
            if (nb[s] > nb[big]) big = s;
        --nb[big];
        --used;
    }
    op->map_seg.assign(G, 0);
    op->map_s0.assign(G, 0);
    op->map_s1.assign(G, 0);
    op->map_blk0.assign(S + 1, 0);
    int last = -1;
    for (int s = 0; s < S; ++s)
        if (sl[s] > 0) last = s;
    int b = 0;
    for (int s = 0; s < S; ++s) {
        op->map_blk0[s] = b;
        const int64_t first = op->seg_row0_h[s] / WAVE;
        for (int64_t i = 0; i < nb[s]; ++i, ++b) {
            op->map_seg[b] = s;
            op->map_s0[b] = first + sl[s] * i / nb[s];
            op->map_s1[b] = first + sl[s] * (i + 1) / nb[s];
        }
        if (s == last)  // the spare blocks join the last running system with an empty range
            for (; b < G; ++b) {
                op->map_seg[b] = s;
                op->map_s0[b] = first + sl[s];
                op->map_s1[b] = first + sl[s];
            }
    }
    op->map_blk0[S] = G;
    upload_map(op, op->map_seg, op->map_s0, op->map_s1, op->map_blk0);
    op->remapped = true;
    return true;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------

// per-segment reduction of the previous kernel's partials
template <int NB>
void launch_fin(pp_batch_s *op, const ppb::BState &st, int fin, int idx = 0)
{
    if (fin == ppb::BF_NONE) return;
    hipLaunchKernelGGL((ppb::kb_fin<NB>), dim3(op->S), dim3(BLOCK), 0, op->stream, op->bt(), st,
                       (const double *)op->partials, fin, idx);
}

void launch_state_init(pp_batch_s *op, double tol, int maxit)
{
    const int m = std::max(op->S * op->NB, op->S);
    hipLaunchKernelGGL(ppb::kb_state_init, dim3((unsigned)((m + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, op->stream,
                       op->bst(tol, maxit), op->S, op->NB);
    hipLaunchKernelGGL(ppb::kb_pad_cols, dim3((unsigned)((op->S + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, op->stream,
                       op->bst(tol, maxit), op->S, op->NB, op->nrhs);
}

// Z = p_k(A-hat) R for all columns; fin = BF_RHO0 / BF_RHO (reduce R.Z)
template <int W, int CPL>
void poly(pp_batch_s *op, const ppb::BState &st, int fin)
{
    const dim3 g(op->G), b(BLOCK);
    const ppb::Batch bt = op->bt();
    const int k = op->k;
    if (k == 0) {
        hipLaunchKernelGGL((ppb::kb_deg0<W, CPL>), g, b, 0, op->stream, bt, st, op->view(false), (const double *)op->R,
                           op->Z, (const double *)op->thinv_d, op->partials, fin);
        launch_fin<W * CPL>(op, st, fin);
        return;
    }
    const bool nt = op->ntload != 0;
    if (!op->mixed()) {
        const ppk::SellView A = op->view(false);
        for (int j = 1; j <= k; ++j) {
            const bool last = (j == k);
            const double *X = j == 1 ? op->R : ((j % 2 == 0) ? op->SA64 : op->SB64);
            const double *old = (j % 2 == 0) ? op->SB64 : op->SA64;
            double *out = last ? op->Z : ((j % 2 == 1) ? op->SA64 : op->SB64);
#define KB64(MODE, LAST, NT)                                                                                           \
    hipLaunchKernelGGL((ppb::kb_cheb<double, double, double, W, CPL, MODE, LAST, NT>), g, b, 0, op->stream, bt, st, A, \
                       X, (const double *)op->R, old, out, (const double *)op->coef_d, j, op->partials, fin)
            const int mode = j == 1 ? 1 : (j == 2 ? 2 : 3);
            if (last) {
                if (mode == 1) { if (nt) KB64(1, true, true); else KB64(1, true, false); }
                else if (mode == 2) { if (nt) KB64(2, true, true); else KB64(2, true, false); }
                else { if (nt) KB64(3, true, true); else KB64(3, true, false); }
                launch_fin<W * CPL>(op, st, fin);
            } else {
                if (mode == 1) { if (nt) KB64(1, false, true); else KB64(1, false, false); }
                else if (mode == 2) { if (nt) KB64(2, false, true); else KB64(2, false, false); }
                else { if (nt) KB64(3, false, true); else KB64(3, false, false); }
            }
#undef KB64
        }
        return;
    }
    const ppk::SellView A = op->view(true);
    hipLaunchKernelGGL((ppb::kb_conv<W, CPL>), g, b, 0, op->stream, bt, st, A, (const double *)op->R, op->R32);
    for (int j = 1; j <= k; ++j) {
        const bool last = (j == k);
        const float *X = j == 1 ? op->R32 : ((j % 2 == 0) ? op->SA : op->SB);
        const float *old = (j % 2 == 0) ? op->SB : op->SA;
        float *out = (j % 2 == 1) ? op->SA : op->SB;
        const int mode = j == 1 ? 1 : (j == 2 ? 2 : 3);
#define KB32(MODE, NT)                                                                                                  \
    hipLaunchKernelGGL((ppb::kb_cheb<float, float, float, W, CPL, MODE, false, NT>), g, b, 0, op->stream, bt, st, A,    \
                       X, (const float *)op->R32, old, out, (const double *)op->coef_d, j, op->partials, fin)
#define KB32L(MODE, NT)                                                                                                 \
    hipLaunchKernelGGL((ppb::kb_cheb<float, double, double, W, CPL, MODE, true, NT>), g, b, 0, op->stream, bt, st, A,   \
                       X, (const double *)op->R, old, op->Z, (const double *)op->coef_d, j, op->partials, fin)
        if (last) {
            if (mode == 1) { if (nt) KB32L(1, true); else KB32L(1, false); }
            else if (mode == 2) { if (nt) KB32L(2, true); else KB32L(2, false); }
            else { if (nt) KB32L(3, true); else KB32L(3, false); }
            launch_fin<W * CPL>(op, st, fin);
        } else {
            if (mode == 1) { if (nt) KB32(1, true); else KB32(1, false); }
            else if (mode == 2) { if (nt) KB32(2, true); else KB32(2, false); }
            else { if (nt) KB32(3, true); else KB32(3, false); }
        }
#undef KB32
#undef KB32L
    }
}

template <int W, int CPL>
void iteration(pp_batch_s *op, const ppb::BState &st)
{
    const dim3 g(op->G), b(BLOCK);
    const ppb::Batch bt = op->bt();
    const ppk::SellView A = op->view(false);
    if (op->ntload)
        hipLaunchKernelGGL((ppb::kb_apply64<W, CPL, 1, true>), g, b, 0, op->stream, bt, st, A, (const double *)op->P,
                           (const double *)nullptr, op->Q, op->partials);
    else
        hipLaunchKernelGGL((ppb::kb_apply64<W, CPL, 1, false>), g, b, 0, op->stream, bt, st, A, (const double *)op->P,
                           (const double *)nullptr, op->Q, op->partials);
    launch_fin<W * CPL>(op, st, ppb::BF_GAMMA);
    hipLaunchKernelGGL((ppb::kb_xr<W, CPL>), g, b, 0, op->stream, bt, st, A, (const double *)op->P,
                       (const double *)op->Q, op->Xh, op->R, op->partials);
    launch_fin<W * CPL>(op, st, ppb::BF_RR);
    poly<W, CPL>(op, st, ppb::BF_RHO);
    hipLaunchKernelGGL((ppb::kb_p<W, CPL>), g, b, 0, op->stream, bt, st, A, (const double *)op->Z, op->P, 0);
}

void upload_coefficients(pp_batch_s *op)
{
    const int S = op->S, k = op->k;
    std::vector<double> coef((size_t)S * std::max(1, k) * 4, 0.0), thinv(S);
    for (int s = 0; s < S; ++s) {
        const double th = (op->lmax[s] + op->lmin[s]) / 2.0 * (1.0 + op->xi);
        const double de = (op->lmax[s] - op->lmin[s]) / 2.0;
        const double si = th / de;
        std::vector<double> rho(k + 1);
        rho[0] = 1.0 / si;
        for (int j = 1; j <= k; ++j) rho[j] = 1.0 / (2.0 * si - rho[j - 1]);
        thinv[s] = 1.0 / th;
        for (int j = 1; j <= k; ++j) {
            double *c = &coef[((size_t)s * k + (j - 1)) * 4];
            if (j == 1) {
                c[0] = 0; c[1] = 0; c[2] = 4.0 * rho[1] / de; c[3] = -2.0 * rho[1] / (de * th);
            } else if (j == 2) {
                c[0] = 2.0 * si * rho[2]; c[1] = 0; c[2] = 2.0 * rho[2] / de - rho[2] * rho[1] / th;
                c[3] = -2.0 * rho[2] / de;
            } else {
                c[0] = 2.0 * si * rho[j]; c[1] = -rho[j] * rho[j - 1]; c[2] = 2.0 * rho[j] / de; c[3] = -2.0 * rho[j] / de;
            }
        }
    }
    dfree(op->coef_d);
    dfree(op->thinv_d);
    op->coef_d = dalloc<double>(coef.size());
    op->thinv_d = dalloc<double>(S);
    HIPCHK(hipMemcpyAsync(op->coef_d, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(op->thinv_d, thinv.data(), sizeof(double) * S, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
}

}  // namespace

extern "C" {

pp_status pp_create_batch(pp_batch *out, int nsys, const int64_t *sys_ptr, int64_t nnz, const int64_t *rowptr,
                          const int32_t *colind, const double *val, int nrhs, unsigned flags, void *stream)
{
    if (!out) return fail(PP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nsys < 1 || !sys_ptr || nnz <= 0 || !rowptr || !colind || !val)
        return fail(PP_ERR_ARG, "nsys >= 1, nnz > 0 and non-NULL arrays required");
    if (nrhs < 1 || nrhs > ppb::NB_MAX) return fail(PP_ERR_ARG, "nrhs must be in [1, 32]");
    if (flags & ~(unsigned)(PP_JACOBI | PP_MIXED | PP_SLICED)) return fail(PP_ERR_ARG, "unknown flags");
    if (sys_ptr[0] != 0) return fail(PP_ERR_ARG, "sys_ptr[0] must be 0");
    for (int s = 0; s < nsys; ++s)
        if (sys_ptr[s + 1] <= sys_ptr[s]) return fail(PP_ERR_ARG, "sys_ptr must be strictly increasing");
    if (sys_ptr[nsys] > (int64_t)INT32_MAX - 1) return fail(PP_ERR_ARG, "n must be below 2^31");
    pp_batch_s *op = new (std::nothrow) pp_batch_s();
    if (!op) return fail(PP_ERR_OOM, "host allocation failed");
    op->S = nsys;
    op->nrhs = nrhs;
    op->NB = nrhs == 1 ? 1 : (nrhs <= 8 ? 8 : 32);
    op->W = op->NB;
    op->CPL = 1;
    op->flags = flags;
    op->ustream = (hipStream_t)stream;
    op->sys_ptr.assign(sys_ptr, sys_ptr + nsys + 1);
    op->n_ext = sys_ptr[nsys];
    op->nnz = nnz;
    (void)hipGetDevice(&op->device);
    pp_status s = build(op, rowptr, colind, val);
    if (s != PP_OK) {
        op->release();
        delete op;
        return s;
    }
    op->stats.n = op->n_ext;
    op->stats.nsys = nsys;
    op->stats.nb = op->NB;
    op->stats.nrhs = nrhs;
    op->stats.w = op->W;
    op->stats.nnz_stored = op->nstored;
    op->stats.grid = op->G;
    op->stats.diag_systems = op->diag_systems;
    *out = op;
    return PP_OK;
}

void pp_destroy_batch(pp_batch op)
{
    if (!op) return;
    (void)hipStreamSynchronize(op->stream);
    op->release();
    delete op;
}

pp_status pp_batch_set_option(pp_batch op, int key, int64_t value)
{
    if (!op) return fail(PP_ERR_ARG, "op is NULL");
    switch (key) {
    case PP_OPT_CHUNK:
        if (value < 0 || value > 256) return fail(PP_ERR_ARG, "chunk must be in [0, 256]");
        op->chunk = (int)value;
        return PP_OK;
    case PP_OPT_NT_LOADS: op->ntload = value != 0; op->g_k = -1; return PP_OK;
    case PP_BOPT_GRAPH: op->use_graph = value != 0; return PP_OK;
    case PP_BOPT_DRIVER:
        if (value < 0 || value > 1) return fail(PP_ERR_ARG, "PP_BOPT_DRIVER must be 0 or 1");
        op->driver = (int)value;
        return PP_OK;
    case PP_OPT_GRID:
        if (value < 0 || value > 8192) return fail(PP_ERR_ARG, "grid must be in [0, 8192]");
        op->pgrid = (int)value;
        return PP_OK;
    case PP_OPT_BARRIER:
        if (value < -1 || value > 2) return fail(PP_ERR_ARG, "PP_OPT_BARRIER must be -1, 0, 1 or 2");
        op->bar_mode = (int)value;
        return PP_OK;
    case PP_OPT_SPIN_LIMIT:
        if (value < 1 || value > (int64_t)1 << 31) return fail(PP_ERR_ARG, "PP_OPT_SPIN_LIMIT must be in [1, 2^31]");
        op->spin = (unsigned int)value;
        return PP_OK;
    case PP_OPT_VERIFY:
        if (value < -1 || value > 1) return fail(PP_ERR_ARG, "PP_OPT_VERIFY must be -1, 0 or 1");
        op->verify = (int)value;
        return PP_OK;
    default: return fail(PP_ERR_ARG, "unknown batch option");
    }
}

pp_status pp_batch_set_layout(pp_batch op, int w)
{
    if (!op) return fail(PP_ERR_ARG, "op is NULL");
    if (w == 0) w = op->NB;
    if (!layout_ok(op->NB, w)) return fail(PP_ERR_ARG, "unsupported lanes-per-row for this block width");
    op->W = w;
    op->CPL = op->NB / w;
    op->stats.w = w;
    return PP_OK;
}

pp_status pp_batch_get_stats(pp_batch op, pp_batch_stats *st)
{
    if (!op || !st) return fail(PP_ERR_ARG, "NULL argument");
    *st = op->stats;
    return PP_OK;
}

pp_status pp_batch_setup(pp_batch op, int k, const double *lambda_min, const double *lambda_max, double scaling)
{
    if (!op || !lambda_min || !lambda_max) return fail(PP_ERR_ARG, "NULL argument");
    if (k < 0 || k > 4096) return fail(PP_ERR_ARG, "degree k out of range [0, 4096]");
    if (!std::isfinite(scaling) || !(scaling >= 0.0)) return fail(PP_ERR_ARG, "scaling must be finite and >= 0");
    for (int s = 0; s < op->S; ++s)
        if (!std::isfinite(lambda_min[s]) || !std::isfinite(lambda_max[s]) || !(lambda_min[s] > 0.0) ||
            !(lambda_max[s] > lambda_min[s]))
            return fail(PP_ERR_ARG, "bounds must satisfy 0 < lambda_min < lambda_max (finite) for every system");
    try {
        op->k = k;
        op->xi = scaling;
        op->lmin.assign(lambda_min, lambda_min + op->S);
        op->lmax.assign(lambda_max, lambda_max + op->S);
        upload_coefficients(op);
        op->g_k = -1;  // re-capture the iteration graph
        op->setup_done = true;
    } catch (std::bad_alloc &) {
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_batch_estimate_bounds(pp_batch op, int steps, double *lambda_min, double *lambda_max)
{
    if (!op || !lambda_min || !lambda_max) return fail(PP_ERR_ARG, "NULL argument");
    if (steps < 1 || steps > ppk::LZ_MAX) return fail(PP_ERR_ARG, "steps must be in [1, 64]");
    try {
        begin_call(op);
        const dim3 g(op->G), b(BLOCK);
        const ppb::Batch bt = op->bt();
        const ppb::BState st = op->bst(0.0, 0);
        const ppk::SellView A = op->view(false);
        launch_state_init(op, 0.0, 0);
        double *v = op->P, *vprev = op->Q, *w = op->Z;
        hipLaunchKernelGGL(ppb::kb_lz_start, g, b, 0, op->stream, bt, st, A, v, op->partials);
        launch_fin<1>(op, st, ppb::BF_LZN);
        hipLaunchKernelGGL(ppb::kb_lz_vec, g, b, 0, op->stream, bt, st, A, v, vprev, (const double *)w, 0, 0);
        for (int j = 0; j < steps; ++j) {
            hipLaunchKernelGGL(ppb::kb_lz_step<0>, g, b, 0, op->stream, bt, st, A, (const double *)v,
                               (const double *)vprev, w, op->partials, j);
            launch_fin<1>(op, st, ppb::BF_LZA, j);
            hipLaunchKernelGGL(ppb::kb_lz_step<1>, g, b, 0, op->stream, bt, st, A, (const double *)v,
                               (const double *)vprev, w, op->partials, j);
            launch_fin<1>(op, st, ppb::BF_LZB, j);
            if (j + 1 < steps)
                hipLaunchKernelGGL(ppb::kb_lz_vec, g, b, 0, op->stream, bt, st, A, v, vprev, (const double *)w, 1, j);
        }
        HIPCHK(hipGetLastError());
        const size_t lzn = (size_t)op->S * (2 * ppk::LZ_MAX + 2);
        std::vector<double> lz(lzn);
        HIPCHK(hipMemcpyAsync(lz.data(), op->d_lz, sizeof(double) * lzn, hipMemcpyDeviceToHost, op->stream));
        // the Lanczos vectors used the CG buffers: restore their zero padding
        const size_t nv = (size_t)op->n_int * op->NB;
        HIPCHK(hipMemsetAsync(op->P, 0, nv * sizeof(double), op->stream));
        HIPCHK(hipMemsetAsync(op->Q, 0, nv * sizeof(double), op->stream));
        HIPCHK(hipMemsetAsync(op->Z, 0, nv * sizeof(double), op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        end_call(op);
        for (int s = 0; s < op->S; ++s) {
            const double *al = &lz[(size_t)s * (2 * ppk::LZ_MAX + 2)];
            const double *be = al + ppk::LZ_MAX;
            int m = steps;
            for (int j = 0; j < steps; ++j) {
                if (!std::isfinite(al[j]) || !std::isfinite(be[j]))
                    return fail(PP_ERR_ARG, "non-finite value in Lanczos");
                if (be[j] == 0.0) { m = j + 1; break; }
            }
            std::vector<double> T((size_t)m * m, 0.0), wv, V;
            for (int j = 0; j < m; ++j) {
                T[(size_t)j * m + j] = al[j];
                if (j + 1 < m) T[(size_t)j * m + j + 1] = T[(size_t)(j + 1) * m + j] = be[j];
            }
            ppeig::jacobi_eig(m, T, wv, V);
            int imin = 0, imax = 0;
            for (int i = 1; i < m; ++i) {
                if (wv[i] < wv[imin]) imin = i;
                if (wv[i] > wv[imax]) imax = i;
            }
            lambda_min[s] = wv[imin];
            lambda_max[s] = wv[imax] + std::fabs(be[m - 1] * V[(size_t)(m - 1) * m + imax]);
        }
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

namespace {

// One run of the batched CG loop from X (unscaled): scaled right-hand sides
// and iterates, the initial residuals and their test, the first polynomial,
// then chunks of iterations (a captured graph) until every column is done,
// and X = D^{-1/2} X-hat.  check_only: stop after the initial test when it
// ends every column (the true-residual check of a converged batch).
// The whole pass in one cooperative launch (ppb::kbp_solve).  Returns false,
// with nothing queued but the barrier reset, when the runtime refuses the
// cooperative grid; the caller then drives the pass from the host.
bool persistent_pass(pp_batch_s *op, const double *B, double *X, double tol, int maxit)
{
    // one right-hand side per system (internal block width 1) only: the
    // multi-column layouts, inlined into one kernel, would spill
    if (op->NB != 1 || op->W != 1 || op->CPL != 1) return false;
    const void *fn = op->mixed() ? (const void *)ppb::kbp_solve<1, 1, true> : (const void *)ppb::kbp_solve<1, 1, false>;
    int occ = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, BLOCK, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, op->device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    // all resident workgroups while a phase has work for them (a slice per
    // wave and more), else 256: the barrier's cost grows with the grid
    // (256 systems of sides 4..8: 0.97 ms on 256 workgroups, 1.10 ms on 363;
    // sides 8..24: 6.2 ms on 768, 8.6 ms on 256)
    int G = std::min(op->G, std::max(0, occ) * std::max(0, cus));
    G = (int)std::min<int64_t>(G, std::max<int64_t>(256, op->nslices / 8));
    if (op->pgrid > 0) G = std::min(G, op->pgrid);
    if (G < 1) return false;
    if (!op->bw) op->bw = dalloc<unsigned long long>((size_t)ppk::GB_LINES * ppk::GB_LINE);
    hipLaunchKernelGGL(ppk::k_zero_u64, dim3(1), dim3(BLOCK), 0, op->stream, op->bw,
                       (int64_t)ppk::GB_LINES * ppk::GB_LINE);
    ppb::BPArgs a;
    a.bt = op->bt();
    a.st = op->bst(tol, maxit);
    a.A = op->view(false);
    a.A32 = op->view(op->mixed());
    a.B = B;
    a.X = X;
    a.dis = op->dis;
    a.Bh = op->Bh; a.Xh = op->Xh; a.R = op->R; a.P = op->P; a.Q = op->Q; a.Z = op->Z;
    a.SA64 = op->SA64; a.SB64 = op->SB64;
    a.R32 = op->R32; a.SA = op->SA; a.SB = op->SB;
    a.partials = op->partials;
    a.coef = op->coef_d;
    a.thinv = op->thinv_d;
    a.nblk = op->G;
    a.k = op->k;
    a.maxit = maxit;
    a.total = op->S * op->NB;
    a.bw = op->bw;
    a.bar_mode = op->bar_mode >= 0 ? op->bar_mode : (G < 32 ? 1 : 2);
    a.spin = op->spin;
    void *args[] = {&a};
    if (hipLaunchCooperativeKernel(fn, dim3(G), dim3(BLOCK), args, 0, op->stream) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    HIPCHK(hipMemcpyAsync(&op->h_abort, op->bw + (size_t)ppk::GB_ABORT * ppk::GB_LINE, sizeof(op->h_abort),
                          hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    if (op->h_abort != 0) op->timed_out = true;
    op->stats.grid = G;
    op->stats.driver = 1;
    return true;
}

void batch_pass(pp_batch_s *op, const double *B, double *X, double tol, int maxit, bool check_only)
{
    if (op->driver == 1) {
        launch_state_init(op, tol, maxit);
        if (persistent_pass(op, B, X, tol, maxit)) return;
    }
    op->stats.grid = op->G;
    op->stats.driver = 0;
    const ppb::BState st = op->bst(tol, maxit);
    const ppb::Batch bt = op->bt();
    const dim3 g(op->G), b(BLOCK);
    launch_state_init(op, tol, maxit);
    const int total = op->S * op->NB;
    int chunk = op->chunk > 0 ? op->chunk : (op->n_int * (int64_t)op->NB >= (1 << 22) ? 2 : 8);
    with_layout(op->W, op->CPL, [&](auto wc, auto cc) {
        constexpr int W = decltype(wc)::value;
        constexpr int CPL = decltype(cc)::value;
        const ppk::SellView A = op->view(false);
        hipLaunchKernelGGL((ppb::kb_init_scale<W, CPL>), g, b, 0, op->stream, bt, st, A, B, (const double *)X,
                           (const double *)op->dis, op->Bh, op->Xh, op->partials);
        launch_fin<W * CPL>(op, st, ppb::BF_BNORM);
        hipLaunchKernelGGL((ppb::kb_apply64<W, CPL, 0, false>), g, b, 0, op->stream, bt, st, A,
                           (const double *)op->Xh, (const double *)op->Bh, op->R, op->partials);
        launch_fin<W * CPL>(op, st, ppb::BF_RR0);
        bool all_done = false;
        if (check_only) {
            HIPCHK(hipMemcpyAsync(&op->h_ndone[0], op->d_ndone, sizeof(int32_t), hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            all_done = op->h_ndone[0] >= total;
        }
        if (!all_done) {
            poly<W, CPL>(op, st, ppb::BF_RHO0);
            hipLaunchKernelGGL((ppb::kb_p<W, CPL>), g, b, 0, op->stream, bt, st, A, (const double *)op->Z, op->P, 1);
            HIPCHK(hipGetLastError());
            // one chunk of iterations, captured once and replayed
            const bool graph = op->use_graph != 0;
            if (graph && (op->g_k != op->k || op->g_chunk != chunk || op->g_tol != tol || op->g_maxit != maxit ||
                          op->g_W != op->W || !op->gexec)) {
                if (op->gexec) HIPCHK(hipGraphExecDestroy(op->gexec));
                op->gexec = nullptr;
                hipGraph_t gr;
                HIPCHK(hipStreamBeginCapture(op->stream, hipStreamCaptureModeThreadLocal));
                for (int i = 0; i < chunk; ++i) iteration<W, CPL>(op, st);
                HIPCHK(hipStreamEndCapture(op->stream, &gr));
                HIPCHK(hipGraphInstantiate(&op->gexec, gr, nullptr, nullptr, 0));
                HIPCHK(hipGraphDestroy(gr));
                op->g_k = op->k; op->g_chunk = chunk; op->g_tol = tol; op->g_maxit = maxit; op->g_W = op->W;
            }
            int enq = 0, c = 0, ndone_mapped = 0;
            const bool balance = op->S > 1;
            while (enq < maxit) {
                if (graph) HIPCHK(hipGraphLaunch(op->gexec, op->stream));
                else
                    for (int i = 0; i < chunk; ++i) iteration<W, CPL>(op, st);
                HIPCHK(hipGetLastError());
                enq += chunk;
                HIPCHK(hipMemcpyAsync(&op->h_ndone[c & 1], op->d_ndone, sizeof(int32_t), hipMemcpyDeviceToHost,
                                      op->stream));
                if (balance)
                    HIPCHK(hipMemcpyAsync(op->h_segdone + (size_t)(c & 1) * op->S, op->d_seg_done,
                                          sizeof(int32_t) * op->S, hipMemcpyDeviceToHost, op->stream));
                HIPCHK(hipEventRecord(op->flag_ev[c & 1], op->stream));
                if (c >= 1) {
                    HIPCHK(hipEventSynchronize(op->flag_ev[(c - 1) & 1]));
                    const int nd = op->h_ndone[(c - 1) & 1];
                    if (nd >= total) break;
                    if (balance && nd > ndone_mapped) {
                        // a system finished (as of chunk c-1): spread the idle workgroups
                        const int32_t *sd = op->h_segdone + (size_t)((c - 1) & 1) * op->S;
                        std::vector<int32_t> done(sd, sd + op->S);
                        if (done != op->seg_done_h) {
                            op->seg_done_h = done;
                            if (rebalance(op, done)) HIPCHK(hipStreamSynchronize(op->stream));
                        }
                        ndone_mapped = nd;
                    }
                }
                ++c;
            }
            if (op->remapped) {  // every system's rows again, for the final scaling and later calls
                upload_map(op, op->blk_seg_h, op->blk_s0_h, op->blk_s1_h, op->seg_blk0_h);
                HIPCHK(hipStreamSynchronize(op->stream));
                op->remapped = false;
            }
            op->seg_done_h.clear();
        }
        hipLaunchKernelGGL((ppb::kb_final<W, CPL>), g, b, 0, op->stream, bt, st, A, (const double *)op->Xh,
                           (const double *)op->dis, X);
        HIPCHK(hipGetLastError());
    });
}

}  // namespace

pp_status pcg_solve_batch(pp_batch op, const double *B, double *X, double tol, int maxit, int *iters, double *relres,
                          int *status)
{
    if (!op || !B || !X) return fail(PP_ERR_ARG, "NULL argument");
    if (B == X) return fail(PP_ERR_ARG, "B and X must not alias");
    if (!std::isfinite(tol) || tol < 0.0) return fail(PP_ERR_ARG, "tol must be finite and >= 0");
    if (maxit < 0) return fail(PP_ERR_ARG, "maxit must be >= 0");
    if (!op->setup_done) return fail(PP_ERR_STATE, "pp_batch_setup must be called before pcg_solve_batch");
    try {
        begin_call(op);
        op->timed_out = false;
        HIPCHK(hipEventRecord(op->solve_ev[0], op->stream));
        // true-residual check at convergence (default: mixed mode only)
        const bool verify = op->verify > 0 || (op->verify < 0 && op->mixed());
        const int total = op->S * op->NB;
        const size_t sn = (size_t)total;
        std::vector<int32_t> it(sn), stt(sn), zb(sn), it_sum(sn, 0);
        std::vector<double> rr(sn), bn(sn);
        int restarts = 0;
        bool verified = false;
        // Pass 0 is the solve.  When every column converged and the check is
        // on, pass 1 starts again from the iterates: its initial residuals are
        // the true residuals, and its initial test either ends every column at
        // once (the usual case) or CG continues from there (a restart, with the
        // iterations left to the column that used most); at most three restarts.
        for (int pass = 0;; ++pass) {
            int used = 0;
            for (size_t i = 0; i < sn; ++i) used = std::max(used, it_sum[i]);
            batch_pass(op, B, X, tol, maxit - used, pass > 0);
            HIPCHK(hipMemcpyAsync(it.data(), op->d_it, sizeof(int32_t) * sn, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipMemcpyAsync(stt.data(), op->d_status, sizeof(int32_t) * sn, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipMemcpyAsync(zb.data(), op->d_zero_b, sizeof(int32_t) * sn, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipMemcpyAsync(rr.data(), op->d_rr, sizeof(double) * sn, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipMemcpyAsync(bn.data(), op->d_bn2, sizeof(double) * sn, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            bool all_ok = true, iterated = false;
            for (int s = 0; s < op->S; ++s)
                for (int c = 0; c < op->nrhs; ++c) {
                    const size_t i = (size_t)s * op->NB + c;
                    it_sum[i] += it[i];
                    if (!zb[i] && stt[i] != PP_OK) all_ok = false;
                    if (!zb[i] && it[i] > 0) iterated = true;
                }
            if (op->timed_out) break;
            if (pass > 0 && !iterated) { verified = all_ok; break; }
            if (pass > 0) ++restarts;
            if (!(verify && all_ok && iterated && pass < 3)) break;
        }
        HIPCHK(hipEventRecord(op->solve_ev[1], op->stream));
        HIPCHK(hipEventSynchronize(op->solve_ev[1]));
        end_call(op);
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, op->solve_ev[0], op->solve_ev[1]));
        op->stats.solve_ms = ms;
        op->stats.graph = op->use_graph;
        op->stats.restarts = restarts;
        op->stats.verified = verified ? 1 : 0;
        pp_status worst = PP_OK;
        int maxits = 0;
        for (int s = 0; s < op->S; ++s)
            for (int c = 0; c < op->nrhs; ++c) {
                const size_t i = (size_t)s * op->NB + c, o = (size_t)s * op->nrhs + c;
                const pp_status sc = zb[i] ? PP_OK : (pp_status)stt[i];
                if (sc == PP_BREAKDOWN || (sc == PP_NOT_CONVERGED && worst == PP_OK)) worst = sc;
                maxits = std::max(maxits, it_sum[i]);
                if (iters) iters[o] = it_sum[i];
                if (status) status[o] = sc;
                if (relres) relres[o] = zb[i] ? 0.0 : (bn[i] > 0 ? std::sqrt(rr[i] / bn[i]) : 0.0);
            }
        op->stats.max_iters = maxits;
        if (op->timed_out)
            return fail(PP_ERR_TIMEOUT, "a grid-barrier wait of the persistent batched solve gave up (PP_OPT_SPIN_LIMIT)");
        return worst;
    } catch (std::bad_alloc &) {
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        return hip_fail(e);
    }
}

pp_status pp_batch_apply(pp_batch op, const double *Rin, double *Zout)
{
    if (!op || !Rin || !Zout) return fail(PP_ERR_ARG, "NULL argument");
    if (Rin == Zout) return fail(PP_ERR_ARG, "R and Z must not alias");
    if (!op->setup_done) return fail(PP_ERR_STATE, "pp_batch_setup must be called before pp_batch_apply");
    try {
        begin_call(op);
        const ppb::BState st = op->bst(0.0, 1);
        const ppb::Batch bt = op->bt();
        const dim3 g(op->G), b(BLOCK);
        launch_state_init(op, 0.0, 1);
        with_layout(op->W, op->CPL, [&](auto wc, auto cc) {
            constexpr int W = decltype(wc)::value;
            constexpr int CPL = decltype(cc)::value;
            const ppk::SellView A = op->view(false);
            // R = D^{-1/2} Rin in the internal layout (Bh holds it), polynomial, Z = D^{-1/2} z
            hipLaunchKernelGGL((ppb::kb_init_scale<W, CPL>), g, b, 0, op->stream, bt, st, A, Rin, Rin,
                               (const double *)op->dis, op->R, op->Xh, op->partials);
            launch_fin<W * CPL>(op, st, ppb::BF_BNORM);
            poly<W, CPL>(op, st, ppb::BF_NONE);
            hipLaunchKernelGGL((ppb::kb_final<W, CPL>), g, b, 0, op->stream, bt, st, A, (const double *)op->Z,
                               (const double *)op->dis, Zout);
        });
        HIPCHK(hipGetLastError());
        end_call(op);
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_batch_autotune(pp_batch op, int *best_w, double *best_us)
{
    if (!op || !best_w) return fail(PP_ERR_ARG, "NULL argument");
    if (!op->setup_done || op->k < 3) return fail(PP_ERR_STATE, "autotune needs pp_batch_setup with k >= 3");
    const int cands[5] = {op->NB, op->NB / 2, op->NB / 4, op->NB / 8, op->NB == 8 ? 1 : 0};
    double best = 1e300;
    int bw = op->W;
    try {
        begin_call(op);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const ppb::BState st = op->bst(0.0, 1);
        launch_state_init(op, 0.0, 1);
        for (int ci = 0; ci < 5; ++ci) {
            const int w = cands[ci];
            bool seen = false;
            for (int cj = 0; cj < ci; ++cj) seen = seen || cands[cj] == w;
            if (w < 1 || seen || !layout_ok(op->NB, w)) continue;
            const int cpl = op->NB / w;
            double us = 0;
            with_layout(w, cpl, [&](auto wc, auto cc) {
                constexpr int W = decltype(wc)::value;
                constexpr int CPL = decltype(cc)::value;
                const dim3 g(op->G), b(BLOCK);
                const ppb::Batch bt = op->bt();
                const bool f32 = op->mixed();
                const ppk::SellView A = op->view(f32);
                auto step = [&]() {
                    if (f32)
                        hipLaunchKernelGGL((ppb::kb_cheb<float, float, float, W, CPL, 3, false, true>), g, b, 0,
                                           op->stream, bt, st, A, (const float *)op->SA, (const float *)op->R32,
                                           (const float *)op->SB, op->SB, (const double *)op->coef_d, 3, op->partials, 0);
                    else
                        hipLaunchKernelGGL((ppb::kb_cheb<double, double, double, W, CPL, 3, false, true>), g, b, 0,
                                           op->stream, bt, st, A, (const double *)op->SA64, (const double *)op->R,
                                           (const double *)op->SB64, op->SB64, (const double *)op->coef_d, 3,
                                           op->partials, 0);
                };
                step();
                HIPCHK(hipEventRecord(e0, op->stream));
                for (int r = 0; r < 5; ++r) step();
                HIPCHK(hipEventRecord(e1, op->stream));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                us = 1000.0 * ms / 5;
            });
            if (us < best) {
                best = us;
                bw = w;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // the timing steps wrote the step buffers: restore zero padding
        const size_t nv = (size_t)op->n_int * op->NB;
        if (op->mixed()) HIPCHK(hipMemsetAsync(op->SB, 0, nv * sizeof(float), op->stream));
        else HIPCHK(hipMemsetAsync(op->SB64, 0, nv * sizeof(double), op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        end_call(op);
    } catch (HipError &e) {
        return hip_fail(e);
    }
    op->W = bw;
    op->CPL = op->NB / bw;
    op->stats.w = bw;
    *best_w = bw;
    if (best_us) *best_us = best;
    return PP_OK;
}

}  // extern "C"
