// C-ABI implementation of include/pp.h: polynomial-preconditioned CG on one
// MI355X.  Host code only queues the HIP kernels of kernels.hpp; every step
// of the solve runs on the device, and CG scalars never leave it until the
// solve ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <thread>
#include "../../include/pp.h"
#include "kernels.hpp"
#include "op.hpp"
#include "dia_plan.hpp"
#include "lowrank.hpp"
#include "persistent.hpp"
#include "reorder.hpp"
#include "stencil2.hpp"
#include "sym_eig.hpp"

using ppk::BLOCK;
using ppk::WAVE;
using ppk::WPB;

#include "common.hpp"

std::string &ppc::last_error()
{
    static thread_local std::string e;
    return e;
}

namespace {

using ppc::dalloc;
using ppc::dfree;
using ppc::fail;
using ppc::HipError;
using ppc::hip_fail;

constexpr int K_MAX = 4096;

}  // namespace



namespace {

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

// Host-side transpose of C (nt x n, given on the device) into per-cell lists
// (cell -> trace rows), sorted by trace row so that the appended entries have
// a fixed order.  C is small (two entries per trace row).
void build_ct(pp_op_s *op, const int64_t *c_rowptr, const int32_t *c_col, const double *c_val,
              int64_t **ctp_d, int32_t **ctt_d, double **ctv_d)
{
    const int64_t nt = op->nt, n = op->n, nnz = op->nnz_c;
    std::vector<int64_t> crp(nt + 1);
    std::vector<int32_t> ccol(nnz);
    std::vector<double> cval(nnz);
    HIPCHK(hipMemcpyAsync(crp.data(), c_rowptr, sizeof(int64_t) * (nt + 1), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(ccol.data(), c_col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(cval.data(), c_val, sizeof(double) * nnz, hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    std::vector<int64_t> ctp(n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) ctp[(size_t)ccol[p] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) ctp[i + 1] += ctp[i];
    std::vector<int64_t> fill(ctp.begin(), ctp.end() - 1);
    std::vector<int32_t> ctt(nnz);
    std::vector<double> ctv(nnz);
    for (int64_t t = 0; t < nt; ++t)  // ascending t -> each list sorted by trace row
        for (int64_t p = crp[t]; p < crp[t + 1]; ++p) {
            const int64_t o = fill[ccol[p]]++;
            ctt[o] = (int32_t)t;
            ctv[o] = cval[p];
        }
    *ctp_d = dalloc<int64_t>(n + 1);
    *ctt_d = dalloc<int32_t>(nnz);
    *ctv_d = dalloc<double>(nnz);
    HIPCHK(hipMemcpyAsync(*ctp_d, ctp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(*ctt_d, ctt.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(*ctv_d, ctv.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
}

int check_csr_dev(pp_op_s *op, int64_t rows, int64_t ncols, int64_t nnz, const int64_t *rp,
                  const int32_t *col, int *flag_d)
{
    HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
    const int64_t g = (rows + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(ppk::k_check_csr, dim3((unsigned)g), dim3(BLOCK), 0, op->stream, rows, ncols,
                       nnz, rp, col, flag_d);
    HIPCHK(hipGetLastError());
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, flag_d, sizeof(int), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    return h;
}

// Symmetric diagonal part of the operator (see SellView): histogram the
// column offsets of the nonzero entries, pick the offsets worth a stored
// diagonal (choose_diagonals), fill them, verify that the covered entries are
// exactly symmetric, then scale.  Explicit zeros are counted nowhere; the
// fill stores them as the zeros they are.  Returns the covered set; nd = 0
// when the matrix does not qualify (more than OFF_SLOTS distinct offsets, no
// dense diagonal, duplicate entries or asymmetric values): every entry then
// stays in the slice part.
ppk::DiaSet build_diagonals(pp_op_s *op, const int64_t *rp, const int32_t *col, const double *val)
{
    using ppk::OFF_SLOTS;
    typedef unsigned long long u64;
    ppk::DiaSet D;
    const int64_t n = op->n;
    struct Tmp {
        u64 *key = nullptr, *cnt = nullptr;
        int *flag = nullptr;
        ~Tmp() { dfree(key); dfree(cnt); dfree(flag); }
    } t;
    t.key = dalloc<u64>(OFF_SLOTS);
    t.cnt = dalloc<u64>(OFF_SLOTS);
    t.flag = dalloc<int>(1);
    std::vector<u64> hk(OFF_SLOTS, ppk::OFF_EMPTY), hc(OFF_SLOTS, 0);
    HIPCHK(hipMemcpyAsync(t.key, hk.data(), sizeof(u64) * OFF_SLOTS, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemsetAsync(t.cnt, 0, sizeof(u64) * OFF_SLOTS, op->stream));
    HIPCHK(hipMemsetAsync(t.flag, 0, sizeof(int), op->stream));
    const unsigned g = (unsigned)std::min<int64_t>(2048, (n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(ppk::k_offsets, dim3(g), dim3(BLOCK), 0, op->stream, n, (int64_t)0, rp, col, val, t.key,
                       t.cnt, t.flag);
    HIPCHK(hipGetLastError());
    int flag = 0;
    HIPCHK(hipMemcpyAsync(hk.data(), t.key, sizeof(u64) * OFF_SLOTS, hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(hc.data(), t.cnt, sizeof(u64) * OFF_SLOTS, hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(&flag, t.flag, sizeof(int), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    if (flag) return D;
    D = choose_diagonals(hk.data(), hc.data(), n);
    if (D.nd == 0) return D;

    const int64_t ds = op->nslices * WAVE;
    op->dval = dalloc<double>((size_t)D.nd * ds);
    HIPCHK(hipMemsetAsync(op->dval, 0, sizeof(double) * D.nd * ds, op->stream));
    HIPCHK(hipMemsetAsync(t.cnt, 0, 2 * sizeof(u64), op->stream));
    HIPCHK(hipMemsetAsync(t.flag, 0, sizeof(int), op->stream));
    const unsigned gr = (unsigned)((n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(ppk::k_dia_fill, dim3(gr), dim3(BLOCK), 0, op->stream, n, (int64_t)0, rp, col, val, D,
                       op->dval, ds, t.cnt, t.flag);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(ppk::k_dia_check, dim3(gr), dim3(BLOCK), 0, op->stream, n, (int64_t)0, rp, col, val, D,
                       (const double *)op->dval, ds, t.flag);
    HIPCHK(hipGetLastError());
    u64 ul[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(ul, t.cnt, 2 * sizeof(u64), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(&flag, t.flag, sizeof(int), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    if (flag || ul[0] != ul[1]) {
        dfree(op->dval);
        return ppk::DiaSet{};
    }
    if (op->mixed()) op->dval32 = dalloc<float>((size_t)D.nd * ds);
    if (op->dval32) HIPCHK(hipMemsetAsync(op->dval32, 0, sizeof(float) * D.nd * ds, op->stream));
    hipLaunchKernelGGL(ppk::k_dia_scale, dim3(gr), dim3(BLOCK), 0, op->stream, n, D, (const double *)op->dis,
                       op->dval, op->dval32, ds, op->kind == 0 ? 1 : 0);
    HIPCHK(hipGetLastError());
    op->nd = D.nd;
    op->dstride = ds;
    for (int d = 0; d < ppk::DMAX; ++d) op->doff[d] = D.off[d];
    return D;
}

// A CSR matrix that neither fits the stored diagonals nor numbers neighbouring
// rows close together (the gathers of a slice spread over many cache lines)
// is renumbered by reverse Cuthill-McKee when that brings the spread down at
// least twofold: op->perm (new -> old) is set and a renumbered device copy is
// returned in *prp, *pcol, *pval (the caller frees it).  Rows longer than 512
// entries (the device sort is quadratic in the row length) keep the order.
bool maybe_reorder(pp_op_s *op, const int64_t *rp, const int32_t *col, const double *val, int64_t **prp,
                   int32_t **pcol, double **pval)
{
    const int64_t n = op->n, nnz = op->nnz_given;
    std::vector<int64_t> hrp(n + 1);
    std::vector<int32_t> hcol(nnz);
    HIPCHK(hipMemcpyAsync(hrp.data(), rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(hcol.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    for (int64_t i = 0; i < n; ++i)
        if (hrp[i + 1] - hrp[i] > 512) return false;
    const std::vector<int64_t> none;
    const double s0 = pprc::gather_spread(n, hrp, hcol, none, none);
    op->spread[0] = op->spread[1] = s0;
    if (s0 <= 0.25) return false;
    const std::vector<int64_t> perm = pprc::rcm(n, hrp, hcol);
    std::vector<int64_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[perm[i]] = i;
    const double s1 = pprc::gather_spread(n, hrp, hcol, perm, iperm);
    if (!(s1 < 0.5 * s0)) return false;
    op->spread[1] = s1;
    std::vector<int64_t> nrp(n + 1, 0);
    std::vector<int32_t> p32(n), ip32(n);
    for (int64_t i = 0; i < n; ++i) {
        nrp[i + 1] = nrp[i] + (hrp[perm[i] + 1] - hrp[perm[i]]);
        p32[i] = (int32_t)perm[i];
        ip32[i] = (int32_t)iperm[i];
    }
    int32_t *ip = dalloc<int32_t>(n);
    struct Free {
        int32_t *&p;
        ~Free() { dfree(p); }
    } f{ip};
    op->perm = dalloc<int32_t>(n);
    *prp = dalloc<int64_t>(n + 1);
    *pcol = dalloc<int32_t>(nnz);
    *pval = dalloc<double>(nnz);
    HIPCHK(hipMemcpyAsync(op->perm, p32.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(ip, ip32.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(*prp, nrp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, op->stream));
    hipLaunchKernelGGL(ppk::k_perm_csr, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, op->stream, n, rp,
                       col, val, (const int32_t *)op->perm, (const int32_t *)ip, (const int64_t *)*prp, *pcol, *pval);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(op->stream));  // host vectors leave scope
    return true;
}

// LDS-staged x tiles (ltile.hpp) for a CSR operator held in slices only, FP64:
// per tile of LT_TS slices, the touched columns merged into segments (gaps
// up to LT_GAP bridged) and a 16-bit staging index per stored slot.  A tile
// that would stage more than LT_CAP values gathers from memory; lt_on stays 0
// when more than a tenth of the tiles would, or when the lanes of a slot row
// mostly read columns that are not consecutive: the staged reads then meet in
// LDS banks (measured: a renumbered irregular operator ran 15 % slower staged,
// the 7-point box in slices 6 % faster).  Tiles are planned on host threads.
void plan_ltiles(pp_op_s *op)
{
    using ppk::LT_TS;
    const int64_t ns = op->nslices, nst = op->nstored;
    if (ns == 0 || nst == 0) return;
    std::vector<int64_t> sp(ns + 1);
    std::vector<int32_t> col(nst);
    HIPCHK(hipMemcpyAsync(sp.data(), op->sp, sizeof(int64_t) * (ns + 1), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipMemcpyAsync(col.data(), op->scol, sizeof(int32_t) * nst, hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    const int64_t nt = (ns + LT_TS - 1) / LT_TS;
    std::vector<std::vector<int32_t>> seg(nt);  // per tile: (first column, length) pairs
    std::vector<uint16_t> lcol(nst);
    std::vector<int> caps(nt, 0);
    std::vector<int32_t> staged(nt, 1);
    const int nth = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<int64_t> consec(nth, 0);  // lanes whose column follows the previous lane's
    auto work = [&](int64_t ta, int64_t tb, int64_t *cons) {
        std::vector<int32_t> c;
        for (int64_t t = ta; t < tb; ++t) {
            const int64_t e0 = sp[t * LT_TS], e1 = sp[std::min(ns, (t + 1) * LT_TS)];
            for (int64_t e = e0 + 1; e < e1; ++e)
                if ((e & 63) != 0 && col[e] == col[e - 1] + 1) ++*cons;
            c.assign(col.begin() + e0, col.begin() + e1);
            std::sort(c.begin(), c.end());
            c.erase(std::unique(c.begin(), c.end()), c.end());
            std::vector<int32_t> &s = seg[t];
            int total = 0;
            for (size_t i = 0; i < c.size();) {
                size_t j = i;
                while (j + 1 < c.size() && c[j + 1] - c[j] <= ppk::LT_GAP) ++j;
                const int len = c[j] - c[i] + 1;
                s.push_back(c[i]);
                s.push_back(len);
                total += len;
                i = j + 1;
            }
            if (total > ppk::LT_CAP) {  // this tile gathers from memory
                staged[t] = 0;
                s.clear();
                continue;
            }
            caps[t] = total;
            // staging index of every slot: offset of its segment plus the column's place in it
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t cv = col[e];
                size_t lo = 0, hi = s.size() / 2;  // last segment starting at or before cv
                while (hi - lo > 1) {
                    const size_t mid = (lo + hi) / 2;
                    if (s[2 * mid] <= cv) lo = mid; else hi = mid;
                }
                int off = 0;
                for (size_t q = 0; q < lo; ++q) off += s[2 * q + 1];
                lcol[e] = (uint16_t)(off + (cv - s[2 * lo]));
            }
        }
    };
    std::vector<std::thread> pool;
    for (int k = 0; k < nth; ++k) pool.emplace_back(work, nt * k / nth, nt * (k + 1) / nth, &consec[k]);
    for (auto &th : pool) th.join();
    int64_t unstaged = 0, cons = 0;
    for (int32_t f : staged) unstaged += f == 0;
    for (int64_t v : consec) cons += v;
    if (10 * unstaged > nt || 2 * cons < nst * 63 / 64) return;
    std::vector<int32_t> seg_ptr(nt + 1, 0), seg_col, seg_lds, seg_len;
    for (int64_t t = 0; t < nt; ++t) {
        seg_ptr[t + 1] = seg_ptr[t] + (int32_t)(seg[t].size() / 2);
        int off = 0;
        for (size_t q = 0; q < seg[t].size(); q += 2) {
            seg_col.push_back(seg[t][q]);
            seg_lds.push_back(off);
            seg_len.push_back(seg[t][q + 1]);
            off += seg[t][q + 1];
        }
    }
    const int64_t nseg = (int64_t)seg_col.size();
    std::vector<int32_t> packed;
    packed.reserve(2 * nt + 1 + 3 * nseg);
    packed.insert(packed.end(), seg_ptr.begin(), seg_ptr.end());
    packed.insert(packed.end(), staged.begin(), staged.end());
    packed.insert(packed.end(), seg_col.begin(), seg_col.end());
    packed.insert(packed.end(), seg_lds.begin(), seg_lds.end());
    packed.insert(packed.end(), seg_len.begin(), seg_len.end());
    op->lt_seg = dalloc<int32_t>(packed.size());
    op->lt_lcol = dalloc<uint16_t>(nst);
    HIPCHK(hipMemcpyAsync(op->lt_seg, packed.data(), sizeof(int32_t) * packed.size(), hipMemcpyHostToDevice,
                          op->stream));
    HIPCHK(hipMemcpyAsync(op->lt_lcol, lcol.data(), sizeof(uint16_t) * nst, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    op->lt_ntiles = nt;
    op->lt_nseg = nseg;
    op->lt_cap = *std::max_element(caps.begin(), caps.end());
    op->lt_on = 1;
}

pp_status build_operator(pp_op_s *op, const int64_t *rp, const int32_t *col, const double *val,
                         const int64_t *c_rowptr, const int32_t *c_col, const double *c_val,
                         const double *m_diag)
{
    const int64_t n = op->n;
    int *flag_d = dalloc<int>(1);
    int64_t *ctp = nullptr;
    int32_t *ctt = nullptr;
    double *ctv = nullptr;
    int64_t *width = nullptr;
    double *dtmp = nullptr;
    int64_t *prp = nullptr;  // renumbered copy of A (maybe_reorder)
    int32_t *pcol = nullptr;
    double *pval = nullptr;
    auto cleanup = [&]() {
        dfree(flag_d); dfree(ctp); dfree(ctt); dfree(ctv); dfree(width); dfree(dtmp);
        dfree(prp); dfree(pcol); dfree(pval);
    };
    try {
        int bad = check_csr_dev(op, n, n, op->nnz_given, rp, col, flag_d);
        if (bad) { cleanup(); return fail(PP_ERR_ARG, "invalid CSR structure of A (row pointers or column indices)"); }
        if (op->schur()) {
            bad = check_csr_dev(op, op->nt, n, op->nnz_c, c_rowptr, c_col, flag_d);
            if (bad) { cleanup(); return fail(PP_ERR_ARG, "invalid CSR structure of C"); }
            // m > 0 check on host (nt is small)
            std::vector<double> mh(op->nt);
            HIPCHK(hipMemcpyAsync(mh.data(), m_diag, sizeof(double) * op->nt, hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            for (double v : mh)
                if (!(v > 0.0) || !std::isfinite(v)) { cleanup(); return fail(PP_ERR_ARG, "m_diag must be positive and finite"); }
            build_ct(op, c_rowptr, c_col, c_val, &ctp, &ctt, &ctv);
        }
        // Jacobi: d = diag(op), dis = d^{-1/2}
        if (op->flags & PP_JACOBI) {
            op->dis = dalloc<double>(n);
            dtmp = dalloc<double>(n);
            HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
            hipLaunchKernelGGL(ppk::k_diag, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                               op->stream, n, rp, col, val, ctp, ctt, ctv, m_diag, dtmp, op->dis, flag_d);
            HIPCHK(hipGetLastError());
            int h = 0;
            HIPCHK(hipMemcpyAsync(&h, flag_d, sizeof(int), hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            if (h) { cleanup(); return fail(PP_ERR_ARG, "Jacobi scaling needs a positive finite diagonal"); }
        }
        op->nslices = (n + WAVE - 1) / WAVE;
        // symmetric diagonal part (unless the caller asked for the slice layout only)
        ppk::DiaSet D;
        if (!(op->flags & PP_SLICED)) D = build_diagonals(op, rp, col, val);
        // slices only: renumber when the gathers of a slice are scattered
        if (op->kind == 0 && D.nd == 0 && !(op->flags & PP_NO_REORDER) &&
            maybe_reorder(op, rp, col, val, &prp, &pcol, &pval)) {
            rp = prp;
            col = pcol;
            val = pval;
            if (op->flags & PP_JACOBI) {
                hipLaunchKernelGGL(ppk::k_diag, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                                   op->stream, n, rp, col, val, (const int64_t *)nullptr, (const int32_t *)nullptr,
                                   (const double *)nullptr, m_diag, dtmp, op->dis, flag_d);
                HIPCHK(hipGetLastError());
            }
            if (!(op->flags & PP_SLICED)) D = build_diagonals(op, rp, col, val);
        }
        // slice part: the entries the diagonal part does not cover, plus trace columns
        width = dalloc<int64_t>(op->nslices);
        op->sp = dalloc<int64_t>(op->nslices + 1);
        const unsigned gs = (unsigned)((op->nslices + WPB - 1) / WPB);
        hipLaunchKernelGGL(ppk::k_slice_width, dim3(gs), dim3(BLOCK), 0, op->stream, n, op->nslices, rp, col, D,
                           (const int64_t *)ctp, width);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(ppk::k_scan_slices, dim3(1), dim3(1024), 0, op->stream, op->nslices,
                           (const int64_t *)width, op->sp);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&op->nstored, op->sp + op->nslices, sizeof(int64_t), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        op->sell = op->nstored > 0 ? 1 : 0;
        op->scol = dalloc<int32_t>(op->nstored);
        op->sval = dalloc<double>(op->nstored);
        if (op->mixed()) op->sval32 = dalloc<float>(op->nstored);
        hipLaunchKernelGGL(ppk::k_slice_fill, dim3(gs), dim3(BLOCK), 0, op->stream, n, op->nslices, n, rp,
                           col, val, D, (const int64_t *)ctp, (const int32_t *)ctt, (const double *)ctv,
                           (const double *)op->dis, (const int64_t *)op->sp, op->scol, op->sval,
                           op->sval32);
        HIPCHK(hipGetLastError());
        if (op->kind == 0 && op->nd == 0 && !op->mixed()) plan_ltiles(op);
        if (op->schur()) {
            const int64_t nt = op->nt;
            op->crp = dalloc<int64_t>(nt + 1);
            op->ccol = dalloc<int32_t>(op->nnz_c);
            op->cm = dalloc<double>(op->nnz_c);
            HIPCHK(hipMemcpyAsync(op->crp, c_rowptr, sizeof(int64_t) * (nt + 1), hipMemcpyDeviceToDevice, op->stream));
            HIPCHK(hipMemcpyAsync(op->ccol, c_col, sizeof(int32_t) * op->nnz_c, hipMemcpyDeviceToDevice, op->stream));
            if (op->mixed()) op->cm32 = dalloc<float>(op->nnz_c);
            hipLaunchKernelGGL(ppk::k_trace_fill, dim3((unsigned)((nt + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                               op->stream, nt, (const int64_t *)c_rowptr, c_col, c_val, m_diag,
                               (const double *)op->dis, op->cm, op->cm32);
            HIPCHK(hipGetLastError());
            op->tw = dalloc<double>(nt);
            if (op->mixed()) op->tw32 = dalloc<float>(nt);
        }
        // work vectors
        op->xh = dalloc<double>(n);
        op->r = dalloc<double>(n);
        op->p = dalloc<double>(n);
        op->q = dalloc<double>(n);
        op->z = dalloc<double>(n);
        op->bh = dalloc<double>(n);
        op->sA = dalloc<double>(n);
        op->sB = dalloc<double>(n);
        if (op->mixed()) {
            op->r32 = dalloc<float>(n);
            op->sA32 = dalloc<float>(n);
            op->sB32 = dalloc<float>(n);
        }
        op->partials = dalloc<double>((size_t)(1 + ppk::LR_MAX) * 8192);
        op->st = dalloc<ppk::State>(1);
        HIPCHK(hipMemsetAsync(op->st, 0, sizeof(ppk::State), op->stream));
        HIPCHK(hipHostMalloc((void **)&op->hst, sizeof(ppk::State), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&op->hflag, 2 * sizeof(int32_t), hipHostMallocDefault));
        for (auto &e : op->flag_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : op->solve_ev) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipStreamSynchronize(op->stream));
    } catch (std::bad_alloc &) {
        cleanup();
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        cleanup();
        char b[256];
        snprintf(b, sizeof b, "HIP error %s in %s (line %d)", hipGetErrorString(e.e), e.what, e.line);
        return fail(PP_ERR_HIP, b);
    }
    cleanup();
    op->stats.n = n;
    op->stats.nnz_stored = op->nstored;
    op->stats.diagonals = op->nd;
    op->stats.nnz_matrix = op->nnz_given + op->nnz_c;
    op->stats.reordered = op->perm ? 1 : 0;
    op->stats.lds_tiles = op->lt_on;
    op->stats.gather_spread = op->spread[1];
    return PP_OK;
}

pp_status create_common(pp_op *out, int kind, int64_t n, int64_t nnz, const int64_t *rp,
                        const int32_t *col, const double *val, int64_t nt, int64_t nnz_c,
                        const int64_t *c_rowptr, const int32_t *c_col, const double *c_val,
                        const double *m_diag, unsigned flags, void *stream)
{
    if (!out) return fail(PP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n <= 0 || nnz <= 0 || !rp || !col || !val) return fail(PP_ERR_ARG, "n, nnz must be positive and arrays non-NULL");
    if (n > (int64_t)INT32_MAX - 1) return fail(PP_ERR_ARG, "n must be below 2^31 (int32 column indices)");
    if (flags & ~(unsigned)(PP_JACOBI | PP_MIXED | PP_SLICED | PP_NO_REORDER)) return fail(PP_ERR_ARG, "unknown flags");
    if (kind == 1) {
        if (nt <= 0 || nnz_c <= 0 || !c_rowptr || !c_col || !c_val || !m_diag)
            return fail(PP_ERR_ARG, "Schur: nt, nnz_c must be positive and arrays non-NULL");
        if (n + nt > (int64_t)INT32_MAX - 1) return fail(PP_ERR_ARG, "n + nt must be below 2^31");
    }
    pp_op_s *op = new (std::nothrow) pp_op_s();
    if (!op) return fail(PP_ERR_OOM, "host allocation failed");
    op->kind = kind;
    op->n = n;
    op->nt = kind == 1 ? nt : 0;
    op->nnz_c = kind == 1 ? nnz_c : 0;
    op->nnz_given = nnz;
    op->flags = flags;
    op->stream = (hipStream_t)stream;
    (void)hipGetDevice(&op->device);
    pp_status s = build_operator(op, rp, col, val, c_rowptr, c_col, c_val, m_diag);
    if (s != PP_OK) {
        op->release();
        delete op;
        return s;
    }
    // one wave of resident workgroups for the streaming kernels: the fused
    // step holds ~70 VGPRs, which caps residency; a grid of exactly the
    // resident count avoids a tail of late workgroups
    int cus = 0, occ = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, op->device) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, (const void *)ppk::k_cheb<double, double, double, double, 3, false, false, false, true>, BLOCK,
            0) == hipSuccess &&
        cus > 0 && occ > 0) {
        op->cus = cus;
        op->grid_auto = std::min(8192, cus * occ);
        op->grid_max = op->grid_auto;
    }
    (void)hipGetLastError();
    // non-temporal streams pay only when a step's working set (about 64 bytes
    // per row in FP64) does not fit in the 256 MB Infinity Cache: below 2^22
    // rows the steps re-read matrix and vectors from it
    op->ntload = n >= (int64_t)1 << 22 ? 1 : 0;
    // 3-D 7-point shape (offsets 0, 1, N, N^2, n = N^2 NZ, no coupling across
    // the x- and y-faces): pairs of Chebyshev steps can share one pass
    if (op->nd == 4 && !op->sell && !op->schur() && op->doff[1] == 1 && op->doff[2] > 1 &&
        op->doff[2] <= ppk::S2_NMAX && op->doff[3] == op->doff[2] * op->doff[2] && n % op->doff[3] == 0) {
        try {
            int *bad = dalloc<int>(1);
            int h = 0;
            HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), op->stream));
            hipLaunchKernelGGL(ppk::k_s2_check, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, op->stream,
                               n, op->doff[2], (const double *)op->dval, op->dstride, bad);
            HIPCHK(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            dfree(bad);
            if (!h) {
                if (op->mixed()) {
                    op->sC32 = dalloc<float>(n);
                    op->sD32 = dalloc<float>(n);
                } else {
                    op->sC = dalloc<double>(n);
                    op->sD = dalloc<double>(n);
                }
                op->s2 = true;
                op->s2N = op->doff[2];
                op->s2NZ = n / op->doff[3];
            }
        } catch (...) {
            // the one-step kernels serve every operator: keep them
            op->s2 = false;
            (void)hipGetLastError();
        }
    }
    *out = op;
    return PP_OK;
}

// ---------------------------------------------------------------------------
// polynomial application (Algorithm 2), queued on the handle's stream
// ---------------------------------------------------------------------------

// reduce the G partials of the previous kernel into the CG state
void enqueue_fin(pp_op_s *op, int G, int fin, int idx = 0)
{
    hipLaunchKernelGGL(ppk::k_fin, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials, G, op->st, fin,
                       idx);
}

struct StepCoef {
    double cx, cold, cr, cA;
};

// coefficients of step j (1-based) in the form out = cx x + cold sold + cr r + cA (A x)
StepCoef step_coef(const pp_op_s *op, int j)
{
    const double th = op->theta, de = op->delta, si = op->sigma;
    const std::vector<double> &rho = op->rho;
    StepCoef c{0, 0, 0, 0};
    if (j == 1) {
        c.cr = 4.0 * rho[1] / de;
        c.cA = -2.0 * rho[1] / (de * th);
    } else if (j == 2) {
        c.cx = 2.0 * si * rho[2];
        c.cr = 2.0 * rho[2] / de - rho[2] * rho[1] / th;
        c.cA = -2.0 * rho[2] / de;
    } else {
        c.cx = 2.0 * si * rho[j];
        c.cold = -rho[j] * rho[j - 1];
        c.cr = 2.0 * rho[j] / de;
        c.cA = -2.0 * rho[j] / de;
    }
    return c;
}

template <typename T, typename XT, typename RT, typename OT, int MODE, bool SCHUR, bool DOT, bool SCALE>
void launch_cheb(pp_op_s *op, const XT *xg, const T *w, const RT *r, const T *sold, OT *out,
                 const StepCoef &c, int fin)
{
    const bool f32 = sizeof(T) == 4;
    if constexpr (sizeof(T) == 8 && sizeof(XT) == 8 && sizeof(RT) == 8 && sizeof(OT) == 8 && !SCHUR) {
        if (op->lt_on && op->lt_use) {
            // LDS-staged x tiles: one workgroup per tile range
            const int g = (int)std::max<int64_t>(1, std::min<int64_t>(op->lt_ntiles, op->grid_max));
            hipLaunchKernelGGL((ppk::k_cheb_lt<MODE, DOT, SCALE>), dim3(g), dim3(BLOCK),
                               sizeof(double) * (size_t)op->lt_cap, op->stream, op->view(false), op->ltview(),
                               (const double *)xg, (const double *)r, (const double *)sold, (double *)out, c.cx,
                               c.cold, c.cr, c.cA, (const double *)op->dis, op->partials, op->st);
            if (DOT && fin != ppk::FIN_NONE) enqueue_fin(op, g, fin);
            return;
        }
    }
    struct FinAfter {
        pp_op_s *op;
        int fin;
        ~FinAfter()
        {
            if (DOT && fin != ppk::FIN_NONE) enqueue_fin(op, op->grid_slices(), fin);
        }
    } after{op, fin};
#define PP_CHEB(NTV, UNITV)                                                                                    \
    hipLaunchKernelGGL((ppk::k_cheb<T, XT, RT, OT, MODE, SCHUR, DOT, SCALE, NTV, UNITV>), dim3(op->grid_slices()), \
                       dim3(BLOCK), 0, op->stream, op->view(f32), xg, w, r, sold, out, c.cx, c.cold, c.cr, c.cA,    \
                       (const double *)op->dis, op->partials, op->st, fin, 0)
    // Jacobi-scaled CSR operator with stored diagonals: the main one is exactly 1, not read
    if constexpr (!SCHUR) {
        if (op->dis != nullptr && op->kind == 0 && op->nd > 0) {
            if (op->ntload) PP_CHEB(true, true);
            else PP_CHEB(false, true);
            return;
        }
    }
    if (op->ntload) PP_CHEB(true, false);
    else PP_CHEB(false, false);
#undef PP_CHEB
}

template <typename T, typename XT, typename RT, typename OT, int MODE, bool SCHUR>
void launch_cheb_rt(pp_op_s *op, const XT *xg, const T *w, const RT *r, const T *sold, OT *out,
                    const StepCoef &c, int fin, bool scale)
{
    if (fin != ppk::FIN_NONE)
        launch_cheb<T, XT, RT, OT, MODE, SCHUR, true, false>(op, xg, w, r, sold, out, c, fin);
    else if (scale)
        launch_cheb<T, XT, RT, OT, MODE, SCHUR, false, true>(op, xg, w, r, sold, out, c, fin);
    else
        launch_cheb<T, XT, RT, OT, MODE, SCHUR, false, false>(op, xg, w, r, sold, out, c, fin);
}

// The fracture kernel for the smallest compiled band bound >= G.
void launch_frac(pp_op_s *op, const double *x, const double *s, const double *q, double *t, double *d,
                 const ppk::State *st)
{
    const ppk::DfnView g = op->dview();
    hipLaunchKernelGGL(ppk::k_dfn_cb, dim3(op->grid_elems(g.nh)), dim3(BLOCK), 0, op->stream, g, x, s, q, t, d, st);
    const size_t lds = sizeof(double) * 2 * (size_t)g.nf;
    const dim3 grid((unsigned)g.F), blk(ppk::DFN_WAVE);
#define PP_FRAC(GM, EX) hipLaunchKernelGGL((ppk::k_dfn_frac<GM, EX>), grid, blk, lds, op->stream, g, t, d, st)
    switch (g.G) {
    case 16: PP_FRAC(16, true); return;
    case 32: PP_FRAC(32, true); return;
    case 48: PP_FRAC(48, true); return;
    case 64: PP_FRAC(64, true); return;
    default: break;
    }
    if (g.G < 16)
        PP_FRAC(16, false);
    else if (g.G < 32)
        PP_FRAC(32, false);
    else if (g.G < 48)
        PP_FRAC(48, false);
    else
        PP_FRAC(64, false);
#undef PP_FRAC
}

// y = D^{-1/2} S_u D^{-1/2} x by Algorithm 3 (DFN): the fracture kernels
// (its three solves with A as two), then the rows of the unknowns.
// live_state: skip once the solve is done.
void enqueue_su(pp_op_s *op, const double *x, double *y, bool live_state)
{
    const ppk::DfnView g = op->dview();
    const ppk::State *st = live_state ? (const ppk::State *)op->st : nullptr;
    launch_frac(op, x, (const double *)op->dis, (const double *)nullptr, op->dfn_t, op->dfn_d, st);
    hipLaunchKernelGGL(ppk::k_dfn_urow, dim3(op->grid_elems(op->n)), dim3(BLOCK), 0, op->stream, g, x,
                       (const double *)op->dis, (const double *)op->dfn_t, (const double *)op->dfn_d, 1.0, -1.0,
                       -1.0, y, st);
}

template <typename T, typename XT, typename RT, typename OT, int MODE>
void launch_step(pp_op_s *op, const XT *xg, const RT *r, const T *sold, OT *out, const StepCoef &c,
                 int fin, bool scale)
{
    if (op->dfn()) {
        // FP64 only (no mixed mode): tw = S-hat x by Algorithm 3, read through the unit entries
        if constexpr (sizeof(T) == 8 && sizeof(XT) == 8) {
            enqueue_su(op, (const double *)xg, op->tw, true);
            launch_cheb_rt<T, XT, RT, OT, MODE, true>(op, xg, (const T *)op->tw, r, sold, out, c, fin, scale);
        }
    } else if (op->schur()) {
        T *w = sizeof(T) == 4 ? (T *)op->tw32 : (T *)op->tw;
        hipLaunchKernelGGL((ppk::k_trace<T, XT>), dim3(op->grid_elems(op->nt)), dim3(BLOCK), 0, op->stream,
                           op->cview(sizeof(T) == 4), xg, w, (const ppk::State *)op->st);
        launch_cheb_rt<T, XT, RT, OT, MODE, true>(op, xg, w, r, sold, out, c, fin, scale);
    } else {
        launch_cheb_rt<T, XT, RT, OT, MODE, false>(op, xg, (const T *)nullptr, r, sold, out, c, fin, scale);
    }
}

// Algorithm 1 (Newton form), FP64:  out = alpha P_j(in) + beta extra, with
// P_0 v = zeta_0 v and P_j v = zeta_j (2 P_{j-1} v - P_{j-1} A P_{j-1} v).
// Every operator application is one fused step; level j >= 2 keeps
// u = P_{j-1}(in) and A u in its own two work vectors, so the recursion holds
// 2 nlev vectors at most.  P_1 v = zeta_1 zeta_0 (2 v - zeta_0 A v) is a
// single fused step, and the outer combination of every level is folded into
// the last step of its second sub-call (extra term).
void newton_level(pp_op_s *op, int j, const double *in, double *out, double alpha, const double *extra,
                  double beta)
{
    const double *zt = op->zeta.data();
    if (j == 1) {
        StepCoef c{0, 0, 0, 0};
        c.cA = -zt[1] * zt[0] * zt[0] * alpha;
        if (extra) {
            c.cx = 2.0 * zt[1] * zt[0] * alpha;
            c.cr = beta;
            launch_step<double, double, double, double, 2>(op, in, extra, (const double *)nullptr, out, c,
                                                           ppk::FIN_NONE, false);
        } else {
            c.cr = 2.0 * zt[1] * zt[0] * alpha;
            launch_step<double, double, double, double, 1>(op, in, in, (const double *)nullptr, out, c,
                                                           ppk::FIN_NONE, false);
        }
        return;
    }
    const int64_t n = op->n;
    double *U = op->nbuf + (size_t)(2 * (j - 2)) * n, *AU = U + n;  // this level's vectors (j >= 2)
    newton_level(op, j - 1, in, U, 1.0, nullptr, 0.0);
    StepCoef c{0, 0, 0, 1.0};  // AU = A U
    launch_step<double, double, double, double, 1>(op, U, U, (const double *)nullptr, AU, c, ppk::FIN_NONE, false);
    // out = alpha zeta_j (2 U - P_{j-1}(AU)) + beta extra
    const double a2 = 2.0 * alpha * zt[j];
    if (extra) {
        hipLaunchKernelGGL(ppk::k_lin2, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n, a2, (const double *)U,
                           beta, extra, U);
        newton_level(op, j - 1, AU, out, -alpha * zt[j], U, 1.0);
    } else {
        newton_level(op, j - 1, AU, out, -alpha * zt[j], U, a2);
    }
}

void enqueue_newton(pp_op_s *op, const double *rr, double *zout, int fin, bool scale)
{
    const int64_t n = op->n;
    const int ge = op->grid_elems(n);
    if (op->nlev == 0)
        hipLaunchKernelGGL(ppk::k_lin2, dim3(ge), dim3(BLOCK), 0, op->stream, n, op->zeta[0], rr, 0.0,
                           (const double *)nullptr, zout);
    else
        newton_level(op, op->nlev, rr, zout, 1.0, nullptr, 0.0);
    if (scale)
        hipLaunchKernelGGL((ppk::k_scale<double, double>), dim3(ge), dim3(BLOCK), 0, op->stream, n,
                           (const double *)zout, (const double *)op->dis, 1.0, zout);
    if (fin != ppk::FIN_NONE) {
        hipLaunchKernelGGL(ppk::k_dot_fin, dim3(ge), dim3(BLOCK), 0, op->stream, n, rr, (const double *)zout,
                           op->partials, op->st, fin);
        enqueue_fin(op, ge, fin);
    }
}

// Steps j and j+1 (both three-term steps) in one pass of k_cheb2_stencil.
// Tiles of a pair launch: y-tiles of S2_TY lines; z-chunks of 32 planes, or
// 16.  A pair workgroup holds a whole CU, so the chunk is taken only if the
// tiles fill whole rounds of CUs at least 90 % (256^3: 256 tiles of 32
// planes); zc = 0 when none does (the one-step kernels are then faster:
// 160^3 and 192^3 measured 25-30 % slower with a part-filled last round, and
// 128^3 on 8-plane chunks, whose recomputed halo planes add a quarter, 7-10 %
// slower with full rounds).  Forced pairs (PP_OPT_TWO_STEP = 2) take 32.
ppk::Stencil2 pair_shape(const pp_op_s *op)
{
    ppk::Stencil2 g;
    g.N = op->s2N;
    g.NZ = op->s2NZ;
    g.n = op->n;
    g.nty = (int)((g.N + ppk::S2_TY - 1) / ppk::S2_TY);
    g.zc = 0;
    const int64_t cus = op->cus;
    for (int zc = ppk::S2_ZC_MAX; zc >= 16; zc /= 2) {
        const int64_t nwg = (int64_t)g.nty * ((g.NZ + zc - 1) / zc);
        const int64_t rounds = (nwg + cus - 1) / cus;
        if (nwg >= cus && 10 * nwg >= 9 * rounds * cus) {
            g.zc = zc;
            break;
        }
    }
    if (g.zc == 0 && op->two_step == 2) g.zc = ppk::S2_ZC_MAX;
    g.nzc = g.zc > 0 ? (int)((g.NZ + g.zc - 1) / g.zc) : 0;
    return g;
}

// Fused pairs of Chebyshev steps for this polynomial (three-term form, FP64,
// a 3-D 7-point box large enough, or forced)
bool use_pairs(const pp_op_s *op)
{
    return op->s2 && op->two_step != 0 && op->form == 0 && pair_shape(op).zc > 0;
}

template <typename T, typename O2 = T>
void launch_pair(pp_op_s *op, const T *sm1, const T *sm2, const T *r, T *o1, O2 *o2, const StepCoef &c1,
                 const StepCoef &c2, bool dot, const double *r64 = nullptr)
{
    const ppk::Stencil2 g = pair_shape(op);
    const dim3 grid((unsigned)(g.nty * g.nzc));
    const T *dv = sizeof(T) == 4 ? (const T *)op->dval32 : (const T *)op->dval;
    const size_t lds = sizeof(T) * (2 * ppk::S2_RY + (ppk::S2_SL ? 2 * (ppk::S2_RY + 2) : 0)) * (size_t)g.N;
    const ppk::State *st = (const ppk::State *)op->st;
#define PP_PAIR(NTV, DOTV, UNITV)                                                                                   \
    hipLaunchKernelGGL((ppk::k_cheb2_stencil<T, NTV, ppk::S2_BS, ppk::S2_SL, DOTV, UNITV, O2>), grid,              \
                       dim3(ppk::S2_BS), lds, op->stream, g, dv, op->dstride, sm1, sm2, r, r64, o1, o2, c1.cx,      \
                       c1.cold, c1.cr, c1.cA, c2.cx, c2.cold, c2.cr, c2.cA, st, op->partials)
#define PP_PAIR_U(NTV, DOTV)                  \
    do {                                      \
        if (unit) PP_PAIR(NTV, DOTV, true);   \
        else PP_PAIR(NTV, DOTV, false);       \
    } while (0)
    // Jacobi scaling: the stored main diagonal is exactly 1 (k_dia_scale), not read
    const bool unit = op->dis != nullptr && op->kind == 0;
    if (op->ntload) {
        if (dot) PP_PAIR_U(true, true);
        else PP_PAIR_U(true, false);
    } else {
        if (dot) PP_PAIR_U(false, true);
        else PP_PAIR_U(false, false);
    }
#undef PP_PAIR_U
#undef PP_PAIR
}

// workgroups of a pair launch (the partials it writes when it ends the polynomial)
int pair_grid(const pp_op_s *op)
{
    const ppk::Stencil2 g = pair_shape(op);
    return g.nty * g.nzc;
}

hipEvent_t pair_event(pp_op_s *op)
{
    if (op->pev_i == op->pev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        op->pev.push_back(e);
    }
    return op->pev[op->pev_i++];
}

// p_k(A-hat) rr with pairs of Chebyshev steps fused (3-D 7-point operators,
// k >= 4): steps (1, 2), (3, 4), ...; step 1 reads r in place of s_{j-1}
// (its coefficients of s_{j-1} and s_{j-2} are zero, as is step 2's of
// s_{j-2}).  When k is even and the output is not scaled, the last pair
// writes zout and reduces rr . zout; otherwise the remaining step(s) run
// alone, the last one with the reduction / scaling.  T: double.  Four step
// buffers rotate: a pair writes s_j and s_{j+1} to two that hold neither input.
template <typename T>
void enqueue_poly_pairs(pp_op_s *op, const double *rr, const T *rT, T *const (&buf)[4], double *zout, int fin,
                        bool scale)
{
    const int k = op->k;
    // the last pair writes z in FP64 (in mixed mode its second step reads r in
    // FP64 for the dot product); partials hold 8192 per column
    const bool last_pair = !scale && k % 2 == 0 && pair_grid(op) <= 8192;
    int ic = -1, io = -1;  // buffers of s_{j-1} and s_{j-2} (-1: r)
    int j = 1;
    const bool timed = op->time_pairs;
    if (timed) HIPCHK(hipEventRecord(pair_event(op), op->stream));
    int pairs = 0;
    while (j + 1 <= k - 1 || (j + 1 == k && last_pair)) {
        const bool ends = j + 1 == k;
        int a = -1, b = -1;
        for (int q = 0; q < 4; ++q)
            if (q != ic && q != io) (a < 0 ? a : b) = q;
        const T *sm1 = ic < 0 ? rT : buf[ic], *sm2 = io < 0 ? rT : buf[io];
        if (!ends)
            launch_pair<T>(op, sm1, sm2, rT, buf[a], buf[b], step_coef(op, j), step_coef(op, j + 1), false);
        else
            launch_pair<T, double>(op, sm1, sm2, rT, buf[a], zout, step_coef(op, j), step_coef(op, j + 1),
                                   fin != ppk::FIN_NONE, sizeof(T) == 8 ? nullptr : rr);
        ++pairs;
        io = a;
        ic = b;
        j += 2;
    }
    if (timed) {
        op->pairs_per_poly = pairs;
        HIPCHK(hipEventRecord(pair_event(op), op->stream));
    }
    if (j > k) {  // the last pair ended the polynomial
        if (fin != ppk::FIN_NONE) enqueue_fin(op, pair_grid(op), fin);
        return;
    }
    if (j <= k - 1) {  // one three-term step left before the last: in place over s_{j-2}
        launch_step<T, T, T, T, 3>(op, buf[ic], rT, buf[io], buf[io], step_coef(op, j), ppk::FIN_NONE, false);
        std::swap(ic, io);
        ++j;
    }
    launch_step<T, T, double, double, 3>(op, buf[ic], rr, buf[io], zout, step_coef(op, k), fin, scale);
}

// z = p_k(A-hat) rr, rr in the scaled space (double).  fin: FIN_NONE,
// FIN_RHO0 or FIN_RHO (reduce rr.z).  scale: multiply the output by dis
// (pp_apply under Jacobi).  r32src: FP32 copy of rr already made (mixed).
void enqueue_poly(pp_op_s *op, const double *rr, double *zout, int fin, bool scale, bool r32_ready = false)
{
    if (op->form == 1) {
        enqueue_newton(op, rr, zout, fin, scale);
        return;
    }
    const int k = op->k;
    if (k >= 4 && use_pairs(op) && !op->mixed()) {
        double *const buf[4] = {op->sA, op->sB, op->sC, op->sD};
        enqueue_poly_pairs<double>(op, rr, rr, buf, zout, fin, scale);
        return;
    }
    if (k == 0) {
        // z = rr / theta (and the dot when requested)
        hipLaunchKernelGGL((ppk::k_scale<double, double>), dim3(op->grid_elems(op->n)), dim3(BLOCK), 0,
                           op->stream, op->n, rr, (const double *)(scale ? op->dis : nullptr), 1.0 / op->theta,
                           zout);
        if (fin != ppk::FIN_NONE) {
            hipLaunchKernelGGL(ppk::k_dot_fin, dim3(op->grid_elems(op->n)), dim3(BLOCK), 0, op->stream, op->n,
                               rr, (const double *)zout, op->partials, op->st, fin);
            enqueue_fin(op, op->grid_elems(op->n), fin);
        }
        return;
    }
    if (!op->mixed()) {
        for (int j = 1; j <= k; ++j) {
            const StepCoef c = step_coef(op, j);
            const bool last = (j == k);
            const int f = last ? fin : ppk::FIN_NONE;
            const bool sc = last && scale;
            double *out = last ? zout : ((j % 2 == 1) ? op->sA : op->sB);
            if (j == 1) {
                launch_step<double, double, double, double, 1>(op, rr, rr, (const double *)nullptr, out, c, f, sc);
            } else if (j == 2) {
                launch_step<double, double, double, double, 2>(op, op->sA, rr, (const double *)nullptr, out, c, f, sc);
            } else {
                // s_{j-1} in the buffer written by step j-1, s_{j-2} in the other
                const double *prev = (j % 2 == 0) ? op->sA : op->sB;
                const double *old = (j % 2 == 0) ? op->sB : op->sA;
                launch_step<double, double, double, double, 3>(op, prev, rr, old, out, c, f, sc);
            }
        }
        return;
    }
    // mixed: r32 = (float) rr (unless the r update wrote it), steps in FP32,
    // last step writes FP64 z
    if (!r32_ready)
        hipLaunchKernelGGL((ppk::k_scale<double, float>), dim3(op->grid_elems(op->n)), dim3(BLOCK), 0, op->stream,
                           op->n, rr, (const double *)nullptr, 1.0, op->r32);
    if (k >= 4 && use_pairs(op)) {
        float *const buf[4] = {op->sA32, op->sB32, op->sC32, op->sD32};
        enqueue_poly_pairs<float>(op, rr, op->r32, buf, zout, fin, scale);
        return;
    }
    for (int j = 1; j <= k; ++j) {
        const StepCoef c = step_coef(op, j);
        const bool last = (j == k);
        const int f = last ? fin : ppk::FIN_NONE;
        const bool sc = last && scale;
        float *out32 = (j % 2 == 1) ? op->sA32 : op->sB32;
        if (!last) {
            if (j == 1)
                launch_step<float, float, float, float, 1>(op, op->r32, op->r32, (const float *)nullptr, out32, c, f, sc);
            else if (j == 2)
                launch_step<float, float, float, float, 2>(op, op->sA32, op->r32, (const float *)nullptr, out32, c, f, sc);
            else {
                const float *prev = (j % 2 == 0) ? op->sA32 : op->sB32;
                const float *old = (j % 2 == 0) ? op->sB32 : op->sA32;
                launch_step<float, float, float, float, 3>(op, prev, op->r32, old, out32, c, f, sc);
            }
        } else {
            // last step: r read in FP64 (for the CG dot), output FP64
            if (j == 1)
                launch_step<float, float, double, double, 1>(op, op->r32, rr, (const float *)nullptr, zout, c, f, sc);
            else if (j == 2)
                launch_step<float, float, double, double, 2>(op, op->sA32, rr, (const float *)nullptr, zout, c, f, sc);
            else {
                const float *prev = (j % 2 == 0) ? op->sA32 : op->sB32;
                const float *old = (j % 2 == 0) ? op->sB32 : op->sA32;
                launch_step<float, float, double, double, 3>(op, prev, rr, old, zout, c, f, sc);
            }
        }
    }
}

}  // namespace

namespace {

// w = M^{-1} C-hat x (Schur only).  live_state: skip once the solve is done.
void enqueue_trace_f64(pp_op_s *op, const double *x, bool live_state = true)
{
    if (!op->schur()) return;
    if (op->dfn()) {
        enqueue_su(op, x, op->tw, live_state);
        return;
    }
    hipLaunchKernelGGL((ppk::k_trace<double, double>), dim3(op->grid_elems(op->nt)), dim3(BLOCK), 0, op->stream,
                       op->cview(false), x, op->tw, (const ppk::State *)(live_state ? op->st : nullptr));
}

// p = z (+ V y) + beta p
void enqueue_p(pp_op_s *op, bool first)
{
    const int ge = op->grid_elems(op->n);
    if (op->lr_p > 0)
        hipLaunchKernelGGL(ppk::k_p_lr, dim3(ge), dim3(BLOCK), 0, op->stream, op->n, op->lr_p,
                           (const double *)op->lr_v, op->n, (const double *)op->z, op->p, (const ppk::State *)op->st,
                           first ? 1 : 0);
    else
        hipLaunchKernelGGL(ppk::k_p, dim3(ge), dim3(BLOCK), 0, op->stream, op->n, (const double *)op->z, op->p,
                           (const ppk::State *)op->st, first ? 1 : 0);
}

// c = V^T (s .* r) and y = Hinv c into the state (s = scale or 1)
void enqueue_lr_c(pp_op_s *op, const double *r, const double *scale)
{
    const int ge = op->grid_elems(op->n), lp = op->lr_p;
    hipLaunchKernelGGL(ppk::k_lr_dots, dim3(ge), dim3(BLOCK), 0, op->stream, op->n, lp, (const double *)op->lr_v,
                       op->n, r, scale, op->partials, (const ppk::State *)op->st);
    hipLaunchKernelGGL(ppk::k_fin_lr, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials, ge, lp,
                       op->st, (int)ppk::LR_FIN_C, lp, (const double *)op->lr_hinv);
}

void enqueue_iteration(pp_op_s *op, hipEvent_t e0, hipEvent_t e1)
{
    const int gs = op->grid_slices(), ge = op->grid_elems(op->n);
    enqueue_trace_f64(op, op->p);
    if (op->schur())
        hipLaunchKernelGGL(ppk::k_pq<true>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false), op->p,
                           (const double *)op->tw, op->q, op->partials, op->st, op->ntload);
    else if (op->dis != nullptr && op->kind == 0 && op->nd > 0)  // unit main diagonal (k_dia_scale): not read
        hipLaunchKernelGGL((ppk::k_pq<false, true>), dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false), op->p,
                           (const double *)nullptr, op->q, op->partials, op->st, op->ntload);
    else
        hipLaunchKernelGGL(ppk::k_pq<false>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false), op->p,
                           (const double *)nullptr, op->q, op->partials, op->st, op->ntload);
    enqueue_fin(op, gs, ppk::FIN_GAMMA);
    const int lp = op->lr_p;
    if (lp > 0) {
        // r update with c = V^T r in the same pass; y = Hinv c in the finaliser
        hipLaunchKernelGGL(ppk::k_xr_lr, dim3(ge), dim3(BLOCK), 0, op->stream, op->n, lp, (const double *)op->lr_v,
                           op->n, (const double *)op->p, (const double *)op->q, op->xh, op->r, op->partials, op->st);
        hipLaunchKernelGGL(ppk::k_fin_lr, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials, ge,
                           1 + lp, op->st, (int)ppk::LR_FIN_RR, lp, (const double *)op->lr_hinv);
    } else {
        // mixed mode: the FP32 copy of r for the polynomial in the same pass
        hipLaunchKernelGGL(ppk::k_xr, dim3(ge), dim3(BLOCK), 0, op->stream, op->n, op->p, op->q, op->xh, op->r,
                           op->partials, op->st, op->mixed() ? op->r32 : (float *)nullptr);
        enqueue_fin(op, ge, ppk::FIN_RR);
    }
    if (e0) (void)hipEventRecord(e0, op->stream);
    enqueue_poly(op, op->r, op->z, ppk::FIN_RHO, false, op->mixed() && lp == 0);
    if (e1) (void)hipEventRecord(e1, op->stream);
    enqueue_p(op, false);
}

hipEvent_t timing_event(pp_op_s *op, size_t i)
{
    while (op->tev.size() <= i) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        op->tev.push_back(e);
    }
    return op->tev[i];
}


}  // namespace

// operators of at most 1024 slices (65536 rows) take the persistent driver by default
constexpr int64_t PERSIST_SMALL_SLICES = 1024;

namespace {

template <bool SCHUR, bool MIXED>
const void *persistent_kernel()
{
    return (const void *)ppk::k_pcg_persistent<SCHUR, MIXED>;
}

const void *pick_persistent(const pp_op_s *op, int *slot)
{
    *slot = (op->schur() ? 2 : 0) + (op->mixed() ? 1 : 0);
    switch (*slot) {
    case 0: return persistent_kernel<false, false>();
    case 1: return persistent_kernel<false, true>();
    case 2: return persistent_kernel<true, false>();
    default: return persistent_kernel<true, true>();
    }
}

// Whole solve in one cooperative launch.  Returns false (nothing queued) when
// the runtime refuses the cooperative grid; the caller then uses the
// stream-driven kernels.
bool persistent_solve(pp_op_s *op, const double *b, double *x, double tol, int maxit)
{
    int slot = 0;
    const void *fn = pick_persistent(op, &slot);
    if (op->persist_occ[slot] == 0) {
        int occ = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, BLOCK, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, op->device) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        op->persist_occ[slot] = std::max(0, occ) * std::max(0, cus);
    }
    int G = (int)std::min<int64_t>({(int64_t)op->persist_occ[slot], (op->nslices + WPB - 1) / WPB, 8192,
                                    (int64_t)op->grid_max});
    // Small operators: one slice per wave, at most 128 workgroups (the
    // two-level barrier costs ~3 us at 128 workgroups, ~4 us at 256; measured
    // Poisson k = 10: 32^3 1.04 ms at 128 workgroups, 1.27 at 32, 1.56 at 16;
    // 40^3 1.35 ms at 128, 1.43 at 250).
    if (op->nslices <= PERSIST_SMALL_SLICES && op->grid_max == op->grid_auto)
        G = (int)std::min<int64_t>(G, 128);
    if (G < 1) return false;
    const int k = op->k;
    if (op->coef_k != k) {
        op->coef_h.assign((size_t)std::max(1, 4 * k), 0.0);
        for (int j = 1; j <= k; ++j) {
            const StepCoef c = step_coef(op, j);
            op->coef_h[4 * (j - 1) + 0] = c.cx;
            op->coef_h[4 * (j - 1) + 1] = c.cold;
            op->coef_h[4 * (j - 1) + 2] = c.cr;
            op->coef_h[4 * (j - 1) + 3] = c.cA;
        }
        dfree(op->coef_d);
        op->coef_d = dalloc<double>(op->coef_h.size());
        HIPCHK(hipMemcpyAsync(op->coef_d, op->coef_h.data(), sizeof(double) * op->coef_h.size(),
                              hipMemcpyHostToDevice, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        op->coef_k = k;
    }
    if (!op->bw) op->bw = dalloc<unsigned long long>((size_t)ppk::GB_LINES * ppk::GB_LINE);
    hipLaunchKernelGGL(ppk::k_zero_u64, dim3(1), dim3(BLOCK), 0, op->stream, op->bw,
                       (int64_t)ppk::GB_LINES * ppk::GB_LINE);
    ppk::PersistArgs a;
    a.A = op->view(false);
    a.A32 = op->view(op->mixed());
    a.Cm = op->cview(false);
    a.Cm32 = op->cview(op->mixed());
    a.b = b;
    a.x = x;
    a.dis = op->dis;
    a.bh = op->bh; a.xh = op->xh; a.r = op->r; a.p = op->p; a.q = op->q; a.z = op->z;
    a.sA = op->sA; a.sB = op->sB; a.tw = op->tw;
    a.r32 = op->r32; a.sA32 = op->sA32; a.sB32 = op->sB32; a.tw32 = op->tw32;
    a.coef = op->coef_d;
    a.partials = op->partials;
    a.st = op->st;
    a.theta_inv = 1.0 / op->theta;
    a.tol = tol;
    a.k = k;
    a.maxit = maxit;
    a.bw = op->bw;
    // the runtime's barrier costs ~0.1 us per workgroup, the flat one about a
    // third of that, the two-level one grows far more slowly (alone in a
    // cooperative launch: 8 workgroups 2.5 / 1.1 / 1.6 us, 32: 5.1 / 1.8 /
    // 2.2 us, 256: 26.8 / 9.5 / 4.2 us, 1024: 104 / 74 / 11 us); inside the
    // solve the two-level one is ahead from 32 workgroups
    a.bar_mode = op->bar_mode >= 0 ? op->bar_mode : (G < 32 ? 1 : 2);
    a.spin = op->spin;
    void *args[] = {&a};
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(BLOCK), args, 0, op->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    op->stats.grid = G;
    op->stats.barrier = a.bar_mode;
    return true;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char *pp_status_str(pp_status s)
{
    switch (s) {
    case PP_OK: return "PP_OK";
    case PP_NOT_CONVERGED: return "PP_NOT_CONVERGED";
    case PP_BREAKDOWN: return "PP_BREAKDOWN";
    case PP_ERR_ARG: return "PP_ERR_ARG";
    case PP_ERR_OOM: return "PP_ERR_OOM";
    case PP_ERR_HIP: return "PP_ERR_HIP";
    case PP_ERR_STATE: return "PP_ERR_STATE";
    case PP_ERR_TIMEOUT: return "PP_ERR_TIMEOUT";
    }
    return "PP_UNKNOWN";
}

const char *pp_last_error(void) { return ppc::last_error().c_str(); }

pp_status pp_create_csr(pp_op *out, int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *colind,
                        const double *val, unsigned flags, void *stream)
{
    return create_common(out, 0, n, nnz, rowptr, colind, val, 0, 0, nullptr, nullptr, nullptr, nullptr, flags,
                         stream);
}

pp_status pp_create_schur(pp_op *out, int64_t n, int64_t nnz_a, const int64_t *a_rowptr, const int32_t *a_col,
                          const double *a_val, int64_t nt, int64_t nnz_c, const int64_t *c_rowptr,
                          const int32_t *c_col, const double *c_val, const double *m_diag, unsigned flags,
                          void *stream)
{
    return create_common(out, 1, n, nnz_a, a_rowptr, a_col, a_val, nt, nnz_c, c_rowptr, c_col, c_val, m_diag,
                         flags, stream);
}

namespace {

// Device copy of a CSR matrix (values scaled by a), after a structure check.
void dfn_copy_csr(pp_op_s *op, const pp_csr &m, double a, int64_t **rp, int32_t **col, double **val)
{
    *rp = dalloc<int64_t>(m.rows + 1);
    *col = dalloc<int32_t>(m.nnz);
    *val = dalloc<double>(m.nnz);
    HIPCHK(hipMemcpyAsync(*rp, m.rowptr, sizeof(int64_t) * (m.rows + 1), hipMemcpyDeviceToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(*col, m.col, sizeof(int32_t) * m.nnz, hipMemcpyDeviceToDevice, op->stream));
    hipLaunchKernelGGL(ppk::k_dfn_axv, dim3(op->grid_elems(m.nnz)), dim3(BLOCK), 0, op->stream, m.nnz, a, m.val,
                       *val);
    HIPCHK(hipGetLastError());
}

// Transpose (rows x cols -> cols rows) of a device CSR, values scaled by a.
void dfn_transpose(pp_op_s *op, int64_t rows, int64_t cols, int64_t nnz, const int64_t *rp, const int32_t *cl,
                   const double *v, double a, int64_t **trp, int32_t **tcol, double **tval)
{
    int64_t *cnt = dalloc<int64_t>(cols);
    struct Free {
        int64_t *&p;
        ~Free() { ppc::dfree(p); }
    } fr{cnt};
    *trp = dalloc<int64_t>(cols + 1);
    *tcol = dalloc<int32_t>(nnz);
    *tval = dalloc<double>(nnz);
    ppk::CsrD m{rp, cl, v};
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int64_t) * cols, op->stream));
    const unsigned gr = (unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + BLOCK - 1) / BLOCK, 8192));
    hipLaunchKernelGGL(ppk::k_t_count, dim3(gr), dim3(BLOCK), 0, op->stream, rows, m, cnt);
    hipLaunchKernelGGL(ppk::k_scan_i64, dim3(1), dim3(1024), 0, op->stream, cols, (const int64_t *)cnt, *trp);
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int64_t) * cols, op->stream));
    hipLaunchKernelGGL(ppk::k_t_fill, dim3(gr), dim3(BLOCK), 0, op->stream, rows, m, a, (const int64_t *)*trp, cnt,
                       *tcol, *tval);
    const unsigned gc = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cols + BLOCK - 1) / BLOCK, 8192));
    hipLaunchKernelGGL(ppk::k_t_sort, dim3(gc), dim3(BLOCK), 0, op->stream, cols, (const int64_t *)*trp, *tcol,
                       *tval);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(op->stream));
}

int read_flag(pp_op_s *op, int *flag_d)
{
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, flag_d, sizeof(int), hipMemcpyDeviceToHost, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    return h;
}

pp_status dfn_build(pp_op_s *op, const pp_dfn_desc &d)
{
    const int64_t F = d.n_frac, G = d.grid, nf = G * G, nh = F * nf, nu = d.gu.rows;
    int *flag_d = dalloc<int>(1);
    int32_t *owner = nullptr, *wg_frac = nullptr;
    int64_t *wg_first = nullptr, *u_end = nullptr;
    double *yscr = nullptr, *dsv = nullptr;
    auto cleanup = [&]() {
        ppc::dfree(flag_d); ppc::dfree(owner); ppc::dfree(wg_frac); ppc::dfree(wg_first); ppc::dfree(u_end);
        ppc::dfree(yscr); ppc::dfree(dsv);
    };
    try {
        const pp_csr *mats[5] = {&d.a, &d.gh, &d.c, &d.b, &d.gu};
        const char *names[5] = {"A", "G^h", "C", "B", "G^u"};
        for (int i = 0; i < 5; ++i)
            if (check_csr_dev(op, mats[i]->rows, mats[i]->cols, mats[i]->nnz, mats[i]->rowptr, mats[i]->col, flag_d)) {
                cleanup();
                return fail(PP_ERR_ARG, std::string("invalid CSR structure of ") + names[i]);
            }
        // checks: A, G^h fracture-local within the band and symmetric; G^u symmetric
        HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
        const unsigned gh_ = (unsigned)std::min<int64_t>((nh + BLOCK - 1) / BLOCK, 8192);
        const unsigned gu_ = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nu + BLOCK - 1) / BLOCK, 8192));
        hipLaunchKernelGGL(ppk::k_dfn_sym, dim3(gh_), dim3(BLOCK), 0, op->stream, nh,
                           ppk::CsrD{d.a.rowptr, d.a.col, d.a.val}, nf, G, flag_d);
        hipLaunchKernelGGL(ppk::k_dfn_sym, dim3(gh_), dim3(BLOCK), 0, op->stream, nh,
                           ppk::CsrD{d.gh.rowptr, d.gh.col, d.gh.val}, nf, G, flag_d);
        hipLaunchKernelGGL(ppk::k_dfn_sym, dim3(gu_), dim3(BLOCK), 0, op->stream, nu,
                           ppk::CsrD{d.gu.rowptr, d.gu.col, d.gu.val}, (int64_t)0, (int64_t)0, flag_d);
        HIPCHK(hipGetLastError());
        int bad = read_flag(op, flag_d);
        if (bad & 1) { cleanup(); return fail(PP_ERR_ARG, "A or G^h has an entry outside its fracture block or band"); }
        if (bad & 2) { cleanup(); return fail(PP_ERR_ARG, "A, G^h or G^u is not symmetric (or has unsorted rows)"); }
        // band factor
        const size_t lbn = (size_t)nh * ppk::dfn_stride((int)G) + ppk::DFN_GMAX + 2;
        op->dfn_Lb = dalloc<double>(lbn);
        HIPCHK(hipMemsetAsync(op->dfn_Lb, 0, sizeof(double) * lbn, op->stream));
        hipLaunchKernelGGL(ppk::k_dfn_band, dim3(gh_), dim3(BLOCK), 0, op->stream, nh, nf, G,
                           ppk::CsrD{d.a.rowptr, d.a.col, d.a.val}, op->dfn_Lb, flag_d);
        hipLaunchKernelGGL(ppk::k_dfn_chol, dim3((unsigned)F), dim3(ppk::DFN_WAVE), 0, op->stream, nh, nf, (int)G,
                           op->dfn_Lb, flag_d);
        HIPCHK(hipGetLastError());
        bad = read_flag(op, flag_d);
        if (bad & 4) { cleanup(); return fail(PP_ERR_ARG, "A is not positive definite (Cholesky pivot <= 0)"); }
        // copies: C, a B, G^h by fracture rows; C^T, a B^T by unknowns; G^u
        dfn_copy_csr(op, d.c, 1.0, &op->dfn_rp[0], &op->dfn_col[0], &op->dfn_val[0]);
        dfn_copy_csr(op, d.b, d.alpha, &op->dfn_rp[1], &op->dfn_col[1], &op->dfn_val[1]);
        dfn_copy_csr(op, d.gh, 1.0, &op->dfn_rp[2], &op->dfn_col[2], &op->dfn_val[2]);
        dfn_transpose(op, nh, nu, d.c.nnz, d.c.rowptr, d.c.col, d.c.val, 1.0, &op->dfn_rp[3], &op->dfn_col[3],
                      &op->dfn_val[3]);
        dfn_transpose(op, nh, nu, d.b.nnz, d.b.rowptr, d.b.col, d.b.val, d.alpha, &op->dfn_rp[4], &op->dfn_col[4],
                      &op->dfn_val[4]);
        dfn_copy_csr(op, d.gu, 1.0, &op->dfn_rp[5], &op->dfn_col[5], &op->dfn_val[5]);
        op->dfn_F = F;
        op->dfn_G = G;
        op->dfn_nh = nh;
        // G^h by entry slots when its rows are short
        {
            HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
            hipLaunchKernelGGL(ppk::k_dfn_maxrow, dim3(gh_), dim3(BLOCK), 0, op->stream, nh,
                               (const int64_t *)op->dfn_rp[2], flag_d);
            HIPCHK(hipGetLastError());
            const int W = read_flag(op, flag_d);
            if (W > 0 && W <= ppk::DFN_ELL_MAX) {
                op->dfn_ghc = dalloc<int32_t>((size_t)W * nh);
                op->dfn_ghv = dalloc<double>((size_t)W * nh);
                hipLaunchKernelGGL(ppk::k_dfn_ghell, dim3(gh_), dim3(BLOCK), 0, op->stream, nh,
                                   ppk::CsrD{op->dfn_rp[2], op->dfn_col[2], op->dfn_val[2]}, W, op->dfn_ghc,
                                   op->dfn_ghv);
                HIPCHK(hipGetLastError());
                op->dfn_ghw = W;
            }
        }
        // the factor by sweep steps for the application
        {
            const size_t qn = (size_t)nh * G + ppk::DFN_WAVE;
            op->dfn_Q = dalloc<double>(2 * qn + nh);
            HIPCHK(hipMemsetAsync(op->dfn_Q, 0, sizeof(double) * (2 * qn + nh), op->stream));
            const ppk::DfnView gq = op->dview();
            hipLaunchKernelGGL(ppk::k_dfn_qcoef, dim3(op->grid_elems(nh * G)), dim3(BLOCK), 0, op->stream, nh, nf,
                               (int)G, (const double *)op->dfn_Lb, const_cast<double *>(gq.Qf),
                               const_cast<double *>(gq.Qb), const_cast<double *>(gq.di2));
            HIPCHK(hipGetLastError());
        }
        // owners of the unknowns, and Algorithm 4 in workgroups of 64 unknowns of one fracture
        std::vector<int32_t> own((size_t)nu);
        std::vector<int32_t> wf;
        std::vector<int64_t> wfirst, uend((size_t)F);
        for (int64_t f = 0; f < F; ++f) {
            for (int64_t j = d.u_off[f]; j < d.u_off[f + 1]; ++j) own[(size_t)j] = (int32_t)f;
            for (int64_t j = d.u_off[f]; j < d.u_off[f + 1]; j += ppk::DFN_WAVE) {
                wf.push_back((int32_t)f);
                wfirst.push_back(j);
            }
            uend[(size_t)f] = d.u_off[f + 1];
        }
        owner = dalloc<int32_t>(nu);
        HIPCHK(hipMemcpyAsync(owner, own.data(), sizeof(int32_t) * nu, hipMemcpyHostToDevice, op->stream));
        HIPCHK(hipMemsetAsync(flag_d, 0, sizeof(int), op->stream));
        const ppk::DfnView g = op->dview();
        hipLaunchKernelGGL(ppk::k_dfn_owner, dim3(gu_), dim3(BLOCK), 0, op->stream, nu, nf, g.ct,
                           (const int32_t *)owner, flag_d);
        HIPCHK(hipGetLastError());
        if (read_flag(op, flag_d) & 8) { cleanup(); return fail(PP_ERR_ARG, "a column of C lies outside the fracture owning it"); }
        const int64_t nwg = (int64_t)wf.size();
        op->dis = dalloc<double>(nu);
        dsv = dalloc<double>(nu);
        if (nwg > 0) {
            wg_frac = dalloc<int32_t>(nwg);
            wg_first = dalloc<int64_t>(nwg);
            u_end = dalloc<int64_t>(F);
            HIPCHK(hipMemcpyAsync(wg_frac, wf.data(), sizeof(int32_t) * nwg, hipMemcpyHostToDevice, op->stream));
            HIPCHK(hipMemcpyAsync(wg_first, wfirst.data(), sizeof(int64_t) * nwg, hipMemcpyHostToDevice, op->stream));
            HIPCHK(hipMemcpyAsync(u_end, uend.data(), sizeof(int64_t) * F, hipMemcpyHostToDevice, op->stream));
            yscr = dalloc<double>((size_t)nwg * nf * ppk::DFN_WAVE);
            hipLaunchKernelGGL(ppk::k_dfn_diag, dim3((unsigned)nwg), dim3(ppk::DFN_WAVE), 0, op->stream, g,
                               (const int32_t *)wg_frac, (const int64_t *)wg_first, (const int64_t *)u_end, yscr, dsv,
                               op->dis, flag_d);
            HIPCHK(hipGetLastError());
        }
        if (read_flag(op, flag_d) & 16) { cleanup(); return fail(PP_ERR_ARG, "diag(S_u) has a non-positive entry"); }
        // the factor by rows served the step-ordered copies and Algorithm 4 (both done: read_flag synchronised)
        ppc::dfree(op->dfn_Lb);
        op->dfn_Lb = nullptr;
        // the operator seen by the fused kernels: one unit entry per row, column n + i
        op->nslices = (nu + WAVE - 1) / WAVE;
        op->nstored = op->nslices * WAVE;
        op->sp = dalloc<int64_t>(op->nslices + 1);
        op->scol = dalloc<int32_t>(op->nstored);
        op->sval = dalloc<double>(op->nstored);
        hipLaunchKernelGGL(ppk::k_dfn_unit, dim3(op->grid_elems(op->nstored)), dim3(BLOCK), 0, op->stream, nu,
                           op->nslices, op->sp, op->scol, op->sval);
        HIPCHK(hipGetLastError());
        op->sell = 1;
        op->nd = 0;
        op->tw = dalloc<double>(nu);
        op->dfn_t = dalloc<double>(nh);
        op->dfn_d = dalloc<double>(nh);
        op->xh = dalloc<double>(nu);
        op->r = dalloc<double>(nu);
        op->p = dalloc<double>(nu);
        op->q = dalloc<double>(nu);
        op->z = dalloc<double>(nu);
        op->bh = dalloc<double>(nu);
        op->sA = dalloc<double>(nu);
        op->sB = dalloc<double>(nu);
        op->partials = dalloc<double>((size_t)(1 + ppk::LR_MAX) * 8192);
        op->st = dalloc<ppk::State>(1);
        HIPCHK(hipMemsetAsync(op->st, 0, sizeof(ppk::State), op->stream));
        HIPCHK(hipHostMalloc((void **)&op->hst, sizeof(ppk::State), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&op->hflag, 2 * sizeof(int32_t), hipHostMallocDefault));
        for (auto &e : op->flag_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : op->solve_ev) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipStreamSynchronize(op->stream));
    } catch (std::bad_alloc &) {
        cleanup();
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        cleanup();
        return hip_fail(e);
    }
    cleanup();
    op->stats.n = nu;
    op->stats.nnz_stored = 0;
    op->stats.diagonals = 0;
    op->stats.nnz_matrix = d.a.nnz + d.gh.nnz + d.c.nnz + d.b.nnz + d.gu.nnz;
    return PP_OK;
}

}  // namespace

pp_status pp_create_dfn(pp_op *out, const pp_dfn_desc *desc, unsigned flags, void *stream)
{
    if (!out) return fail(PP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!desc) return fail(PP_ERR_ARG, "desc is NULL");
    const pp_dfn_desc &d = *desc;
    if (flags & ~(unsigned)PP_JACOBI) return fail(PP_ERR_ARG, "DFN operator: only PP_JACOBI (implied) is accepted");
    if (d.n_frac < 1 || d.grid < 1 || d.grid > ppk::DFN_GMAX)
        return fail(PP_ERR_ARG, "n_frac must be >= 1 and grid in [1, 64]");
    const int64_t nh = d.n_frac * d.grid * d.grid, nu = d.gu.rows;
    if (nh > (int64_t)INT32_MAX - 1 || nu < 1 || nu > (int64_t)INT32_MAX / 2)
        return fail(PP_ERR_ARG, "sizes out of range (n_h < 2^31, 1 <= n_u < 2^30)");
    if (d.a.rows != nh || d.a.cols != nh || d.gh.rows != nh || d.gh.cols != nh || d.c.rows != nh ||
        d.b.rows != nh || d.c.cols != nu || d.b.cols != nu || d.gu.cols != nu)
        return fail(PP_ERR_ARG, "block sizes disagree (A, G^h: n_h x n_h; C, B: n_h x n_u; G^u: n_u x n_u)");
    const pp_csr *mats[5] = {&d.a, &d.gh, &d.c, &d.b, &d.gu};
    for (const pp_csr *m : mats)
        if (!m->rowptr || m->nnz < 0 || (m->nnz > 0 && (!m->col || !m->val)))
            return fail(PP_ERR_ARG, "NULL CSR array");
    if (d.a.nnz < 1) return fail(PP_ERR_ARG, "A is empty");
    if (!d.u_off || d.u_off[0] != 0 || d.u_off[d.n_frac] != nu) return fail(PP_ERR_ARG, "u_off must run from 0 to n_u");
    for (int64_t f = 0; f < d.n_frac; ++f)
        if (d.u_off[f + 1] < d.u_off[f]) return fail(PP_ERR_ARG, "u_off must be non-decreasing");
    if (!std::isfinite(d.alpha)) return fail(PP_ERR_ARG, "alpha must be finite");
    pp_op_s *op = new (std::nothrow) pp_op_s();
    if (!op) return fail(PP_ERR_OOM, "host allocation failed");
    op->kind = 2;
    op->n = nu;
    op->nt = nu;
    op->nnz_given = d.a.nnz;
    op->flags = PP_JACOBI;
    op->stream = (hipStream_t)stream;
    (void)hipGetDevice(&op->device);
    op->ntload = 0;
    pp_status s = dfn_build(op, d);
    if (s != PP_OK) {
        op->release();
        delete op;
        return s;
    }
    *out = op;
    return PP_OK;
}

pp_status pp_dfn_rhs(pp_op op, const double *q, double *r)
{
    if (!op || !q || !r) return fail(PP_ERR_ARG, "NULL argument");
    if (!op->dfn()) return fail(PP_ERR_ARG, "not a DFN operator");
    try {
        const ppk::DfnView g = op->dview();
        launch_frac(op, (const double *)nullptr, (const double *)nullptr, q, op->dfn_t, op->dfn_d,
                    (const ppk::State *)nullptr);
        hipLaunchKernelGGL(ppk::k_dfn_urow, dim3(op->grid_elems(op->n)), dim3(BLOCK), 0, op->stream, g,
                           (const double *)nullptr, (const double *)nullptr, (const double *)op->dfn_t,
                           (const double *)op->dfn_d, 0.0, 1.0, 1.0, r, (const ppk::State *)nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(op->stream));
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_dfn_recover(pp_op op, const double *q, const double *u, double *h, double *p)
{
    if (!op || !q || !u || !h || !p) return fail(PP_ERR_ARG, "NULL argument");
    if (!op->dfn()) return fail(PP_ERR_ARG, "not a DFN operator");
    if (h == p) return fail(PP_ERR_ARG, "h and p must not alias");
    try {
        launch_frac(op, u, (const double *)nullptr, q, h, p, (const ppk::State *)nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(op->stream));
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

void pp_destroy(pp_op op)
{
    if (!op) return;
    (void)hipStreamSynchronize(op->stream);
    op->release();
    delete op;
}

pp_status pp_setup(pp_op op, int k, double lambda_min, double lambda_max, double scaling)
{
    if (!op) return fail(PP_ERR_ARG, "op is NULL");
    if (k < 0 || k > K_MAX) return fail(PP_ERR_ARG, "degree k out of range [0, 4096]");
    if (!std::isfinite(lambda_min) || !std::isfinite(lambda_max) || !(lambda_min > 0.0) ||
        !(lambda_max > lambda_min))
        return fail(PP_ERR_ARG, "bounds must satisfy 0 < lambda_min < lambda_max (finite)");
    if (!std::isfinite(scaling) || !(scaling >= 0.0)) return fail(PP_ERR_ARG, "scaling must be finite and >= 0");
    op->k = k;
    op->lmin = lambda_min;
    op->lmax = lambda_max;
    op->xi = scaling;
    op->theta = (lambda_max + lambda_min) / 2.0 * (1.0 + scaling);
    op->delta = (lambda_max - lambda_min) / 2.0;
    op->sigma = op->theta / op->delta;
    op->rho.assign((size_t)k + 1, 0.0);
    op->rho[0] = 1.0 / op->sigma;
    for (int j = 1; j <= k; ++j) op->rho[j] = 1.0 / (2.0 * op->sigma - op->rho[j - 1]);
    op->form = 0;
    op->setup_done = true;
    return PP_OK;
}

pp_status pp_setup_newton(pp_op op, int nlev, double lambda_min, double lambda_max, double scaling)
{
    if (!op) return fail(PP_ERR_ARG, "op is NULL");
    if (nlev < 0 || nlev > 12) return fail(PP_ERR_ARG, "nlev must be in [0, 12]");
    const pp_status s = pp_setup(op, (1 << nlev) - 1, lambda_min, lambda_max, scaling);
    if (s != PP_OK) return s;
    try {
        if (nlev >= 2 && op->nbuf_levels < nlev - 1) {
            dfree(op->nbuf);
            op->nbuf = dalloc<double>((size_t)2 * (nlev - 1) * op->n);
            op->nbuf_levels = nlev - 1;
        }
    } catch (std::bad_alloc &) {
        op->setup_done = false;
        return fail(PP_ERR_OOM, "device allocation failed");
    }
    // zeta_0 = 1 / theta-bar; zeta_1 from the left end a = theta-bar - delta of
    // the (shifted) interval; zeta_i = 2 / (1 + 2 zeta_{i-1} - zeta_{i-1}^2)
    op->zeta.assign((size_t)nlev + 1, 0.0);
    op->zeta[0] = 1.0 / op->theta;
    if (nlev >= 1) {
        const double az = (op->theta - op->delta) * op->zeta[0];
        op->zeta[1] = 2.0 / (1.0 + 2.0 * az - az * az);
    }
    for (int i = 2; i <= nlev; ++i)
        op->zeta[i] = 2.0 / (1.0 + 2.0 * op->zeta[i - 1] - op->zeta[i - 1] * op->zeta[i - 1]);
    op->nlev = nlev;
    op->form = 1;
    return PP_OK;
}

pp_status pp_set_option(pp_op op, int key, int64_t value)
{
    if (!op) return fail(PP_ERR_ARG, "op is NULL");
    switch (key) {
    case PP_OPT_GRID:
        if (value < 0 || value > 8192) return fail(PP_ERR_ARG, "grid must be in [0, 8192]");
        op->grid_max = value == 0 ? op->grid_auto : (int)value;
        return PP_OK;
    case PP_OPT_CHUNK:
        if (value < 0 || value > 4096) return fail(PP_ERR_ARG, "chunk must be in [0, 4096]");
        op->chunk = (int)value;
        return PP_OK;
    case PP_OPT_TIMING: op->timing = value != 0; return PP_OK;
    case PP_OPT_DRIVER:
        if (value < -1 || value > 1) return fail(PP_ERR_ARG, "driver: 0 (stream-driven), 1 (persistent), -1 (auto)");
        op->driver = (int)value;
        return PP_OK;
    case PP_OPT_NT_LOADS: op->ntload = value != 0; return PP_OK;
    case PP_OPT_TWO_STEP:
        if (value < 0 || value > 2) return fail(PP_ERR_ARG, "PP_OPT_TWO_STEP must be 0, 1 or 2");
        op->two_step = (int)value;
        return PP_OK;
    case PP_OPT_VERIFY:
        if (value < -1 || value > 1) return fail(PP_ERR_ARG, "PP_OPT_VERIFY must be -1, 0 or 1");
        op->verify = (int)value;
        return PP_OK;
    case PP_OPT_RITZ:
        if (value < 0 || value > 1) return fail(PP_ERR_ARG, "PP_OPT_RITZ must be 0 or 1");
        op->ritz_poly = (int)value;
        return PP_OK;
    case PP_OPT_LDS_TILES:
        if (value < 0 || value > 1) return fail(PP_ERR_ARG, "PP_OPT_LDS_TILES must be 0 or 1");
        op->lt_use = (int)value;
        return PP_OK;
    case PP_OPT_BARRIER:
        if (value < -1 || value > 2) return fail(PP_ERR_ARG, "PP_OPT_BARRIER must be -1, 0, 1 or 2");
        op->bar_mode = (int)value;
        return PP_OK;
    case PP_OPT_SPIN_LIMIT:
        if (value < 1 || value > (int64_t)1 << 31) return fail(PP_ERR_ARG, "PP_OPT_SPIN_LIMIT must be in [1, 2^31]");
        op->spin = (unsigned int)value;
        return PP_OK;
    default: return fail(PP_ERR_ARG, "unknown option");
    }
}

pp_status pp_get_stats(pp_op op, pp_stats *st)
{
    if (!op || !st) return fail(PP_ERR_ARG, "NULL argument");
    *st = op->stats;
    st->two_step = use_pairs(op) ? 1 : 0;
    st->unit_diagonal = op->dis != nullptr && op->kind == 0 && op->nd > 0 ? 1 : 0;
    return PP_OK;
}

pp_status pp_operator_apply(pp_op op, const double *x, double *y)
{
    if (!op || !x || !y) return fail(PP_ERR_ARG, "NULL argument");
    if (x == y) return fail(PP_ERR_ARG, "x and y must not alias");
    try {
        const int64_t n = op->n;
        const double *src = x;
        if (op->perm) {
            // P x into the operator's numbering (y comes back through P^T below)
            hipLaunchKernelGGL(ppk::k_gather_scale, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n, x,
                               (const int32_t *)op->perm, (const double *)nullptr, 1.0, op->z);
            src = op->z;
        }
        if (op->dis) {
            // A = D^{1/2} A-hat D^{1/2}: xh = x / dis, y = (A-hat xh) / dis
            hipLaunchKernelGGL(ppk::k_div, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n, src,
                               (const double *)op->dis, op->bh);
            src = op->bh;
        }
        enqueue_trace_f64(op, src, false);
        double *dst = op->dis || op->perm ? op->sA : y;
        if (op->schur())
            hipLaunchKernelGGL((ppk::k_spmv<double, true>), dim3(op->grid_slices()), dim3(BLOCK), 0, op->stream,
                               op->view(false), src, (const double *)op->tw, dst, op->ntload);
        else
            hipLaunchKernelGGL((ppk::k_spmv<double, false>), dim3(op->grid_slices()), dim3(BLOCK), 0, op->stream,
                               op->view(false), src, (const double *)nullptr, dst, op->ntload);
        if (op->dis)
            hipLaunchKernelGGL(ppk::k_div, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n,
                               (const double *)op->sA, (const double *)op->dis, op->perm ? op->sB : y);
        if (op->perm)
            hipLaunchKernelGGL(ppk::k_scatter, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n,
                               (const double *)(op->dis ? op->sB : op->sA), (const int32_t *)op->perm, y);
        HIPCHK(hipGetLastError());
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_apply(pp_op op, const double *r, double *z)
{
    if (!op || !r || !z) return fail(PP_ERR_ARG, "NULL argument");
    if (r == z) return fail(PP_ERR_ARG, "r and z must not alias");
    if (!op->setup_done) return fail(PP_ERR_STATE, "pp_setup must be called before pp_apply");
    try {
        const int64_t n = op->n;
        // the polynomial kernels check the device state: make sure it is live
        hipLaunchKernelGGL(ppk::k_state_init, dim3(1), dim3(64), 0, op->stream, op->st, 0.0, 0);
        const double *rr = r;
        if (op->perm) {
            // the caller's numbering in and out: bh = D^{-1/2} P r, z = P^T z'
            hipLaunchKernelGGL(ppk::k_gather_scale, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n, r,
                               (const int32_t *)op->perm, (const double *)op->dis, 1.0, op->bh);
            rr = op->bh;
        } else if (op->dis) {
            hipLaunchKernelGGL((ppk::k_scale<double, double>), dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream,
                               n, r, (const double *)op->dis, 1.0, op->bh);
            rr = op->bh;
        }
        double *zz = op->perm ? op->z : z;
        enqueue_poly(op, rr, zz, ppk::FIN_NONE, op->dis != nullptr);
        if (op->lr_p > 0) {
            // z += D^{-1/2} V Hinv V^T D^{-1/2} r
            enqueue_lr_c(op, rr, nullptr);
            hipLaunchKernelGGL(ppk::k_lr_axpy, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n, op->lr_p,
                               (const double *)op->lr_v, n, (const double *)op->dis, zz, (const ppk::State *)op->st);
        }
        if (op->perm)
            hipLaunchKernelGGL(ppk::k_scatter, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n,
                               (const double *)zz, (const int32_t *)op->perm, z);
        HIPCHK(hipGetLastError());
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

namespace {

// One stream-driven run of the CG loop from x (unscaled, device): b-hat and
// x-hat from b and x, the initial residual and its test, the first
// polynomial, then chunks of iterations until the done flag is seen, and
// x = D^{-1/2} x-hat.  The state must have been reset (k_state_init) with
// this run's iteration budget.  timed: record the per-polynomial events.
void stream_pass(pp_op_s *op, const double *b, double *x, bool timed, size_t &ev_i)
{
    const int64_t n = op->n;
    const int gs = op->grid_slices(), ge = op->grid_elems(n);
    hipLaunchKernelGGL(ppk::k_init_scale, dim3(ge), dim3(BLOCK), 0, op->stream, n, b, (const double *)x,
                       (const double *)op->dis, op->bh, op->xh, op->partials, op->st, (const int32_t *)op->perm);
    enqueue_fin(op, ge, ppk::FIN_BNORM);
    enqueue_trace_f64(op, op->xh);
    if (op->schur())
        hipLaunchKernelGGL(ppk::k_init_resid<true>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                           (const double *)op->xh, (const double *)op->tw, (const double *)op->bh, op->r,
                           op->partials, op->st, op->ntload);
    else
        hipLaunchKernelGGL(ppk::k_init_resid<false>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                           (const double *)op->xh, (const double *)nullptr, (const double *)op->bh, op->r,
                           op->partials, op->st, op->ntload);
    enqueue_fin(op, gs, ppk::FIN_RR0);
    if (op->lr_p > 0) enqueue_lr_c(op, op->r, nullptr);
    hipEvent_t e0 = timed ? timing_event(op, ev_i++) : nullptr;
    hipEvent_t e1 = timed ? timing_event(op, ev_i++) : nullptr;
    if (e0) HIPCHK(hipEventRecord(e0, op->stream));
    enqueue_poly(op, op->r, op->z, ppk::FIN_RHO0, false);
    if (e1) HIPCHK(hipEventRecord(e1, op->stream));
    enqueue_p(op, true);
    HIPCHK(hipGetLastError());

    int chunk = op->chunk;
    if (chunk <= 0) chunk = n >= (1 << 20) ? 1 : (n >= (1 << 16) ? 4 : 16);
    // the state's own budget ends the loop on the device; the host stops
    // queueing once the flag it polls (one chunk behind) is set
    const int maxit = op->pass_maxit;
    int enq = 0, c = 0;
    while (enq < maxit) {
        const int m = std::min(chunk, maxit - enq);
        for (int i = 0; i < m; ++i) {
            hipEvent_t ea = timed ? timing_event(op, ev_i++) : nullptr;
            hipEvent_t eb = timed ? timing_event(op, ev_i++) : nullptr;
            enqueue_iteration(op, ea, eb);
        }
        HIPCHK(hipGetLastError());
        enq += m;
        HIPCHK(hipMemcpyAsync(&op->hflag[c & 1], &op->st->done, sizeof(int32_t), hipMemcpyDeviceToHost,
                              op->stream));
        HIPCHK(hipEventRecord(op->flag_ev[c & 1], op->stream));
        if (c >= 1) {
            HIPCHK(hipEventSynchronize(op->flag_ev[(c - 1) & 1]));
            if (op->hflag[(c - 1) & 1]) break;
        }
        ++c;
    }
    hipLaunchKernelGGL(ppk::k_final_x, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)op->xh,
                       (const double *)op->dis, x, (const ppk::State *)op->st, (const int32_t *)op->perm);
}

}  // namespace

pp_status pcg_solve(pp_op op, const double *b, double *x, double tol, int maxit, int *iters, double *relres)
{
    if (!op || !b || !x) return fail(PP_ERR_ARG, "NULL argument");
    if (b == x) return fail(PP_ERR_ARG, "b and x must not alias");
    if (!std::isfinite(tol) || tol < 0.0) return fail(PP_ERR_ARG, "tol must be finite and >= 0");
    if (maxit < 0) return fail(PP_ERR_ARG, "maxit must be >= 0");
    if (!op->setup_done) return fail(PP_ERR_STATE, "pp_setup must be called before pcg_solve");
    try {
        HIPCHK(hipEventRecord(op->solve_ev[0], op->stream));
        // persistent driver: on request, or by default for small operators whose
        // polynomial runs single steps (few workgroups and cheap barriers beat
        // a kernel boundary per step there; measured to 32^3)
        const bool small = op->driver == -1 && op->nslices <= PERSIST_SMALL_SLICES && !use_pairs(op);
        const bool want_persist = (op->driver == 1 || small) && op->lr_p == 0 && op->form == 0 && !op->dfn() &&
                                  !op->perm;
        // true-residual check at convergence (default: mixed mode only)
        const bool verify = op->verify > 0 || (op->verify < 0 && op->mixed());
        size_t ev_i = 0;
        op->pev_i = 0;
        op->pairs_per_poly = 0;
        op->time_pairs = op->timing;
        int it_total = 0, restarts = 0, first_it = 0;
        int64_t applies = 0, dots = 0;
        bool persisted = false, zero_b = false, verified = false;
        pp_status ret = PP_OK;
        double rel = 0.0;
        // Pass 0 is the solve.  When it converges and the check is on, pass 1
        // starts again from the iterate: its initial residual b-hat - A-hat x-hat
        // is the true residual, and its initial test either ends the solve at
        // once (the usual case) or CG continues from there (a restart); at most
        // three restarts.
        for (int pass = 0;; ++pass) {
            const int left = maxit - it_total;
            op->pass_maxit = left;
            hipLaunchKernelGGL(ppk::k_state_init, dim3(1), dim3(64), 0, op->stream, op->st, tol, left);
            const bool pers = pass == 0 && want_persist && persistent_solve(op, b, x, tol, left);
            if (!pers) stream_pass(op, b, x, pass == 0 && op->timing, ev_i);
            if (pass == 0) persisted = pers;
            op->time_pairs = false;  // pair events: first pass only
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(op->hst, op->st, sizeof(ppk::State), hipMemcpyDeviceToHost, op->stream));
            HIPCHK(hipStreamSynchronize(op->stream));
            const ppk::State &s = *op->hst;
            const int it = s.it;
            ret = (pp_status)s.status;
            rel = s.bnorm2 > 0 ? std::sqrt(s.rr / s.bnorm2) : 0.0;
            zero_b = s.zero_b != 0;
            if (zero_b) { ret = PP_OK; rel = 0.0; break; }
            it_total += it;
            if (pass == 0) first_it = it;
            // initial residual (1) + initial preconditioner (k, unless the initial
            // test ended the run) + per iteration A p (1) and, except after the
            // last iteration, the preconditioner (k)
            const int64_t polys = it > 0 ? it : (ret == PP_BREAKDOWN ? 1 : 0);
            applies += 1 + (int64_t)op->k * polys + it;
            // and, with a rank-p correction, p more values reduced at the start and in every iteration
            dots += it > 0 || ret == PP_BREAKDOWN ? 1 + 3LL * it + (int64_t)op->lr_p * (1 + it) : 1;
            if (pass > 0 && it == 0) { verified = ret == PP_OK; break; }
            if (pass > 0) ++restarts;
            if (!(verify && ret == PP_OK && it > 0 && pass < 3)) break;
        }
        HIPCHK(hipEventRecord(op->solve_ev[1], op->stream));
        HIPCHK(hipEventSynchronize(op->solve_ev[1]));
        if (iters) *iters = it_total;
        if (relres) *relres = rel;
        op->stats.iters = it_total;
        op->stats.status = ret;
        op->stats.relres = rel;
        op->stats.op_applies = zero_b ? 0 : applies;
        op->stats.dots = zero_b ? 0 : dots;
        op->stats.restarts = restarts;
        op->stats.true_relres = verified ? rel : -1.0;
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, op->solve_ev[0], op->solve_ev[1]));
        op->stats.solve_ms = ms;
        op->time_pairs = false;
        op->stats.cheb_ms = 0;
        op->stats.cheb_steps = 0;
        op->stats.pair_ms = 0;
        op->stats.pair_launches = 0;
        op->stats.driver = persisted ? 1 : 0;
        if (!persisted) op->stats.grid = op->grid_slices();
        if (!persisted) op->stats.barrier = -1;
        if (ret == PP_ERR_TIMEOUT) ppc::last_error() = "a grid-barrier wait of the persistent driver gave up (PP_OPT_SPIN_LIMIT)";
        if (op->timing && !zero_b && !persisted) {
            // first pass only: pairs 0 .. polys-1 ran (the initial one and one per iteration but the last)
            const int64_t polys = first_it > 0 ? first_it : 1;
            double tot = 0;
            for (int64_t i = 0; i < polys && (size_t)(2 * i + 1) < ev_i; ++i) {
                float t = 0;
                HIPCHK(hipEventElapsedTime(&t, op->tev[2 * i], op->tev[2 * i + 1]));
                tot += t;
            }
            op->stats.cheb_ms = tot;
            op->stats.cheb_steps = (int64_t)op->k * polys;
            // one run of pairs per polynomial application, in the same order
            double pt = 0;
            int64_t runs = 0;
            for (int64_t i = 0; i < polys && (size_t)(2 * i + 1) < op->pev_i; ++i) {
                float t = 0;
                HIPCHK(hipEventElapsedTime(&t, op->pev[2 * i], op->pev[2 * i + 1]));
                pt += t;
                ++runs;
            }
            op->stats.pair_ms = pt;
            op->stats.pair_launches = runs * op->pairs_per_poly;
        }
        return ret;
    } catch (HipError &e) {
        return hip_fail(e);
    }
}

namespace {

// H = V^T A-hat V (p operator applications), inverted on the host by
// Gauss-Jordan elimination with partial pivoting; false if H is singular or
// not finite.
bool lowrank_hinv(pp_op_s *op, int p, const double *V, std::vector<double> &hinv)
{
    const int64_t n = op->n;
    const int gs = op->grid_slices(), ge = op->grid_elems(n);
    double *out = dalloc<double>(ppk::LR_MAX + 2);
    struct Free {
        double *&p;
        ~Free() { dfree(p); }
    } f{out};
    std::vector<double> h((size_t)p * 2 * p, 0.0), col(p), nrm(2);
    op->lr_theta.assign(p, 0.0);
    op->lr_res.assign(p, 0.0);
    for (int j = 0; j < p; ++j) {
        const double *vj = V + (int64_t)j * n;
        enqueue_trace_f64(op, vj, false);
        if (op->schur())
            hipLaunchKernelGGL((ppk::k_spmv<double, true>), dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false), vj,
                               (const double *)op->tw, op->q, op->ntload);
        else
            hipLaunchKernelGGL((ppk::k_spmv<double, false>), dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                               vj, (const double *)nullptr, op->q, op->ntload);
        hipLaunchKernelGGL(ppk::k_lr_dots, dim3(ge), dim3(BLOCK), 0, op->stream, n, p, V, n, (const double *)op->q,
                           (const double *)nullptr, op->partials, (const ppk::State *)nullptr);
        hipLaunchKernelGGL(ppk::k_colsum, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials, ge, p,
                           out);
        // ||v_j||^2, then theta = v^T A v / v^T v and ||A v_j - theta v_j||^2
        hipLaunchKernelGGL(ppk::k_lr_dots, dim3(ge), dim3(BLOCK), 0, op->stream, n, 1, vj, n, vj,
                           (const double *)nullptr, op->partials, (const ppk::State *)nullptr);
        hipLaunchKernelGGL(ppk::k_colsum, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials, ge, 1,
                           out + p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(col.data(), out, sizeof(double) * p, hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipMemcpyAsync(nrm.data(), out + p, sizeof(double), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        for (int i = 0; i < p; ++i) h[(size_t)i * 2 * p + j] = col[i];  // H_ij = V_i^T A V_j
        const double vv = nrm[0] > 0.0 ? nrm[0] : 1.0, th = col[j] / vv;
        hipLaunchKernelGGL(ppk::k_resid_norm2, dim3(ge), dim3(BLOCK), 0, op->stream, n, th, vj,
                           (const double *)op->q, op->partials);
        hipLaunchKernelGGL(ppk::k_colsum, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials, ge, 1,
                           out + p + 1);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(nrm.data() + 1, out + p + 1, sizeof(double), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        op->lr_theta[j] = th;
        op->lr_res[j] = std::sqrt(nrm[1]) / (std::fabs(th) * std::sqrt(vv) + 1e-300);
    }
    for (int i = 0; i < p; ++i) h[(size_t)i * 2 * p + p + i] = 1.0;
    for (int c = 0; c < p; ++c) {
        int piv = c;
        for (int i = c + 1; i < p; ++i)
            if (std::fabs(h[(size_t)i * 2 * p + c]) > std::fabs(h[(size_t)piv * 2 * p + c])) piv = i;
        const double d = h[(size_t)piv * 2 * p + c];
        if (!(std::fabs(d) > 0.0) || !std::isfinite(d)) return false;
        if (piv != c)
            for (int j = 0; j < 2 * p; ++j) std::swap(h[(size_t)c * 2 * p + j], h[(size_t)piv * 2 * p + j]);
        for (int j = 0; j < 2 * p; ++j) h[(size_t)c * 2 * p + j] /= d;
        for (int i = 0; i < p; ++i) {
            if (i == c) continue;
            const double fct = h[(size_t)i * 2 * p + c];
            for (int j = 0; j < 2 * p; ++j) h[(size_t)i * 2 * p + j] -= fct * h[(size_t)c * 2 * p + j];
        }
    }
    hinv.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            hinv[(size_t)i * p + j] = h[(size_t)i * 2 * p + p + j];
            if (!std::isfinite(hinv[(size_t)i * p + j])) return false;
        }
    return true;
}

}  // namespace

pp_status pp_lowrank_set(pp_op op, int p, const double *V)
{
    if (!op) return fail(PP_ERR_ARG, "NULL operator");
    if (p < 0 || p > ppk::LR_MAX) return fail(PP_ERR_ARG, "rank must be in [0, 8]");
    if (p > 0 && !V) return fail(PP_ERR_ARG, "V is NULL");
    try {
        if (p == 0) {
            op->lr_p = 0;
            return PP_OK;
        }
        const int64_t n = op->n;
        if (!op->lr_v) op->lr_v = dalloc<double>((size_t)ppk::LR_MAX * n);
        if (!op->lr_hinv) op->lr_hinv = dalloc<double>((size_t)ppk::LR_MAX * ppk::LR_MAX);
        if (V != op->lr_v && op->perm) {
            for (int j = 0; j < p; ++j)  // into the operator's numbering
                hipLaunchKernelGGL(ppk::k_gather_scale, dim3(op->grid_elems(n)), dim3(BLOCK), 0, op->stream, n,
                                   V + (size_t)j * n, (const int32_t *)op->perm, (const double *)nullptr, 1.0,
                                   op->lr_v + (size_t)j * n);
            HIPCHK(hipGetLastError());
        } else if (V != op->lr_v) {
            HIPCHK(hipMemcpyAsync(op->lr_v, V, sizeof(double) * (size_t)p * n, hipMemcpyDeviceToDevice, op->stream));
        }
        std::vector<double> hinv;
        if (!lowrank_hinv(op, p, op->lr_v, hinv)) {
            op->lr_p = 0;
            return fail(PP_ERR_ARG, "V^T A V is singular or not finite");
        }
        HIPCHK(hipMemcpyAsync(op->lr_hinv, hinv.data(), sizeof(double) * hinv.size(), hipMemcpyHostToDevice,
                              op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        op->lr_p = p;
    } catch (std::bad_alloc &) {
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_lowrank_ritz(pp_op op, int steps, int p, double *theta)
{
    if (!op) return fail(PP_ERR_ARG, "NULL operator");
    if (steps < 1 || steps > ppk::LZ_MAX) return fail(PP_ERR_ARG, "steps must be in [1, 64]");
    if (p < 1 || p > ppk::LR_MAX || p > steps) return fail(PP_ERR_ARG, "rank must be in [1, min(8, steps)]");
    const bool poly = op->ritz_poly != 0;
    if (poly && (!op->setup_done || op->form != 0))
        return fail(PP_ERR_STATE, "PP_OPT_RITZ = 1 needs a Chebyshev polynomial (pp_setup) first");
    double *Q = nullptr, *S = nullptr, *coef = nullptr;
    struct Free {
        double *&a, *&b, *&c;
        ~Free() { dfree(a); dfree(b); dfree(c); }
    } f{Q, S, coef};
    try {
        const int64_t n = op->n;
        const int gs = op->grid_slices(), ge = op->grid_elems(n);
        Q = dalloc<double>((size_t)steps * n);
        // the polynomial uses sA..sD: its Lanczos vectors live in r, p, z
        double *v = poly ? op->r : op->sA, *vprev = poly ? op->p : op->sB, *w = poly ? op->z : op->q;
        if (poly) coef = dalloc<double>(ppk::LR_MAX);
        // the Lanczos recurrence of pp_estimate_bounds, keeping every basis vector
        hipLaunchKernelGGL(ppk::k_state_init, dim3(1), dim3(64), 0, op->stream, op->st, 0.0, 0);
        hipLaunchKernelGGL(ppk::k_lz_start, dim3(ge), dim3(BLOCK), 0, op->stream, n, v, op->partials, op->st,
                           (const int32_t *)op->perm);
        enqueue_fin(op, ge, ppk::FIN_LZ_NORM0);
        hipLaunchKernelGGL(ppk::k_lz_norm, dim3(ge), dim3(BLOCK), 0, op->stream, n, v, (const ppk::State *)op->st);
        hipLaunchKernelGGL((ppk::k_scale<double, double>), dim3(ge), dim3(BLOCK), 0, op->stream, n,
                           (const double *)v, (const double *)nullptr, 0.0, vprev);
        for (int j = 0; j < steps && poly; ++j) {
            // w = p_k(A-hat) v, then the three-term Lanczos step and a full
            // reorthogonalisation of w against the basis so far (blocks of LR_MAX)
            HIPCHK(hipMemcpyAsync(Q + (size_t)j * n, v, sizeof(double) * n, hipMemcpyDeviceToDevice, op->stream));
            enqueue_poly(op, v, w, ppk::FIN_NONE, false);
            hipLaunchKernelGGL(ppk::k_lz_wsub, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)v,
                               (const double *)vprev, w, op->partials, op->st, j);
            enqueue_fin(op, ge, ppk::FIN_LZ_ALPHA, j);
            hipLaunchKernelGGL(ppk::k_lz_orth, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)v, w,
                               op->partials, op->st, j);
            for (int c0 = 0; c0 <= j; c0 += ppk::LR_MAX) {
                const int pc = std::min(ppk::LR_MAX, j + 1 - c0);
                const double *Qc = Q + (size_t)c0 * n;
                hipLaunchKernelGGL(ppk::k_lr_dots, dim3(ge), dim3(BLOCK), 0, op->stream, n, pc, Qc, n,
                                   (const double *)w, (const double *)nullptr, op->partials,
                                   (const ppk::State *)nullptr);
                hipLaunchKernelGGL(ppk::k_colsum, dim3(1), dim3(BLOCK), 0, op->stream, (const double *)op->partials,
                                   ge, pc, coef);
                hipLaunchKernelGGL(ppk::k_lr_sub, dim3(ge), dim3(BLOCK), 0, op->stream, n, pc, Qc, n,
                                   (const double *)coef, w);
            }
            hipLaunchKernelGGL(ppk::k_dot_fin, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)w,
                               (const double *)w, op->partials, op->st, (int)ppk::FIN_LZ_BETA);
            enqueue_fin(op, ge, ppk::FIN_LZ_BETA, j);
            if (j + 1 < steps)
                hipLaunchKernelGGL(ppk::k_lz_next, dim3(ge), dim3(BLOCK), 0, op->stream, n, vprev, v,
                                   (const double *)w, (const ppk::State *)op->st, j);
        }
        for (int j = 0; j < steps && !poly; ++j) {
            HIPCHK(hipMemcpyAsync(Q + (size_t)j * n, v, sizeof(double) * n, hipMemcpyDeviceToDevice, op->stream));
            enqueue_trace_f64(op, v);
            if (op->schur())
                hipLaunchKernelGGL(ppk::k_lz_apply<true>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                                   (const double *)v, (const double *)op->tw, (const double *)vprev, w,
                                   op->partials, op->st, j, op->ntload);
            else
                hipLaunchKernelGGL(ppk::k_lz_apply<false>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                                   (const double *)v, (const double *)nullptr, (const double *)vprev, w,
                                   op->partials, op->st, j, op->ntload);
            enqueue_fin(op, gs, ppk::FIN_LZ_ALPHA, j);
            hipLaunchKernelGGL(ppk::k_lz_orth, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)v, w,
                               op->partials, op->st, j);
            enqueue_fin(op, ge, ppk::FIN_LZ_BETA, j);
            if (j + 1 < steps)
                hipLaunchKernelGGL(ppk::k_lz_next, dim3(ge), dim3(BLOCK), 0, op->stream, n, vprev, v,
                                   (const double *)w, (const ppk::State *)op->st, j);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(op->hst, op->st, sizeof(ppk::State), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        int m = steps;
        for (int j = 0; j < steps; ++j) {
            if (!std::isfinite(op->hst->lz_alpha[j]) || !std::isfinite(op->hst->lz_beta[j]))
                return fail(PP_ERR_ARG, "non-finite value in Lanczos (operator not finite?)");
            if (op->hst->lz_beta[j] == 0.0) { m = j + 1; break; }
        }
        if (p > m) return fail(PP_ERR_ARG, "the Krylov space is smaller than the rank asked for");
        std::vector<double> T((size_t)m * m, 0.0), wv, E;
        for (int j = 0; j < m; ++j) {
            T[(size_t)j * m + j] = op->hst->lz_alpha[j];
            if (j + 1 < m) {
                T[(size_t)j * m + j + 1] = op->hst->lz_beta[j];
                T[(size_t)(j + 1) * m + j] = op->hst->lz_beta[j];
            }
        }
        ppeig::jacobi_eig(m, T, wv, E);
        std::vector<int> idx(m);
        for (int i = 0; i < m; ++i) idx[i] = i;
        // smallest Ritz values of A-hat; of p_k(A-hat) the largest
        std::sort(idx.begin(), idx.end(), [&](int a, int b) { return poly ? wv[a] > wv[b] : wv[a] < wv[b]; });
        std::vector<double> Sh((size_t)m * p);
        for (int j = 0; j < m; ++j)
            for (int c = 0; c < p; ++c) Sh[(size_t)j * p + c] = E[(size_t)j * m + idx[c]];
        if (theta)
            for (int c = 0; c < p; ++c) theta[c] = wv[idx[c]];
        S = dalloc<double>(Sh.size());
        HIPCHK(hipMemcpyAsync(S, Sh.data(), sizeof(double) * Sh.size(), hipMemcpyHostToDevice, op->stream));
        if (!op->lr_v) op->lr_v = dalloc<double>((size_t)ppk::LR_MAX * n);
        if (!op->lr_hinv) op->lr_hinv = dalloc<double>((size_t)ppk::LR_MAX * ppk::LR_MAX);
        hipLaunchKernelGGL(ppk::k_lr_combine, dim3(ge), dim3(BLOCK), 0, op->stream, n, m, p, (const double *)Q,
                           (const double *)S, op->lr_v);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(op->stream));  // Sh leaves scope
    } catch (std::bad_alloc &) {
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        return hip_fail(e);
    }
    const pp_status s = pp_lowrank_set(op, p, op->lr_v);
    // of p_k(A-hat) the Ritz values are not eigenvalue estimates of A-hat: report v^T A-hat v
    if (s == PP_OK && poly && theta)
        for (int c = 0; c < p; ++c) theta[c] = op->lr_theta[c];
    return s;
}

pp_status pp_lowrank_info(pp_op op, double *theta, double *resid)
{
    if (!op) return fail(PP_ERR_ARG, "NULL operator");
    for (int c = 0; c < op->lr_p; ++c) {
        if (theta) theta[c] = op->lr_theta[c];
        if (resid) resid[c] = op->lr_res[c];
    }
    return PP_OK;
}

pp_status pp_lowrank_get(pp_op op, int *p, double *V)
{
    if (!op || !p) return fail(PP_ERR_ARG, "NULL argument");
    *p = op->lr_p;
    if (V && op->lr_p > 0) {
        try {
            if (op->perm) {
                for (int j = 0; j < op->lr_p; ++j)  // back to the caller's numbering
                    hipLaunchKernelGGL(ppk::k_scatter, dim3(op->grid_elems(op->n)), dim3(BLOCK), 0, op->stream,
                                       op->n, (const double *)op->lr_v + (size_t)j * op->n,
                                       (const int32_t *)op->perm, V + (size_t)j * op->n);
                HIPCHK(hipGetLastError());
            } else {
                HIPCHK(hipMemcpyAsync(V, op->lr_v, sizeof(double) * (size_t)op->lr_p * op->n,
                                      hipMemcpyDeviceToDevice, op->stream));
            }
        } catch (HipError &e) {
            return hip_fail(e);
        }
    }
    return PP_OK;
}

pp_status pp_estimate_bounds(pp_op op, int steps, double *lambda_min, double *lambda_max)
{
    if (!op || !lambda_min || !lambda_max) return fail(PP_ERR_ARG, "NULL argument");
    if (steps < 1 || steps > ppk::LZ_MAX) return fail(PP_ERR_ARG, "steps must be in [1, 64]");
    try {
        const int64_t n = op->n;
        const int gs = op->grid_slices(), ge = op->grid_elems(n);
        double *v = op->sA, *vprev = op->sB, *w = op->q;
        hipLaunchKernelGGL(ppk::k_state_init, dim3(1), dim3(64), 0, op->stream, op->st, 0.0, 0);
        hipLaunchKernelGGL(ppk::k_lz_start, dim3(ge), dim3(BLOCK), 0, op->stream, n, v, op->partials, op->st,
                           (const int32_t *)op->perm);
        enqueue_fin(op, ge, ppk::FIN_LZ_NORM0);
        hipLaunchKernelGGL(ppk::k_lz_norm, dim3(ge), dim3(BLOCK), 0, op->stream, n, v, (const ppk::State *)op->st);
        hipLaunchKernelGGL((ppk::k_scale<double, double>), dim3(ge), dim3(BLOCK), 0, op->stream, n,
                           (const double *)v, (const double *)nullptr, 0.0, vprev);
        for (int j = 0; j < steps; ++j) {
            enqueue_trace_f64(op, v);
            if (op->schur())
                hipLaunchKernelGGL(ppk::k_lz_apply<true>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                                   (const double *)v, (const double *)op->tw, (const double *)vprev, w,
                                   op->partials, op->st, j, op->ntload);
            else
                hipLaunchKernelGGL(ppk::k_lz_apply<false>, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                                   (const double *)v, (const double *)nullptr, (const double *)vprev, w,
                                   op->partials, op->st, j, op->ntload);
            enqueue_fin(op, gs, ppk::FIN_LZ_ALPHA, j);
            hipLaunchKernelGGL(ppk::k_lz_orth, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)v, w,
                               op->partials, op->st, j);
            enqueue_fin(op, ge, ppk::FIN_LZ_BETA, j);
            if (j + 1 < steps)
                hipLaunchKernelGGL(ppk::k_lz_next, dim3(ge), dim3(BLOCK), 0, op->stream, n, vprev, v,
                                   (const double *)w, (const ppk::State *)op->st, j);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(op->hst, op->st, sizeof(ppk::State), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        int m = steps;
        for (int j = 0; j < steps; ++j) {
            if (!std::isfinite(op->hst->lz_alpha[j]) || !std::isfinite(op->hst->lz_beta[j]))
                return fail(PP_ERR_ARG, "non-finite value in Lanczos (operator not finite?)");
            if (op->hst->lz_beta[j] == 0.0) { m = j + 1; break; }
        }
        std::vector<double> T((size_t)m * m, 0.0), wv, V;
        for (int j = 0; j < m; ++j) {
            T[(size_t)j * m + j] = op->hst->lz_alpha[j];
            if (j + 1 < m) {
                T[(size_t)j * m + j + 1] = op->hst->lz_beta[j];
                T[(size_t)(j + 1) * m + j] = op->hst->lz_beta[j];
            }
        }
        ppeig::jacobi_eig(m, T, wv, V);
        int imin = 0, imax = 0;
        for (int i = 1; i < m; ++i) {
            if (wv[i] < wv[imin]) imin = i;
            if (wv[i] > wv[imax]) imax = i;
        }
        const double pad = std::fabs(op->hst->lz_beta[m - 1] * V[(size_t)(m - 1) * m + imax]);
        *lambda_min = wv[imin];
        *lambda_max = wv[imax] + pad;
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

}  // extern "C"
