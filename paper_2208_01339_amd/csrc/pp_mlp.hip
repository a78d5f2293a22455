// C-ABI implementation of the learned-bounds entry points of include/pp.h:
// operator features, the bounds/scaling MLP (forward, gradients, Adam
// training) and the prediction with its fallback to Lanczos.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "mlp.hpp"
#include "op.hpp"

using ppc::dalloc;
using ppc::dfree;
using ppc::fail;
using ppc::hip_fail;
using ppc::HipError;
using ppk::BLOCK;

struct pp_mlp_s {
    int n_in = 0, hidden = 0, depth = 0, n_out = 0;
    hipStream_t stream = nullptr;
    int64_t nparam = 0;
    std::vector<int64_t> w_off, b_off;  // per layer offsets into the parameter vector
    std::vector<int> fan_in, fan_out;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    // activations for a batch of at most bmax rows
    int bmax = 0;
    std::vector<float *> Z, H, dZ;  // per layer [bmax][fan_out]
    float *dY = nullptr;
    double *loss_d = nullptr;
    double *loss_h = nullptr;  // pinned
    int adam_t = 0;
    double in_mean[32], in_std[32], out_mean[8], out_std[8];
    bool have_norm = false;

    int layers() const { return depth + 1; }

    void release()
    {
        dfree(params); dfree(grads); dfree(m); dfree(v); dfree(dY); dfree(loss_d);
        for (auto &p : Z) dfree(p);
        for (auto &p : H) dfree(p);
        for (auto &p : dZ) dfree(p);
        if (loss_h) (void)hipHostFree(loss_h);
        loss_h = nullptr;
    }
};

namespace {

constexpr int BMAX = 1024;
constexpr int NFEAT = 16;

// splitmix64: deterministic parameter initialisation on the host
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

unsigned grid1(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// forward pass; the output layer lands in Z.back() (no activation)
void forward(pp_mlp_s *mp, int batch, const float *X)
{
    const float *in = X;
    int ld_in = mp->n_in;
    for (int l = 0; l < mp->layers(); ++l) {
        const int K = mp->fan_in[l], N = mp->fan_out[l];
        const bool last = (l == mp->layers() - 1);
        hipLaunchKernelGGL((ppm::km_mm<false, false>), dim3(grid1((int64_t)batch * N)), dim3(BLOCK), 0, mp->stream, batch,
                           N, K, in, ld_in, (const float *)(mp->params + mp->w_off[l]), N,
                           (const float *)(mp->params + mp->b_off[l]), mp->Z[l], N, last ? 0 : 1,
                           (const float *)nullptr, mp->H[l]);
        in = mp->H[l];
        ld_in = N;
    }
}

// loss and gradients into mp->grads (flat, same layout as params)
void backward(pp_mlp_s *mp, int batch, const float *X, const float *T)
{
    const int Lc = mp->layers();
    const int NO = mp->n_out;
    hipLaunchKernelGGL(ppm::km_loss, dim3(1), dim3(BLOCK), 0, mp->stream, batch, NO, (const float *)mp->Z[Lc - 1], T,
                       mp->dY, mp->loss_d);
    const float *dz = mp->dY;
    for (int l = Lc - 1; l >= 0; --l) {
        const int K = mp->fan_in[l], N = mp->fan_out[l];
        const float *hin = l == 0 ? X : mp->H[l - 1];
        // dW[K][N] = hin^T dz
        hipLaunchKernelGGL((ppm::km_mm<true, false>), dim3(grid1((int64_t)K * N)), dim3(BLOCK), 0, mp->stream, K, N,
                           batch, hin, K, dz, N, (const float *)nullptr, mp->grads + mp->w_off[l], N, 0,
                           (const float *)nullptr, (float *)nullptr);
        hipLaunchKernelGGL(ppm::km_colsum, dim3(grid1(N)), dim3(BLOCK), 0, mp->stream, batch, N, dz,
                           mp->grads + mp->b_off[l]);
        if (l > 0) {
            // dZ_{l-1}[batch][K] = (dz W^T) * relu'(Z_{l-1})
            hipLaunchKernelGGL((ppm::km_mm<false, true>), dim3(grid1((int64_t)batch * K)), dim3(BLOCK), 0, mp->stream,
                               batch, K, N, dz, N, (const float *)(mp->params + mp->w_off[l]), N,
                               (const float *)nullptr, mp->dZ[l - 1], K, 2, (const float *)mp->Z[l - 1],
                               (float *)nullptr);
            dz = mp->dZ[l - 1];
        }
    }
}

}  // namespace

extern "C" {

pp_status pp_mlp_create(pp_mlp *out, int n_in, int hidden, int depth, int n_out, uint64_t seed, void *stream)
{
    if (!out) return fail(PP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_in > 32 || hidden < 1 || hidden > 1024 || depth < 1 || depth > 8 || n_out < 1 || n_out > 8)
        return fail(PP_ERR_ARG, "sizes out of range (n_in <= 32, hidden <= 1024, depth <= 8, n_out <= 8)");
    pp_mlp_s *mp = new (std::nothrow) pp_mlp_s();
    if (!mp) return fail(PP_ERR_OOM, "host allocation failed");
    mp->n_in = n_in; mp->hidden = hidden; mp->depth = depth; mp->n_out = n_out;
    mp->stream = (hipStream_t)stream;
    try {
        int64_t off = 0;
        for (int l = 0; l <= depth; ++l) {
            const int fi = l == 0 ? n_in : hidden, fo = l == depth ? n_out : hidden;
            mp->fan_in.push_back(fi);
            mp->fan_out.push_back(fo);
            mp->w_off.push_back(off);
            off += (int64_t)fi * fo;
            mp->b_off.push_back(off);
            off += fo;
        }
        mp->nparam = off;
        // He-uniform weights, zero biases
        std::vector<float> p(off, 0.0f);
        uint64_t s = seed;
        for (int l = 0; l <= depth; ++l) {
            const double bound = std::sqrt(6.0 / mp->fan_in[l]);
            for (int64_t i = 0; i < (int64_t)mp->fan_in[l] * mp->fan_out[l]; ++i) {
                const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
                p[mp->w_off[l] + i] = (float)((2.0 * u - 1.0) * bound);
            }
        }
        mp->params = dalloc<float>(off);
        mp->grads = dalloc<float>(off);
        mp->m = dalloc<float>(off);
        mp->v = dalloc<float>(off);
        HIPCHK(hipMemcpyAsync(mp->params, p.data(), sizeof(float) * off, hipMemcpyHostToDevice, mp->stream));
        HIPCHK(hipMemsetAsync(mp->m, 0, sizeof(float) * off, mp->stream));
        HIPCHK(hipMemsetAsync(mp->v, 0, sizeof(float) * off, mp->stream));
        HIPCHK(hipMemsetAsync(mp->grads, 0, sizeof(float) * off, mp->stream));
        mp->bmax = BMAX;
        for (int l = 0; l <= depth; ++l) {
            mp->Z.push_back(dalloc<float>((size_t)BMAX * mp->fan_out[l]));
            mp->H.push_back(dalloc<float>((size_t)BMAX * mp->fan_out[l]));
            mp->dZ.push_back(dalloc<float>((size_t)BMAX * mp->fan_out[l]));
        }
        mp->dY = dalloc<float>((size_t)BMAX * n_out);
        mp->loss_d = dalloc<double>(1);
        HIPCHK(hipHostMalloc((void **)&mp->loss_h, sizeof(double), hipHostMallocDefault));
        HIPCHK(hipStreamSynchronize(mp->stream));
    } catch (std::bad_alloc &) {
        mp->release();
        delete mp;
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        mp->release();
        delete mp;
        return hip_fail(e);
    }
    for (int i = 0; i < 32; ++i) { mp->in_mean[i] = 0.0; mp->in_std[i] = 1.0; }
    for (int i = 0; i < 8; ++i) { mp->out_mean[i] = 0.0; mp->out_std[i] = 1.0; }
    *out = mp;
    return PP_OK;
}

void pp_mlp_destroy(pp_mlp mp)
{
    if (!mp) return;
    (void)hipStreamSynchronize(mp->stream);
    mp->release();
    delete mp;
}

pp_status pp_mlp_num_params(pp_mlp mp, int64_t *count)
{
    if (!mp || !count) return fail(PP_ERR_ARG, "NULL argument");
    *count = mp->nparam;
    return PP_OK;
}

pp_status pp_mlp_get_params(pp_mlp mp, float *dst)
{
    if (!mp || !dst) return fail(PP_ERR_ARG, "NULL argument");
    try {
        HIPCHK(hipMemcpyAsync(dst, mp->params, sizeof(float) * mp->nparam, hipMemcpyDeviceToDevice, mp->stream));
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_mlp_set_params(pp_mlp mp, const float *src)
{
    if (!mp || !src) return fail(PP_ERR_ARG, "NULL argument");
    try {
        HIPCHK(hipMemcpyAsync(mp->params, src, sizeof(float) * mp->nparam, hipMemcpyDeviceToDevice, mp->stream));
        HIPCHK(hipMemsetAsync(mp->m, 0, sizeof(float) * mp->nparam, mp->stream));
        HIPCHK(hipMemsetAsync(mp->v, 0, sizeof(float) * mp->nparam, mp->stream));
        mp->adam_t = 0;
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_mlp_set_normalization(pp_mlp mp, const double *in_mean, const double *in_std, const double *out_mean,
                                   const double *out_std)
{
    if (!mp || !in_mean || !in_std || !out_mean || !out_std) return fail(PP_ERR_ARG, "NULL argument");
    for (int i = 0; i < mp->n_in; ++i) {
        if (!(in_std[i] > 0) || !std::isfinite(in_mean[i])) return fail(PP_ERR_ARG, "input std must be > 0");
        mp->in_mean[i] = in_mean[i];
        mp->in_std[i] = in_std[i];
    }
    for (int i = 0; i < mp->n_out; ++i) {
        if (!(out_std[i] > 0) || !std::isfinite(out_mean[i])) return fail(PP_ERR_ARG, "output std must be > 0");
        mp->out_mean[i] = out_mean[i];
        mp->out_std[i] = out_std[i];
    }
    mp->have_norm = true;
    return PP_OK;
}

pp_status pp_mlp_forward(pp_mlp mp, int batch, const float *X, float *Y)
{
    if (!mp || !X || !Y) return fail(PP_ERR_ARG, "NULL argument");
    if (batch < 1 || batch > BMAX) return fail(PP_ERR_ARG, "batch must be in [1, 1024]");
    try {
        forward(mp, batch, X);
        HIPCHK(hipMemcpyAsync(Y, mp->Z.back(), sizeof(float) * batch * mp->n_out, hipMemcpyDeviceToDevice,
                              mp->stream));
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_mlp_loss_grad(pp_mlp mp, int batch, const float *X, const float *T, float *grad, double *loss)
{
    if (!mp || !X || !T) return fail(PP_ERR_ARG, "NULL argument");
    if (batch < 1 || batch > BMAX) return fail(PP_ERR_ARG, "batch must be in [1, 1024]");
    try {
        forward(mp, batch, X);
        backward(mp, batch, X, T);
        if (grad)
            HIPCHK(hipMemcpyAsync(grad, mp->grads, sizeof(float) * mp->nparam, hipMemcpyDeviceToDevice, mp->stream));
        HIPCHK(hipMemcpyAsync(mp->loss_h, mp->loss_d, sizeof(double), hipMemcpyDeviceToHost, mp->stream));
        HIPCHK(hipStreamSynchronize(mp->stream));
        if (loss) *loss = *mp->loss_h;
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_mlp_train_step(pp_mlp mp, int batch, const float *X, const float *T, float lr, double *loss)
{
    if (!mp || !X || !T) return fail(PP_ERR_ARG, "NULL argument");
    if (batch < 1 || batch > BMAX) return fail(PP_ERR_ARG, "batch must be in [1, 1024]");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(PP_ERR_ARG, "lr must be positive");
    try {
        forward(mp, batch, X);
        backward(mp, batch, X, T);
        mp->adam_t += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = (float)(1.0 - std::pow(0.9, mp->adam_t)), c2 = (float)(1.0 - std::pow(0.999, mp->adam_t));
        hipLaunchKernelGGL(ppm::km_adam, dim3(grid1(mp->nparam)), dim3(BLOCK), 0, mp->stream, mp->nparam, mp->params,
                           (const float *)mp->grads, mp->m, mp->v, lr, b1, b2, 1e-8f, c1, c2);
        HIPCHK(hipGetLastError());
        if (loss) {
            HIPCHK(hipMemcpyAsync(mp->loss_h, mp->loss_d, sizeof(double), hipMemcpyDeviceToHost, mp->stream));
            HIPCHK(hipStreamSynchronize(mp->stream));
            *loss = *mp->loss_h;
        }
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

// ---------------------------------------------------------------------------
// operator features
// ---------------------------------------------------------------------------

pp_status pp_features(pp_op op, int power_steps, double *f)
{
    if (!op || !f) return fail(PP_ERR_ARG, "NULL argument");
    if (power_steps < 2 || power_steps > 64 || power_steps % 2) return fail(PP_ERR_ARG, "power_steps: even, 2..64");
    try {
        const int64_t n = op->n;
        const int gs = op->grid_slices(), ge = op->grid_elems(n);
        double *stats = nullptr, *part = nullptr;
        stats = dalloc<double>(16 + 64 + 2);
        part = dalloc<double>((size_t)std::max(gs, ge) * ppm::NSTAT);
        const double *ts = nullptr;
        if (op->schur()) {
            hipLaunchKernelGGL(ppm::k_trace_abs, dim3((unsigned)((op->nt + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, op->stream,
                               op->cview(false), op->tw);
            ts = op->tw;
        }
        hipLaunchKernelGGL(ppm::k_feat_rows, dim3(gs), dim3(BLOCK), 0, op->stream, op->view(false),
                           (const double *)op->dis, ts, part);
        hipLaunchKernelGGL(ppm::k_feat_fin, dim3(1), dim3(64), 0, op->stream, (const double *)part, gs, stats);
        // power iteration on A-hat, then on (c I - A-hat) with c = Gershgorin upper bound (stats[4])
        double *v = op->sA, *w = op->sB, *y = op->q;
        for (int shifted = 0; shifted < 2; ++shifted) {
            hipLaunchKernelGGL(ppk::k_lz_start, dim3(ge), dim3(BLOCK), 0, op->stream, n, v, part,
                               (ppk::State *)nullptr, (const int32_t *)op->perm);
            for (int t = 0; t < power_steps; ++t) {
                if (op->schur()) {
                    hipLaunchKernelGGL((ppk::k_trace<double, double>), dim3(op->grid_elems(op->nt)), dim3(BLOCK), 0,
                                       op->stream, op->cview(false), (const double *)v, op->tw,
                                       (const ppk::State *)nullptr);
                    hipLaunchKernelGGL((ppk::k_spmv<double, true>), dim3(gs), dim3(BLOCK), 0, op->stream,
                                       op->view(false), (const double *)v, (const double *)op->tw, y, 0);
                } else {
                    hipLaunchKernelGGL((ppk::k_spmv<double, false>), dim3(gs), dim3(BLOCK), 0, op->stream,
                                       op->view(false), (const double *)v, (const double *)nullptr, y, 0);
                }
                hipLaunchKernelGGL(ppm::k_pow_dots, dim3(ge), dim3(BLOCK), 0, op->stream, n, (const double *)v,
                                   (const double *)y, w, (const double *)(stats + 4), shifted, part);
                hipLaunchKernelGGL(ppm::k_pow_fin, dim3(1), dim3(64), 0, op->stream, (const double *)part, ge,
                                   stats + 16 + shifted * 32 + t);
                std::swap(v, w);
            }
        }
        HIPCHK(hipGetLastError());
        std::vector<double> h(16 + 64);
        HIPCHK(hipMemcpyAsync(h.data(), stats, sizeof(double) * h.size(), hipMemcpyDeviceToHost, op->stream));
        HIPCHK(hipStreamSynchronize(op->stream));
        dfree(stats);
        dfree(part);
        const double nn = (double)n;
        const double mean = h[0] / nn;
        const double var = std::max(0.0, h[1] / nn - mean * mean);
        const int P = power_steps;
        const double rq = h[16 + P - 1];                   // last Rayleigh quotient of A-hat
        const double lmin_est = h[4] - h[16 + 32 + P - 1];  // c - RQ of (c I - A-hat)
        f[0] = std::log10(nn);
        f[1] = (double)op->nnz_given / nn;
        f[2] = mean;
        f[3] = std::sqrt(var);
        f[4] = h[2];
        f[5] = h[3];
        f[6] = h[4];            // Gershgorin upper bound of lambda_max
        f[7] = h[5] / nn;       // mean off-diagonal absolute row sum
        f[8] = h[6];            // Gershgorin lower bound (A part)
        // Rayleigh quotients after P/4, P/2, 3P/4 and P operator applications
        const int q1 = std::max(1, P / 4), q2 = std::max(1, P / 2), q3 = std::max(1, 3 * P / 4);
        f[9] = h[16 + q1 - 1];
        f[10] = h[16 + q2 - 1];
        f[11] = h[16 + q3 - 1];
        f[12] = rq;
        f[13] = lmin_est;
        f[14] = h[7];           // longest row
        f[15] = std::log10(std::max(rq, 1e-300) / std::max(std::fabs(lmin_est), 1e-12));
    } catch (std::bad_alloc &) {
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        return hip_fail(e);
    }
    return PP_OK;
}

pp_status pp_predict_bounds(pp_op op, pp_mlp mp, int power_steps, double *lambda_min, double *lambda_max,
                            double *scaling, int *fallback)
{
    if (!op || !mp || !lambda_min || !lambda_max || !scaling || !fallback) return fail(PP_ERR_ARG, "NULL argument");
    if (mp->n_in != NFEAT || mp->n_out != 3) return fail(PP_ERR_ARG, "MLP must map 16 features to 3 outputs");
    if (!mp->have_norm) return fail(PP_ERR_STATE, "pp_mlp_set_normalization must be called first");
    double f[NFEAT];
    pp_status s = pp_features(op, power_steps, f);
    if (s != PP_OK) return s;
    float xin[NFEAT], yout[3];
    for (int i = 0; i < NFEAT; ++i) xin[i] = (float)((f[i] - mp->in_mean[i]) / mp->in_std[i]);
    float *xd = nullptr, *yd = nullptr;
    try {
        xd = dalloc<float>(NFEAT);
        yd = dalloc<float>(3);
        HIPCHK(hipMemcpyAsync(xd, xin, sizeof(xin), hipMemcpyHostToDevice, mp->stream));
        forward(mp, 1, xd);
        HIPCHK(hipMemcpyAsync(yd, mp->Z.back(), sizeof(float) * 3, hipMemcpyDeviceToDevice, mp->stream));
        HIPCHK(hipMemcpyAsync(yout, yd, sizeof(yout), hipMemcpyDeviceToHost, mp->stream));
        HIPCHK(hipStreamSynchronize(mp->stream));
    } catch (std::bad_alloc &) {
        dfree(xd); dfree(yd);
        return fail(PP_ERR_OOM, "device allocation failed");
    } catch (HipError &e) {
        dfree(xd); dfree(yd);
        return hip_fail(e);
    }
    dfree(xd);
    dfree(yd);
    const double lo = std::exp((double)yout[0] * mp->out_std[0] + mp->out_mean[0]);
    const double hi = std::exp((double)yout[1] * mp->out_std[1] + mp->out_mean[1]);
    const double xi = std::max(0.0, std::pow(10.0, (double)yout[2] * mp->out_std[2] + mp->out_mean[2]) - 1e-5);
    // violation checks: RQ <= lambda_max <= Gershgorin upper bound, 0 < lambda_min < lambda_max
    const double rq = f[12], gup = f[6];
    const bool bad = !std::isfinite(lo) || !std::isfinite(hi) || !std::isfinite(xi) || !(lo > 0.0) || !(hi > lo) ||
                     hi < rq || hi > gup * (1.0 + 1e-12) || xi > 0.1;
    if (!bad) {
        *lambda_min = lo;
        *lambda_max = hi;
        *scaling = xi;
        *fallback = 0;
        return PP_OK;
    }
    *fallback = 1;
    *scaling = 0.0;
    return pp_estimate_bounds(op, 20, lambda_min, lambda_max);
}

}  // extern "C"
