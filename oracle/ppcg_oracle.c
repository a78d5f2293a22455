/*
 * CPU oracle for polynomial-preconditioned Conjugate Gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 reference that
 * the GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the GPU library never does, and
 * the two share no code.  Everything here is written for a reader to compare
 * by eye with the paper: plain loops, left-to-right sums, no blocking, no
 * fusion.  Build with -ffp-contract=off so that no FMA changes the rounding of
 * the printed formulas.  The checker build has no threads.  The few OpenMP
 * pragmas on row loops and dot products are read only by a second build
 * (-fopenmp), used solely to time the oracle on all host cores; that build
 * sums dot products in another order and is never a parity reference.
 *
 * Paper: Bergamaschi, Ferronato, Isotton, Janna, Martinez, "Parallel
 * matrix-free polynomial preconditioners with application to flow simulations
 * in discrete fracture networks" (arXiv 2208.01339).
 *
 * Contents and the passage each follows:
 *   orc_op_apply     y = A x for a CSR matrix, or for the Schur-shaped
 *                    operator y = A_ff x + C^T (M^{-1} (C x)) (the
 *                    G - W^T M^{-1} Z pattern of section 4.2, eq. (schur),
 *                    with a diagonal middle block), optionally symmetrically
 *                    scaled by D^{-1/2} (section 3, W = D^{-1/2}; section 4.3).
 *   orc_op_diag      diag of that operator without forming it (the analogue
 *                    of Algorithm 4 for the Schur shape).
 *   orc_cheb_coeffs  theta-bar, delta, sigma and rho_j: section 2.2 eqs.
 *                    (polycheb)/(rhocheb) with theta replaced by
 *                    theta-bar = (beta+alpha)/2 (1+xi), eq. (thetamod).
 *   orc_cheb_apply   z = p_k(A) r from the recurrence of the polynomials,
 *                    section 2.2 eq. (polycheb) (what Algorithm 2 computes).
 *   orc_newton_apply z = P_nlev r, Algorithm 1 (degree 2^nlev - 1).
 *   orc_pcg          CG preconditioned by p_k(A), standard Hestenes-Stiefel
 *                    loop; counts operator applications and dot products as
 *                    reported in Table tab11.
 *   orc_pcg_newton   the same loop preconditioned by P_nlev of Algorithm 1.
 *   orc_lowrank_setup, orc_lowrank_apply, orc_pcg_lowrank
 *                    the spectral low-rank correction of section 3.1:
 *                    P = P_0 + V (V^T A V)^{-1} V^T with P_0 = p_k(A), and CG
 *                    preconditioned by it (one extra dot product per column
 *                    of V per iteration, as in the rank-one rows of tab11).
 *   orc_lanczos      plain Lanczos tridiagonalisation (no
 *                    reorthogonalisation) used to estimate the extremal
 *                    eigenvalues alpha, beta that section 2 assumes known.
 *   orc_fmix32_start Lanczos start vector from the MurmurHash3 32-bit
 *                    finaliser of the row index.
 *   orc_dfn_*        the DFN Schur complement of sections 4.2-4.3 (operator
 *                    kind 2): the exact Cholesky factor of the block-diagonal
 *                    A (orc_dfn_factor), y = S_u r from the expansion of
 *                    eq. (schur) (used by orc_op_apply), diag(S_u) from the
 *                    same expansion (orc_op_diag; the quantity Algorithm 4
 *                    computes), the reduced right-hand side
 *                    r = W^T M^{-1} f_1 and the recovery of h and p after the
 *                    solve for u (section 4.2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Blocks of the DFN system (section 4.1, eq. (sys)) in the unknowns (h, u, p):
 * A (n_h x n_h, block diagonal SPD, one block of nf = G*G rows per fracture,
 * entries within distance G of the diagonal), G^h (n_h x n_h, same blocks),
 * C, B (n_h x n_u), G^u (n_u x n_u), the scalar alpha.  All CSR. */
typedef struct {
    int64_t n_frac, G, nf, nh, nu;
    const int64_t *arp; const int32_t *aci; const double *av;
    const int64_t *ghrp; const int32_t *ghci; const double *ghv;
    const int64_t *crp; const int32_t *cci; const double *cv;
    const int64_t *brp; const int32_t *bci; const double *bv;
    const int64_t *gurp; const int32_t *guci; const double *guv;
    double alpha;
    double *L;                 /* band factor, row-major: L[i (G+1) + k] = L(i, i-k) */
    double *w1, *w2, *w3, *w4; /* scratch, n_h doubles each                         */
    double *wu;                /* scratch, n_u doubles                               */
} orc_dfn;

typedef struct {
    int32_t kind;          /* 0 = CSR matrix, 1 = Schur-shaped, 2 = DFN S_u      */
    int32_t pad0;
    int64_t n;             /* order of the operator                              */
    const int64_t *arp;    /* A (or A_ff): CSR row pointers, n + 1               */
    const int32_t *aci;    /* A: column indices                                  */
    const double *av;      /* A: values                                          */
    int64_t nt;            /* Schur: rows of C (trace cell pairs)                */
    const int64_t *crp;    /* Schur: C row pointers, nt + 1                      */
    const int32_t *cci;    /* Schur: C column indices (cells)                    */
    const double *cv;      /* Schur: C values                                    */
    const double *m;       /* Schur: diagonal of M, nt                           */
    const double *dis;     /* D^{-1/2} for symmetric scaling, or NULL            */
    double *work_n;        /* scratch, n doubles                                 */
    double *work_nt;       /* scratch, nt doubles (Schur only)                   */
    int64_t n_apply;       /* operator applications performed (counter)          */
    orc_dfn *dfn;          /* kind 2: the DFN blocks and factor                  */
} orc_op;

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2, ORC_ERR_ARG = -1 };

/* ------------------------------------------------------------------------ */
/* vectors                                                                   */
/* ------------------------------------------------------------------------ */

double orc_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    #pragma omp parallel for schedule(static) reduction(+ : s)
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* operators                                                                 */
/* ------------------------------------------------------------------------ */

/* y = A x for a CSR matrix. */
void orc_csr_matvec(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                    const double *x, double *y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * x[ci[p]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* DFN Schur complement (sections 4.2 and 4.3)                              */
/* ------------------------------------------------------------------------ */

/* y = M^T x for a CSR matrix M with n rows (y has M's column count, zeroed here). */
static void csr_tmatvec(int64_t n, int64_t ncol, const int64_t *rp, const int32_t *ci, const double *v,
                        const double *x, double *y)
{
    for (int64_t j = 0; j < ncol; ++j) y[j] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) y[ci[p]] += v[p] * x[i];
}

/* Exact Cholesky factor of A, block by block (Cholesky-Banachiewicz, by rows):
 *   L(i,j) = (a_ij - sum_{m<j} L(i,m) L(j,m)) / L(j,j),   j < i
 *   L(i,i) = sqrt(a_ii - sum_{m<i} L(i,m)^2)
 * with m, j restricted to the band of the block.  Returns ORC_ERR_ARG when an
 * entry of A lies outside its fracture's block or band, or a pivot is not
 * positive (A not SPD). */
int orc_dfn_factor(orc_dfn *d)
{
    const int64_t G = d->G, nf = d->nf, W = G + 1;
    for (int64_t i = 0; i < d->nh * W; ++i) d->L[i] = 0.0;
    for (int64_t i = 0; i < d->nh; ++i) {
        const int64_t f0 = (i / nf) * nf;
        for (int64_t p = d->arp[i]; p < d->arp[i + 1]; ++p) {
            const int64_t j = d->aci[p];
            if (j < f0 || j >= f0 + nf || j > i + G || j < i - G) return ORC_ERR_ARG;
            if (j <= i) d->L[i * W + (i - j)] += d->av[p];
        }
    }
    for (int64_t i = 0; i < d->nh; ++i) {
        const int64_t f0 = (i / nf) * nf;
        const int64_t j0 = i - G > f0 ? i - G : f0;
        for (int64_t j = j0; j < i; ++j) {
            double s = d->L[i * W + (i - j)];
            const int64_t m0 = j - G > j0 ? j - G : j0;
            for (int64_t m = m0; m < j; ++m) s -= d->L[i * W + (i - m)] * d->L[j * W + (j - m)];
            d->L[i * W + (i - j)] = s / d->L[j * W];
        }
        double s = d->L[i * W];
        for (int64_t m = j0; m < i; ++m) s -= d->L[i * W + (i - m)] * d->L[i * W + (i - m)];
        if (!(s > 0.0)) return ORC_ERR_ARG;
        d->L[i * W] = sqrt(s);
    }
    return ORC_OK;
}

/* x = A^{-1} b = L^{-T} (L^{-1} b) with A = L L^T, fracture by fracture
 * (section 4.2).  x may alias b. */
void orc_dfn_ainv(const orc_dfn *d, const double *b, double *x)
{
    const int64_t G = d->G, nf = d->nf, W = G + 1;
    for (int64_t i = 0; i < d->nh; ++i) x[i] = b[i];
    for (int64_t f0 = 0; f0 < d->nh; f0 += nf) {
        /* L y = b */
        for (int64_t i = f0; i < f0 + nf; ++i) {
            double s = x[i];
            const int64_t j0 = i - G > f0 ? i - G : f0;
            for (int64_t j = j0; j < i; ++j) s -= d->L[i * W + (i - j)] * x[j];
            x[i] = s / d->L[i * W];
        }
        /* L^T x = y */
        for (int64_t i = f0 + nf - 1; i >= f0; --i) {
            double s = x[i];
            const int64_t j1 = i + G < f0 + nf - 1 ? i + G : f0 + nf - 1;
            for (int64_t j = i + 1; j <= j1; ++j) s -= d->L[j * W + (j - i)] * x[j];
            x[i] = s / d->L[i * W];
        }
    }
}

/* y = S_u r from the expansion of the Schur complement (section 4.2, eq. (schur)):
 *   S_u(a) = G^u - a B^T A^{-1} C - a C^T A^{-1} B + C^T A^{-1} G^h A^{-1} C,
 * one term after the other, each A^{-1} by the two triangular solves with
 * the exact factor.  A^{-1} C r is formed once and used by the second and the
 * last term.  (Algorithm 3 evaluates the same products in another grouping.) */
void orc_dfn_su(orc_dfn *d, const double *r, double *y)
{
    const int64_t nh = d->nh, nu = d->nu;
    double *cr = d->w1, *ainv_cr = d->w2, *tmp = d->w3, *tmp2 = d->w4, *term = d->wu;
    /* term 1: G^u r */
    orc_csr_matvec(nu, d->gurp, d->guci, d->guv, r, y);
    /* term 2: - a B^T (A^{-1} C r) */
    orc_csr_matvec(nh, d->crp, d->cci, d->cv, r, cr);
    orc_dfn_ainv(d, cr, ainv_cr);
    csr_tmatvec(nh, nu, d->brp, d->bci, d->bv, ainv_cr, term);
    for (int64_t j = 0; j < nu; ++j) y[j] -= d->alpha * term[j];
    /* term 3: - a C^T (A^{-1} B r) */
    orc_csr_matvec(nh, d->brp, d->bci, d->bv, r, tmp);
    orc_dfn_ainv(d, tmp, tmp2);
    csr_tmatvec(nh, nu, d->crp, d->cci, d->cv, tmp2, term);
    for (int64_t j = 0; j < nu; ++j) y[j] -= d->alpha * term[j];
    /* term 4: + C^T A^{-1} G^h (A^{-1} C r) */
    orc_csr_matvec(nh, d->ghrp, d->ghci, d->ghv, ainv_cr, tmp);
    orc_dfn_ainv(d, tmp, tmp2);
    csr_tmatvec(nh, nu, d->crp, d->cci, d->cv, tmp2, term);
    for (int64_t j = 0; j < nu; ++j) y[j] += term[j];
}

/* diag(S_u) without forming S_u (section 4.3): entry i of the expansion above
 * is, with c_i, b_i the i-th columns of C and B and z_i = A^{-1} c_i (A and
 * so A^{-1} symmetric, hence c_i^T A^{-1} b_i = b_i^T z_i):
 *   (S_u)_ii = (G^u)_ii - 2 a b_i^T z_i + z_i^T G^h z_i,
 * which Algorithm 4 groups as (G^u)_ii + z_i^T (G^h z_i - 2 a b_i).  One
 * column at a time; a block whose part of c_i is zero has a zero part of z_i
 * and is not solved. */
void orc_dfn_diag(orc_dfn *d, double *ds)
{
    const int64_t nh = d->nh, nu = d->nu, G = d->G, nf = d->nf, W = G + 1;
    double *c = d->w1, *z = d->w2, *ghz = d->w3, *b = d->w4;
    for (int64_t i = 0; i < nu; ++i) {
        for (int64_t r = 0; r < nh; ++r) c[r] = 0.0, b[r] = 0.0;
        for (int64_t r = 0; r < nh; ++r) {
            for (int64_t p = d->crp[r]; p < d->crp[r + 1]; ++p)
                if (d->cci[p] == i) c[r] += d->cv[p];
            for (int64_t p = d->brp[r]; p < d->brp[r + 1]; ++p)
                if (d->bci[p] == i) b[r] += d->bv[p];
        }
        /* z_i = A^{-1} c_i, block by block */
        for (int64_t f0 = 0; f0 < nh; f0 += nf) {
            int nonzero = 0;
            for (int64_t r = f0; r < f0 + nf; ++r) nonzero |= c[r] != 0.0;
            if (!nonzero) {
                for (int64_t r = f0; r < f0 + nf; ++r) z[r] = 0.0;
                continue;
            }
            for (int64_t r = f0; r < f0 + nf; ++r) {
                double s = c[r];
                const int64_t j0 = r - G > f0 ? r - G : f0;
                for (int64_t j = j0; j < r; ++j) s -= d->L[r * W + (r - j)] * z[j];
                z[r] = s / d->L[r * W];
            }
            for (int64_t r = f0 + nf - 1; r >= f0; --r) {
                double s = z[r];
                const int64_t j1 = r + G < f0 + nf - 1 ? r + G : f0 + nf - 1;
                for (int64_t j = r + 1; j <= j1; ++j) s -= d->L[j * W + (j - r)] * z[j];
                z[r] = s / d->L[r * W];
            }
        }
        double gii = 0.0;
        for (int64_t p = d->gurp[i]; p < d->gurp[i + 1]; ++p)
            if (d->guci[p] == i) gii += d->guv[p];
        orc_csr_matvec(nh, d->ghrp, d->ghci, d->ghv, z, ghz);
        ds[i] = gii - 2.0 * d->alpha * orc_dot(nh, b, z) + orc_dot(nh, z, ghz);
    }
}

/* r = W^T M^{-1} f_1 with f_1 = (q, 0):  r = a B^T A^{-1} q - C^T A^{-1} G^h A^{-1} q. */
void orc_dfn_rhs(orc_dfn *d, const double *q, double *r)
{
    const int64_t nh = d->nh, nu = d->nu;
    double *a1 = d->w1, *g = d->w2, *a2 = d->w3;
    orc_dfn_ainv(d, q, a1);
    orc_csr_matvec(nh, d->ghrp, d->ghci, d->ghv, a1, g);
    orc_dfn_ainv(d, g, a2);
    csr_tmatvec(nh, nu, d->brp, d->bci, d->bv, a1, r);
    csr_tmatvec(nh, nu, d->crp, d->cci, d->cv, a2, d->wu);
    for (int64_t j = 0; j < nu; ++j) r[j] = d->alpha * r[j] - d->wu[j];
}

/* h = A^{-1} (q + C u),  p = A^{-1} (a B u - G^h h). */
void orc_dfn_recover(orc_dfn *d, const double *q, const double *u, double *h, double *p)
{
    const int64_t nh = d->nh;
    double *v = d->w1, *g = d->w2;
    orc_csr_matvec(nh, d->crp, d->cci, d->cv, u, v);
    for (int64_t i = 0; i < nh; ++i) v[i] = q[i] + v[i];
    orc_dfn_ainv(d, v, h);
    orc_csr_matvec(nh, d->brp, d->bci, d->bv, u, v);
    orc_csr_matvec(nh, d->ghrp, d->ghci, d->ghv, h, g);
    for (int64_t i = 0; i < nh; ++i) v[i] = d->alpha * v[i] - g[i];
    orc_dfn_ainv(d, v, p);
}

/* y = op x (unscaled).  Schur: y = A_ff x + C^T (M^{-1} (C x)).  DFN: S_u x. */
static void op_apply_raw(const orc_op *op, const double *x, double *y)
{
    if (op->kind == 2) {
        orc_dfn_su(op->dfn, x, y);
        return;
    }
    orc_csr_matvec(op->n, op->arp, op->aci, op->av, x, y);
    if (op->kind == 1) {
        double *w = op->work_nt;
        /* w = C x */
        orc_csr_matvec(op->nt, op->crp, op->cci, op->cv, x, w);
        /* w = M^{-1} w */
        for (int64_t t = 0; t < op->nt; ++t) w[t] = w[t] / op->m[t];
        /* y += C^T w, one row of C at a time */
        for (int64_t t = 0; t < op->nt; ++t)
            for (int64_t p = op->crp[t]; p < op->crp[t + 1]; ++p)
                y[op->cci[p]] += op->cv[p] * w[t];
    }
}

/* y = op-hat x, with op-hat = D^{-1/2} op D^{-1/2} when dis is set. */
void orc_op_apply(orc_op *op, const double *x, double *y)
{
    op->n_apply += 1;
    if (op->dis == NULL) {
        op_apply_raw(op, x, y);
        return;
    }
    double *t = op->work_n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < op->n; ++i) t[i] = op->dis[i] * x[i];
    op_apply_raw(op, t, y);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < op->n; ++i) y[i] = op->dis[i] * y[i];
}

/* d = diag(op), unscaled.  CSR: a_ii.  Schur: (A_ff)_ii + sum_t C_ti^2 / M_t.
 * DFN: Algorithm 4. */
void orc_op_diag(const orc_op *op, double *d)
{
    if (op->kind == 2) {
        orc_dfn_diag(op->dfn, d);
        return;
    }
    for (int64_t i = 0; i < op->n; ++i) {
        double s = 0.0;
        for (int64_t p = op->arp[i]; p < op->arp[i + 1]; ++p)
            if (op->aci[p] == i) s += op->av[p];
        d[i] = s;
    }
    if (op->kind == 1) {
        for (int64_t t = 0; t < op->nt; ++t)
            for (int64_t p = op->crp[t]; p < op->crp[t + 1]; ++p)
                d[op->cci[p]] += op->cv[p] * op->cv[p] / op->m[t];
    }
}

/* ------------------------------------------------------------------------ */
/* Chebyshev polynomial preconditioner                                       */
/* ------------------------------------------------------------------------ */

/*
 * theta-bar = (lmax + lmin)/2 * (1 + xi)   (eq. thetamod: xi moves the centre)
 * delta     = (lmax - lmin)/2              (unchanged by xi)
 * sigma     = theta-bar / delta
 * rho_0 = 1/sigma, rho_j = 1/(2 sigma - rho_{j-1})   (eq. rhocheb)
 * rho must have room for k + 1 entries (k >= 0).
 */
int orc_cheb_coeffs(int k, double lmin, double lmax, double xi,
                    double *theta_bar, double *delta, double *sigma, double *rho)
{
    if (k < 0 || !(lmin > 0.0) || !(lmax > lmin) || !(xi >= 0.0)) return ORC_ERR_ARG;
    double th = (lmax + lmin) / 2.0 * (1.0 + xi);
    double de = (lmax - lmin) / 2.0;
    double si = th / de;
    *theta_bar = th;
    *delta = de;
    *sigma = si;
    rho[0] = 1.0 / si;
    for (int j = 1; j <= k; ++j) rho[j] = 1.0 / (2.0 * si - rho[j - 1]);
    return ORC_OK;
}

/*
 * z = p_k(op-hat) r, from the recurrence that defines the polynomials
 * (section 2.2, eq. (polycheb), theta replaced by theta-bar of eq. (thetamod)):
 *   p_{-1} = 0,   p_0 = 1/theta,
 *   p_j(x) = rho_j (2 sigma (1 - x/theta) p_{j-1}(x) - rho_{j-1} p_{j-2}(x) + 2/delta),
 * taken at the operator and applied to r.  With s_j = p_j(A) r:
 *   s_{-1} = 0,  s_0 = r / theta,
 *   s_j = rho_j (2 sigma (s_{j-1} - A s_{j-1} / theta) - rho_{j-1} s_{j-2} + (2/delta) r).
 * One operator application per degree, k in all.  Algorithm 2 forms the same
 * vectors (its first step is s_1 with s_{-1} = 0 written out).
 * work must hold 3 n doubles.
 */
int orc_cheb_apply(orc_op *op, int k, double lmin, double lmax, double xi,
                   const double *r, double *z, double *work)
{
    int64_t n = op->n;
    double th, de, si;
    double *rho = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    if (!rho) return ORC_ERR_ARG;
    int st = orc_cheb_coeffs(k, lmin, lmax, xi, &th, &de, &si, rho);
    if (st != ORC_OK) { free(rho); return st; }
    double *s_prev = work, *s = work + n, *as = work + 2 * n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        s_prev[i] = 0.0;          /* s_{-1} */
        s[i] = r[i] / th;         /* s_0    */
    }
    for (int j = 1; j <= k; ++j) {
        orc_op_apply(op, s, as);
        const double rj = rho[j], rjm1 = rho[j - 1];
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double next = rj * (2.0 * si * (s[i] - as[i] / th) - rjm1 * s_prev[i] + (2.0 / de) * r[i]);
            s_prev[i] = s[i];
            s[i] = next;
        }
    }
    memcpy(z, s, sizeof(double) * (size_t)n);
    free(rho);
    return ORC_OK;
}

/*
 * Algorithm 1 (Newton form), applied recursively:
 *   P_0 r = zeta_0 r,   P_{j+1} r = zeta_{j+1} (2 P_j r - P_j A P_j r).
 * zeta_0 = 1/theta-bar (= 2/(alpha+beta) when xi = 0);
 * zeta_1 = 2 / (1 + 2 a zeta_0 - (a zeta_0)^2) with a the left end of the
 * interval [theta-bar - delta, theta-bar + delta] (a = alpha when xi = 0);
 * zeta_i = 2 / (1 + 2 zeta_{i-1} - zeta_{i-1}^2), i >= 2  (eq. zetaNewt).
 */
static void newton_level(orc_op *op, int j, const double *zeta, const double *r, double *out,
                         double *ws)
{
    int64_t n = op->n;
    if (j == 0) {
        for (int64_t i = 0; i < n; ++i) out[i] = zeta[0] * r[i];
        return;
    }
    double *u = ws, *au = ws + n, *pau = ws + 2 * n, *next = ws + 3 * n;
    newton_level(op, j - 1, zeta, r, u, next);
    orc_op_apply(op, u, au);
    newton_level(op, j - 1, zeta, au, pau, next);
    for (int64_t i = 0; i < n; ++i) out[i] = zeta[j] * (2.0 * u[i] - pau[i]);
}

int orc_newton_apply(orc_op *op, int nlev, double lmin, double lmax, double xi,
                     const double *r, double *z)
{
    if (nlev < 0 || nlev > 20 || !(lmin > 0.0) || !(lmax > lmin) || !(xi >= 0.0)) return ORC_ERR_ARG;
    double th = (lmax + lmin) / 2.0 * (1.0 + xi);
    double de = (lmax - lmin) / 2.0;
    double a = th - de;
    double zeta[21];
    zeta[0] = 1.0 / th;
    if (nlev >= 1) {
        double az = a * zeta[0];
        zeta[1] = 2.0 / (1.0 + 2.0 * az - az * az);
    }
    for (int i = 2; i <= nlev; ++i) zeta[i] = 2.0 / (1.0 + 2.0 * zeta[i - 1] - zeta[i - 1] * zeta[i - 1]);
    double *ws = (double *)malloc(sizeof(double) * (size_t)op->n * (size_t)(3 * nlev + 1));
    if (!ws) return ORC_ERR_ARG;
    newton_level(op, nlev, zeta, r, z, ws);
    free(ws);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* PCG                                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t iters;
    int32_t status;
    double relres;      /* ||r_hat|| / ||b_hat|| of the recursive residual */
    int64_t n_apply;    /* operator applications, preconditioner included  */
    int64_t n_dot;      /* dot products, excluding ||b_hat||              */
} orc_pcg_stats;

/*
 * Solve op x = b by CG preconditioned with p_k(op-hat) (op-hat = scaled op when
 * op->dis is set: the system solved is D^{-1/2} A D^{-1/2} x_hat = D^{-1/2} b,
 * x = D^{-1/2} x_hat; the tolerance applies to ||r_hat|| / ||b_hat||).
 * On entry x holds x0; on exit the last iterate.
 *
 *   r = b - A x0;  z = P r;  p = z;  rho = r.z
 *   for it = 1..maxit:
 *     q = A p;  gamma = p.q;  alpha = rho / gamma
 *     x += alpha p;  r -= alpha q
 *     if ||r|| <= tol ||b|| : converged after it iterations
 *     z = P r;  rho' = r.z;  beta = rho' / rho;  p = z + beta p;  rho = rho'
 */
/*
 * Spectral low-rank correction (section 3.1).  V: n x p, column j at
 * V[j*n .. j*n+n-1] (vectors of the scaled operator when op->dis is set).
 * orc_lowrank_setup forms H = V^T A V with p operator applications and its
 * inverse by Gauss-Jordan elimination with partial pivoting (p is small);
 * Hinv: p x p row-major.  Returns ORC_ERR_ARG if H is singular.
 */
int orc_lowrank_setup(orc_op *op, int p, const double *V, double *Hinv)
{
    int64_t n = op->n;
    if (p < 1 || p > 64) return ORC_ERR_ARG;
    double *av = (double *)malloc(sizeof(double) * (size_t)n);
    double *h = (double *)malloc(sizeof(double) * (size_t)p * 2 * p);
    if (!av || !h) { free(av); free(h); return ORC_ERR_ARG; }
    /* augmented [H | I] */
    for (int j = 0; j < p; ++j) {
        orc_op_apply(op, V + (size_t)j * n, av);
        for (int i = 0; i < p; ++i) h[(size_t)i * 2 * p + j] = orc_dot(n, V + (size_t)i * n, av);
    }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) h[(size_t)i * 2 * p + p + j] = (i == j) ? 1.0 : 0.0;
    int ret = ORC_OK;
    for (int c = 0; c < p && ret == ORC_OK; ++c) {
        int piv = c;
        for (int i = c + 1; i < p; ++i)
            if (fabs(h[(size_t)i * 2 * p + c]) > fabs(h[(size_t)piv * 2 * p + c])) piv = i;
        if (!(fabs(h[(size_t)piv * 2 * p + c]) > 0.0)) { ret = ORC_ERR_ARG; break; }
        if (piv != c)
            for (int j = 0; j < 2 * p; ++j) {
                double t = h[(size_t)c * 2 * p + j];
                h[(size_t)c * 2 * p + j] = h[(size_t)piv * 2 * p + j];
                h[(size_t)piv * 2 * p + j] = t;
            }
        double d = h[(size_t)c * 2 * p + c];
        for (int j = 0; j < 2 * p; ++j) h[(size_t)c * 2 * p + j] /= d;
        for (int i = 0; i < p; ++i) {
            if (i == c) continue;
            double f = h[(size_t)i * 2 * p + c];
            for (int j = 0; j < 2 * p; ++j) h[(size_t)i * 2 * p + j] -= f * h[(size_t)c * 2 * p + j];
        }
    }
    if (ret == ORC_OK)
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j) Hinv[(size_t)i * p + j] = h[(size_t)i * 2 * p + p + j];
    free(av);
    free(h);
    return ret;
}

/* z += V Hinv V^T r  (p dot products; counted in *ndot when given) */
static void lowrank_add(int64_t n, int p, const double *V, const double *Hinv, const double *r, double *z,
                        int64_t *ndot)
{
    double c[64], y[64];
    for (int j = 0; j < p; ++j) c[j] = orc_dot(n, V + (size_t)j * n, r);
    if (ndot) *ndot += p;
    for (int i = 0; i < p; ++i) {
        double s = 0.0;
        for (int j = 0; j < p; ++j) s += Hinv[(size_t)i * p + j] * c[j];
        y[i] = s;
    }
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < p; ++j) s += V[(size_t)j * n + i] * y[j];
        z[i] += s;
    }
}

/* z = (p_k(A) + V (V^T A V)^{-1} V^T) r ; work: 3 n doubles */
int orc_lowrank_apply(orc_op *op, int k, double lmin, double lmax, double xi, int p, const double *V,
                      const double *Hinv, const double *r, double *z, double *work)
{
    int ret = orc_cheb_apply(op, k, lmin, lmax, xi, r, z, work);
    if (ret != ORC_OK) return ret;
    if (p > 0) lowrank_add(op->n, p, V, Hinv, r, z, NULL);
    return ORC_OK;
}

/* The polynomial part of the preconditioner: p_k(A) r (Chebyshev, nlev < 0)
 * or P_nlev r (Newton form of Algorithm 1, degree 2^nlev - 1). */
static int poly_apply(orc_op *op, int k, int nlev, double lmin, double lmax, double xi, const double *r,
                      double *z, double *work)
{
    if (nlev >= 0) return orc_newton_apply(op, nlev, lmin, lmax, xi, r, z);
    return orc_cheb_apply(op, k, lmin, lmax, xi, r, z, work);
}

static int pcg_core(orc_op *op, int k, int nlev, double lmin, double lmax, double xi, int lr_p,
                    const double *V, const double *Hinv, const double *b, double *x, double tol, int maxit,
                    orc_pcg_stats *st);

int orc_pcg(orc_op *op, int k, double lmin, double lmax, double xi, const double *b, double *x,
            double tol, int maxit, orc_pcg_stats *st)
{
    return pcg_core(op, k, -1, lmin, lmax, xi, 0, NULL, NULL, b, x, tol, maxit, st);
}

/* CG preconditioned by the Newton form P_nlev of Algorithm 1 (section 2.1). */
int orc_pcg_newton(orc_op *op, int nlev, double lmin, double lmax, double xi, const double *b, double *x,
                   double tol, int maxit, orc_pcg_stats *st)
{
    if (nlev < 0 || nlev > 20) return ORC_ERR_ARG;
    return pcg_core(op, 0, nlev, lmin, lmax, xi, 0, NULL, NULL, b, x, tol, maxit, st);
}

/* CG preconditioned by P = p_k(A) + V Hinv V^T (Hinv from orc_lowrank_setup). */
int orc_pcg_lowrank(orc_op *op, int k, double lmin, double lmax, double xi, int p, const double *V,
                    const double *Hinv, const double *b, double *x, double tol, int maxit, orc_pcg_stats *st)
{
    if (p < 0 || p > 64) return ORC_ERR_ARG;
    return pcg_core(op, k, -1, lmin, lmax, xi, p, V, Hinv, b, x, tol, maxit, st);
}

static int pcg_core(orc_op *op, int k, int nlev, double lmin, double lmax, double xi, int lr_p,
                    const double *V, const double *Hinv, const double *b, double *x, double tol, int maxit,
                    orc_pcg_stats *st)
{
    int64_t n = op->n;
    memset(st, 0, sizeof(*st));
    double *bh = (double *)malloc(sizeof(double) * (size_t)n * 9);
    if (!bh) return ORC_ERR_ARG;
    double *xh = bh + n, *r = bh + 2 * n, *z = bh + 3 * n, *p = bh + 4 * n, *q = bh + 5 * n;
    double *cw = bh + 6 * n;
    int64_t apply0 = op->n_apply;
    int ret = ORC_OK;

    int x0_zero = 1;
    for (int64_t i = 0; i < n; ++i) {
        double di = op->dis ? op->dis[i] : 1.0;
        bh[i] = di * b[i];
        xh[i] = x[i] / di;
        if (x[i] != 0.0) x0_zero = 0;
    }
    double bnorm = sqrt(orc_dot(n, bh, bh));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        st->status = ORC_OK;
        free(bh);
        return ORC_OK;
    }
    if (x0_zero) {
        memcpy(r, bh, sizeof(double) * (size_t)n);
    } else {
        orc_op_apply(op, xh, q);
        for (int64_t i = 0; i < n; ++i) r[i] = bh[i] - q[i];
        double rr0 = orc_dot(n, r, r);
        if (sqrt(rr0) <= tol * bnorm) {
            st->relres = sqrt(rr0) / bnorm;
            goto done;
        }
    }
    ret = poly_apply(op, k, nlev, lmin, lmax, xi, r, z, cw);
    if (ret != ORC_OK) goto done;
    if (lr_p > 0) lowrank_add(n, lr_p, V, Hinv, r, z, &st->n_dot);
    double rho = orc_dot(n, r, z);
    st->n_dot += 1;
    if (!(rho > 0.0) || !isfinite(rho)) { ret = ORC_BREAKDOWN; goto done; }
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rr = 0.0;
    ret = ORC_NOT_CONVERGED;
    for (int it = 1; it <= maxit; ++it) {
        orc_op_apply(op, p, q);
        double gamma = orc_dot(n, p, q);
        st->n_dot += 1;
        if (!(gamma > 0.0) || !isfinite(gamma)) { ret = ORC_BREAKDOWN; break; }
        double alpha = rho / gamma;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            xh[i] = xh[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        st->iters = it;
        rr = orc_dot(n, r, r);
        st->n_dot += 1;
        st->relres = sqrt(rr) / bnorm;
        if (!isfinite(rr)) { ret = ORC_BREAKDOWN; break; }
        if (sqrt(rr) <= tol * bnorm) { ret = ORC_OK; break; }
        if (it == maxit) { ret = ORC_NOT_CONVERGED; break; }
        poly_apply(op, k, nlev, lmin, lmax, xi, r, z, cw);
        if (lr_p > 0) lowrank_add(n, lr_p, V, Hinv, r, z, &st->n_dot);
        double rho_new = orc_dot(n, r, z);
        st->n_dot += 1;
        if (!(rho_new > 0.0) || !isfinite(rho_new)) { ret = ORC_BREAKDOWN; break; }
        double beta = rho_new / rho;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
done:
    for (int64_t i = 0; i < n; ++i) {
        double di = op->dis ? op->dis[i] : 1.0;
        x[i] = di * xh[i];
    }
    st->status = ret;
    st->n_apply = op->n_apply - apply0;
    free(bh);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* Lanczos                                                                   */
/* ------------------------------------------------------------------------ */

/* MurmurHash3 32-bit finaliser (fmix32). */
static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* v_i = fmix32(i) / 2^32 - 0.5, i = 0..n-1 (0-based row index, low 32 bits). */
void orc_fmix32_start(int64_t n, double *v)
{
    for (int64_t i = 0; i < n; ++i) v[i] = (double)fmix32((uint32_t)i) / 4294967296.0 - 0.5;
}

/*
 * m steps of Lanczos on op-hat from the fmix32 start vector, no
 * reorthogonalisation:
 *   v_1 = v / ||v||,  beta_0 v_0 = 0
 *   w = A v_j - beta_{j-1} v_{j-1};  alpha_j = v_j.w;  w -= alpha_j v_j
 *   beta_j = ||w||;  v_{j+1} = w / beta_j
 * Outputs alpha_1..alpha_m and beta_1..beta_m (beta_m couples T_m to the
 * next Lanczos vector).  Returns the number of steps done (< m on an exact
 * invariant subspace, beta_j == 0).
 */
int orc_lanczos(orc_op *op, int m, double *alpha, double *beta)
{
    int64_t n = op->n;
    double *v = (double *)malloc(sizeof(double) * (size_t)n * 3);
    if (!v) return -1;
    double *vprev = v + n, *w = v + 2 * n;
    orc_fmix32_start(n, v);
    double nv = sqrt(orc_dot(n, v, v));
    for (int64_t i = 0; i < n; ++i) { v[i] = v[i] / nv; vprev[i] = 0.0; }
    double bprev = 0.0;
    int done = 0;
    for (int j = 0; j < m; ++j) {
        orc_op_apply(op, v, w);
        for (int64_t i = 0; i < n; ++i) w[i] = w[i] - bprev * vprev[i];
        double a = orc_dot(n, v, w);
        for (int64_t i = 0; i < n; ++i) w[i] = w[i] - a * v[i];
        double b = sqrt(orc_dot(n, w, w));
        alpha[j] = a;
        beta[j] = b;
        done = j + 1;
        if (b == 0.0) break;
        for (int64_t i = 0; i < n; ++i) {
            vprev[i] = v[i];
            v[i] = w[i] / b;
        }
        bprev = b;
    }
    free(v);
    return done;
}
