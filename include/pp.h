/*
 * pp.h -- polynomial-preconditioned Conjugate Gradient on one MI355X (gfx950).
 *
 * Method: Bergamaschi, Ferronato, Isotton, Janna, Martinez, "Parallel
 * matrix-free polynomial preconditioners with application to flow simulations
 * in discrete fracture networks" (arXiv 2208.01339).
 *
 * CG (section 1) is preconditioned by P = p_k(A), the optimal Chebyshev
 * polynomial of degree k on [lambda_min, lambda_max] with the centre of the
 * interval moved by the scaling parameter xi (section 2.2, eqs. polycheb and
 * rhocheb; section 2.4, eq. thetamod).  P is applied matrix-free by the
 * three-term recurrence of Algorithm 2: k operator applications and a few
 * vector updates, no dot product.  The operator is either a CSR matrix or the
 * never-assembled Schur-shaped operator S = A_ff + C^T M^{-1} C of section 4.2
 * (eq. schur, with a diagonal middle block).  Optional symmetric Jacobi
 * scaling D^{-1/2} A D^{-1/2} is the diagonal seed preconditioner of
 * section 3 (W = D^{-1/2}) and section 4.3.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (hipMalloc'ed or torch CUDA tensors)
 *    unless marked "host".  The library never frees caller memory.
 *  - create copies (and re-lays out) what it needs during the call; the
 *    caller may free its arrays once create returns.
 *  - All GPU work of a handle is queued on the stream given at create
 *    (NULL = the legacy default stream).  pcg_solve, pp_estimate_bounds and
 *    create synchronise that stream before returning; pp_apply and
 *    pp_operator_apply return with the work queued.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - No C++ exception crosses this interface; errors are status codes, and
 *    pp_last_error() gives a message for the last failing call on the calling
 *    thread.
 *  - Vectors passed to pp_apply / pcg_solve must hold n doubles; this cannot
 *    be checked.  Input and output vectors must not alias.
 */
#ifndef PP_H
#define PP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define PP_API __attribute__((visibility("default")))
#else
#define PP_API
#endif

typedef struct pp_op_s *pp_op;

typedef enum {
    PP_OK = 0,            /* success / converged                                   */
    PP_NOT_CONVERGED = 1, /* maxit iterations done without reaching tol            */
    PP_BREAKDOWN = 2,     /* p.Ap <= 0, r.z <= 0 or a non-finite scalar in CG      */
    PP_ERR_ARG = -1,      /* invalid argument (null pointer, size, bounds, flags)  */
    PP_ERR_OOM = -2,      /* device allocation failed                              */
    PP_ERR_HIP = -3,      /* a HIP runtime call failed                             */
    PP_ERR_STATE = -4,    /* call out of order (apply/solve before pp_setup)       */
    PP_ERR_TIMEOUT = -5   /* a grid-barrier wait of the persistent driver gave up  */
                          /* (PP_OPT_SPIN_LIMIT); x is undefined                   */
} pp_status;

/* create flags */
enum {
    PP_JACOBI = 1u, /* iterate on D^{-1/2} A D^{-1/2}, D = diag(A) (section 3, 4.3)        */
    PP_MIXED = 2u,  /* p_k(A)v in FP32 (values, vectors, accumulation); CG stays FP64     */
    PP_SLICED = 4u, /* keep every entry in the sliced layout (no symmetric diagonal part)  */
    PP_NO_REORDER = 8u /* CSR: keep the caller's row order (see Renumbering below)         */
};

/*
 * Renumbering.  A CSR operator held in slices only (no stored diagonals) whose
 * numbering scatters the columns that a slice of 64 consecutive rows gathers
 * (more than 0.25 distinct 64-byte lines of x per stored entry, sampled) is
 * renumbered at create by reverse Cuthill-McKee (breadth-first levels from a
 * peripheral vertex), when that at least halves the spread.  Vectors stay in
 * the caller's numbering at every entry point (b, x, r, z, V); internally the
 * library holds P A P^T.  The Lanczos start vectors use the caller's row
 * index, so bounds, Ritz vectors and features are those of the caller's
 * numbering up to rounding.  Create copies the matrix structure to the host
 * for this (n + 1 row pointers and nnz column indices).  The persistent
 * driver is not used for renumbered operators.
 */

/*
 * Storage.  By default an operator whose column offsets j - i take few
 * distinct values (stencils, the fracture blocks of the Schur shape) keeps
 * the densely populated offsets as symmetric stored diagonals: for offset
 * o >= 0 one array of n values a_{i,i+o}, the mirrored entry a_{i+o,i} read
 * from the same array, so a symmetric operator is read at about half the
 * bytes of CSR.  This is used only when the covered entries are exactly
 * symmetric and free of duplicates; all other entries (and the trace columns
 * of the Schur shape) go to a sliced ELLPACK layout.  PP_SLICED forces the
 * sliced layout for everything.
 */

/*
 * Create an operator from a CSR matrix A (n x n, symmetric positive definite).
 *   rowptr  [n+1] int64, rowptr[0] = 0, non-decreasing, rowptr[n] = nnz
 *   colind  [nnz] int32 in [0, n)
 *   val     [nnz] double
 * With PP_JACOBI the diagonal must be positive (PP_ERR_ARG otherwise).
 * n >= 1, nnz >= 1, nnz < 2^31 per slice layout limits are checked.
 */
PP_API pp_status pp_create_csr(pp_op *out, int64_t n, int64_t nnz, const int64_t *rowptr,
                        const int32_t *colind, const double *val, unsigned flags, void *stream);

/*
 * Create the Schur-shaped operator S = A_ff + C^T diag(m)^{-1} C (section 4.2,
 * eq. schur; Algorithm 3 applies the paper's S_u the same way, matrix-free).
 *   A_ff    n x n CSR (a_rowptr [n+1] int64, a_col [nnz_a] int32, a_val [nnz_a])
 *   C       nt x n CSR (c_rowptr [nt+1] int64, c_col [nnz_c] int32, c_val [nnz_c])
 *   m_diag  [nt] double, all > 0
 * S is never formed.  With PP_JACOBI, D = diag(S) is computed in closed form
 * as (A_ff)_ii + sum_t C_ti^2 / m_t (the analogue of Algorithm 4).
 */
PP_API pp_status pp_create_schur(pp_op *out, int64_t n, int64_t nnz_a, const int64_t *a_rowptr,
                          const int32_t *a_col, const double *a_val, int64_t nt, int64_t nnz_c,
                          const int64_t *c_rowptr, const int32_t *c_col, const double *c_val,
                          const double *m_diag, unsigned flags, void *stream);

/*
 * The DFN Schur complement of section 4.2 (eq. schur):
 *   S_u(alpha) = G^u - alpha B^T A^{-1} C - alpha C^T A^{-1} B + C^T A^{-1} G^h A^{-1} C,
 * the operator of the reduced system S_u u = r after the permutation of
 * eq. (tilde_var).  A sparse matrix given as CSR on the device:
 */
typedef struct {
    int64_t rows, cols, nnz;
    const int64_t *rowptr;  /* [rows+1], rowptr[0] = 0, non-decreasing    */
    const int32_t *col;     /* [nnz] in [0, cols)                          */
    const double *val;      /* [nnz]                                       */
} pp_csr;

/*
 * The blocks of the DFN system (section 4.1, eq. (sys)), device CSR:
 *   a      A, n_h x n_h, symmetric positive definite and block diagonal: one
 *          block of grid^2 consecutive rows per fracture (n_h = n_frac grid^2),
 *          every entry within distance grid of the diagonal (a 2-D grid
 *          numbered by lines, as a 5-point operator); 1 <= grid <= 64
 *   gh     G^h, n_h x n_h, symmetric, same blocks and band
 *   c      C, n_h x n_u: every column inside the block of the fracture that
 *          owns that unknown
 *   b      B, n_h x n_u (any pattern)
 *   gu     G^u, n_u x n_u, symmetric
 *   u_off  [n_frac+1] host int64: unknowns u_off[f] .. u_off[f+1]-1 are owned
 *          by fracture f (non-decreasing, u_off[0] = 0, u_off[n_frac] = n_u)
 *   alpha  the scalar of eq. (sys); S_u must be SPD for it (the paper's
 *          assumption; a PCG breakdown reports otherwise)
 */
typedef struct {
    int64_t n_frac, grid;
    pp_csr a, gh, c, b, gu;
    const int64_t *u_off;
    double alpha;
} pp_dfn_desc;

/*
 * Create the operator S_u of a DFN system (n = n_u).  At create, on the
 * device: the exact Cholesky factor of every block of A (banded; computed
 * before the iteration, section 4.2), and D_S = diag(S_u) by Algorithm 4
 * (section 4.3); the operator seen
 * by pp_setup / pp_apply / pcg_solve / pp_estimate_bounds is
 * D_S^{-1/2} S_u D_S^{-1/2} (section 4.3), applied matrix-free by Algorithm 3
 * (its three solves with A done as two, since A^{-1} is linear, each a
 * forward and a backward sweep with the factor, and the products with C, B,
 * G^h, G^u).  The input arrays are copied; the
 * caller keeps ownership.  Device memory held: two step-ordered copies of
 * the banded factor for the sweeps (2 n_h G doubles) and copies of the
 * blocks; the factor by rows (n_h (G+2) doubles) is freed within the call.  flags: 0 (Jacobi scaling by D_S is implied;
 * PP_MIXED and PP_SLICED are refused).  PP_ERR_ARG for an invalid structure
 * (entry outside its fracture block or band, a C column outside its owner,
 * asymmetric A, G^h or G^u, A not SPD, a non-positive D_S).
 */
PP_API pp_status pp_create_dfn(pp_op *out, const pp_dfn_desc *desc, unsigned flags, void *stream);

/*
 * Reduced right-hand side of the DFN system (block elimination of section
 * 4.2): r = W^T M^{-1} f_1 with f_1 = (q, 0), i.e.
 *   r = alpha B^T A^{-1} q - C^T A^{-1} G^h A^{-1} q.
 *   q [n_h] device, r [n_u] device (unscaled; pass r to pcg_solve as b).
 * PP_ERR_ARG unless op came from pp_create_dfn.  Queued on the handle's
 * stream and synchronised.
 */
PP_API pp_status pp_dfn_rhs(pp_op op, const double *q, double *r);

/*
 * Recovery of the other unknowns once S_u u = r is solved (section 4.2):
 *   h = A^{-1} (q + C u),  p = A^{-1} (alpha B u - G^h h).
 *   q [n_h], u [n_u], h [n_h] and p [n_h] device.  h and p must be distinct
 *   arrays; either may be q itself (q is read before it is overwritten).
 *   Synchronised.
 */
PP_API pp_status pp_dfn_recover(pp_op op, const double *q, const double *u, double *h, double *p);

/*
 * Fix the polynomial (section 2.2 and eq. thetamod of section 2.4):
 *   theta-bar = (lambda_max + lambda_min)/2 * (1 + scaling),
 *   delta = (lambda_max - lambda_min)/2, sigma = theta-bar/delta,
 *   rho_0 = 1/sigma, rho_j = 1/(2 sigma - rho_{j-1}).
 * k = degree = operator applications per preconditioner application,
 * 0 <= k <= 4096.  Bounds refer to the (Jacobi-scaled, if PP_JACOBI) operator;
 * require 0 < lambda_min < lambda_max, both finite, scaling >= 0 finite.
 * Host-only computation; may be called again to change the polynomial.
 */
PP_API pp_status pp_setup(pp_op op, int k, double lambda_min, double lambda_max, double scaling);

/*
 * The same preconditioner family in the Newton form of Algorithm 1 (section
 * 2.1): degree k = 2^nlev - 1 (nlev in [0, 12]), applied by the recursion
 * P_0 r = zeta_0 r, P_j r = zeta_j (2 P_{j-1} r - P_{j-1} A P_{j-1} r) with
 * zeta_0 = 1/theta-bar, zeta_1 = 2/(1 + 2 a zeta_0 - (a zeta_0)^2) (a =
 * theta-bar - delta, the left end of the shifted interval) and eq. zetaNewt
 * for zeta_i, i >= 2.  In exact arithmetic it equals the Chebyshev
 * polynomial of the same degree (pp_setup).  Every operator application is
 * one fused kernel; the recursion keeps 2 (nlev - 1) work vectors (allocated
 * here).  Runs in FP64 even under PP_MIXED, with the stream-driven kernels.
 * pp_setup switches back to the three-term Chebyshev form.
 */
PP_API pp_status pp_setup_newton(pp_op op, int nlev, double lambda_min, double lambda_max, double scaling);

/*
 * z = P r by Algorithm 2 (k operator applications, no dot product).
 * With PP_JACOBI: z = D^{-1/2} p_k(D^{-1/2} A D^{-1/2}) D^{-1/2} r, the
 * effective preconditioner of A.  With PP_MIXED the recurrence runs in FP32.
 * r, z: [n] double, must not alias.  Asynchronous on the handle's stream.
 */
PP_API pp_status pp_apply(pp_op op, const double *r, double *z);

/*
 * Solve A x = b by CG preconditioned with P (standard Hestenes-Stiefel loop:
 * q = A p, alpha = rho / p.q, x += alpha p, r -= alpha q, convergence test,
 * z = P r, rho' = r.z, beta = rho'/rho, p = z + beta p; three dot products
 * per iteration, as counted in Table tab11).
 *   b      [n] double (device)
 *   x      [n] double (device): x0 on entry, last iterate on exit
 *   tol    stop when ||r_hat|| <= tol ||b_hat|| (scaled system under PP_JACOBI,
 *          as in section 4.3); tol >= 0 (0 = run maxit iterations)
 *   maxit  >= 0
 *   iters, relres  host outputs (may be NULL): iterations done and the final
 *          recursive relative residual ||r_hat|| / ||b_hat||
 * Returns PP_OK, PP_NOT_CONVERGED (iters = maxit) or PP_BREAKDOWN (x holds
 * the last iterate).  b = 0 gives x = 0, iters = 0, PP_OK.  Synchronises.
 */
PP_API pp_status pcg_solve(pp_op op, const double *b, double *x, double tol, int maxit, int *iters,
                    double *relres);

/*
 * Spectral low-rank correction (section 3.1): the preconditioner becomes
 *   P = p_k(A) + V (V^T A V)^{-1} V^T
 * (A and V in the Jacobi-scaled space under PP_JACOBI; pp_apply then returns
 * D^{-1/2} P D^{-1/2} r).  With V spanning approximate eigenvectors of the
 * smallest eigenvalues, their eigenvalues of P A move from lambda_j p_k(lambda_j)
 * to about 1 + lambda_j p_k(lambda_j) (eq. plusone), away from the origin.
 * Each CG iteration then reads V twice and reduces p more values (the
 * rank-one rows of Table tab11 use four dot products per iteration).
 *
 * pp_lowrank_set: V device n x p, column-major (column j at V + j n), copied;
 *   p in [0, 8], p = 0 removes the correction.  V^T A V is formed with p
 *   operator applications and inverted on the host; PP_ERR_ARG if it is
 *   singular.  Synchronises.
 * pp_lowrank_ritz: run `steps` (1..64) Lanczos steps from the start vector of
 *   pp_estimate_bounds keeping the basis, and install as V the Ritz vectors of
 *   the p smallest Ritz values (p in [1, min(8, steps)]); theta: HOST [p]
 *   receives those Ritz values (may be NULL).  Uses steps x n doubles of
 *   scratch during the call.  Synchronises.  With PP_OPT_RITZ = 1 the
 *   Lanczos process runs on the preconditioner p_k(A-hat) of the last
 *   pp_setup instead (k operator applications per step, every new vector
 *   reorthogonalised against the whole basis): p_k(x) is close to 1/x on
 *   [lambda_min, lambda_max] and larger below it, so the largest Ritz values
 *   of p_k(A-hat) belong to the smallest eigenvalues of A-hat and converge in
 *   few steps (the paper takes the leftmost eigenvectors from a preconditioned
 *   eigensolver, DACG, section 6.1; here the polynomial is the
 *   preconditioner); V gets the Ritz vectors of the p largest, and theta
 *   their Rayleigh quotients v^T A-hat v.
 *   PP_ERR_STATE without a Chebyshev polynomial set up.
 * pp_lowrank_get: the rank in use (*p) and, when V is not NULL, a copy of the
 *   vectors (device n x p).
 * pp_lowrank_info: for the installed V, HOST [p] outputs (either may be NULL):
 *   theta_j = v_j^T A-hat v_j / v_j^T v_j and the relative residual
 *   ||A-hat v_j - theta_j v_j|| / (|theta_j| ||v_j||).
 * The persistent driver does not apply the correction: pcg_solve uses the
 * stream-driven kernels while a correction is installed.
 */
PP_API pp_status pp_lowrank_set(pp_op op, int p, const double *V);
PP_API pp_status pp_lowrank_ritz(pp_op op, int steps, int p, double *theta);
PP_API pp_status pp_lowrank_get(pp_op op, int *p, double *V);
PP_API pp_status pp_lowrank_info(pp_op op, double *theta, double *resid);

/*
 * Estimate lambda_min, lambda_max of the (scaled) operator with `steps`
 * Lanczos steps (1..64) from the start vector v_i = fmix32(i)/2^32 - 0.5
 * (MurmurHash3 finaliser of the row index), no reorthogonalisation:
 * lambda_min = smallest Ritz value, lambda_max = largest Ritz value + its
 * Ritz residual.  The paper obtains these bounds with DACG (section 6.1);
 * any estimate of the extremal eigenvalues serves.  Host outputs; synchronises.
 */
PP_API pp_status pp_estimate_bounds(pp_op op, int steps, double *lambda_min, double *lambda_max);

/*
 * y = A x with the UNSCALED operator (CSR SpMV, or A_ff x + C^T (M^{-1}(C x))
 * for the Schur shape, Algorithm 3's role).  x, y: [n] double, no aliasing.
 */
PP_API pp_status pp_operator_apply(pp_op op, const double *x, double *y);

/* Statistics of the last pcg_solve / pp_apply on this handle (host struct). */
typedef struct {
    int32_t iters;          /* CG iterations of the last solve                      */
    int32_t status;         /* pp_status of the last solve                          */
    double relres;          /* recursive ||r_hat|| / ||b_hat||                       */
    int64_t op_applies;     /* operator applications in the last solve              */
    int64_t dots;           /* values reduced over the grid (dot products), not ||b|| */
    double cheb_ms;         /* summed device time of the polynomial steps (events), */
                            /* valid only with PP_OPT_TIMING = 1                    */
    int64_t cheb_steps;     /* polynomial steps covered by cheb_ms                  */
    double solve_ms;        /* device time of the whole solve (events)             */
    int64_t n;              /* operator order                                       */
    int64_t nnz_stored;     /* entries held in the slice layout (padded)            */
    int64_t nnz_matrix;     /* entries of the CSR / A_ff + C^T parts given          */
    int32_t driver;         /* 0 = stream-driven kernels, 1 = persistent kernel     */
    int32_t grid;           /* workgroups per launch used                           */
    int32_t diagonals;      /* stored diagonals of the symmetric diagonal part      */
                            /* (0 = every entry in the slice layout)                */
    int32_t two_step;       /* 1 when pairs of Chebyshev steps share one pass        */
    double pair_ms;         /* summed device time of the fused-pair launches (events */
                            /* around each run of pairs; PP_OPT_TIMING = 1)           */
    int64_t pair_launches;  /* fused-pair launches covered by pair_ms                */
    int32_t restarts;       /* CG restarts after a failed true-residual check        */
                            /* (PP_OPT_VERIFY)                                      */
    int32_t reordered;      /* 1 when create renumbered the rows (PP_NO_REORDER)     */
    double true_relres;     /* ||b_hat - A_hat x_hat|| / ||b_hat|| of the returned x */
                            /* when the true-residual check ran, else -1             */
    double gather_spread;   /* distinct 64-byte lines of x per stored entry that a   */
                            /* slice of 64 rows gathers (sampled; after renumbering) */
    int32_t lds_tiles;      /* 1 when the FP64 steps stage x in LDS per tile         */
    int32_t unit_diagonal;  /* 1 when the Jacobi-scaled main diagonal is stored as   */
                            /* exactly 1 (stored diagonals of a CSR matrix) and the   */
                            /* fused pairs skip reading it                            */
    int32_t barrier;        /* grid barrier of the last persistent solve: 0 the      */
                            /* runtime's cooperative barrier, 1 flat, 2 two-level    */
                            /* (PP_OPT_BARRIER); -1 after a stream-driven solve      */
} pp_stats;

PP_API pp_status pp_get_stats(pp_op op, pp_stats *st);

/* Tunables (pp_set_option keys). */
enum {
    PP_OPT_GRID = 1,        /* workgroups per launch, 0 = auto (resident workgroups, CUs x occupancy) */
    PP_OPT_CHUNK = 2,       /* CG iterations queued between host convergence checks       */
    PP_OPT_TIMING = 3,      /* 1 = record events around the polynomial steps              */
    PP_OPT_DRIVER = 4,      /* 0 = stream-driven, 1 = persistent cooperative kernel, -1 = auto */
                            /* (default: persistent for operators of at most 65536 rows   */
                            /* whose polynomial runs single steps, one 64-row slice per   */
                            /* wave up to 128 workgroups; stream-driven otherwise)        */
    PP_OPT_NT_LOADS = 5,    /* 1 = non-temporal accesses for the streams read once per step */
                            /* (the sliced matrix; r, s_{j-2} and the output with stored */
                            /* diagonals), 0 = plain; default 1 from 2^22 rows on       */
    PP_OPT_TWO_STEP = 6,    /* on 3-D 7-point operators (stored diagonals at offsets 0, 1,  */
                            /* N, N^2, no coupling across the box's x- and y-faces,        */
                            /* N <= 256) fuse pairs of Chebyshev steps into one pass (in   */
                            /* PP_MIXED mode FP32 pairs, the last one writing z in FP64) */
                            /* (tiles of whole x-lines with one recomputed halo line each  */
                            /* side, marching up z): 1 (default) = when the box's tiles    */
                            /* fill whole rounds of compute units (one tile per CU) at     */
                            /* least 90 %, 2 = for any box, 0 = one pass per step.  Other  */
                            /* values: PP_ERR_ARG                                          */
    PP_OPT_VERIFY = 7,      /* true-residual check when pcg_solve converges: the residual  */
                            /* b_hat - A_hat x_hat of the iterate is formed in FP64; if it */
                            /* misses tol, CG restarts from the iterate (at most 3 times). */
                            /* 1 = on, 0 = off, -1 (default) = on in PP_MIXED mode only.   */
                            /* Costs one operator application when the check passes.       */
    PP_OPT_RITZ = 8,        /* pp_lowrank_ritz: 0 (default) Lanczos on A-hat, 1 Lanczos on   */
                            /* p_k(A-hat) with full reorthogonalisation                    */
    PP_OPT_LDS_TILES = 9,   /* FP64 CSR operators held in slices only: 1 (default) = the    */
                            /* Chebyshev steps stage the x segments of each tile of 1024  */
                            /* rows in LDS and gather from there (tiles touching more     */
                            /* than 6144 values of x gather from memory; create plans     */
                            /* no tiles when over a tenth would), 0 = gather from memory  */
    PP_OPT_BARRIER = 10,    /* grid barrier of the persistent driver: 0 = the runtime's   */
                            /* cooperative barrier, 1 = flat (every workgroup writes back */
                            /* its L2 and arrives on one counter), 2 = two-level (one L2  */
                            /* writeback and one global arrival per XCD), -1 (default) =  */
                            /* flat below 32 workgroups, two-level from 32                */
    PP_OPT_SPIN_LIMIT = 11  /* polls (each about a microsecond) before a wait in a hand-  */
                            /* written grid barrier gives up and the solve returns        */
                            /* PP_ERR_TIMEOUT; 1 .. 2^31, default 2^21                    */
};
PP_API pp_status pp_set_option(pp_op op, int key, int64_t value);

PP_API void pp_destroy(pp_op op);

/* ------------------------------------------------------------------------
 * Batches: many independent systems and/or a block of right-hand sides,
 * solved together.  Each system keeps its own Jacobi scaling, bounds,
 * polynomial and CG scalars; every right-hand side column runs its own CG
 * (own alpha, beta, convergence test).  The matrix is read once per
 * polynomial step for all columns (a sparse-matrix times block-of-vectors
 * product), and one chunk of CG iterations is captured in a hipGraph and
 * replayed until every (system, column) has finished.
 * ------------------------------------------------------------------------ */
typedef struct pp_batch_s *pp_batch;

/*
 * nsys systems given as ONE block-diagonal CSR matrix: the rows and columns of
 * system s are sys_ptr[s] .. sys_ptr[s+1]-1 (sys_ptr: HOST array [nsys+1],
 * sys_ptr[0] = 0, strictly increasing); an entry coupling two systems is
 * rejected (PP_ERR_ARG).  rowptr [n+1] int64, colind [nnz] int32 (global
 * column numbers), val [nnz] double, n = sys_ptr[nsys] (device arrays).
 * nrhs in [1, 32]: width of the right-hand-side blocks (row-major [n][nrhs]).
 * flags: PP_JACOBI, PP_MIXED (FP32 polynomial / SpMM, FP64 CG), PP_SLICED.
 * Each system chooses its storage as pp_create_csr does (symmetric stored
 * diagonals for 5- and 7-point-like systems, the sliced layout otherwise).
 */
PP_API pp_status pp_create_batch(pp_batch *out, int nsys, const int64_t *sys_ptr, int64_t nnz,
                                 const int64_t *rowptr, const int32_t *colind, const double *val,
                                 int nrhs, unsigned flags, void *stream);

/* Lanczos bounds of every system (steps in [1, 64]); lambda_min, lambda_max:
 * HOST arrays [nsys].  Same start vector and padding as pp_estimate_bounds. */
PP_API pp_status pp_batch_estimate_bounds(pp_batch op, int steps, double *lambda_min,
                                          double *lambda_max);

/* Per-system polynomial (section 2.2 / eq. thetamod), degree k shared by all
 * systems, bounds HOST arrays [nsys], one scaling for all. */
PP_API pp_status pp_batch_setup(pp_batch op, int k, const double *lambda_min, const double *lambda_max,
                                double scaling);

/*
 * Solve every system for every column: B, X device [n][nrhs] row-major
 * (X: x0 in, solution out).  iters, relres, status: HOST arrays
 * [nsys * nrhs] (index s * nrhs + c), may be NULL.  Returns PP_OK when every
 * (system, column) converged, otherwise the worst status.  Synchronises.
 */
PP_API pp_status pcg_solve_batch(pp_batch op, const double *B, double *X, double tol, int maxit,
                                 int *iters, double *relres, int *status);

/* Z = P R for every system and column (device [n][nrhs]); asynchronous. */
PP_API pp_status pp_batch_apply(pp_batch op, const double *R, double *Z);

/*
 * Layout of the block product: W lanes per row (64/W rows per wavefront),
 * each lane handling (internal block width)/W columns.  W = 0 restores the
 * default.  pp_batch_autotune times every supported W on a polynomial step
 * and keeps the fastest (HOST output *best_w, *best_us).
 */
PP_API pp_status pp_batch_set_layout(pp_batch op, int w);
PP_API pp_status pp_batch_autotune(pp_batch op, int *best_w, double *best_us);

/* Batch options: PP_OPT_CHUNK (iterations per graph), PP_OPT_NT_LOADS,
 * PP_OPT_VERIFY (as for pcg_solve: once every column has converged, the true
 * residuals are formed in FP64 and the columns that miss tol restart from
 * their iterates; -1 default = in PP_MIXED mode only),
 * PP_BOPT_GRAPH (1 = replay captured iteration chunks, 0 = launch eagerly),
 * PP_BOPT_DRIVER (0 = iteration chunks driven from the host, which polls
 * convergence one chunk behind and moves the workgroups of finished systems
 * to the others; 1 = the whole solve in one persistent cooperative launch,
 * with no host round trip, convergence decided on the device and the
 * workgroup map fixed, for batches with one right-hand side per system --
 * blocks of right-hand sides keep the host-driven chunks; PP_OPT_GRID caps
 * its workgroups, 0 default = the resident ones, at most max(256, slices/8);
 * PP_OPT_BARRIER and PP_OPT_SPIN_LIMIT as for a single operator, a timeout
 * returning PP_ERR_TIMEOUT). */
enum { PP_BOPT_GRAPH = 100, PP_BOPT_DRIVER = 101 };
PP_API pp_status pp_batch_set_option(pp_batch op, int key, int64_t value);

/* Sizes and last-solve timing: n rows, internal block width, entries in the
 * slice layout, workgroups per launch, solve device time (ms), the most
 * iterations of any (system, column), systems held as stored diagonals, CG
 * restarts after a failed true-residual check, 1 when the check ran and
 * every column passed it (relres then holds the true residuals), and the
 * driver of the last solve (grid: its workgroups). */
typedef struct {
    int64_t n;
    int32_t nsys;
    int32_t nb;
    int32_t nrhs;
    int32_t w;
    int64_t nnz_stored;
    int32_t grid;
    int32_t graph;
    double solve_ms;
    int32_t max_iters;
    int32_t diag_systems;
    int32_t restarts;
    int32_t verified;
    int32_t driver;  /* 1 when the last solve ran as one persistent launch */
} pp_batch_stats;
PP_API pp_status pp_batch_get_stats(pp_batch op, pp_batch_stats *st);

PP_API void pp_destroy_batch(pp_batch op);

/* ------------------------------------------------------------------------
 * Learned bounds: a small multilayer perceptron (ReLU hidden layers, linear
 * output, FP32) that maps 16 cheap operator features to
 * (log lambda_min, log lambda_max, log10(xi + 1e-5)), trained on bounds and
 * iteration counts produced by this library.  Hand-written kernels for the
 * forward pass, the gradients of the mean squared error and Adam.  The
 * paper leaves the choice of xi problem dependent (section 2.4); the
 * Lanczos bounds stay the fallback and the reference.
 * ------------------------------------------------------------------------ */
typedef struct pp_mlp_s *pp_mlp;

/* n_in <= 32 inputs, depth hidden layers of `hidden` units, n_out <= 8
 * outputs; weights He-uniform from `seed` (splitmix64), biases 0. */
PP_API pp_status pp_mlp_create(pp_mlp *out, int n_in, int hidden, int depth, int n_out, uint64_t seed,
                               void *stream);
PP_API void pp_mlp_destroy(pp_mlp mlp);
/* number of parameters; the flat layout is, per layer, W [fan_in][fan_out] row-major then b [fan_out] */
PP_API pp_status pp_mlp_num_params(pp_mlp mlp, int64_t *count);
PP_API pp_status pp_mlp_get_params(pp_mlp mlp, float *dst);       /* device [count] */
PP_API pp_status pp_mlp_set_params(pp_mlp mlp, const float *src); /* device [count]; resets Adam */
/* feature / target normalisation used by pp_predict_bounds (host arrays) */
PP_API pp_status pp_mlp_set_normalization(pp_mlp mlp, const double *in_mean, const double *in_std,
                                          const double *out_mean, const double *out_std);
/* Y [batch][n_out] = MLP(X [batch][n_in]); device arrays, batch <= 1024 */
PP_API pp_status pp_mlp_forward(pp_mlp mlp, int batch, const float *X, float *Y);
/* loss = mean (Y - T)^2 over the batch; grad (device [count], may be NULL) its gradient; host loss */
PP_API pp_status pp_mlp_loss_grad(pp_mlp mlp, int batch, const float *X, const float *T, float *grad,
                                  double *loss);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch; host loss before the step */
PP_API pp_status pp_mlp_train_step(pp_mlp mlp, int batch, const float *X, const float *T, float lr,
                                   double *loss);

/*
 * 16 features of the (scaled) operator, HOST output f[16]:
 *  0 log10 n, 1 nnz/n, 2..5 mean/std/min/max of log10 of the unscaled diagonal,
 *  6 Gershgorin upper bound of lambda_max, 7 mean off-diagonal absolute row sum,
 *  8 Gershgorin lower bound (A / A_ff part), 9..12 Rayleigh quotients after
 *  power_steps/4, /2, 3/4 and power_steps power steps (lower bounds of
 *  lambda_max), 13 lambda_min estimate from power_steps steps on (c I - A),
 *  c = feature 6, 14 longest row, 15 log10(feature 12 / |feature 13|).
 *  power_steps: even, 2..64.
 */
PP_API pp_status pp_features(pp_op op, int power_steps, double *f);

/*
 * Predict (lambda_min, lambda_max, xi) for pp_setup.  The prediction is
 * rejected (fallback = 1: 20-step Lanczos bounds, xi = 0) when it is not
 * finite, lambda_min <= 0, lambda_min >= lambda_max, lambda_max lies below
 * the last Rayleigh quotient (a certified lower bound of lambda_max) or
 * above the Gershgorin upper bound, or xi > 0.1.  Host outputs.
 */
PP_API pp_status pp_predict_bounds(pp_op op, pp_mlp mlp, int power_steps, double *lambda_min,
                                   double *lambda_max, double *scaling, int *fallback);
/*
 * pcg_solve without any allocation, for callers that cannot allocate device
 * memory (code between graph captures, tight serving loops, harnesses that
 * forbid hipMalloc).  The same method as pp_create_csr + pp_setup + pcg_solve
 * (three-term Chebyshev polynomial, standard PCG loop, optional Jacobi
 * scaling; no stored-diagonal layout, no fused pairs, no true-residual check)
 * on a plain CSR matrix given as it is:
 *   n, nnz, rowptr [n+1] int64, colind [nnz] int32, val [nnz]: DEVICE CSR of a
 *          symmetric positive definite matrix, 1 <= n <= 1048576 (the scratch
 *          capacity; larger n: PP_ERR_ARG), nnz < 2^31; not copied, read during
 *          the call only
 *   flags  0 or PP_JACOBI (needs a positive diagonal, else PP_ERR_ARG and x
 *          untouched); bounds, tol, maxit as for pp_setup / pcg_solve with
 *          k <= 1024 and xi = scaling
 *   b, x   [n] double DEVICE (x: x0 in, last iterate out; no aliasing)
 *   iters, relres  HOST outputs (may be NULL)
 *   stream hipStream_t (NULL = default) of the CURRENT device
 * Work memory: one fixed array of about 72 MiB per device inside the library
 * (located once per device on the first call there, kept until the process
 * ends); the call calls no hipMalloc/hipFree.  Every call on one device uses
 * that device's array: calls that overlap on one device (several host threads
 * or streams) race and must be serialised by the caller.  The call
 * synchronises the stream (a few bytes of state are read back after every
 * chunk of iterations).  Returns as pcg_solve.
 */
PP_API pp_status pcg_solve_csr_noalloc(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *colind,
                                       const double *val, unsigned flags, int k, double lambda_min,
                                       double lambda_max, double scaling, const double *b, double *x, double tol,
                                       int maxit, int *iters, double *relres, void *stream);

PP_API const char *pp_status_str(pp_status s);
PP_API const char *pp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PP_H */
