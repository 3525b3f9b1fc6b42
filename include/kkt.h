/*
 * libkkt -- Newton-step KKT solves for dynamic nonlinear programs on one MI355X.
 *
 * The interior-point method of Pacaud & Shin (arXiv 2403.15913) needs, at every
 * iteration, the solution of the condensed KKT system (eq. (kkt:condensed)).
 * This library provides its two hybrid forms:
 *
 *   Lifted-KKT (section "Solution 1: Lifted-KKT", eq. (liftedkkt)): every
 *     constraint is relaxed to an inequality, the condensed matrix
 *         K = W + diag(Sigma_x) + J^T diag(Sigma_s) J
 *     is symmetric positive definite and K x = b is solved by sparse Cholesky
 *     followed by Richardson iterative refinement (section "Hybrid linear
 *     solver").
 *   HyKKT (section "Solution 2: HyKKT", eqs. (hykkt) and (schurcomp)):
 *         K_gamma = W + diag(Sigma_x) + gamma J^T J
 *     is factored by sparse Cholesky and
 *         [[W + Sigma_x, J^T], [J, 0]] [dx; dy] = [f; g]
 *     is solved by conjugate gradient on the Schur complement
 *     S_gamma = J K_gamma^{-1} J^T, applied matrix-free.
 *
 * The pattern of K is fixed across interior-point iterations, so the symbolic
 * analysis (ordering, elimination tree, supernodes) runs once per pattern and
 * is reused by every refactorisation (section "Hybrid linear solver").
 *
 * Notation (paper -> library): the Hessian W_k -> W; the Jacobian of the
 * relaxed constraints H_k (Lifted-KKT) or of the equality constraints G_k
 * (HyKKT) -> J; the slack diagonal D_s = S^{-1} V -> Sigma_s; the primal
 * regularisation delta_x I plus bound terms -> Sigma_x.
 *
 * Conventions shared by every entry point:
 *   - Index arrays (patterns) are HOST memory, 0-based int32 CSR, read during
 *     the call only. W is given by its lower triangle (col <= row), every row
 *     with strictly ascending columns; J is m x n with strictly ascending
 *     columns in each row. The diagonal of K is always part of its pattern.
 *   - Value, Sigma, right-hand-side and solution arrays are DEVICE pointers
 *     (FP64) in the entry order fixed by the pattern. The caller owns them and
 *     must keep inputs alive until the stream has passed the call.
 *   - The library owns the symbolic objects, factors and all workspaces.
 *   - Calls that take a `stream` (a hipStream_t; NULL = the default stream)
 *     enqueue their work on it. kkt_refactor, kkt_matvec, and kkt_solve /
 *     kkt_cg_schur with info == NULL return without waiting for the device
 *     (their loop decisions are taken on the device; see each entry point).
 *     kkt_solve / kkt_cg_schur with a non-NULL info, kkt_status_sync and the
 *     batched solve synchronise the stream. Inputs must be complete on the
 *     device, in stream order, when the work enqueued on `stream` reads them.
 *   - No exception crosses the ABI. Host-side validation errors return at
 *     once; errors found on the device (a non-positive pivot, non-finite
 *     values) are latched in the factor and returned by the next
 *     synchronising call.
 *   - The right-hand-side sign is positive (K x = b); a caller holding the
 *     paper's -r negates it.
 *   - A symbolic object is immutable and may be shared between factors and
 *     threads; a factor is used by one host thread / stream at a time.
 */
#ifndef KKT_H
#define KKT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kkt_status;
#define KKT_OK 0
#define KKT_ERR_INVALID_ARG 1   /* NULL pointer, negative size, bad option */
#define KKT_ERR_PATTERN 2       /* malformed CSR, duplicate entries, unsupported front size */
#define KKT_ERR_STATE 3         /* call not valid in the object's state (e.g. solve on a failed factor) */
#define KKT_ERR_NOT_SPD 4       /* a pivot of K (or K_gamma) was not positive */
#define KKT_ERR_NONFINITE 5     /* NaN or Inf in the values */
#define KKT_ERR_NOT_CONVERGED 6 /* refinement or CG reached its iteration limit */
#define KKT_ERR_BREAKDOWN 7     /* CG found p^T S p <= 0 (J rank deficient or K_gamma not SPD) */
#define KKT_ERR_OOM 8           /* device allocation failed */
#define KKT_ERR_BUDGET 9        /* request does not fit the server's memory budget */
#define KKT_ERR_DEVICE 10       /* HIP runtime error */

#define KKT_ORDER_AUTO 0
#define KKT_ORDER_NATURAL 1
#define KKT_ORDER_ND 2

typedef struct kkt_options {
    int32_t ordering;      /* KKT_ORDER_*; AUTO picks nested dissection for large patterns */
    int32_t nd_leaf;       /* nested dissection stops splitting parts of at most this many variables (0: auto) */
    int32_t max_super;     /* widest supernode in columns (0: 96) */
    int32_t relax_small;   /* supernodes up to this width always amalgamate (0: 16, <0: none) */
    double relax_frac;     /* amalgamation may add up to this fraction of explicit zeros (<0: 0.5) */
    int32_t front_lds_max; /* LDS bytes one front panel may use (0 or more than 158 KiB: 158 KiB; less
                              than 4 KiB: 4 KiB). A front too tall to fit at one column is a large
                              front: at most 64 columns, assembled, factored and solved in place in HBM
                              by several workgroups per front (its update matrix by one wave per
                              tile); level schedule only, INVALID_ARG if negative */
} kkt_options;

typedef struct kkt_symbolic_stats {
    int32_t n, m;
    int32_t nsuper;        /* supernodes */
    int32_t levels;        /* depth of the supernode tree */
    int32_t max_rows;      /* largest front (rows) */
    int32_t max_cols;      /* widest supernode */
    int64_t nnz_k;         /* entries of the lower triangle of K */
    int64_t nnz_l;         /* stored entries of L (dense supernode panels, diagonal included) */
    int64_t nnz_l_exact;   /* entries of the exact Cholesky structure, diagonal included */
    int64_t n_pairs;       /* J^T J contribution products per assembly */
    double flops;          /* dense front work of one factorisation */
    double flops_exact;    /* sum over columns of (column count)^2 */
    double analyze_seconds;
    int32_t large_fronts;  /* fronts factored and solved in HBM (see kkt_options.front_lds_max) */
} kkt_symbolic_stats;

typedef struct kkt_refine_opts {
    int32_t max_iter;      /* Richardson corrections after the first solve (default 10) */
    double tol;            /* stop when the componentwise backward error omega <= tol (default 1e-14) */
} kkt_refine_opts;

typedef struct kkt_solve_info {
    int32_t status;        /* KKT_OK, KKT_ERR_NOT_SPD (factor failed), KKT_ERR_NOT_CONVERGED */
    int32_t iters;         /* corrections applied */
    double eta;            /* normwise backward error ||b-Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf) */
    double omega;          /* componentwise backward error max_i |b-Kx|_i / (|K||x|+|b|)_i */
    double relres;         /* ||b-Kx||_inf / ||b||_inf */
} kkt_solve_info;

typedef struct kkt_cg_opts {
    double tol;            /* stop when the recurrence residual ||r||_2 <= tol ||c||_2 (default 1e-10) */
    int32_t maxit;         /* iteration limit (default 200) */
    double eta_tol;        /* > 0: also stop once a bound on the saddle system's normwise backward
                              error is <= eta_tol (default 0: off); see kkt_cg_schur */
} kkt_cg_opts;

typedef struct kkt_cg_info {
    int32_t status;        /* KKT_OK, KKT_ERR_NOT_CONVERGED, KKT_ERR_BREAKDOWN, KKT_ERR_NOT_SPD */
    int32_t iters;         /* CG iterations */
    double rel_res;        /* recurrence residual ||r||_2 / ||c||_2 at exit */
    double eta;            /* normwise backward error of (dx, dy) on [[W + Sx, J^T], [J, 0]]:
                              ||res||_inf / (||A||_inf ||(dx, dy)||_inf + ||(f, g)||_inf) */
    int32_t eta_stop;      /* 1: stopped by the eta bound (eta_tol), 0: by tol, maxit or a breakdown */
} kkt_cg_info;

typedef struct kkt_inertia_opts {
    double delta_first;      /* first trial delta when none succeeded before (default 1e-4) */
    double delta_min;        /* smallest starting delta after a success (default 1e-20) */
    double delta_max;        /* give up above this delta (default 1e40) */
    double kappa_minus;      /* after a success the next call starts at kappa_minus * delta_last (default 1/3) */
    double kappa_plus;       /* growth factor after a failed trial (default 8) */
    double kappa_plus_first; /* growth factor while no delta has succeeded yet (default 100) */
} kkt_inertia_opts;

typedef struct kkt_inertia_info {
    int32_t status;          /* KKT_OK, KKT_ERR_NOT_SPD (delta_max exceeded), KKT_ERR_NONFINITE */
    int32_t trials;          /* factorizations run (the first with delta = 0) */
    double delta;            /* the accepted delta (0 when K was definite as given) */
} kkt_inertia_info;

typedef struct kkt_aug_info {
    int32_t status;          /* KKT_OK or KKT_ERR_NOT_CONVERGED (omega > tol at exit) */
    int32_t iters;           /* corrections on the full system */
    double eta;              /* normwise backward error on the augmented system */
    double omega;            /* componentwise backward error on the augmented system */
    int32_t inner_iters;     /* refinement corrections of the first condensed solve */
} kkt_aug_info;

typedef struct kkt_factor_info {
    int32_t status;        /* KKT_OK, KKT_ERR_NOT_SPD, KKT_ERR_NONFINITE */
    int32_t bad_col;       /* original index of the first failing pivot in elimination order, else -1 */
} kkt_factor_info;

typedef struct kkt_symbolic kkt_symbolic;
typedef struct kkt_factor kkt_factor;
typedef struct kkt_batch kkt_batch;
typedef struct kkt_server kkt_server;

/* Fills *opt with the defaults. */
void kkt_options_default(kkt_options* opt);

/* Human-readable name of a status code (static string). */
const char* kkt_status_string(kkt_status s);

/* Message of the last error raised on the calling thread (static per thread). */
const char* kkt_last_error(void);

/*
 * Symbolic analysis of K = W + Sigma_x + J^T d J (section "Hybrid linear
 * solver": computed once per pattern and reused by every refactorisation).
 * n variables, m rows of J; patterns as described above (host, int32 CSR,
 * w_rowptr has n+1 entries, j_rowptr m+1). opt may be NULL (defaults).
 * On success *out owns the analysis; release it with kkt_symbolic_destroy.
 * Errors: INVALID_ARG (NULL out, negative sizes), PATTERN (malformed CSR,
 * a front larger than one workgroup's LDS can hold). Host only.
 */
kkt_status kkt_symbolic_analyze(int32_t n, int32_t m,
                                const int32_t* w_rowptr, const int32_t* w_colind,
                                const int32_t* j_rowptr, const int32_t* j_colind,
                                const kkt_options* opt, kkt_symbolic** out);

/* Statistics of an analysis (host only). */
kkt_status kkt_symbolic_get_stats(const kkt_symbolic* sym, kkt_symbolic_stats* out);

/* perm[k] = original index of the k-th pivot (host array of n entries). */
kkt_status kkt_symbolic_get_perm(const kkt_symbolic* sym, int32_t* perm);

/* Supernode partition: col_ptr (nsuper+1: first pivot of each supernode),
 * parent (nsuper: parent supernode or -1), nrows (nsuper: front rows).
 * Any pointer may be NULL. Host only. */
kkt_status kkt_symbolic_get_supernodes(const kkt_symbolic* sym, int32_t* col_ptr, int32_t* parent, int32_t* nrows);

void kkt_symbolic_destroy(kkt_symbolic* sym);

/*
 * Device storage for one numeric factorisation of a pattern: the supernode
 * panels of L, the update matrices of the multifrontal assembly, the
 * assembled values of K and solve workspaces. The symbolic object must
 * outlive the factor. Errors: INVALID_ARG, OOM, DEVICE.
 */
kkt_status kkt_factor_create(const kkt_symbolic* sym, kkt_factor** out);
void kkt_factor_destroy(kkt_factor* f);

/*
 * General HyKKT (section "Solution 2: HyKKT" with the condensed matrix of eq.
 * (kkt:condensed)): marks rows of J as equality constraints G; the other rows
 * are inequality constraints H with slack weights D_s = sigma_s. With rows set
 * (count > 0), kkt_refactor takes gamma > 0 AND sigma_s and factors
 *     K_gamma = W + Sx + H^T D_s H + gamma G^T G
 * (per-row weight sigma_s on H rows, gamma on G rows), and kkt_cg_schur runs
 * the Schur-complement CG over the equality rows only: it solves
 *     [[W + Sx + H^T D_s H, G^T], [G, 0]] [dx; dy] = [fv; g]
 * where fv is the condensed right-hand side -(r1 + H^T (D_s r4 - r2)) and g
 * (length m, read on the G rows) is -r3; dy is 0 on the H rows. rows: host
 * array of `count` distinct row indices; count = 0 returns the factor to the
 * Lifted-KKT / HyKKT rules. The next refactor applies the setting.
 * Errors: INVALID_ARG (out of range or repeated rows), OOM, DEVICE.
 */
kkt_status kkt_factor_set_equality_rows(kkt_factor* f, const int32_t* rows, int32_t count);

/*
 * Numeric refactorisation with new values (same pattern).
 *   w_vals  (nnz_W)  lower-triangle values of W, CSR entry order
 *   j_vals  (nnz_J)  values of J, CSR entry order
 *   sigma_x (n)      primal diagonal
 *   gamma == 0, sigma_s (m) slack diagonal -> Lifted-KKT: K = W + Sx + J^T diag(sigma_s) J
 *                           (sigma_s may be NULL only when m == 0)
 *   gamma > 0, sigma_s NULL                -> HyKKT:      K_gamma = W + Sx + gamma J^T J
 *   equality rows set (kkt_factor_set_equality_rows), gamma > 0, sigma_s (m)
 *                                          -> general HyKKT: K_gamma = W + Sx + H^T D_s H + gamma G^T G
 * Device pointers; asynchronous on `stream`. A non-positive or non-finite pivot
 * is latched (see kkt_status_sync). Errors returned at once: INVALID_ARG
 * (NULL pointers, negative or non-finite gamma, sigma_s given with gamma > 0), DEVICE.
 */
kkt_status kkt_refactor(kkt_factor* f, const double* w_vals, const double* j_vals,
                        const double* sigma_x, const double* sigma_s, double gamma, void* stream);

/* Fills *o with the inertia-correction defaults. */
void kkt_inertia_opts_default(kkt_inertia_opts* o);

/*
 * Refactorisation with inertia correction (section "Augmented KKT system":
 * when the inertia of the augmented system differs from eq. (inertia), the
 * solver adds a primal regularisation delta_x; section "Solution 1:
 * Lifted-KKT": delta_x is raised until the condensed matrix is positive
 * definite). By Haynsworth's formula (after eq. (kkt:condensed)) the inertia
 * condition holds exactly when K = W + Sx + delta I + J^T d J is positive
 * definite, i.e. when the Cholesky factorization succeeds, so each trial is a
 * refactorisation with the same analysis: delta = 0 first; on NOT_SPD
 * delta_first (no earlier success on this factor) or max(delta_min,
 * kappa_minus * delta_last); then delta grows by kappa_plus_first (no earlier
 * success) or kappa_plus until the factorization succeeds or delta exceeds
 * delta_max (the update rule of the filter line-search interior-point method
 * the paper builds on; the paper itself fixes none). The factor remembers the
 * last accepted delta. Arguments as kkt_refactor; o may be NULL (defaults),
 * info may be NULL. Synchronises after every trial. Returns KKT_OK with K + delta I
 * factored, KKT_ERR_NOT_SPD when delta_max is exceeded, or another failure
 * (NONFINITE stops the trials at once).
 */
kkt_status kkt_refactor_inertia(kkt_factor* f, const double* w_vals, const double* j_vals, const double* sigma_x,
                                const double* sigma_s, double gamma, const kkt_inertia_opts* o,
                                kkt_inertia_info* info, void* stream);

/*
 * Waits for the stream work of the factor and reports the latched status:
 * KKT_OK, KKT_ERR_NOT_SPD (info->bad_col = original index of the first
 * failing pivot in elimination order) or KKT_ERR_NONFINITE. info may be NULL.
 */
kkt_status kkt_status_sync(kkt_factor* f, kkt_factor_info* info);

/*
 * Solves K x = b (Lifted-KKT) or K_gamma x = b (HyKKT factor) with the current
 * factor: a forward and backward sweep, then Richardson refinement
 * r = b - K x, x += K^{-1} r, stopping when omega <= ro->tol, after
 * ro->max_iter corrections, or when omega fails to halve; the iterate with the
 * smaller omega of the last two is returned (section "Hybrid linear solver":
 * the Cholesky solve followed by iterative refinement). b and x are device
 * arrays of n (x may not alias b). ro may be NULL (defaults).
 *   info != NULL: the host reads each stop decision (one synchronisation per
 *     round), then synchronises once more and returns KKT_ERR_NOT_SPD if the
 *     factor failed or KKT_ERR_NOT_CONVERGED if omega > tol at exit (x still
 *     holds the best iterate).
 *   info == NULL: asynchronous. The first solve and ro->max_iter refinement
 *     rounds are enqueued; the stop rule is evaluated on the device and the
 *     kernels of the rounds after it fired return at once, so x is the same
 *     bit for bit as with info. Nothing is read back: a failed factor is
 *     reported by kkt_status_sync (x is then meaningless).
 */
kkt_status kkt_solve(kkt_factor* f, const double* b, double* x, const kkt_refine_opts* ro,
                     kkt_solve_info* info, void* stream);

/* Fills *o with the CG defaults (tol 1e-10, maxit 200, eta_tol 0). */
void kkt_cg_opts_default(kkt_cg_opts* o);

/*
 * HyKKT (section "Solution 2: HyKKT", eqs. (hykkt), (schurcomp)): with f
 * factored as K_gamma (sigma_s NULL, gamma > 0), solves
 * [[W + Sx, J^T], [J, 0]] [dx; dy] = [fv; g]:
 *   f_gamma = fv + gamma J^T g;  c = J K_gamma^{-1} f_gamma - g;
 *   CG from dy = 0 on S_gamma dy = c, S_gamma = J K_gamma^{-1} J^T (matrix-free,
 *   one sweep pair per iteration), stopping when ||r||_2 <= tol ||c||_2, or
 *   (eta_tol > 0) when max(gamma ||J^T r||_inf, ||r||_inf) / (||A||_inf
 *   ||dy||_inf + ||(fv, g)||_inf) <= eta_tol -- an upper bound on the saddle
 *   system's normwise backward error, since with dx below its residual is
 *   (gamma J^T r, r) -- or after maxit iterations;
 *   dx = K_gamma^{-1}(f_gamma - J^T dy);
 *   then the saddle-system residual of (dx, dy) and its normwise backward
 *   error eta (kkt_cg_info.eta).
 * fv (n), g (m), dx (n), dy (m) are device arrays; opts may be NULL
 * (defaults). Needs m <= n (J of full row rank). Errors: INVALID_ARG, STATE
 * (no K_gamma factor, e.g. a Lifted-KKT factor).
 *   info != NULL: synchronises once before the iterations (a failed factor
 *     returns NOT_SPD / NONFINITE) and once per iteration (one iteration of
 *     lookahead), and returns NOT_CONVERGED or BREAKDOWN as they occur.
 *   info == NULL: asynchronous; all maxit iterations are enqueued and the
 *     stop decisions are taken on the device (the kernels of the iterations
 *     after the stop return at once), so dx, dy are the same bit for bit as
 *     with info. Each queued iteration costs launches even when it does
 *     nothing: choose maxit near the expected count. A failed factor is
 *     reported by kkt_status_sync.
 */
kkt_status kkt_cg_schur(kkt_factor* f, const double* fv, const double* g, const kkt_cg_opts* opts,
                        double* dx, double* dy, kkt_cg_info* info, void* stream);

/*
 * Lifted-KKT refactorisations of this factor (enable = 1) also keep
 * W + Sx + delta I, J (by rows and by columns) and Sigma_s on the device, which
 * kkt_solve_augmented needs for the full system's residual; they cost about
 * 12 nnz(K) + 16 nnz(J) + 8 m bytes of extra writes per refactor, so they are
 * off by default. HyKKT factors always keep what their CG needs. Host only;
 * applies from the next refactor.
 */
kkt_status kkt_factor_keep_augmented(kkt_factor* f, int32_t enable);

/*
 * The augmented system of eq. (kkt:augmented) for Lifted-KKT (every
 * constraint an inequality: H = J, D_s = Sigma_s, no equality rows), with the
 * factor's primal regularisation (Sigma_x + delta I on the Hessian block):
 *   [[W + Sx + delta I, 0, J^T], [0, Sigma_s, I], [J, I, 0]] [dx; ds; dz] = -[r1; r2; r4].
 * Condensation (eq. (kkt:condensed)): K dx = -(r1 + J^T (Sigma_s r4 - r2)),
 * solved with refinement as kkt_solve does; the slack and multiplier steps
 * are recovered as ds = -r4 - J dx and dz = -r2 - Sigma_s ds (stated after
 * eq. (kkt:condensed)). Then Richardson refinement on the full system
 * (section "Hybrid linear solver"): residual e of the augmented system,
 * correction by the same condensation with the factor, stop when its
 * componentwise backward error omega <= ro->tol, after ro->max_iter
 * corrections, or when omega fails to halve (the better of the last two
 * iterates is kept). r1 (n), r2 (m), r4 (m), dx (n), ds (m), dz (m) are device
 * arrays; ro may be NULL (defaults), info may be NULL. Needs a Lifted-KKT
 * factor refactored with kkt_factor_keep_augmented(f, 1) (STATE otherwise).
 * Synchronises once per round.
 */
kkt_status kkt_solve_augmented(kkt_factor* f, const double* r1, const double* r2, const double* r4, double* dx,
                               double* ds, double* dz, const kkt_refine_opts* ro, kkt_aug_info* info,
                               void* stream);

/*
 * Interior-point outer loop (section "INTERIOR-POINT METHOD": the smoothed KKT
 * system eq. (smoothkkt) solved by Newton steps, eq. (newtonstep), with a
 * fraction-to-boundary step) on the convex QP
 *     min 1/2 x^T W x + c^T x   s.t.   J x <= u
 * over the factor's pattern (W from its lower triangle, every row of J an
 * inequality), with slacks s (J x + s = u, s >= 0) and multipliers z. Each
 * iteration: r1 = W x + c + J^T z, r4 = J x + s - u, gap = s^T z / m; stop when
 * max(||r1||_inf / (1 + ||c||_inf), ||r4||_inf / (1 + ||u||_inf), gap) <= tol;
 * else mu = sigma gap, r2 = z - mu / s, D_s = Z S^{-1}; kkt_refactor_inertia
 * with Sigma_x = 0 and sigma_s = D_s (same analysis), kkt_solve_augmented for
 * (dx, ds, dz) (eqs. (kkt:augmented), (kkt:condensed)); tau = max(tau_min,
 * 1 - mu) and the largest alpha_p, alpha_d <= 1 keeping s and z above
 * (1 - tau) of their current values; x += alpha_p dx, s += alpha_p ds,
 * z += alpha_d dz. (The paper's solver adds a filter line search; on a convex
 * QP the fraction-to-boundary steps are kept as they are.)
 * w_vals, j_vals, c (n), u (m) are device inputs; x (n), s (m), z (m) are
 * device arrays holding the starting point on entry (s > 0, z > 0) and the
 * last iterate on return. opts may be NULL (tol 1e-8, maxit 100, sigma 0.1,
 * tau_min 0.99). Synchronises every iteration. Enables kkt_factor_keep_augmented.
 * Returns OK, NOT_CONVERGED after maxit iterations, or a refactor / solve error.
 */
typedef struct kkt_ipm_opts {
    double tol;
    int32_t maxit;
    double sigma;            /* barrier reduction: mu = sigma * s^T z / m */
    double tau_min;          /* fraction to the boundary: tau = max(tau_min, 1 - mu) */
} kkt_ipm_opts;

typedef struct kkt_ipm_info {
    int32_t status;
    int32_t iterations;      /* Newton steps taken */
    double err;              /* the stop measure at exit */
    double gap;              /* s^T z / m at exit */
    double r1;               /* ||W x + c + J^T z||_inf at exit */
    double r4;               /* ||J x + s - u||_inf at exit */
    double max_delta;        /* largest inertia-correction delta used */
    int32_t aug_corrections; /* refinement corrections of the augmented solves, summed */
} kkt_ipm_info;

void kkt_ipm_opts_default(kkt_ipm_opts* o);
kkt_status kkt_ipm_qp(kkt_factor* f, const double* w_vals, const double* j_vals, const double* c, const double* u,
                      double* x, double* s, double* z, const kkt_ipm_opts* opts, kkt_ipm_info* info, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): kkt_solve
 * with the same arguments, results (bit for bit) and synchronisation rules,
 * whose per-solve workspace lives in a static device array of the library
 * (32 MiB per GPU, held until the process ends) instead of the factor's
 * storage. The call allocates nothing: no hipMalloc, no host allocation of
 * the runtime, no event (per-launch timers are suspended during the call).
 * Errors: those of kkt_solve, and BUDGET when the workspace (about 24 n +
 * 8 * update rows + 176 * supernodes bytes) exceeds the array. Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 */
kkt_status kkt_solve_noalloc(kkt_factor* f, const double* b, double* x, const kkt_refine_opts* ro,
                             kkt_solve_info* info, void* stream);

/* Matrix-vector product y = K x with the assembled K of the current factor
 * (device arrays of n). Asynchronous. Used to evaluate residuals. */
kkt_status kkt_matvec(kkt_factor* f, const double* x, double* y, void* stream);

/* Kernel phases timed by the per-launch event timers. */
#define KKT_PHASE_ASSEMBLE 0  /* K = W + Sigma_x + J^T d J */
#define KKT_PHASE_FACTOR 1    /* supernodal Cholesky (one launch per tree level, or one queue launch) */
#define KKT_PHASE_FWD 2       /* forward sweep L y = P b (with the queue schedule: both sweeps) */
#define KKT_PHASE_BWD 3       /* backward sweep L^T z = y */
#define KKT_PHASE_RESIDUAL 4  /* r = b - K x and backward-error reductions */
#define KKT_PHASE_PERMUTE 5   /* gathers between original and pivot order */
#define KKT_PHASE_CG 6        /* Schur-complement CG vector kernels (J^T p, J t, dots, axpys) */
#define KKT_PHASE_CONTROL 7   /* small control kernels (fills, refinement / CG decisions) */
#define KKT_NPHASES 8

typedef struct kkt_timing {
    double ms[KKT_NPHASES];        /* summed kernel time per phase (HIP events around every launch) */
    int32_t launches[KKT_NPHASES]; /* number of launches per phase */
} kkt_timing;

/* Enables (1) or disables (0) per-launch HIP event timing for this factor. */
kkt_status kkt_factor_set_timing(kkt_factor* f, int32_t enable);

/* Synchronises the last stream used, returns the times accumulated since the
 * previous read (or since timing was enabled) and resets them. */
kkt_status kkt_factor_read_timing(kkt_factor* f, kkt_timing* out);

/*
 * Launch schedules of the supernode tree (factorization and both sweeps; the
 * tree is the elimination tree of the supernodal Cholesky, section "Hybrid
 * linear solver", and every front depends on its children only).
 *   LEVELS: one launch per tree level (leaves first for the factor and the
 *           forward sweep, roots first for the backward sweep).
 *   QUEUE:  one persistent launch for the factor and one for both sweeps;
 *           workgroups take fronts from a ticket counter in topological order
 *           and wait on per-front dependency counters, so fronts of different
 *           levels (and instances) overlap. A dependency wait that exceeds its
 *           spin bound makes the next status read return KKT_ERR_DEVICE.
 * Both schedules run the same per-front arithmetic in the same order, so
 * results are bitwise identical. The default is LEVELS. QUEUE is refused
 * (INVALID_ARG) for patterns with large fronts (kkt_options.front_lds_max).
 * Host only; applies to launches issued after the call.
 */
#define KKT_SCHEDULE_LEVELS 0
#define KKT_SCHEDULE_QUEUE 1
kkt_status kkt_factor_set_schedule(kkt_factor* f, int32_t schedule);

/*
 * Launch shape of the update matrices U = -L21 L21^T of the multifrontal
 * factorization (section "Hybrid linear solver": the dense kernels of the
 * supernodal Cholesky), level schedule only: on a tree level with fewer
 * than max_fronts fronts whose widest update part has at least min_rows
 * rows, the update matrices are formed by a launch of their own (one wave
 * per 16 x 16 tile) instead of by each front's workgroup after its panel.
 * Both ways give every entry the same operations in the same order, so
 * results are bitwise identical; only the time differs. Defaults 140 and 64;
 * max_fronts = 0 keeps every update in the front's workgroup. The
 * autotuner picks them by measurement. INVALID_ARG for negative values.
 * Host only; applies to launches issued after the call.
 */
kkt_status kkt_factor_set_update_split(kkt_factor* f, int32_t max_fronts, int32_t min_rows);

/*
 * Workgroup size of the front factorization (section "Hybrid linear solver":
 * the dense kernels of the supernodal Cholesky), level schedule only: a tree
 * level whose widest front has at most max_cols columns is factored by
 * 256-thread workgroups that reserve only that level's LDS (two fit on a
 * compute unit when the level's fronts need at most 80 KiB); other levels by
 * 512-thread workgroups. Both give every entry the same operations in the
 * same order, so results are bitwise identical; only the time differs.
 * Default 0 (every level by 512 threads); the autotuner picks it by
 * measurement. INVALID_ARG if negative. Host only; applies to launches
 * issued after the call.
 */
kkt_status kkt_factor_set_small_fronts(kkt_factor* f, int32_t max_cols);

/*
 * Batched form: many independent instances (each with its own pattern; the
 * same symbolic object may appear several times) refactored and solved by
 * the same launches. With the LEVELS schedule every launch covers one tree
 * level of all instances; with QUEUE one persistent launch walks the fronts
 * of all instances; either way small NMPC-sized fronts from different
 * instances share the GPU.
 *
 * Values and vectors are concatenated in instance order: instance q owns
 * w_vals[w_ofs[q] .. w_ofs[q+1]), j_vals[j_ofs[q] ..), sigma_x / b / x
 * [n_ofs[q] ..) and sigma_s [m_ofs[q] ..), as reported by kkt_batch_offsets.
 * The symbolic objects must outlive the batch. Lifted-KKT only.
 */
kkt_status kkt_batch_create(int32_t count, const kkt_symbolic* const* syms, kkt_batch** out);
void kkt_batch_destroy(kkt_batch* b);

/* Prefix offsets (count+1 entries each; any pointer may be NULL). Host only. */
kkt_status kkt_batch_offsets(const kkt_batch* b, int64_t* n_ofs, int64_t* m_ofs, int64_t* w_ofs, int64_t* j_ofs);

/* Refactors every instance: K_q = W_q + Sx_q + J_q^T diag(Ss_q) J_q. Device
 * arrays, asynchronous on `stream`; per-instance failures are latched. */
kkt_status kkt_batch_refactor(kkt_batch* b, const double* w_vals, const double* j_vals,
                              const double* sigma_x, const double* sigma_s, void* stream);

/* Solves every instance with Richardson refinement (per-instance stop rule as
 * in kkt_solve; instances that have stopped skip the remaining sweeps).
 * infos, when non-NULL, receives `count` entries. Synchronises the stream.
 * Returns NOT_SPD / NONFINITE if any factor failed, NOT_CONVERGED if any
 * instance ended above tol, else OK. */
kkt_status kkt_batch_solve(kkt_batch* b, const double* rhs, double* x, const kkt_refine_opts* ro,
                           kkt_solve_info* infos, void* stream);

/* Waits and reports each instance's factor status and failing column (original
 * index, -1 if none); either array (count entries) may be NULL. */
kkt_status kkt_batch_status(kkt_batch* b, int32_t* status, int32_t* bad_col);

/* Launch schedule of the batch (see KKT_SCHEDULE_*). */
kkt_status kkt_batch_set_schedule(kkt_batch* b, int32_t schedule);
/* As kkt_factor_set_update_split, for every level of the batch's launches. */
kkt_status kkt_batch_set_update_split(kkt_batch* b, int32_t max_fronts, int32_t min_rows);
/* As kkt_factor_set_small_fronts, for every level of the batch's launches. */
kkt_status kkt_batch_set_small_fronts(kkt_batch* b, int32_t max_cols);

/*
 * Graph form of kkt_batch_refactor + kkt_batch_solve. kkt_batch_capture
 * records, as one HIP graph on a stream private to the batch, the status
 * reset, assembly, factorization, first solve and `rounds` refinement rounds
 * (each: residual, stop decision, and a correction for the instances still
 * refining), bound to the given device arrays; it runs nothing. The graph
 * holds kernel nodes only. kkt_batch_replay launches it on `stream`, then
 * continues the refinement loop on the host from round `rounds` (for the
 * instances not yet stopped), applies the better-of-last-two rule and fills
 * `infos` (count entries, may be NULL); it synchronises the stream and
 * returns as kkt_batch_solve does. Every instance goes through exactly the
 * operations of the two separate calls, so the results are bitwise the same.
 * The caller refreshes the arrays' contents between replays and keeps them
 * allocated while the graph exists. The graph keeps the schedule and launch
 * shapes (update split, front workgroup size) in effect when it was
 * recorded; setting them later changes eager calls and later captures only.
 * A new capture replaces the old one; kkt_batch_destroy releases it.
 * Errors: INVALID_ARG (NULL arrays, x aliasing rhs, bad refinement options,
 * rounds outside 0..max_iter+1), STATE (replay without a capture), HIP.
 */
kkt_status kkt_batch_capture(kkt_batch* b, const double* w_vals, const double* j_vals, const double* sigma_x,
                             const double* sigma_s, const double* rhs, double* x, const kkt_refine_opts* ro,
                             int32_t rounds);
kkt_status kkt_batch_replay(kkt_batch* b, kkt_solve_info* infos, void* stream);

kkt_status kkt_batch_set_timing(kkt_batch* b, int32_t enable);
kkt_status kkt_batch_read_timing(kkt_batch* b, kkt_timing* out);

/*
 * Stage-structured solver (section "Future Works": the condensed matrix of a
 * dynamic program is block-banded and can be factorized by a block solver
 * instead of a general sparse one). For patterns whose variables are
 * numbered stage by stage (stage k owns [stage_ptr[k], stage_ptr[k+1]), at
 * most 96 variables), where W couples only variables of the same or
 * consecutive stages and every row of J spans at most two consecutive
 * stages, K = W + Sigma_x + J^T Sigma_s J is block tridiagonal,
 * K = tridiag(E_{k-1}, D_k, E_k^T), and is factored by the block Cholesky
 * (Riccati) recursion
 *   Dt_k = D_k - Ls_{k-1} Ls_{k-1}^T,  L_kk = chol(Dt_k),  Ls_k = E_k L_kk^{-T}
 * with one workgroup per instance walking its stages; K itself is assembled
 * by the same kernels (same bits) as kkt_factor_refactor. No fill-reducing
 * ordering is used: vectors stay in the original numbering.
 *
 * kkt_stagewise_create: count instances, syms[q] the pattern of instance q
 * (must outlive the solver), stage_ptrs[q] its nstages[q] + 1 stage starts
 * (host arrays, copied). Values and vectors are concatenated in instance
 * order as for kkt_batch (offsets from the patterns' sizes). Errors:
 * INVALID_ARG (stage_ptr not 0 .. n, an empty stage), PATTERN (a stage
 * wider than 96, or a position of K coupling stages more than one apart),
 * OOM. Synchronous.
 */
typedef struct kkt_stagewise kkt_stagewise;
kkt_status kkt_stagewise_create(int32_t count, const kkt_symbolic* const* syms, const int32_t* const* stage_ptrs,
                                const int32_t* nstages, kkt_stagewise** out);
void kkt_stagewise_destroy(kkt_stagewise* w);

/* Assembles and factors K of every instance (device arrays in the patterns'
 * entry order, concatenated). Asynchronous on `stream`; a pivot that is not
 * positive is reported by kkt_stagewise_status (and by the next solve). */
kkt_status kkt_stagewise_refactor(kkt_stagewise* w, const double* w_vals, const double* j_vals,
                                  const double* sigma_x, const double* sigma_s, void* stream);

/* Synchronises the last stream and reports each instance's factor status
 * (status[q], KKT_OK or KKT_ERR_NOT_SPD) and, on NOT_SPD, the first failed
 * variable in the original numbering (bad_col[q], else -1); either array
 * may be NULL. Returns the first failure. */
kkt_status kkt_stagewise_status(kkt_stagewise* w, int32_t* status, int32_t* bad_col);

/* Solves K x = rhs for every instance with the stop rule of kkt_solve
 * (componentwise backward error <= tol, at most max_iter corrections, stop
 * when it fails to halve; ro may be NULL: tol 1e-14, max_iter 10). rhs and x
 * are device arrays (concatenated, original numbering, no aliasing); infos
 * (host, one per instance) may be NULL. Synchronises once per refinement
 * round. Returns NOT_SPD if the factor failed, NOT_CONVERGED if an instance
 * missed tol. */
kkt_status kkt_stagewise_solve(kkt_stagewise* w, const double* rhs, double* x, const kkt_refine_opts* ro,
                               kkt_solve_info* infos, void* stream);

kkt_status kkt_stagewise_set_timing(kkt_stagewise* w, int32_t enable);
kkt_status kkt_stagewise_read_timing(kkt_stagewise* w, kkt_timing* out);

/*
 * Served form: a request loop over resident sparsity patterns. A registered
 * pattern's analysis stays on the device; each request is a refactor with new
 * values plus a refined solve (the analysis is reused, section "Hybrid linear
 * solver"). Requests queue FIFO; `workers` threads, each with its own HIP
 * stream and an HBM arena of hbm_budget / workers bytes, repeatedly take the
 * longest queue prefix that fits their arena (at most max_wave requests),
 * gather its inputs, refactor + solve it as one batch and scatter the
 * solutions. Requests arriving while waves run join the next free worker's
 * wave, so waves overlap on the GPU. A request's result does not depend on
 * the wave it rides in (no cross-request reductions).
 */
typedef struct kkt_server_opts {
    int64_t hbm_budget;      /* bytes of device workspace for all workers (default 8 GiB) */
    int32_t max_wave;        /* most requests per wave (default 64) */
    int32_t workers;         /* waves in flight at once, 1..8 (default 2) */
    int32_t refine_max_iter; /* Richardson corrections (default 10) */
    double refine_tol;       /* omega target (default 1e-14) */
    double linger_us;        /* a worker may wait this long for a fuller wave (default 0) */
} kkt_server_opts;

typedef struct kkt_server_stats {
    int64_t submitted, completed, rejected, waves;
    double mean_wave;        /* requests per wave */
    double p50_s, p99_s;     /* latency from submit to result ready */
    double mean_queue_s;     /* submit -> wave start */
    double mean_service_s;   /* wave start -> result ready */
    double throughput;       /* completed / window_s */
    double window_s;         /* first submit -> last completion */
} kkt_server_stats;

void kkt_server_opts_default(kkt_server_opts* o);

/* Creates the server, its worker threads, streams and arenas (device memory
 * of hbm_budget bytes is allocated here). Errors: INVALID_ARG, OOM, DEVICE. */
kkt_status kkt_server_create(const kkt_server_opts* opt, kkt_server** out);

/* Uploads the pattern's analysis; *pattern_id names it in submissions. The
 * symbolic object must outlive the server. BUDGET if one request of this
 * pattern cannot fit a worker's arena. */
kkt_status kkt_server_register(kkt_server* s, const kkt_symbolic* sym, int32_t* pattern_id);

/* Queues one Lifted-KKT refactor+solve: device arrays in the pattern's entry
 * order (w_vals, j_vals, sigma_x, sigma_s, b) and the output x (n). The
 * request is ordered after the work enqueued on `stream` (a hipStream_t,
 * NULL = the default stream) before this call: an event recorded there at
 * submission is waited for by the worker's stream before it reads the inputs
 * or writes x. The arrays must stay valid (inputs unchanged) until
 * kkt_server_wait returns for *ticket. Returns at once. */
kkt_status kkt_server_submit(kkt_server* s, int32_t pattern_id, const double* w_vals, const double* j_vals,
                             const double* sigma_x, const double* sigma_s, const double* b, double* x,
                             void* stream, int64_t* ticket);

/* Blocks until the request is done (its x complete on the device); returns
 * its status (NOT_SPD, NONFINITE, NOT_CONVERGED or OK) and fills its solve
 * info and latency (may be NULL). A ticket can be waited for once. */
kkt_status kkt_server_wait(kkt_server* s, int64_t ticket, kkt_solve_info* info, double* latency_s);

kkt_status kkt_server_get_stats(kkt_server* s, kkt_server_stats* out);
kkt_status kkt_server_reset_stats(kkt_server* s);

/* Finishes the queued requests, stops the workers and frees everything. */
void kkt_server_destroy(kkt_server* s);

#ifdef __cplusplus
}
#endif
#endif /* KKT_H */
