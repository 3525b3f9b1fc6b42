/*
 * Sparse FP64 oracle: TEST INFRASTRUCTURE ONLY.
 *
 * Called from Python (ctypes) by the tests and by the CPU-baseline leg of the
 * benchmark; the library never links or calls it. It shares no code with the
 * library: its own elimination tree, its own factorisation, its own solves.
 *
 * What it computes (Pacaud & Shin, arXiv 2403.15913):
 *   - a sparse LDL^T with static (diagonal, no interchange) pivots of a
 *     symmetric matrix under a given symmetric ordering. On the condensed
 *     matrix K (eq. (kkt:condensed), eq. (liftedkkt)) it is the Cholesky
 *     factorisation written as L D L^T, and all pivots positive is exactly
 *     "K positive definite". On the 2x2 saddle-point form of eq. (hykkt)
 *     with each constraint ordered after its last primal variable, the
 *     pivots are nonzero and their signs give the inertia.
 *   - Richardson iterative refinement on K (section "Hybrid linear solver":
 *     backsolve followed by Richardson iterations).
 *   - the HyKKT solve: factor K_gamma = K + gamma J^T J, form
 *     f_gamma = f + gamma J^T g, run conjugate gradient on
 *     S_gamma = J K_gamma^{-1} J^T (eq. (schurcomp)) from y0 = 0 and recover
 *     dx = K_gamma^{-1}(f_gamma - J^T dy).
 *
 * Matrices are CSR with 64-bit row pointers and 32-bit column indices. A
 * symmetric matrix is passed with both triangles. perm[k] is the original
 * index of the k-th pivot.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n;
    int64_t *Lp;     /* column pointers of strictly lower L, n+1 */
    int *Lnz;        /* entries per column */
    int *Li;         /* row indices (pivot order) */
    double *Lx;
    double *D;
    int *parent;     /* elimination tree */
    int *perm;       /* pivot k -> original index */
    int *pinv;       /* original index -> pivot */
} ora_ldl;

void ora_ldl_free(ora_ldl *F) {
    if (!F) return;
    free(F->Lp); free(F->Lnz); free(F->Li); free(F->Lx); free(F->D);
    free(F->parent); free(F->perm); free(F->pinv); free(F);
}

/* Entries of column k of the permuted matrix C = P A P^T with row <= k:
 * those are row k of C restricted to columns <= k, read from row perm[k] of A. */

/*
 * Factor. Returns 0 on success, 1 if pivot k is zero or not finite
 * (*bad = original index of that pivot), 2 on allocation failure,
 * 3 if any input value is not finite (*bad = original row).
 */
int ora_ldl_factor(int n, const int64_t *Ap, const int *Ai, const double *Ax,
                   const int *perm, ora_ldl **out, int *bad) {
    *out = NULL;
    *bad = -1;
    ora_ldl *F = (ora_ldl *)calloc(1, sizeof(ora_ldl));
    if (!F) return 2;
    F->n = n;
    F->Lp = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    F->Lnz = (int *)calloc(n > 0 ? n : 1, sizeof(int));
    F->D = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    F->parent = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    F->perm = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    F->pinv = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *flag = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    if (!F->Lp || !F->Lnz || !F->D || !F->parent || !F->perm || !F->pinv || !flag) {
        free(flag); ora_ldl_free(F); return 2;
    }
    for (int k = 0; k < n; k++) { F->perm[k] = perm[k]; F->pinv[perm[k]] = k; }

    /* symbolic: elimination tree and column counts by walking the tree from
     * every off-diagonal entry of each row of the upper triangle */
    for (int k = 0; k < n; k++) {
        F->parent[k] = -1;
        flag[k] = k;
        int ok = perm[k];
        for (int64_t p = Ap[ok]; p < Ap[ok + 1]; p++) {
            int i = F->pinv[Ai[p]];
            if (i >= k) continue;
            while (flag[i] != k) {
                if (F->parent[i] == -1) F->parent[i] = k;
                F->Lnz[i]++;
                flag[i] = k;
                i = F->parent[i];
            }
        }
    }
    F->Lp[0] = 0;
    for (int k = 0; k < n; k++) F->Lp[k + 1] = F->Lp[k] + F->Lnz[k];
    int64_t nnzL = F->Lp[n];
    F->Li = (int *)malloc(sizeof(int) * (nnzL > 0 ? nnzL : 1));
    F->Lx = (double *)malloc(sizeof(double) * (nnzL > 0 ? nnzL : 1));
    double *Y = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    int *pattern = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    if (!F->Li || !F->Lx || !Y || !pattern) {
        free(flag); free(Y); free(pattern); ora_ldl_free(F); return 2;
    }

    /* numeric: row k of L from a sparse triangular solve whose pattern is the
     * reach of column k's entries in the elimination tree */
    for (int k = 0; k < n; k++) flag[k] = -1;
    for (int k = 0; k < n; k++) {
        int top = n;
        flag[k] = k;
        F->Lnz[k] = 0;
        int ok = perm[k];
        for (int64_t p = Ap[ok]; p < Ap[ok + 1]; p++) {
            if (!isfinite(Ax[p])) { *bad = ok; free(flag); free(Y); free(pattern); ora_ldl_free(F); return 3; }
            int i = F->pinv[Ai[p]];
            if (i > k) continue;
            Y[i] += Ax[p];
            int len = 0;
            while (flag[i] != k) {          /* climb until an already marked node */
                pattern[len++] = i;
                flag[i] = k;
                i = F->parent[i];
            }
            while (len > 0) pattern[--top] = pattern[--len];
        }
        double d = Y[k];
        Y[k] = 0.0;
        for (; top < n; top++) {
            int i = pattern[top];
            double yi = Y[i];
            Y[i] = 0.0;
            int64_t p0 = F->Lp[i], p1 = F->Lp[i] + F->Lnz[i];
            for (int64_t p = p0; p < p1; p++) Y[F->Li[p]] -= F->Lx[p] * yi;
            double lki = yi / F->D[i];
            d -= lki * yi;
            F->Li[p1] = k;
            F->Lx[p1] = lki;
            F->Lnz[i]++;
        }
        F->D[k] = d;
        if (d == 0.0 || !isfinite(d)) {
            *bad = ok;
            free(flag); free(Y); free(pattern);
            *out = F;          /* partial factor kept for inspection */
            return 1;
        }
    }
    free(flag); free(Y); free(pattern);
    *out = F;
    return 0;
}

int64_t ora_ldl_nnz(const ora_ldl *F) { return F->Lp[F->n]; }

/* (positive, zero, negative) pivot counts over the first `upto` pivots (all if upto < 0) */
void ora_ldl_inertia(const ora_ldl *F, int upto, int *pos, int *zero, int *neg) {
    int n = (upto < 0 || upto > F->n) ? F->n : upto;
    *pos = *zero = *neg = 0;
    for (int k = 0; k < n; k++) {
        if (F->D[k] > 0) (*pos)++; else if (F->D[k] < 0) (*neg)++; else (*zero)++;
    }
}

void ora_ldl_get_d(const ora_ldl *F, double *d) { memcpy(d, F->D, sizeof(double) * F->n); }
void ora_ldl_get_parent(const ora_ldl *F, int *parent) { memcpy(parent, F->parent, sizeof(int) * F->n); }
void ora_ldl_get_colcounts(const ora_ldl *F, int *cnt) { memcpy(cnt, F->Lnz, sizeof(int) * F->n); }

/* x = A^{-1} b through P^T L^{-T} D^{-1} L^{-1} P; work has length n */
void ora_ldl_solve(const ora_ldl *F, const double *b, double *x, double *work) {
    int n = F->n;
    for (int k = 0; k < n; k++) work[k] = b[F->perm[k]];
    for (int j = 0; j < n; j++) {
        double yj = work[j];
        if (yj != 0.0)
            for (int64_t p = F->Lp[j]; p < F->Lp[j] + F->Lnz[j]; p++) work[F->Li[p]] -= F->Lx[p] * yj;
    }
    for (int k = 0; k < n; k++) work[k] /= F->D[k];
    for (int j = n - 1; j >= 0; j--) {
        double s = work[j];
        for (int64_t p = F->Lp[j]; p < F->Lp[j] + F->Lnz[j]; p++) s -= F->Lx[p] * work[F->Li[p]];
        work[j] = s;
    }
    for (int k = 0; k < n; k++) x[F->perm[k]] = work[k];
}

/* r = b - A x for a CSR matrix; also returns |A||x| + |b| in den (if non-NULL) */
static void residual(int n, const int64_t *Ap, const int *Ai, const double *Ax,
                     const double *x, const double *b, double *r, double *den) {
    for (int i = 0; i < n; i++) {
        double s = 0.0, a = 0.0;
        for (int64_t p = Ap[i]; p < Ap[i + 1]; p++) {
            double t = Ax[p] * x[Ai[p]];
            s += t;
            a += fabs(t);
        }
        r[i] = b[i] - s;
        if (den) den[i] = a + fabs(b[i]);
    }
}

static double inf_norm_mat(int n, const int64_t *Ap, const double *Ax) {
    double nm = 0.0;
    for (int i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = Ap[i]; p < Ap[i + 1]; p++) s += fabs(Ax[p]);
        if (s > nm) nm = s;
    }
    return nm;
}

/*
 * Richardson refinement on A (symmetric, full CSR) with the factor F.
 * x <- A^{-1} b, then repeatedly r = b - A x, omega = max_i |r_i| / (|A||x|+|b|)_i,
 * eta = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf); stop when omega <= tol,
 * after maxit corrections, or when omega fails to halve; otherwise x += A^{-1} r.
 * The iterate with the smallest omega is returned. Returns the number of
 * corrections applied.
 */
int ora_refine(int n, const int64_t *Ap, const int *Ai, const double *Ax, const ora_ldl *F,
               const double *b, double *x, int maxit, double tol, double *eta, double *omega) {
    double *r = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *den = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *best = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double nA = inf_norm_mat(n, Ap, Ax), nb = 0.0;
    for (int i = 0; i < n; i++) if (fabs(b[i]) > nb) nb = fabs(b[i]);
    ora_ldl_solve(F, b, x, w);
    double best_om = INFINITY, best_eta = INFINITY, prev = INFINITY;
    int it = 0, applied = 0;
    for (;;) {
        residual(n, Ap, Ai, Ax, x, b, r, den);
        double om = 0.0, rn = 0.0, xn = 0.0;
        for (int i = 0; i < n; i++) {
            double ri = fabs(r[i]);
            double q = den[i] > 0 ? ri / den[i] : (ri > 0 ? INFINITY : 0.0);
            if (q > om) om = q;
            if (ri > rn) rn = ri;
            if (fabs(x[i]) > xn) xn = fabs(x[i]);
        }
        double et = (nA * xn + nb) > 0 ? rn / (nA * xn + nb) : 0.0;
        if (om < best_om) { best_om = om; best_eta = et; memcpy(best, x, sizeof(double) * n); applied = it; }
        if (om <= tol || it >= maxit || (it > 0 && om > 0.5 * prev)) break;
        prev = om;
        ora_ldl_solve(F, r, d, w);
        for (int i = 0; i < n; i++) x[i] += d[i];
        it++;
    }
    memcpy(x, best, sizeof(double) * n);
    *eta = best_eta;
    *omega = best_om;
    free(r); free(den); free(d); free(w); free(best);
    return applied;
}

/*
 * HyKKT with K_gamma already factored in F. J is m x n CSR.
 * Returns 0 converged, 6 max iterations, 7 breakdown (p^T S p <= 0).
 */
int ora_hykkt_cg(int n, int m, const int64_t *Jp, const int *Ji, const double *Jx,
                 const ora_ldl *F, double gamma, const double *f, const double *g,
                 double tol, int maxit, double *dx, double *dy, int *iters, double *true_res) {
    double *fg = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *t = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *u = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *c = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    double *r = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    double *p = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    double *q = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    int status = 6;
    /* f_gamma = f + gamma J^T g */
    memcpy(fg, f, sizeof(double) * n);
    for (int i = 0; i < m; i++)
        for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) fg[Ji[k]] += gamma * Jx[k] * g[i];
    /* c = J K_gamma^{-1} f_gamma - g */
    ora_ldl_solve(F, fg, t, w);
    for (int i = 0; i < m; i++) {
        double s = 0.0;
        for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) s += Jx[k] * t[Ji[k]];
        c[i] = s - g[i];
    }
    double cn = 0.0;
    for (int i = 0; i < m; i++) { dy[i] = 0.0; r[i] = c[i]; p[i] = c[i]; cn += c[i] * c[i]; }
    double rr = cn;
    cn = sqrt(cn);
    int it = 0;
    if (sqrt(rr) <= tol * cn) status = 0;
    while (status == 6 && it < maxit) {
        it++;
        /* q = J K_gamma^{-1} J^T p */
        memset(u, 0, sizeof(double) * n);
        for (int i = 0; i < m; i++)
            for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) u[Ji[k]] += Jx[k] * p[i];
        ora_ldl_solve(F, u, t, w);
        double pq = 0.0;
        for (int i = 0; i < m; i++) {
            double s = 0.0;
            for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) s += Jx[k] * t[Ji[k]];
            q[i] = s;
            pq += p[i] * s;
        }
        if (!(pq > 0.0)) { status = 7; break; }
        double a = rr / pq, rr2 = 0.0;
        for (int i = 0; i < m; i++) { dy[i] += a * p[i]; r[i] -= a * q[i]; rr2 += r[i] * r[i]; }
        if (sqrt(rr2) <= tol * cn) { status = 0; break; }
        double beta = rr2 / rr;
        for (int i = 0; i < m; i++) p[i] = r[i] + beta * p[i];
        rr = rr2;
    }
    *iters = it;
    /* dx = K_gamma^{-1}(f_gamma - J^T dy) */
    memcpy(u, fg, sizeof(double) * n);
    for (int i = 0; i < m; i++)
        for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) u[Ji[k]] -= Jx[k] * dy[i];
    ora_ldl_solve(F, u, dx, w);
    /* true Schur residual ||c - S dy||_2 / ||c||_2 */
    memset(u, 0, sizeof(double) * n);
    for (int i = 0; i < m; i++)
        for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) u[Ji[k]] += Jx[k] * dy[i];
    ora_ldl_solve(F, u, t, w);
    double res = 0.0;
    for (int i = 0; i < m; i++) {
        double s = 0.0;
        for (int64_t k = Jp[i]; k < Jp[i + 1]; k++) s += Jx[k] * t[Ji[k]];
        res += (c[i] - s) * (c[i] - s);
    }
    *true_res = cn > 0 ? sqrt(res) / cn : sqrt(res);
    free(fg); free(t); free(u); free(w); free(c); free(r); free(p); free(q);
    return status;
}
