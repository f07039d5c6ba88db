/*
 * CPU oracle for forward-error-oriented iterative refinement of the
 * eigenvectors of a real symmetric matrix (Terao & Ozaki, arXiv 2602.19090).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the GPU library never does, and the
 * two share no code, header or table.
 *
 * What it computes, and where each piece comes from:
 *
 *  or_refine_dd_step   One iteration of the Ogita-Aishima refinement,
 *                      Algorithm 1 (Sec. 2.4), entirely in double-double with
 *                      no splitting: V = A X, r_i = 1 - x_i^T x_i,
 *                      lambda_i = x_i^T v_i / (1 - r_i), W = X^T (V - X D),
 *                      e_ij = w_ij / (lambda_j - lambda_i), e_ii = r_i / 2,
 *                      X <- X + X E. Iterated to its fixed point this gives
 *                      X_true, the eigenvectors of the stored matrix.
 *  or_refine_dd_step_grouped
 *                      The same step with strongly coupled columns grouped (an
 *                      extension for near-tied or badly mixed eigenvectors,
 *                      which the paper leaves for future work, Sec. 5): columns
 *                      i and j are linked when their first-order correction is
 *                      large (|e_ij| > tau); for each linked group C (2..128
 *                      columns) the exact Rayleigh-Ritz problem on
 *                      span(X_C), T y = mu G y with G = X_C^T X_C and
 *                      T = X_C^T A X_C = W_CC + G_CC D_C, replaces the
 *                      first-order entries of the group's columns.
 *  or_method_step      One iteration of the proposed method (Sec. 3): beta
 *                      from the implementation rule of Sec. 4.1 (floor form,
 *                      xi = n), X^(1) = truncation of X to the grid that beta
 *                      fixes (eq. tau/x, Sec. 3.3), then Algorithm 1 on X^(1)
 *                      with every product exact to double-double.
 *  or_split_s7         Exponent-aligned 7-bit digit planes of a matrix, per
 *                      row or per column (the integer re-expression of the
 *                      error-free splitting of Sec. 2.3).
 *  or_slice_gemm_i64   Exact integer products of digit planes (int64).
 *  or_sigma_split      The FP64 splitting of eq. (a)/(x) with
 *                      sigma = 0.75 * 2^ceil(log2 v) * 2^alpha (Sec. 2.3).
 *  or_beta_rule        beta of Sec. 4.1 (floor form, xi = n) and the slice
 *                      count that the truncation grid implies.
 *  or_secular_rank1    Eigenpairs of diag(d) + rho u u^T from the secular
 *                      equation (a textbook route independent of Algorithm 1,
 *                      used to pin the double-double refinement).
 *
 * Matrices are column-major: element (i, j) at i + j*ld.
 *
 * The double-double matrix product tiles its loops for the cache, but each
 * output element accumulates its k terms one by one in index order, exactly
 * as the plain triple loop does; the tiling changes no arithmetic.
 *
 * Build with -ffp-contract=off (error-free transformations must not be
 * contracted into fused operations).
 */
#include "dd.h"

#include <float.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Double-double matrix product C = op(A) * B, op(A) = A or A^T (m x k),     */
/* B (k x n). Low words may be NULL (zero).                                  */
/* ------------------------------------------------------------------------ */
#define TI 64
#define TJ 16
#define TP 128

int or_dd_gemm(int transA, int m, int n, int k,
               const double *Ah, const double *Al, int lda,
               const double *Bh, const double *Bl, int ldb,
               double *Ch, double *Cl, int ldc)
{
    if (m < 0 || n < 0 || k < 0) return -1;
    int ntj = (n + TJ - 1) / TJ, nti = (m + TI - 1) / TI;
    int ntiles = ntj * nti;
#pragma omp parallel
    {
        double *ah = (double *)malloc(sizeof(double) * TP * TI);
        double *al = (double *)malloc(sizeof(double) * TP * TI);
        double *sh = (double *)malloc(sizeof(double) * TJ * TI);
        double *sl = (double *)malloc(sizeof(double) * TJ * TI);
#pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < ntiles; ++t) {
            int j0 = (t / nti) * TJ, i0 = (t % nti) * TI;
            int nj = (n - j0 < TJ) ? n - j0 : TJ;
            int ni = (m - i0 < TI) ? m - i0 : TI;
            for (int q = 0; q < TJ * TI; ++q) { sh[q] = 0.0; sl[q] = 0.0; }
            for (int p0 = 0; p0 < k; p0 += TP) {
                int np = (k - p0 < TP) ? k - p0 : TP;
                /* pack op(A)(i0.., p0..) as ah[pp*TI + ii] */
                for (int pp = 0; pp < np; ++pp)
                    for (int ii = 0; ii < ni; ++ii) {
                        size_t src = transA ? IX(p0 + pp, i0 + ii, lda) : IX(i0 + ii, p0 + pp, lda);
                        ah[pp * TI + ii] = Ah[src];
                        al[pp * TI + ii] = Al ? Al[src] : 0.0;
                    }
                for (int jj = 0; jj < nj; ++jj) {
                    double *shj = sh + jj * TI, *slj = sl + jj * TI;
                    for (int pp = 0; pp < np; ++pp) {
                        size_t bi = IX(p0 + pp, j0 + jj, ldb);
                        dd_t b = { Bh[bi], Bl ? Bl[bi] : 0.0 };
                        const double *ahp = ah + pp * TI, *alp = al + pp * TI;
                        for (int ii = 0; ii < ni; ++ii) {
                            dd_t a = { ahp[ii], alp[ii] };
                            dd_t prod = dd_mul(a, b);
                            dd_t acc = { shj[ii], slj[ii] };
                            acc = dd_add_pair(acc, prod);
                            shj[ii] = acc.hi;
                            slj[ii] = acc.lo;
                        }
                    }
                }
            }
            for (int jj = 0; jj < nj; ++jj)
                for (int ii = 0; ii < ni; ++ii) {
                    Ch[IX(i0 + ii, j0 + jj, ldc)] = sh[jj * TI + ii];
                    if (Cl) Cl[IX(i0 + ii, j0 + jj, ldc)] = sl[jj * TI + ii];
                }
        }
        free(ah); free(al); free(sh); free(sl);
    }
    return 0;
}

/* Column dot product x_i^T y_j in double-double, terms in index order. */
static dd_t dd_dot_cols(int n, const double *xh, const double *xl, const double *yh, const double *yl)
{
    dd_t acc = dd_from(0.0);
    for (int p = 0; p < n; ++p) {
        dd_t a = { xh[p], xl ? xl[p] : 0.0 };
        dd_t b = { yh[p], yl ? yl[p] : 0.0 };
        acc = dd_add_pair(acc, dd_mul(a, b));
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 in double-double (one iteration).                             */
/*   A: FP64 symmetric n x n.  X = Xh + Xl: DD, updated in place.            */
/*   lam_h/lam_l: the Rayleigh quotients of the input X (output).            */
/*   r_h: r_i = 1 - x_i^T x_i (output, may be NULL).                         */
/*   E_h: the correction matrix (output, may be NULL).                       */
/*   emax: max |e_ij| (output).                                              */
/* Returns 0, or -3 when two Rayleigh quotients coincide exactly.            */
/* ------------------------------------------------------------------------ */
static int grouped_correction(int n, const double *Xh, const double *Xl, const dd_t *lam,
                              const double *Wh, const double *Wl, double *Eh, double *El,
                              double tau, int *groups_out);
int or_refine_dd_step_grouped(int n, const double *A, double *Xh, double *Xl,
                              double *lam_h, double *lam_l, double *r_h, double *E_h,
                              double *emax, double tau, int *groups_out);

int or_refine_dd_step(int n, const double *A, double *Xh, double *Xl,
                      double *lam_h, double *lam_l, double *r_h, double *E_h, double *emax)
{
    return or_refine_dd_step_grouped(n, A, Xh, Xl, lam_h, lam_l, r_h, E_h, emax, 0.0, NULL);
}

int or_refine_dd_step_grouped(int n, const double *A, double *Xh, double *Xl,
                              double *lam_h, double *lam_l, double *r_h, double *E_h,
                              double *emax, double tau, int *groups_out)
{
    size_t nn = (size_t)n * n;
    double *Vh = (double *)malloc(sizeof(double) * nn), *Vl = (double *)malloc(sizeof(double) * nn);
    double *Wh = (double *)malloc(sizeof(double) * nn), *Wl = (double *)malloc(sizeof(double) * nn);
    dd_t *lam = (dd_t *)malloc(sizeof(dd_t) * n), *rr = (dd_t *)malloc(sizeof(dd_t) * n);
    if (!Vh || !Vl || !Wh || !Wl || !lam || !rr) return -5;
    int status = 0;

    /* V = A X (exact products, double-double sums) */
    or_dd_gemm(0, n, n, n, A, NULL, n, Xh, Xl, n, Vh, Vl, n);

    /* r_i = 1 - x_i^T x_i and the Rayleigh quotients lambda_i */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double *xh = Xh + IX(0, i, n), *xl = Xl + IX(0, i, n);
        dd_t s = dd_dot_cols(n, xh, xl, xh, xl);
        rr[i] = dd_sub(dd_from(1.0), s);
        dd_t xv = dd_dot_cols(n, xh, xl, Vh + IX(0, i, n), Vl + IX(0, i, n));
        lam[i] = dd_div(xv, dd_sub(dd_from(1.0), rr[i]));
    }

    /* V <- V - X D, then W = X^T (V - X D) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int p = 0; p < n; ++p) {
            size_t q = IX(p, j, n);
            dd_t v = { Vh[q], Vl[q] };
            dd_t x = { Xh[q], Xl[q] };
            v = dd_sub(v, dd_mul(x, lam[j]));
            Vh[q] = v.hi; Vl[q] = v.lo;
        }
    or_dd_gemm(1, n, n, n, Xh, Xl, n, Vh, Vl, n, Wh, Wl, n);

    /* the correction matrix E (first order; stored in W unless groups are formed,
       which need W itself) */
    double *Eh = Wh, *El = Wl;
    if (tau > 0.0) {
        Eh = (double *)malloc(sizeof(double) * nn);
        El = (double *)malloc(sizeof(double) * nn);
        if (!Eh || !El) return -5;
    }
    for (int j = 0; j < n && status == 0; ++j)
        for (int i = 0; i < n; ++i) {
            size_t q = IX(i, j, n);
            dd_t e;
            if (i == j) {
                e = rr[i];
                e.hi *= 0.5; e.lo *= 0.5;
            } else {
                dd_t den = dd_sub(lam[j], lam[i]);
                if (den.hi == 0.0) { status = -3; break; }
                dd_t w = { Wh[q], Wl[q] };
                e = dd_div(w, den);
            }
            Eh[q] = e.hi; El[q] = e.lo;
        }
    if (groups_out) *groups_out = 0;
    if (status == 0 && tau > 0.0)
        status = grouped_correction(n, Xh, Xl, lam, Wh, Wl, Eh, El, tau, groups_out);
    double m = 0.0;
    for (size_t q = 0; q < nn; ++q) {
        if (E_h) E_h[q] = Eh[q];
        if (fabs(Eh[q]) > m) m = fabs(Eh[q]);
    }
    if (Eh != Wh) {
        memcpy(Wh, Eh, sizeof(double) * nn);
        memcpy(Wl, El, sizeof(double) * nn);
        free(Eh); free(El);
    }

    if (status == 0) {
        /* X <- X + X E (products and sum in double-double) */
        or_dd_gemm(0, n, n, n, Xh, Xl, n, Wh, Wl, n, Vh, Vl, n);
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nn; ++q) {
            dd_t x = { Xh[q], Xl[q] };
            dd_t u = { Vh[q], Vl[q] };
            x = dd_add(x, u);
            Xh[q] = x.hi; Xl[q] = x.lo;
        }
    }
    for (int i = 0; i < n; ++i) {
        if (lam_h) lam_h[i] = lam[i].hi;
        if (lam_l) lam_l[i] = lam[i].lo;
        if (r_h) r_h[i] = rr[i].hi;
    }
    if (emax) *emax = m;
    free(Vh); free(Vl); free(Wh); free(Wl); free(lam); free(rr);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Grouped correction (Rayleigh-Ritz on strongly coupled columns).           */
/* ------------------------------------------------------------------------ */
#define OR_GROUP_MAX 128

static int uf_find(int *par, int a)
{
    while (par[a] != a) { par[a] = par[par[a]]; a = par[a]; }
    return a;
}

/* Symmetric eigenproblem of the k x k DD matrix M (row-major, overwritten):
   cyclic Jacobi rotations until every off-diagonal entry is below 1e-32 of
   the largest diagonal entry. Q (row-major) receives the eigenvectors as
   columns; the eigenvalues are left on M's diagonal. */
static void dd_jacobi(int k, dd_t *M, dd_t *Q)
{
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) Q[a * k + b] = dd_from(a == b ? 1.0 : 0.0);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double dmax = 0.0, off = 0.0;
        for (int a = 0; a < k; ++a) dmax = fmax(dmax, fabs(M[a * k + a].hi));
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) off = fmax(off, fabs(M[a * k + b].hi));
        if (off <= 1e-32 * dmax || off == 0.0) break;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                dd_t apq = M[p * k + q];
                if (apq.hi == 0.0) continue;
                /* theta = (a_qq - a_pp) / (2 a_pq); t = sign(theta) / (|theta| + sqrt(theta^2 + 1)) */
                dd_t theta = dd_div(dd_sub(M[q * k + q], M[p * k + p]), dd_mul_d(apq, 2.0));
                dd_t at = theta.hi < 0.0 ? dd_neg(theta) : theta;
                dd_t t;
                if (at.hi > 1e30) t = dd_div(dd_from(0.5), at);
                else t = dd_div(dd_from(1.0), dd_add(at, dd_sqrt(dd_add(dd_mul(at, at), dd_from(1.0)))));
                if (theta.hi < 0.0) t = dd_neg(t);
                dd_t c = dd_div(dd_from(1.0), dd_sqrt(dd_add(dd_mul(t, t), dd_from(1.0))));
                dd_t sn = dd_mul(t, c);
                for (int r = 0; r < k; ++r) {          /* M <- M J (columns p, q) */
                    dd_t mp = M[r * k + p], mq = M[r * k + q];
                    M[r * k + p] = dd_sub(dd_mul(c, mp), dd_mul(sn, mq));
                    M[r * k + q] = dd_add(dd_mul(sn, mp), dd_mul(c, mq));
                }
                for (int r = 0; r < k; ++r) {          /* M <- J^T M (rows p, q) */
                    dd_t mp = M[p * k + r], mq = M[q * k + r];
                    M[p * k + r] = dd_sub(dd_mul(c, mp), dd_mul(sn, mq));
                    M[q * k + r] = dd_add(dd_mul(sn, mp), dd_mul(c, mq));
                }
                for (int r = 0; r < k; ++r) {          /* Q <- Q J */
                    dd_t qp = Q[r * k + p], qq = Q[r * k + q];
                    Q[r * k + p] = dd_sub(dd_mul(c, qp), dd_mul(sn, qq));
                    Q[r * k + q] = dd_add(dd_mul(sn, qp), dd_mul(c, qq));
                }
            }
    }
}

/* Replaces the first-order columns of E for every linked group (see the file
   header). Group members are kept in ascending index order c_0 < ... < c_{k-1};
   each member column receives the Ritz vector closest to it (largest entry
   first) with the sign that makes its own entry positive. For a member column
   c_b with Ritz vector y and
   value mu:  e_{c_a c_b} = y_a - [a == b]  and, for rows i outside the group,
   e_{i c_b} = (sum_a w_{i c_a} y_a) / (mu - lambda_i). */
static int grouped_correction(int n, const double *Xh, const double *Xl, const dd_t *lam,
                              const double *Wh, const double *Wl, double *Eh, double *El,
                              double tau, int *groups_out)
{
    int *par = (int *)malloc(sizeof(int) * n);
    int *size = (int *)calloc((size_t)n, sizeof(int));
    if (!par || !size) return -5;
    for (int j = 0; j < n; ++j) par[j] = j;
    /* link columns i and j whenever |e_ij| > tau (i != j) */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            if (i == j || !(fabs(Eh[IX(i, j, n)]) > tau)) continue;
            int a = uf_find(par, j), b = uf_find(par, i);
            if (a != b) par[a < b ? b : a] = a < b ? a : b;
        }
    for (int j = 0; j < n; ++j) size[uf_find(par, j)]++;
    int ngroups = 0, status = 0;
    int *mem = (int *)malloc(sizeof(int) * OR_GROUP_MAX);
    dd_t *G = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *T = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *L = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *M = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *Q = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *Y = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *mu = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX);
    dd_t *Ynew = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX * OR_GROUP_MAX);
    dd_t *munew = (dd_t *)malloc(sizeof(dd_t) * OR_GROUP_MAX);
    dd_t *Ecol = (dd_t *)malloc(sizeof(dd_t) * (size_t)n * OR_GROUP_MAX);
    if (!mem || !G || !T || !L || !M || !Q || !Y || !mu || !Ynew || !munew || !Ecol) return -5;
    for (int root = 0; root < n && status == 0; ++root) {
        if (uf_find(par, root) != root || size[root] < 2 || size[root] > OR_GROUP_MAX) continue;
        int k = 0;
        for (int j = 0; j < n; ++j)
            if (uf_find(par, j) == root) mem[k++] = j;
        ++ngroups;
        /* G = X_C^T X_C and T = W_CC + G_CC D_C, symmetrised */
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                const size_t ca = IX(0, mem[a], n), cb = IX(0, mem[b], n);
                G[a * k + b] = dd_dot_cols(n, Xh + ca, Xl + ca, Xh + cb, Xl + cb);
            }
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                size_t q = IX(mem[a], mem[b], n);
                dd_t w = { Wh[q], Wl[q] };
                T[a * k + b] = dd_add(w, dd_mul(G[a * k + b], lam[mem[b]]));
            }
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) {
                dd_t avg = dd_add(T[a * k + b], T[b * k + a]);
                avg.hi *= 0.5; avg.lo *= 0.5;
                T[a * k + b] = avg; T[b * k + a] = avg;
            }
        /* Cholesky G = L L^T */
        for (int a = 0; a < k * k; ++a) L[a] = dd_from(0.0);
        for (int a = 0; a < k && status == 0; ++a) {
            dd_t d = G[a * k + a];
            for (int c = 0; c < a; ++c) d = dd_sub(d, dd_mul(L[a * k + c], L[a * k + c]));
            if (!(d.hi > 0.0)) { status = -3; break; }
            L[a * k + a] = dd_sqrt(d);
            for (int b = a + 1; b < k; ++b) {
                dd_t v = G[b * k + a];
                for (int c = 0; c < a; ++c) v = dd_sub(v, dd_mul(L[b * k + c], L[a * k + c]));
                L[b * k + a] = dd_div(v, L[a * k + a]);
            }
        }
        if (status != 0) break;
        /* M = L^-1 T L^-T: forward substitution on the columns, then on the rows */
        for (int b = 0; b < k; ++b)
            for (int a = 0; a < k; ++a) {
                dd_t v = T[a * k + b];
                for (int c = 0; c < a; ++c) v = dd_sub(v, dd_mul(L[a * k + c], M[c * k + b]));
                M[a * k + b] = dd_div(v, L[a * k + a]);
            }
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                dd_t v = M[a * k + b];
                for (int c = 0; c < b; ++c) v = dd_sub(v, dd_mul(T[a * k + c], L[b * k + c]));
                T[a * k + b] = dd_div(v, L[b * k + b]);   /* T now holds M */
            }
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) M[a * k + b] = T[a * k + b];
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) {
                dd_t avg = dd_add(M[a * k + b], M[b * k + a]);
                avg.hi *= 0.5; avg.lo *= 0.5;
                M[a * k + b] = avg; M[b * k + a] = avg;
            }
        dd_jacobi(k, M, Q);
        /* Y = L^-T Q: back substitution */
        for (int b = 0; b < k; ++b)
            for (int a = k - 1; a >= 0; --a) {
                dd_t v = Q[a * k + b];
                for (int c = a + 1; c < k; ++c) v = dd_sub(v, dd_mul(L[c * k + a], Y[c * k + b]));
                Y[a * k + b] = dd_div(v, L[a * k + a]);
            }
        for (int b = 0; b < k; ++b) mu[b] = M[b * k + b];
        /* assignment: repeatedly give the Ritz vector with the largest remaining entry
           |y_a| (over unassigned members a and vectors) to member a, so that each column
           keeps the Ritz vector closest to it (first indices on ties) */
        int used_v[OR_GROUP_MAX], used_c[OR_GROUP_MAX];
        for (int a = 0; a < k; ++a) { used_v[a] = 0; used_c[a] = 0; }
        for (int step = 0; step < k; ++step) {
            int ba = -1, bv = -1;
            double best = -1.0;
            for (int a = 0; a < k; ++a) {
                if (used_c[a]) continue;
                for (int v = 0; v < k; ++v) {
                    if (used_v[v]) continue;
                    double x = fabs(Y[a * k + v].hi);
                    if (x > best) { best = x; ba = a; bv = v; }
                }
            }
            used_c[ba] = 1; used_v[bv] = 1;
            munew[ba] = mu[bv];
            const int flip = Y[ba * k + bv].hi < 0.0;
            for (int r = 0; r < k; ++r) Ynew[r * k + ba] = flip ? dd_neg(Y[r * k + bv]) : Y[r * k + bv];
        }
        /* new columns of E for the members */
        for (int b = 0; b < k; ++b) {
            dd_t *ec = Ecol + (size_t)b * n;
            for (int i = 0; i < n; ++i) {
                int in_group = -1;
                for (int a = 0; a < k; ++a)
                    if (mem[a] == i) in_group = a;
                if (in_group >= 0) {
                    dd_t y = Ynew[in_group * k + b];
                    ec[i] = (in_group == b) ? dd_sub(y, dd_from(1.0)) : y;
                } else {
                    dd_t num = dd_from(0.0);
                    for (int a = 0; a < k; ++a) {
                        size_t q = IX(i, mem[a], n);
                        dd_t w = { Wh[q], Wl[q] };
                        num = dd_add(num, dd_mul(w, Ynew[a * k + b]));
                    }
                    dd_t den = dd_sub(munew[b], lam[i]);
                    if (den.hi == 0.0) { status = -3; break; }
                    ec[i] = dd_div(num, den);
                }
            }
        }
        for (int b = 0; b < k && status == 0; ++b)
            for (int i = 0; i < n; ++i) {
                size_t q = IX(i, mem[b], n);
                Eh[q] = Ecol[(size_t)b * n + i].hi;
                El[q] = Ecol[(size_t)b * n + i].lo;
            }
    }
    if (groups_out) *groups_out = ngroups;
    free(par); free(size); free(mem); free(G); free(T); free(L); free(M); free(Q); free(Y);
    free(mu); free(Ynew); free(munew); free(Ecol);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Exponents and 7-bit digit planes.                                         */
/* ------------------------------------------------------------------------ */

/* frexp exponent: |v| < 2^e and |v| >= 2^(e-1) for v != 0; 0 for v == 0. */
static int exp_above(double v)
{
    int e = 0;
    if (v == 0.0) return 0;
    (void)frexp(v, &e);
    return e;
}

/* ceil(log2 v) for v > 0, exactly: v = f 2^e with f in [0.5, 1). */
static int ceil_log2(double v)
{
    int e = 0;
    double f = frexp(v, &e);
    return (f == 0.5) ? e - 1 : e;
}

/* Digit planes of M (m x ncols, column-major, leading dim ld).
 * by_rows == 0: one exponent per column j, e_j with max_i |M_ij| < 2^e_j;
 *               plane layout (i, j) -> i + j*m (K = row index contiguous).
 * by_rows == 1: one exponent per row i; plane layout (i, j) -> j + i*ncols.
 * Digit r (1..k) of an entry a with scale e is
 *     sign(a) * floor(|a| 2^(7r - e)) mod 128,
 * i.e. the r-th base-128 digit of the truncated magnitude, computed here by
 * repeated exact multiplication by 128. Planes are stored plane-major:
 * plane r-1 starts at planes + (r-1) * m * ncols.
 * trunc_out (optional, same layout as M with leading dim m): the value the
 * first k digits represent. Returns 0, or -4 when an exponent is outside the
 * range where the scaling is exact. */
int or_split_s7(int by_rows, int m, int ncols, const double *M, int ld, int k,
                int *exps, int8_t *planes, double *trunc_out)
{
    int nvec = by_rows ? m : ncols, len = by_rows ? ncols : m;
    size_t plane_sz = (size_t)m * ncols;
    int status = 0;
    for (int v = 0; v < nvec; ++v) {
        double mx = 0.0;
        for (int t = 0; t < len; ++t) {
            double a = by_rows ? M[IX(v, t, ld)] : M[IX(t, v, ld)];
            if (fabs(a) > mx) mx = fabs(a);
        }
        int e = exp_above(mx);
        if (mx != 0.0 && (e < -900 || e > 900)) status = -4;
        exps[v] = e;
        for (int t = 0; t < len; ++t) {
            int i = by_rows ? v : t, j = by_rows ? t : v;
            double a = M[IX(i, j, ld)];
            size_t off = by_rows ? (size_t)i * ncols + j : (size_t)j * m + i;
            double y = ldexp(fabs(a), -e);  /* in [0, 1) */
            int sgn = (a < 0.0) ? -1 : 1;
            double val = 0.0;
            for (int r = 1; r <= k; ++r) {
                double t128 = y * 128.0;
                double d = floor(t128);
                y = t128 - d;
                planes[(size_t)(r - 1) * plane_sz + off] = (int8_t)(sgn * (int)d);
                val += ldexp(d, e - 7 * r);
            }
            if (trunc_out) trunc_out[IX(i, j, m)] = (a < 0.0) ? -val : val;
        }
    }
    return status;
}

/* C(i, j) = sum_p Ap[p + i*lda] * Bp[p + j*ldb]   (exact, int64).
 * C is column-major m x n. */
int or_slice_gemm_i64(int m, int n, int K, const int8_t *Ap, int lda,
                      const int8_t *Bp, int ldb, int64_t *C)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            int64_t s = 0;
            const int8_t *a = Ap + (size_t)i * lda, *b = Bp + (size_t)j * ldb;
            for (int p = 0; p < K; ++p) s += (int64_t)a[p] * (int64_t)b[p];
            C[IX(i, j, m)] = s;
        }
    return 0;
}

/* The FP64 splitting of eq. (a) (by_rows = 1, sigma_i per row) or eq. (x)
 * (by_rows = 0, tau_j per column): for r = 1..ns,
 *   v = max |current remainder| along the row/column,
 *   sigma = 0.75 * 2^ceil(log2 v) * 2^alpha   (0 if v == 0),
 *   slice = fl((sigma + a) - sigma),  a <- fl(a - slice).
 * slices: ns matrices of m x ncols (leading dim m), then the remainder. */
int or_sigma_split(int by_rows, int m, int ncols, const double *M, int ld, int alpha, int ns,
                   double *slices)
{
    size_t sz = (size_t)m * ncols;
    double *rem = slices + (size_t)ns * sz;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ncols; ++j)
        for (int i = 0; i < m; ++i) rem[IX(i, j, m)] = M[IX(i, j, ld)];
    int nvec = by_rows ? m : ncols;
    double *sig = (double *)malloc(sizeof(double) * (size_t)(nvec > 0 ? nvec : 1));
    if (!sig) return -5;
    for (int r = 0; r < ns; ++r) {
        double *out = slices + (size_t)r * sz;
        /* sigma of each row / column from the maximum of its current remainder (the
         * traversal order does not change a maximum) */
        if (by_rows) {
#pragma omp parallel for schedule(static)
            for (int ib = 0; ib < m; ib += 64) {
                int ie = ib + 64 < m ? ib + 64 : m;
                double mx[64];
                for (int i = ib; i < ie; ++i) mx[i - ib] = 0.0;
                for (int j = 0; j < ncols; ++j)
                    for (int i = ib; i < ie; ++i) {
                        double a = fabs(rem[IX(i, j, m)]);
                        if (a > mx[i - ib]) mx[i - ib] = a;
                    }
                for (int i = ib; i < ie; ++i)
                    sig[i] = (mx[i - ib] == 0.0) ? 0.0 : ldexp(0.75, ceil_log2(mx[i - ib]) + alpha);
            }
        } else {
#pragma omp parallel for schedule(static)
            for (int j = 0; j < ncols; ++j) {
                double mx = 0.0;
                for (int i = 0; i < m; ++i) {
                    double a = fabs(rem[IX(i, j, m)]);
                    if (a > mx) mx = a;
                }
                sig[j] = (mx == 0.0) ? 0.0 : ldexp(0.75, ceil_log2(mx) + alpha);
            }
        }
        /* slice = fl((sigma + a) - sigma), a <- fl(a - slice) */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ncols; ++j)
            for (int i = 0; i < m; ++i) {
                size_t q = IX(i, j, m);
                double sigma = by_rows ? sig[i] : sig[j];
                volatile double s1 = sigma + rem[q];
                double sl = s1 - sigma;
                out[q] = sl;
                rem[q] = rem[q] - sl;
            }
    }
    free(sig);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* beta of Sec. 4.1 (floor form, xi = n unless given):                       */
/*   beta = floor(log2( (1/(0.75u)) sqrt( xi delta g / (L S) ) )),           */
/*   g = min_{i != j} |lam_i - lam_j|, L = max |lam_k|,                      */
/*   S = sum_j 2^(2 ceil(log2 w_j)), w_j = max_i |x_ij|.                     */
/* Evaluation order (both sides of any comparison use it):                   */
/*   q = ((xi * delta) * g) / (L * S);  t = sqrt(q) / (0.75 * 2^-53);        */
/*   beta = e - 1 where t = f 2^e, f in [0.5, 1)  (exact floor of log2 t).   */
/* The grid of X^(1) in column j is then 2^(c_j + beta - 54) (the rounding   */
/* bound u * ufp(tau_j) of eq. (minamihata)); with 7-bit planes starting at  */
/* e_j (w_j < 2^e_j) the number of planes is                                 */
/*   kx = ceil((54 - beta + max_j (e_j - c_j)) / 7), clamped to [1, kx_max].  */
/* Returns 0, or -3 if g == 0, or -2 if an input is not finite.              */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* The rule itself, from the column maxima w_j of X (w_j = 0: an empty column). */
int or_beta_core(int n, const double *lam, const double *w, double delta, double xi,
                 int kx_max, int *beta_out, int *kx_out, double *gap_out, double *lmax_out,
                 double *S_out);

int or_beta_rule(int n, const double *lam, const double *X, int ldx, double delta, double xi,
                 int kx_max, int *beta_out, int *kx_out, double *gap_out, double *lmax_out,
                 double *S_out)
{
    double *w = (double *)malloc(sizeof(double) * n);
    for (int j = 0; j < n; ++j) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) {
            double a = fabs(X[IX(i, j, ldx)]);
            if (!isfinite(a)) { free(w); return -2; }
            if (a > m) m = a;
        }
        w[j] = m;
    }
    int st = or_beta_core(n, lam, w, delta, xi, kx_max, beta_out, kx_out, gap_out, lmax_out,
                          S_out);
    free(w);
    return st;
}

int or_beta_core(int n, const double *lam, const double *wmax, double delta, double xi,
                 int kx_max, int *beta_out, int *kx_out, double *gap_out, double *lmax_out,
                 double *S_out)
{
    double *s = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        if (!isfinite(lam[i])) { free(s); return -2; }
        s[i] = lam[i];
    }
    qsort(s, n, sizeof(double), cmp_double);
    double g = INFINITY, L = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        double d = s[i + 1] - s[i];
        if (d < g) g = d;
    }
    for (int i = 0; i < n; ++i)
        if (fabs(lam[i]) > L) L = fabs(lam[i]);
    free(s);
    double S = 0.0;
    int extra = 0;
    for (int j = 0; j < n; ++j) {
        double w = wmax[j];
        if (w == 0.0) continue;
        int c = ceil_log2(w), e = exp_above(w);
        S += ldexp(1.0, 2 * c);
        if (e - c > extra) extra = e - c;
    }
    if (gap_out) *gap_out = g;
    if (lmax_out) *lmax_out = L;
    if (S_out) *S_out = S;
    if (n > 1 && !(g > 0.0)) return -3;
    if (xi <= 0.0) xi = (double)n;
    double q = ((xi * delta) * g) / (L * S);
    double t = sqrt(q) / (0.75 * ldexp(1.0, -53));
    int e = 0;
    (void)frexp(t, &e);
    int beta = e - 1;
    int num = 54 - beta + extra;
    int kx = (num <= 0) ? 1 : (num + 6) / 7;
    if (kx < 1) kx = 1;
    if (kx > kx_max) kx = kx_max;
    *beta_out = beta;
    *kx_out = kx;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One iteration of the proposed method (Sec. 3) with exact products:        */
/*   1. beta and kx from the rule above (lam = previous eigenvalue estimates)*/
/*   2. X^(1): truncation of X to kx 7-bit planes per column                 */
/*   3. Algorithm 1 on X^(1) in double-double                                */
/* Outputs: X1 (FP64), Xnew_h/Xnew_l, lam_h/lam_l (Rayleigh quotients of     */
/* X^(1)), r_h, emax, beta, kx.                                              */
/* ------------------------------------------------------------------------ */
int or_method_step_grouped(int n, const double *A, const double *X, const double *lam_prev,
                           double delta, double xi, int kx_max, int kx_force,
                           double *X1, double *Xnew_h, double *Xnew_l, double *lam_h,
                           double *lam_l, double *r_h, double *emax, int *beta_out, int *kx_out,
                           double tau, int *groups_out);

int or_method_step(int n, const double *A, const double *X, const double *lam_prev,
                   double delta, double xi, int kx_max, int kx_force,
                   double *X1, double *Xnew_h, double *Xnew_l, double *lam_h, double *lam_l,
                   double *r_h, double *emax, int *beta_out, int *kx_out)
{
    return or_method_step_grouped(n, A, X, lam_prev, delta, xi, kx_max, kx_force, X1, Xnew_h,
                                  Xnew_l, lam_h, lam_l, r_h, emax, beta_out, kx_out, 0.0, NULL);
}

int or_method_step_grouped(int n, const double *A, const double *X, const double *lam_prev,
                           double delta, double xi, int kx_max, int kx_force,
                           double *X1, double *Xnew_h, double *Xnew_l, double *lam_h,
                           double *lam_l, double *r_h, double *emax, int *beta_out, int *kx_out,
                           double tau, int *groups_out)
{
    int beta = 0, kx = 0;
    int st = or_beta_rule(n, lam_prev, X, n, delta, xi, kx_max, &beta, &kx, NULL, NULL, NULL);
    if (st != 0) return st;
    if (kx_force > 0) kx = kx_force;
    *beta_out = beta;
    *kx_out = kx;
    size_t nn = (size_t)n * n;
    int *ex = (int *)malloc(sizeof(int) * n);
    int8_t *pl = (int8_t *)malloc(nn * (size_t)kx);
    st = or_split_s7(0, n, n, X, n, kx, ex, pl, X1);
    free(ex); free(pl);
    if (st != 0) return st;
    for (size_t q = 0; q < nn; ++q) { Xnew_h[q] = X1[q]; Xnew_l[q] = 0.0; }
    return or_refine_dd_step_grouped(n, A, Xnew_h, Xnew_l, lam_h, lam_l, r_h, NULL, emax, tau,
                                     groups_out);
}

/* ------------------------------------------------------------------------ */
/* Eigenpairs of diag(d) + rho u u^T, rho > 0, d strictly ascending (DD).    */
/* The j-th eigenvalue lies in (d_j, d_{j+1}) (last one in                   */
/* (d_n, d_n + rho u^T u]) and solves 1 + rho sum_i u_i^2 / (d_i - lambda)=0 */
/* (increasing in lambda on each interval). It is located by bisection in    */
/* double-double on the offset from the nearer pole, and the eigenvector is  */
/* (D - lambda I)^-1 u normalised.                                           */
/* Outputs: lam (DD), X (DD, column-major n x n).                            */
/* ------------------------------------------------------------------------ */
static dd_t secular_f(int n, const double *dh, const double *dl, const double *u, double rho,
                      dd_t origin, dd_t mu)
{
    /* 1 + rho * sum u_i^2 / ((d_i - origin) - mu) */
    dd_t s = dd_from(0.0);
    for (int i = 0; i < n; ++i) {
        dd_t di = { dh[i], dl[i] };
        dd_t den = dd_sub(dd_sub(di, origin), mu);
        dd_t num = two_prod(u[i], u[i]);
        s = dd_add(s, dd_div(num, den));
    }
    return dd_add(dd_from(1.0), dd_mul_d(s, rho));
}

int or_secular_rank1(int n, const double *dh, const double *dl, double rho, const double *u,
                     double *lam_h, double *lam_l, double *Xh, double *Xl, int idx_lo, int idx_hi)
{
    if (rho <= 0.0) return -1;
    for (int i = 0; i + 1 < n; ++i)
        if (!(dh[i] < dh[i + 1] || (dh[i] == dh[i + 1] && dl[i] < dl[i + 1]))) return -1;
    dd_t utu = dd_from(0.0);
    for (int i = 0; i < n; ++i) utu = dd_add(utu, two_prod(u[i], u[i]));
    if (idx_lo < 0) idx_lo = 0;
    if (idx_hi > n || idx_hi <= 0) idx_hi = n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = idx_lo; j < idx_hi; ++j) {
        dd_t dj = { dh[j], dl[j] };
        dd_t width;
        if (j + 1 < n) {
            dd_t dj1 = { dh[j + 1], dl[j + 1] };
            width = dd_sub(dj1, dj);
        } else {
            width = dd_mul_d(utu, rho);
        }
        /* choose the nearer pole as origin */
        dd_t half = { width.hi * 0.5, width.lo * 0.5 };
        dd_t origin = dj;
        int from_right = 0;
        if (j + 1 < n) {
            dd_t fm = secular_f(n, dh, dl, u, rho, dj, half);
            if (fm.hi < 0.0) { /* root in (mid, d_{j+1}) */
                origin.hi = dh[j + 1]; origin.lo = dl[j + 1];
                from_right = 1;
            }
        }
        /* bisection on mu in (0, half] (left origin) or (-half, 0) (right) */
        dd_t lo = dd_from(0.0), hi = (j + 1 < n) ? half : width;
        if (from_right) { lo = dd_neg(half); hi = dd_from(0.0); }
        for (int it = 0; it < 400; ++it) {
            dd_t mid = dd_add(lo, hi);
            mid.hi *= 0.5; mid.lo *= 0.5;
            if ((mid.hi == lo.hi && mid.lo == lo.lo) || (mid.hi == hi.hi && mid.lo == hi.lo)) break;
            dd_t f = secular_f(n, dh, dl, u, rho, origin, mid);
            if (f.hi < 0.0) lo = mid; else hi = mid;
        }
        dd_t mu = dd_add(lo, hi);
        mu.hi *= 0.5; mu.lo *= 0.5;
        dd_t lam = dd_add(origin, mu);
        lam_h[j] = lam.hi; lam_l[j] = lam.lo;
        /* eigenvector */
        dd_t nrm = dd_from(0.0);
        for (int i = 0; i < n; ++i) {
            dd_t di = { dh[i], dl[i] };
            dd_t den = dd_sub(dd_sub(di, origin), mu);
            dd_t x = dd_div(dd_from(u[i]), den);
            Xh[IX(i, j, n)] = x.hi; Xl[IX(i, j, n)] = x.lo;
            nrm = dd_add(nrm, dd_mul(x, x));
        }
        dd_t s = dd_sqrt(nrm);
        for (int i = 0; i < n; ++i) {
            dd_t x = { Xh[IX(i, j, n)], Xl[IX(i, j, n)] };
            x = dd_div(x, s);
            Xh[IX(i, j, n)] = x.hi; Xl[IX(i, j, n)] = x.lo;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Scalar entry points for exact-rational checks of the primitives above.    */
/* ------------------------------------------------------------------------ */
void or_two_sum(double a, double b, double *s, double *e) { dd_t r = two_sum(a, b); *s = r.hi; *e = r.lo; }
void or_two_prod(double a, double b, double *p, double *e) { dd_t r = two_prod(a, b); *p = r.hi; *e = r.lo; }
void or_dd_binop(int op, double ah, double al, double bh, double bl, double *rh, double *rl)
{
    dd_t a = { ah, al }, b = { bh, bl }, r;
    switch (op) {
    case 0: r = dd_add(a, b); break;
    case 1: r = dd_mul(a, b); break;
    case 2: r = dd_div(a, b); break;
    case 3: r = dd_sqrt(a); break;
    default: r = dd_add_pair(a, b); break;
    }
    *rh = r.hi; *rl = r.lo;
}
