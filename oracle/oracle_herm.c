/*
 * CPU oracle, complex Hermitian case: the refinement of Algorithm 1 for a
 * Hermitian matrix A = A^H (the extension that Sec. 5 names as future work).
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: loaded by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the GPU library.
 *
 * Complex matrices are held as separate real and imaginary parts, each
 * column-major n x n (element (i, j) at i + j*n); double-double matrices as
 * (hi, lo) pairs of such parts.
 *
 *  or_herm_dd_step     One iteration of Algorithm 1 with every operation in
 *                      complex double-double: V = A X, r_i = 1 - x_i^H x_i,
 *                      lambda_i = Re(x_i^H v_i) / (1 - r_i) (x^H A x is real
 *                      for Hermitian A), W = X^H (V - X D),
 *                      e_ij = w_ij / (lambda_j - lambda_i), e_ii = r_i / 2,
 *                      X <- X + X E. Each complex product is the sum of two
 *                      real double-double products per part (or_dd_gemm).
 *                      Iterated to its fixed point this gives X_true.
 *  or_herm_beta_rule   beta and k_X of Sec. 4.1 applied to the complex X: the
 *                      column maximum w_j is the largest |real part| or
 *                      |imaginary part| in column j (both parts are cut to
 *                      the same grid), everything else as in the real rule.
 *  or_herm_method_step beta, then X^(1) = each part of each column of X
 *                      truncated to k_X 7-bit digits below 2^(e_j) (e_j from
 *                      the column maximum above; this is or_split_s7 applied
 *                      to the stacked 2n x n matrix [Re X; Im X]), then
 *                      or_herm_dd_step on X^(1).
 *
 * Build with -ffp-contract=off.
 */
#include "dd.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

int or_dd_gemm(int transA, int m, int n, int k, const double *Ah, const double *Al, int lda,
               const double *Bh, const double *Bl, int ldb, double *Ch, double *Cl, int ldc);
int or_split_s7(int by_rows, int m, int ncols, const double *M, int ld, int k, int *exps,
                int8_t *planes, double *trunc_out);
int or_beta_core(int n, const double *lam, const double *w, double delta, double xi,
                 int kx_max, int *beta_out, int *kx_out, double *gap_out, double *lmax_out,
                 double *S_out);

/* A complex double-double matrix: real part (rh, rl), imaginary part (ih, il). */
typedef struct {
    double *rh, *rl, *ih, *il;
} zdd;

static int zdd_alloc(size_t nn, zdd *z)
{
    z->rh = (double *)calloc(nn, sizeof(double));
    z->rl = (double *)calloc(nn, sizeof(double));
    z->ih = (double *)calloc(nn, sizeof(double));
    z->il = (double *)calloc(nn, sizeof(double));
    return (z->rh && z->rl && z->ih && z->il) ? 0 : -5;
}

static void zdd_free(zdd *z)
{
    free(z->rh); free(z->rl); free(z->ih); free(z->il);
}

/* C = op(A) B, n x n, op(A) = A (conj = 0) or A^H (conj = 1):
 *   A B:    Re = Ar Br - Ai Bi,      Im = Ar Bi + Ai Br
 *   A^H B:  Re = Ar^T Br + Ai^T Bi,  Im = Ar^T Bi - Ai^T Br
 * A's low parts may be null (an FP64 matrix). */
static int zgemm_dd(int conj, int n, const double *Arh, const double *Arl, const double *Aih,
                    const double *Ail, const zdd *B, zdd *C)
{
    size_t nn = (size_t)n * n;
    zdd T;
    if (zdd_alloc(nn, &T) != 0) { zdd_free(&T); return -5; }
    /* C.r <- Ar Br, T.r <- Ai Bi, C.i <- Ar Bi, T.i <- Ai Br */
    or_dd_gemm(conj, n, n, n, Arh, Arl, n, B->rh, B->rl, n, C->rh, C->rl, n);
    or_dd_gemm(conj, n, n, n, Aih, Ail, n, B->ih, B->il, n, T.rh, T.rl, n);
    or_dd_gemm(conj, n, n, n, Arh, Arl, n, B->ih, B->il, n, C->ih, C->il, n);
    or_dd_gemm(conj, n, n, n, Aih, Ail, n, B->rh, B->rl, n, T.ih, T.il, n);
    const double sg = conj ? 1.0 : -1.0;   /* sign of the Ai Bi term in the real part */
    for (size_t q = 0; q < nn; ++q) {
        dd_t cr = { C->rh[q], C->rl[q] }, tr = { T.rh[q], T.rl[q] };
        dd_t ci = { C->ih[q], C->il[q] }, ti = { T.ih[q], T.il[q] };
        tr.hi *= sg; tr.lo *= sg;
        ti.hi *= -sg; ti.lo *= -sg;
        cr = dd_add(cr, tr);
        ci = dd_add(ci, ti);
        C->rh[q] = cr.hi; C->rl[q] = cr.lo;
        C->ih[q] = ci.hi; C->il[q] = ci.lo;
    }
    zdd_free(&T);
    return 0;
}

/* sum_p a_p b_p over n terms in double-double, index order. */
static dd_t dot_dd(int n, const double *ah, const double *al, const double *bh, const double *bl)
{
    dd_t acc = dd_from(0.0);
    for (int p = 0; p < n; ++p) {
        dd_t a = { ah[p], al[p] }, b = { bh[p], bl[p] };
        acc = dd_add_pair(acc, dd_mul(a, b));
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 for Hermitian A in complex double-double (one iteration).     */
/*   Ar, Ai: FP64 parts of A.  X = (Xrh + Xrl) + i (Xih + Xil): updated.     */
/*   lam_h/lam_l, r_h: as in the real step.  emax: max_ij |e_ij| (modulus).  */
/* Returns 0, or -3 when two Rayleigh quotients coincide exactly.            */
/* ------------------------------------------------------------------------ */
int or_herm_dd_step(int n, const double *Ar, const double *Ai, double *Xrh, double *Xrl,
                    double *Xih, double *Xil, double *lam_h, double *lam_l, double *r_h,
                    double *emax)
{
    size_t nn = (size_t)n * n;
    zdd X = { Xrh, Xrl, Xih, Xil }, V, W;
    int st = zdd_alloc(nn, &V);
    if (st == 0) st = zdd_alloc(nn, &W);
    dd_t *lam = (dd_t *)malloc(sizeof(dd_t) * n), *rr = (dd_t *)malloc(sizeof(dd_t) * n);
    if (st != 0 || !lam || !rr) { zdd_free(&V); zdd_free(&W); free(lam); free(rr); return -5; }

    /* V = A X */
    zgemm_dd(0, n, Ar, NULL, Ai, NULL, &X, &V);

    /* r_i = 1 - x_i^H x_i, lambda_i = Re(x_i^H v_i) / (1 - r_i) */
    for (int i = 0; i < n; ++i) {
        size_t c = HX(0, i, n);
        dd_t s = dd_add(dot_dd(n, Xrh + c, Xrl + c, Xrh + c, Xrl + c),
                        dot_dd(n, Xih + c, Xil + c, Xih + c, Xil + c));
        rr[i] = dd_sub(dd_from(1.0), s);
        dd_t xv = dd_add(dot_dd(n, Xrh + c, Xrl + c, V.rh + c, V.rl + c),
                         dot_dd(n, Xih + c, Xil + c, V.ih + c, V.il + c));
        lam[i] = dd_div(xv, dd_sub(dd_from(1.0), rr[i]));
    }

    /* V <- V - X D (lambda real), then W = X^H (V - X D) */
    for (int j = 0; j < n; ++j)
        for (int p = 0; p < n; ++p) {
            size_t q = HX(p, j, n);
            dd_t vr = { V.rh[q], V.rl[q] }, vi = { V.ih[q], V.il[q] };
            dd_t xr = { Xrh[q], Xrl[q] }, xi = { Xih[q], Xil[q] };
            vr = dd_sub(vr, dd_mul(xr, lam[j]));
            vi = dd_sub(vi, dd_mul(xi, lam[j]));
            V.rh[q] = vr.hi; V.rl[q] = vr.lo;
            V.ih[q] = vi.hi; V.il[q] = vi.lo;
        }
    zgemm_dd(1, n, Xrh, Xrl, Xih, Xil, &V, &W);

    /* E (stored in W): e_ij = w_ij / (lambda_j - lambda_i), e_ii = r_i / 2 */
    int status = 0;
    double m = 0.0;
    for (int j = 0; j < n && status == 0; ++j)
        for (int i = 0; i < n; ++i) {
            size_t q = HX(i, j, n);
            dd_t er, ei;
            if (i == j) {
                er = rr[i];
                er.hi *= 0.5; er.lo *= 0.5;
                ei = dd_from(0.0);
            } else {
                dd_t den = dd_sub(lam[j], lam[i]);
                if (den.hi == 0.0) { status = -3; break; }
                dd_t wr = { W.rh[q], W.rl[q] }, wi = { W.ih[q], W.il[q] };
                er = dd_div(wr, den);
                ei = dd_div(wi, den);
            }
            W.rh[q] = er.hi; W.rl[q] = er.lo;
            W.ih[q] = ei.hi; W.il[q] = ei.lo;
            double a = sqrt(er.hi * er.hi + ei.hi * ei.hi);
            if (a > m) m = a;
        }

    if (status == 0) {
        /* X <- X + X E */
        zgemm_dd(0, n, Xrh, Xrl, Xih, Xil, &W, &V);
        for (size_t q = 0; q < nn; ++q) {
            dd_t xr = { Xrh[q], Xrl[q] }, xi = { Xih[q], Xil[q] };
            dd_t ur = { V.rh[q], V.rl[q] }, ui = { V.ih[q], V.il[q] };
            xr = dd_add(xr, ur);
            xi = dd_add(xi, ui);
            Xrh[q] = xr.hi; Xrl[q] = xr.lo;
            Xih[q] = xi.hi; Xil[q] = xi.lo;
        }
    }
    for (int i = 0; i < n; ++i) {
        if (lam_h) lam_h[i] = lam[i].hi;
        if (lam_l) lam_l[i] = lam[i].lo;
        if (r_h) r_h[i] = rr[i].hi;
    }
    if (emax) *emax = m;
    zdd_free(&V); zdd_free(&W); free(lam); free(rr);
    return status;
}

/* Column maxima over both parts: w_j = max_i max(|Re x_ij|, |Im x_ij|). */
static int herm_colmax(int n, const double *Xr, const double *Xi, double *w)
{
    for (int j = 0; j < n; ++j) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) {
            double a = fabs(Xr[HX(i, j, n)]), b = fabs(Xi[HX(i, j, n)]);
            if (!isfinite(a) || !isfinite(b)) return -2;
            if (a > m) m = a;
            if (b > m) m = b;
        }
        w[j] = m;
    }
    return 0;
}

int or_herm_beta_rule(int n, const double *lam, const double *Xr, const double *Xi, double delta,
                      double xi, int kx_max, int *beta_out, int *kx_out)
{
    double *w = (double *)malloc(sizeof(double) * n);
    if (!w) return -5;
    int st = herm_colmax(n, Xr, Xi, w);
    if (st == 0)
        st = or_beta_core(n, lam, w, delta, xi, kx_max, beta_out, kx_out, NULL, NULL, NULL);
    free(w);
    return st;
}

/* One iteration of the proposed method for Hermitian A with exact products. Outputs:
 * X1 parts (FP64), the new X as complex double-double, lambda, r, emax, beta, kx. */
int or_herm_method_step(int n, const double *Ar, const double *Ai, const double *Xr,
                        const double *Xi, const double *lam_prev, double delta, double xi,
                        int kx_max, int kx_force, double *X1r, double *X1i, double *Xnr_h,
                        double *Xnr_l, double *Xni_h, double *Xni_l, double *lam_h,
                        double *lam_l, double *r_h, double *emax, int *beta_out, int *kx_out)
{
    int beta = 0, kx = 0;
    int st = or_herm_beta_rule(n, lam_prev, Xr, Xi, delta, xi, kx_max, &beta, &kx);
    if (st != 0) return st;
    if (kx_force > 0) kx = kx_force;
    *beta_out = beta;
    *kx_out = kx;
    size_t nn = (size_t)n * n;
    /* the stacked 2n x n matrix [Re X; Im X]: one exponent per column over both parts */
    double *S = (double *)malloc(sizeof(double) * 2 * nn);
    double *T = (double *)malloc(sizeof(double) * 2 * nn);
    int *ex = (int *)malloc(sizeof(int) * n);
    int8_t *pl = (int8_t *)malloc(2 * nn * (size_t)kx);
    if (!S || !T || !ex || !pl) { free(S); free(T); free(ex); free(pl); return -5; }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            S[HX(i, j, 2 * n)] = Xr[HX(i, j, n)];
            S[HX(n + i, j, 2 * n)] = Xi[HX(i, j, n)];
        }
    st = or_split_s7(0, 2 * n, n, S, 2 * n, kx, ex, pl, T);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            X1r[HX(i, j, n)] = T[HX(i, j, 2 * n)];
            X1i[HX(i, j, n)] = T[HX(n + i, j, 2 * n)];
        }
    free(S); free(T); free(ex); free(pl);
    if (st != 0) return st;
    for (size_t q = 0; q < nn; ++q) {
        Xnr_h[q] = X1r[q]; Xnr_l[q] = 0.0;
        Xni_h[q] = X1i[q]; Xni_l[q] = 0.0;
    }
    return or_herm_dd_step(n, Ar, Ai, Xnr_h, Xnr_l, Xni_h, Xni_l, lam_h, lam_l, r_h, emax);
}
