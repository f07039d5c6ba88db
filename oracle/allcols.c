/*
 * Element-wise and column passes of the all-column forward-error check: one
 * double-double step of Algorithm 1 (Sec. 2.4) from a given X, whose matrix
 * products come from exact FP64 slice products (the Ozaki scheme of Sec. 2.3)
 * on the host's BLAS (oracle/dd_numpy.py).
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the GPU library includes, links or
 * calls this file, and it shares no code with it.
 *
 * Matrices are column-major n x m (element (i, j) at i + j*n). Compile with
 * -ffp-contract=off (dd.h).
 */
#include <math.h>
#include <stddef.h>

#include "dd.h"

/* acc <- acc + P element-wise in double-double (TwoSum of the high words, the
 * error added to the low word). Every P here is an exact slice product. */
void or_dd_acc(size_t count, double *acc_h, double *acc_l, const double *P)
{
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < (long long)count; ++q) {
        dd_t s = two_sum(acc_h[q], P[q]);
        acc_h[q] = s.hi;
        acc_l[q] += s.lo;
    }
}

/* (h, l) <- FastTwoSum(h, l) element-wise (renormalise an accumulation). */
void or_dd_norm(size_t count, double *h, double *l)
{
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < (long long)count; ++q) {
        dd_t s = fast_two_sum(h[q], l[q]);
        h[q] = s.hi;
        l[q] = s.lo;
    }
}

/* The column pass of Algorithm 1 on V = Vh + Vl = A X (double-double): for each
 * column j, in a fixed order along i,
 *   xx_j = x_j^T x_j, xv_j = x_j^T v_j        (double-double dots),
 *   r_j = 1 - xx_j, lambda_j = xv_j / xx_j    (= x^T v / (1 - r)),
 * then V <- V - x_j lambda_j (the residual, double-double), in place. */
void or_colpass(int n, int m, const double *X, double *Vh, double *Vl, double *lam_h,
                double *lam_l, double *r_h, double *r_l)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < m; ++j) {
        const double *x = X + (size_t)j * n;
        double *vh = Vh + (size_t)j * n, *vl = Vl + (size_t)j * n;
        dd_t xx = dd_from(0.0), xv = dd_from(0.0);
        for (int i = 0; i < n; ++i) {
            xx = dd_add(xx, two_prod(x[i], x[i]));
            dd_t v = { vh[i], vl[i] };
            xv = dd_add(xv, dd_mul_d(v, x[i]));
        }
        dd_t r = dd_sub(dd_from(1.0), xx);
        dd_t lam = dd_div(xv, xx);
        lam_h[j] = lam.hi;
        lam_l[j] = lam.lo;
        r_h[j] = r.hi;
        r_l[j] = r.lo;
        for (int i = 0; i < n; ++i) {
            dd_t v = { vh[i], vl[i] };
            dd_t res = dd_sub(v, dd_mul_d(lam, x[i]));
            vh[i] = res.hi;
            vl[i] = res.lo;
        }
    }
}

/* E~ of Algorithm 1 from W = Wh + Wl (n x n): e_ij = w_ij / (lambda_j - lambda_i)
 * for i != j (the difference of the double-double eigenvalues, then the quotient
 * of double-double values rounded to FP64), e_jj = r_j / 2; eps_j = max over
 * i != j of |e_ij|. E may alias neither W. */
void or_form_e(int n, const double *Wh, const double *Wl, const double *lam_h,
               const double *lam_l, const double *r_h, const double *r_l, double *E,
               double *eps)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        dd_t lj = { lam_h[j], lam_l[j] };
        double mx = 0.0;
        for (int i = 0; i < n; ++i) {
            size_t q = (size_t)j * n + i;
            if (i == j) {
                E[q] = 0.5 * (r_h[j] + r_l[j]);
                continue;
            }
            dd_t li = { lam_h[i], lam_l[i] };
            dd_t w = { Wh[q], Wl[q] };
            dd_t e = dd_div(w, dd_sub(lj, li));
            E[q] = e.hi;
            if (fabs(e.hi) > mx) mx = fabs(e.hi);
        }
        eps[j] = mx;
    }
}
