// Kernels of the FP64 plain form (see plain.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace refeig {

// X^(1) = fl((tau_j + x) - tau_j), tau_j = 0.75 * 2^(c_j + beta) (0 for a zero column).
void launch_x1_rn(const double *X, int ldx, int n, const int *c, const double *mx, int beta,
                  double *X1, hipStream_t s);
// ns FP64 slices of the columns of M (n x n), each n x n with leading dimension n.
void launch_sigma_split_cols(const double *M, int ld, int n, int alpha, int ns, double *S,
                             hipStream_t s);
// (Vh, Vl) += P elementwise in pair arithmetic (first != 0: initialise with P).
void launch_dd_accum(const double *P, double *Vh, double *Vl, size_t count, int first,
                     hipStream_t s);
// r_j, lambda_j and Res = V - X^(1) D from the double-word V.
void launch_colpass_dd(const double *Vh, const double *Vl, const double *X1, int n, double *lam,
                       double *r, double *Res, int *flags, hipStream_t s);
// E~ from W (FP64) and column maxima of |E~| (bit patterns, zeroed by the caller).
void launch_etilde(const double *W, const double *lam, const double *r, int n, double *E,
                   unsigned long long *colmax, int *flags, hipStream_t s);
// X = X^(1) + U.
void launch_update(const double *X1, const double *U, int n, double *X, int ldx, hipStream_t s);

}  // namespace refeig
