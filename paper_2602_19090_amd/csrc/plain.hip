// gfx950 kernels for the FP64 "plain form" of the refinement: the same
// iteration (Algorithm 1 with the first slice X^(1), Sec. 3) whose accurate
// product V = A X^(1) is the FP64 Ozaki scheme of Sec. 2.3: error-free FP64
// slices (eq. a / x) whose pairwise products are exact DGEMMs on FP64 MFMA,
// summed in double-word arithmetic. W and X^(1) E~ are single DGEMMs, as in the
// paper's cost count (n_A + 2 products per iteration). The DGEMMs run in
// rocBLAS; these kernels do the splitting, the sums and the column pass.
//
// Compiled with -ffp-contract=off: fl((sigma + a) - sigma) and TwoSum must be
// evaluated exactly as written.
#include "plain.h"

#include <float.h>

namespace refeig {

namespace {

__device__ __forceinline__ void p_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ __forceinline__ void p_fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}
__device__ __forceinline__ void p_two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = fma(a, b, -p);
}
struct pdd {
  double h, l;
};
__device__ __forceinline__ pdd p_dd_add(pdd a, pdd b) {
  double s, e, t, f;
  p_two_sum(a.h, b.h, s, e);
  p_two_sum(a.l, b.l, t, f);
  e += t;
  p_fast_two_sum(s, e, s, e);
  e += f;
  p_fast_two_sum(s, e, s, e);
  return {s, e};
}
__device__ __forceinline__ int p_ceil_log2(double v) {
  if (v == 0.0) return 0;
  int e;
  double f = frexp(v, &e);
  return (f == 0.5) ? e - 1 : e;
}

template <int NT>
__device__ __forceinline__ double p_block_max(double v, double *scratch) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  double m = scratch[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) m = fmax(m, scratch[q]);
  return m;
}
template <int NT>
__device__ __forceinline__ pdd p_block_dd_sum(pdd v, double *scratch) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    pdd w = {__shfl_xor(v.h, o), __shfl_xor(v.l, o)};
    v = p_dd_add(v, w);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    scratch[2 * w] = v.h;
    scratch[2 * w + 1] = v.l;
  }
  __syncthreads();
  pdd s = {scratch[0], scratch[1]};
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) s = p_dd_add(s, pdd{scratch[2 * q], scratch[2 * q + 1]});
  return s;
}

constexpr int kNT = 1024;

// X^(1) of eq. (x): tau_j = 0.75 * 2^(c_j + beta), x1 = fl((tau_j + x) - tau_j).
__global__ __launch_bounds__(256) void k_x1_rn(const double *__restrict__ X, int ldx, int n,
                                               const int *__restrict__ c, const double *mx,
                                               int beta, double *__restrict__ X1) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const double x = X[(size_t)j * ldx + i];
  if (mx[j] == 0.0) {
    X1[(size_t)j * n + i] = 0.0;
    return;
  }
  const double tau = ldexp(0.75, c[j] + beta);
  const double t = tau + x;
  X1[(size_t)j * n + i] = t - tau;
}

// Column-wise FP64 splitting of eq. (a)/(x): for r = 1..ns, sigma from the
// current remainder's column maximum, slice = fl((sigma + a) - sigma),
// remainder = fl(a - slice). One block per column, the column in registers.
template <int EPT>
__global__ __launch_bounds__(kNT) void k_sigma_split_cols(const double *__restrict__ M, int ld,
                                                          int n, int alpha, int ns,
                                                          double *__restrict__ S) {
  __shared__ double scratch[kNT / 64];
  const int j = blockIdx.x, tid = threadIdx.x;
  double rem[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kNT * q;
    rem[q] = (i < n) ? M[(size_t)j * ld + i] : 0.0;
  }
  for (int r = 0; r < ns; ++r) {
    double m = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) m = fmax(m, fabs(rem[q]));
    m = p_block_max<kNT>(m, scratch);
    const double sigma = (m == 0.0) ? 0.0 : ldexp(0.75, p_ceil_log2(m) + alpha);
    double *out = S + (size_t)r * n * n + (size_t)j * n;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int i = tid + kNT * q;
      const double t = sigma + rem[q];
      const double sl = t - sigma;
      rem[q] = rem[q] - sl;
      if (i < n) out[i] = sl;
    }
  }
}

// (Vh, Vl) += P in pair arithmetic; the first call initialises.
__global__ __launch_bounds__(256) void k_dd_accum(const double *__restrict__ P, double *Vh,
                                                  double *Vl, size_t count, int first) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  if (first) {
    Vh[q] = P[q];
    Vl[q] = 0.0;
    return;
  }
  double s, e;
  p_two_sum(Vh[q], P[q], s, e);
  e += Vl[q];
  p_fast_two_sum(s, e, Vh[q], Vl[q]);
}

// Column pass of Algorithm 1 from a double-word V: r_j, lambda_j, Res (FP64).
template <int EPT>
__global__ __launch_bounds__(kNT) void k_colpass_dd(const double *__restrict__ Vh,
                                                    const double *__restrict__ Vl,
                                                    const double *__restrict__ X1, int n,
                                                    double *lam, double *r,
                                                    double *__restrict__ Res, int *flags) {
  __shared__ double scratch[2 * (kNT / 64)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const size_t off = (size_t)j * n;
  pdd sx = {0.0, 0.0}, sv = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kNT * q;
    if (i < n) {
      const double x = X1[off + i], vh = Vh[off + i], vl = Vl[off + i];
      double p, pe, s, e;
      p_two_prod(x, x, p, pe);
      p_two_sum(sx.h, p, s, e);
      e += sx.l + pe;
      p_fast_two_sum(s, e, sx.h, sx.l);
      p_two_prod(x, vh, p, pe);
      p_two_sum(sv.h, p, s, e);
      e += sv.l + (pe + x * vl);
      p_fast_two_sum(s, e, sv.h, sv.l);
    }
  }
  sx = p_block_dd_sum<kNT>(sx, scratch);
  sv = p_block_dd_sum<kNT>(sv, scratch);
  pdd rj = p_dd_add(pdd{1.0, 0.0}, pdd{-sx.h, -sx.l});
  pdd den = p_dd_add(pdd{1.0, 0.0}, pdd{-rj.h, -rj.l});
  double q1 = sv.h / den.h, p, pe, s, e;
  p_two_prod(q1, den.h, p, pe);
  p_two_sum(sv.h, -p, s, e);
  e = ((e - pe) + sv.l) - q1 * den.l;
  const double lj = q1 + (s + e) / den.h;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kNT * q;
    if (i < n) {
      const double x = X1[off + i];
      double pp, ppe, ss, ee;
      p_two_prod(x, lj, pp, ppe);
      p_two_sum(Vh[off + i], -pp, ss, ee);
      Res[off + i] = ss + ((ee + Vl[off + i]) - ppe);
    }
  }
  if (tid == 0) {
    lam[j] = lj;
    r[j] = rj.h;
    if (!(fabs(lj) <= DBL_MAX)) atomicOr(flags, 1);
  }
}

// E~ from W: e_ij = w_ij / (lambda_j - lambda_i), e_jj = r_j / 2; column maxima
// of |e| as ordered integer bit patterns (non-negative doubles order like their bits).
__global__ __launch_bounds__(256) void k_etilde(const double *__restrict__ W, const double *lam,
                                                const double *r, int n, double *__restrict__ E,
                                                unsigned long long *colmax, int *flags) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  double e = 0.0;
  if (i < n) {
    const size_t q = (size_t)j * n + i;
    if (i == j) {
      e = 0.5 * r[j];
    } else {
      const double den = lam[j] - lam[i];
      if (den == 0.0) atomicOr(flags, 2);
      else e = W[q] / den;
    }
    E[q] = e;
  }
  double m = fabs(e);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(colmax + j, (unsigned long long)__double_as_longlong(m));
}

__global__ __launch_bounds__(256) void k_update(const double *__restrict__ X1,
                                                const double *__restrict__ U, int n,
                                                double *__restrict__ X, int ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  X[(size_t)j * ldx + i] = X1[(size_t)j * n + i] + U[(size_t)j * n + i];
}

}  // namespace

void launch_x1_rn(const double *X, int ldx, int n, const int *c, const double *mx, int beta,
                  double *X1, hipStream_t s) {
  hipLaunchKernelGGL(k_x1_rn, dim3((n + 255) / 256, n), dim3(256), 0, s, X, ldx, n, c, mx, beta,
                     X1);
}

void launch_sigma_split_cols(const double *M, int ld, int n, int alpha, int ns, double *S,
                             hipStream_t s) {
  const int ept = (n + kNT - 1) / kNT;
  if (ept <= 1)
    hipLaunchKernelGGL(k_sigma_split_cols<1>, dim3(n), dim3(kNT), 0, s, M, ld, n, alpha, ns, S);
  else if (ept <= 2)
    hipLaunchKernelGGL(k_sigma_split_cols<2>, dim3(n), dim3(kNT), 0, s, M, ld, n, alpha, ns, S);
  else if (ept <= 4)
    hipLaunchKernelGGL(k_sigma_split_cols<4>, dim3(n), dim3(kNT), 0, s, M, ld, n, alpha, ns, S);
  else
    hipLaunchKernelGGL(k_sigma_split_cols<8>, dim3(n), dim3(kNT), 0, s, M, ld, n, alpha, ns, S);
}

void launch_dd_accum(const double *P, double *Vh, double *Vl, size_t count, int first,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_dd_accum, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, P, Vh, Vl,
                     count, first);
}

void launch_colpass_dd(const double *Vh, const double *Vl, const double *X1, int n, double *lam,
                       double *r, double *Res, int *flags, hipStream_t s) {
  const int ept = (n + kNT - 1) / kNT;
  if (ept <= 1)
    hipLaunchKernelGGL(k_colpass_dd<1>, dim3(n), dim3(kNT), 0, s, Vh, Vl, X1, n, lam, r, Res, flags);
  else if (ept <= 2)
    hipLaunchKernelGGL(k_colpass_dd<2>, dim3(n), dim3(kNT), 0, s, Vh, Vl, X1, n, lam, r, Res, flags);
  else if (ept <= 4)
    hipLaunchKernelGGL(k_colpass_dd<4>, dim3(n), dim3(kNT), 0, s, Vh, Vl, X1, n, lam, r, Res, flags);
  else
    hipLaunchKernelGGL(k_colpass_dd<8>, dim3(n), dim3(kNT), 0, s, Vh, Vl, X1, n, lam, r, Res, flags);
}

void launch_etilde(const double *W, const double *lam, const double *r, int n, double *E,
                   unsigned long long *colmax, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_etilde, dim3((n + 255) / 256, n), dim3(256), 0, s, W, lam, r, n, E, colmax,
                     flags);
}

void launch_update(const double *X1, const double *U, int n, double *X, int ldx, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3((n + 255) / 256, n), dim3(256), 0, s, X1, U, n, X, ldx);
}

}  // namespace refeig
