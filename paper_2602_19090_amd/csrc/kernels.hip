// gfx950 (MI355X) kernels for Ozaki-scheme eigenvector refinement.
//
// Data layout (npad = n rounded up to 256, P = npad * npad):
//   digit planes   int8, plane-major. A plane holds a GEMM operand of R rows
//                  (row m, reduction index k) K-blocked: K is cut into 64-byte
//                  blocks and block b stores its 64 bytes of every row in turn,
//                  element (m, k) at ((k >> 6) * R + m) * 64 + (k & 63). The
//                  64-byte K-slice of 256 consecutive rows that one GEMM stage
//                  needs is then one contiguous 16 KB run (full cache lines).
//   slot C_d       int32 n x n per pair diagonal d, element (i, j) at j*npad + i,
//                  i.e. column-major, so the column epilogues read columns
//                  contiguously.
//
// Every floating-point expression in this file is compiled with
// -ffp-contract=off: the error-free transformations (TwoSum, the exact product
// via fma) must not be contracted or reassociated.
#include "kernels.h"
#include "work.h"
#include <hip/hip_ext.h>

#include <float.h>
#include <limits.h>
#include <algorithm>
#include <type_traits>

namespace refeig {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Offset of element (row m, reduction index k) in a K-blocked plane of `rows` rows.
__device__ __forceinline__ size_t kb_off(int m, int k, int rows) {
  return ((size_t)(k >> 6) * rows + m) * 64 + (k & 63);
}

// Global-memory view of a pointer that the compiler cannot place itself (pointers read from a
// descriptor are generic): loads and stores through it are global, not flat, instructions, so
// they count in vmcnt only and an LDS wait does not also wait for them.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gview(const T *p) {
  return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gview_w(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// ---------------------------------------------------------------- scalar helpers
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}
__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = fma(a, b, -p);
}
struct ddv {
  double h, l;
};
__device__ __forceinline__ ddv dd_add(ddv a, ddv b) {
  double s, e, t, f;
  two_sum(a.h, b.h, s, e);
  two_sum(a.l, b.l, t, f);
  e += t;
  fast_two_sum(s, e, s, e);
  e += f;
  fast_two_sum(s, e, s, e);
  return {s, e};
}
// a + p where p is an exact product given as (p, q) with |q| <= ulp(p)/2.
__device__ __forceinline__ ddv dd_add_prod(ddv a, double p, double q) {
  double s, e;
  two_sum(a.h, p, s, e);
  e += a.l + q;
  fast_two_sum(s, e, s, e);
  return {s, e};
}
// (a) / (b) to about 100 bits, rounded to one double.
__device__ __forceinline__ double dd_div_to_d(ddv a, ddv b) {
  double q1 = a.h / b.h;
  double p, pe;
  two_prod(q1, b.h, p, pe);
  double s, e;
  two_sum(a.h, -p, s, e);
  e = ((e - pe) + a.l) - q1 * b.l;
  double rem = s + e;
  double q2 = rem / b.h;
  return q1 + q2;
}

// a / b to double-word: the FP64 quotient q1 (as dd_div_to_d) and its correction q2.
__device__ __forceinline__ ddv dd_div_to_dd(ddv a, ddv b) {
  double q1 = a.h / b.h;
  double p, pe;
  two_prod(q1, b.h, p, pe);
  double s, e;
  two_sum(a.h, -p, s, e);
  e = ((e - pe) + a.l) - q1 * b.l;
  double rem = s + e;
  double q2 = rem / b.h;
  ddv r;
  fast_two_sum(q1, q2, r.h, r.l);
  return r;
}
// (a_h + a_l) - (b_h + b_l) rounded to FP64, with the high parts subtracted exactly.
__device__ __forceinline__ double dd_diff(double ah, double al, double bh, double bl) {
  double s, e;
  two_sum(ah, -bh, s, e);
  return s + (e + (al - bl));
}

// floor(log2 v) + 1 for v > 0 (so v < 2^e), 0 for v == 0.
__device__ __forceinline__ int exp_above(double v) {
  if (v == 0.0) return 0;
  unsigned long long b = (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffULL;
  int be = (int)(b >> 52);
  if (be != 0) return be - 1022;
  return (64 - __clzll((long long)b)) - 1074;
}
// ceil(log2 v) for v > 0, 0 for v == 0.
__device__ __forceinline__ int ceil_log2(double v) {
  if (v == 0.0) return 0;
  unsigned long long b = (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffULL;
  int e = exp_above(v);
  unsigned long long mant = b & 0x000fffffffffffffULL;
  bool pow2 = ((b >> 52) != 0) ? (mant == 0) : (__popcll(b) == 1);
  return pow2 ? e - 1 : e;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ ddv wave_dd_sum(ddv v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ddv w = {__shfl_xor(v.h, o), __shfl_xor(v.l, o)};
    v = dd_add(v, w);
  }
  return v;
}
// Block-wide max; every thread gets the result. scratch: >= nwaves doubles.
template <int NT>
__device__ __forceinline__ double block_max(double v, double *scratch) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  // over the waves' maxima: lane l takes wave l mod NW's, then an xor butterfly
  constexpr int NW = NT / 64;
  static_assert(NW >= 1 && NW <= 64 && (NW & (NW - 1)) == 0, "power-of-two wave count");
  double m = scratch[threadIdx.x & (NW - 1)];
#pragma unroll
  for (int o = NW / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  return m;
}
// Across the waves of a block: lane l of every wave takes partial l mod NW from scratch (stride
// 2 doubles) and the lanes combine them by an xor butterfly.
template <int NW>
__device__ __forceinline__ ddv cross_wave_dd_sum(const double *scratch, int stride) {
  const int q = threadIdx.x & (NW - 1);
  ddv v = {scratch[stride * q], scratch[stride * q + 1]};
#pragma unroll
  for (int o = NW / 2; o > 0; o >>= 1) {
    ddv w = {__shfl_xor(v.h, o), __shfl_xor(v.l, o)};
    v = dd_add(v, w);
  }
  return v;
}
// Block-wide double-word sums in a fixed order (deterministic); every thread gets the result.
// Within a wave and then over the waves' partials the terms meet in xor butterflies: dd_add is
// commutative, so every lane ends with the same value, after log2(NT) additions instead of a
// serial pass over the waves. scratch: >= 2 (one sum) or 4 (two sums) doubles per wave.
template <int NT>
__device__ __forceinline__ ddv block_dd_sum(ddv v, double *scratch) {
  constexpr int NW = NT / 64;
  static_assert(NW >= 1 && NW <= 64 && (NW & (NW - 1)) == 0, "power-of-two wave count");
  v = wave_dd_sum(v);
  if constexpr (NW == 1) {
    return v;
  } else {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      scratch[2 * w] = v.h;
      scratch[2 * w + 1] = v.l;
    }
    __syncthreads();
    return cross_wave_dd_sum<NW>(scratch, 2);
  }
}
template <int NT>
__device__ __forceinline__ void block_dd_sum2(ddv &a, ddv &b, double *scratch) {
  constexpr int NW = NT / 64;
  static_assert(NW >= 1 && NW <= 64 && (NW & (NW - 1)) == 0, "power-of-two wave count");
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const ddv wa = {__shfl_xor(a.h, o), __shfl_xor(a.l, o)};
    const ddv wb = {__shfl_xor(b.h, o), __shfl_xor(b.l, o)};
    a = dd_add(a, wa);
    b = dd_add(b, wb);
  }
  if constexpr (NW > 1) {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      scratch[4 * w] = a.h;
      scratch[4 * w + 1] = a.l;
      scratch[4 * w + 2] = b.h;
      scratch[4 * w + 3] = b.l;
    }
    __syncthreads();
    a = cross_wave_dd_sum<NW>(scratch, 4);
    b = cross_wave_dd_sum<NW>(scratch + 2, 4);
  }
}

// ---------------------------------------------------------------- column statistics
__device__ __forceinline__ void colstats_body(const double *__restrict__ M, int ld, int rows,
                                                  int cols, int *e, int *c, double *mx,
                                                  int *flags, const int *__restrict__ colmap,
                                                  double *ss, int bx) {
  __shared__ double scratch[4];
  const int j = bx;
  if (j >= cols) {
    if (threadIdx.x == 0) {
      e[j] = 0;
      c[j] = 0;
      if (mx) mx[j] = 0.0;
      if (ss) ss[j] = 0.0;
    }
    return;
  }
  const double *col = M + (size_t)(colmap ? colmap[j] : j) * ld;
  double m = 0.0, q = 0.0;
  int bad = 0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    double a = fabs(col[i]);
    if (!(a <= DBL_MAX)) bad = 1;
    else {
      m = fmax(m, a);
      q += a * a;
    }
  }
  if (bad) atomicOr(flags, FLAG_NONFINITE);
  if (ss) {   // sum of squares (for a product bound; plain FP64 is enough)
    q = wave_sum(q);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) ss[j] = (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
    __syncthreads();
  }
  m = block_max<256>(m, scratch);
  if (threadIdx.x == 0) {
    int ee = exp_above(m);
    e[j] = ee;
    c[j] = ceil_log2(m);
    if (mx) mx[j] = m;
    if (m != 0.0 && (ee < -400 || ee > 400)) atomicOr(flags, FLAG_RANGE);
  }
}

__global__ __launch_bounds__(256) void k_colstats(const double *__restrict__ M, int ld, int rows,
                                                  int cols, int *e, int *c, double *mx,
                                                  int *flags, const int *__restrict__ colmap,
                                                  double *ss) {
  colstats_body(M, ld, rows, cols, e, c, mx, flags, colmap, ss, blockIdx.x);
}

// Nonzeros of column j of the symmetric A (= row j), block per column; the maximum goes
// to *kmax (atomicMax on an int the caller zeroed).
__global__ __launch_bounds__(256) void k_row_nnz(const double *__restrict__ A, int lda, int n,
                                                 int *kmax) {
  __shared__ double scratch[4];
  const int j = blockIdx.x;
  const double *col = A + (size_t)j * lda;
  double cnt = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) cnt += (col[i] != 0.0) ? 1.0 : 0.0;
  // counts are small integers: a maximum reduction over per-wave sums is exact
  cnt = wave_sum(cnt);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(kmax, (int)(scratch[0] + scratch[1] + scratch[2] + scratch[3]));
}

void launch_row_nonzeros(const double *A, int lda, int n, int *kmax, hipStream_t s) {
  hipLaunchKernelGGL(k_row_nnz, dim3(n), dim3(256), 0, s, A, lda, n, kmax);
}

void launch_colstats(const double *M, int ld, int rows, int cols, int cols_pad, int *e, int *c,
                     double *mx, int *flags, hipStream_t s, const int *colmap, double *ss) {
  hipLaunchKernelGGL(k_colstats, dim3(cols_pad), dim3(256), 0, s, M, ld, rows, cols, e, c, mx,
                     flags, colmap, ss);
}

// ---------------------------------------------------------------- digit planes
constexpr int kMaxPlanesSplit = 18;
constexpr int kMaxPlanesT = 9;
constexpr int kSplitRow = 80;  // LDS row stride of a staged 64 x 64 digit tile (16-byte aligned)
constexpr int kTStride = 80;   // LDS row stride of the complex splitter's transpose tile

// One block splits a 64 x 64 tile (rows i0.., columns j0..) of M; thread (ig, jg) holds the
// 4 x 4 micro-tile of rows i0 + 4 ig .. + 3 and columns j0 + 4 jg .. + 3. Per plane, each
// thread packs its 16 digits into four column words (4 rows of one column) and, for the
// transposed layout, four row words (4 columns of one row), stages them in LDS, and the
// block writes each layout's tile as one contiguous 4 KiB run (in the K-blocked layout a
// 64 x 64 tile is contiguous), 16 bytes per thread. Reads and the X^(1) writes take 32
// contiguous bytes per thread and column.
template <bool WITH_T>
__device__ __forceinline__ void split_cols_body(const double *__restrict__ M, int ld, int rows,
                                                    int cols, const int *__restrict__ e, int k,
                                                    int8_t *__restrict__ planes, size_t pstride,
                                                    int rpad, int cpad, double *__restrict__ trunc,
                                                    int ldt, int8_t *__restrict__ planesT,
                                                    size_t pstrideT, int kT,
                                                    const int *__restrict__ colmap,
                                                    const int *__restrict__ kdev, int bx, int by) {
  __shared__ __attribute__((aligned(16))) int8_t sC[64 * kSplitRow];
  if (kdev) {
    k = *kdev;
    kT = WITH_T ? k : 0;
  }
  __shared__ __attribute__((aligned(16))) int8_t sR[WITH_T ? 64 * kSplitRow : 16];
  const int i0 = bx * 64, j0 = by * 64;
  const int tid = threadIdx.x, ig = tid & 15, jg = tid >> 4;
  const int kk = (WITH_T && kT > k) ? kT : k;
  const int ib = i0 + 4 * ig;
  // 16-byte aligned runs of 4 rows
  const bool vec = (ld % 2 == 0) && ((uintptr_t)M % 16 == 0) && ib + 3 < rows;
  double y[4][4], val[4][4];
  bool neg[4][4];
  int ej[4];
  const double *colp[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + 4 * jg + c;
    ej[c] = (j < cols) ? e[j] : 0;
    colp[c] = (j < cols) ? M + (size_t)(colmap ? colmap[j] : j) * ld : nullptr;
    double a[4];
    if (colp[c] && vec) {
      const double2 lo = *(const double2 *)(colp[c] + ib);
      const double2 hi = *(const double2 *)(colp[c] + ib + 2);
      a[0] = lo.x; a[1] = lo.y; a[2] = hi.x; a[3] = hi.y;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = (colp[c] && ib + u < rows) ? colp[c][ib + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      y[u][c] = ldexp(fabs(a[u]), -ej[c]);
      neg[u][c] = a[u] < 0.0;
      val[u][c] = 0.0;
    }
  }
  const int rr = tid >> 2, q16 = (tid & 3) * 16;   // this thread's 16 bytes of a staged tile
#pragma unroll 1
  for (int t = 0; t < kk; ++t) {
    unsigned cw[4] = {0u, 0u, 0u, 0u}, rw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double t128 = y[u][c] * 128.0;
        const double d = floor(t128);
        y[u][c] = t128 - d;
        if (t < k) val[u][c] += ldexp(d, ej[c] - 7 * (t + 1));
        const unsigned b = (unsigned)((neg[u][c] ? -(int)d : (int)d) & 0xff);
        cw[c] |= b << (8 * u);
        rw[u] |= b << (8 * c);
      }
    if (t < k)
#pragma unroll
      for (int c = 0; c < 4; ++c) *(unsigned *)(sC + (4 * jg + c) * kSplitRow + 4 * ig) = cw[c];
    if (WITH_T && t < kT)
#pragma unroll
      for (int u = 0; u < 4; ++u) *(unsigned *)(sR + (4 * ig + u) * kSplitRow + 4 * jg) = rw[u];
    __syncthreads();
    // tile rows j0 + rr of the column layout, i0 + rr of the transposed one
    if (t < k)
      *(v4i *)(planes + (size_t)t * pstride + kb_off(j0 + rr, i0 + q16, cpad)) =
          *(const v4i *)(sC + rr * kSplitRow + q16);
    if (WITH_T && t < kT)
      *(v4i *)(planesT + (size_t)t * pstrideT + kb_off(i0 + rr, j0 + q16, rpad)) =
          *(const v4i *)(sR + rr * kSplitRow + q16);
    __syncthreads();
  }
  if (trunc) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + 4 * jg + c;
      if (j >= cols) continue;
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = neg[u][c] ? -val[u][c] : val[u][c];
      double *out = trunc + (size_t)j * ldt + ib;
      if (ib + 3 < rows && ldt % 2 == 0 && (uintptr_t)trunc % 16 == 0) {
        *(double2 *)out = double2{v[0], v[1]};
        *(double2 *)(out + 2) = double2{v[2], v[3]};
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (ib + u < rows) out[u] = v[u];
      }
    }
  }
}

template <bool WITH_T>
__global__ __launch_bounds__(256) void k_split_cols(const double *__restrict__ M, int ld, int rows,
                                                    int cols, const int *__restrict__ e, int k,
                                                    int8_t *__restrict__ planes, size_t pstride,
                                                    int rpad, int cpad, double *__restrict__ trunc,
                                                    int ldt, int8_t *__restrict__ planesT,
                                                    size_t pstrideT, int kT,
                                                    const int *__restrict__ colmap,
                                                    const int *__restrict__ kdev) {
  split_cols_body<WITH_T>(M, ld, rows, cols, e, k, planes, pstride, rpad, cpad, trunc, ldt, planesT, pstrideT, kT, colmap, kdev, blockIdx.x, blockIdx.y);
}

void launch_split_cols(const double *M, int ld, int rows, int cols, const int *e, int k,
                       int8_t *planes, size_t pstride, int rpad, int cpad, double *trunc, int ldt,
                       int8_t *planesT, size_t pstrideT, int kT, hipStream_t s,
                       const int *colmap, const int *kdev) {
  dim3 grid(rpad / 64, cpad / 64);
  if (planesT && kT > 0)
    hipLaunchKernelGGL(k_split_cols<true>, grid, dim3(256), 0, s, M, ld, rows, cols, e, k, planes,
                       pstride, rpad, cpad, trunc, ldt, planesT, pstrideT, kT, colmap, kdev);
  else
    hipLaunchKernelGGL(k_split_cols<false>, grid, dim3(256), 0, s, M, ld, rows, cols, e, k, planes,
                       pstride, rpad, cpad, trunc, ldt, (int8_t *)nullptr, (size_t)0, 0, colmap,
                       kdev);
}

// ---------------------------------------------------------------- INT8 slice GEMM
// One block computes one 128 x 128 tile of one diagonal slot:
//   C_d[m][p] = sum over pairs (s, d - s) of sum_k L_s[m][k] R_{d-s}[p][k].
// 4 waves in a 2 x 2 arrangement, each 64 x 64 = 2 x 2 MFMA 32x32x32 blocks.
// K advances 128 bytes per LDS stage; the next stage is prefetched into
// registers while the current one feeds the matrix cores.
constexpr int GBM = 128, GBN = 128, GBK = 128, GLDS = GBK + 16;

// One 128 x 128 output tile (rows m0.., columns n0..) of slot `slot` (body of k_slice_gemm
// and of the grouped persistent form).
__device__ __forceinline__ void gemm128_item(const int8_t *__restrict__ Lp,
                                             const int8_t *__restrict__ Rp, size_t pstride,
                                             int npad, int kdim, int kl, int kr, int d_min,
                                             int32_t *__restrict__ C, int same,
                                             const int *__restrict__ mods,
                                             const int *__restrict__ vblk, int m0, int n0,
                                             int slot) {
  __shared__ __attribute__((aligned(16))) int8_t sL[GBM * GLDS];
  __shared__ __attribute__((aligned(16))) int8_t sR[GBN * GLDS];
  // vblk (same-plane products, per 256-row block of L: slot count, level)
  int roff = 0;
  if (vblk) {
    const int mb = m0 / 256;
    if (slot >= vblk[2 * mb]) return;
    roff = vblk[2 * mb + 1] * kCrtMax;
  }
  const int d = d_min + slot;
  // same: slot q multiplies plane q + 1 of both operands (one pair); else the pairs of
  // diagonal d, planes (s, d - s)
  const int s_lo = same ? slot + 1 : max(1, d - kr), s_hi = same ? slot + 1 : min(kl, d - 1);
  const int rsum = same ? 2 * (slot + 1) : d;   // R plane of pair s: rsum - s
  const int npairs = s_hi - s_lo + 1;
  const int KT = kdim / GBK;
  const int T = npairs * KT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  v16i acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

  v4i gL[4], gR[4];
  // thread's 16 bytes h of a stage: row c/8, bytes 16 (c%8) of the stage's 128 (c = tid + 256h),
  // i.e. K-block (c%8)/4 of the stage at kb_off(row, 16 (c%4)): a fixed offset from the stage's
  // first K-block. Stages are loaded in order: the next is K-block 2 ik of pair s_lo + ip,
  // whose first K-block starts at lsrc / rsrc (the next pair's L plane follows, R precedes).
  uint32_t hoff[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int c = tid + 256 * h, row = c >> 3, col = (c & 7) * 16;
    hoff[h] = (uint32_t)((col >> 6) * npad * 64 + row * 64 + (col & 63));
  }
  const size_t kstride = (size_t)npad * GBK;   // two 64-deep K-blocks
  const int8_t *lpair = Lp + (size_t)(s_lo - 1) * pstride + (size_t)m0 * 64;
  const int8_t *rpair = Rp + (size_t)(roff + rsum - s_lo - 1) * pstride + (size_t)n0 * 64;
  const int8_t *lsrc = lpair, *rsrc = rpair;
  int ik = 0;
  auto load = [&]() {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      gL[h] = *gview((const v4i *)(lsrc + hoff[h]));
      gR[h] = *gview((const v4i *)(rsrc + hoff[h]));
    }
    const bool wrap = ++ik == KT;
    ik = wrap ? 0 : ik;
    lpair = wrap ? lpair + pstride : lpair;
    rpair = wrap ? rpair - pstride : rpair;
    lsrc = wrap ? lpair : lsrc + kstride;
    rsrc = wrap ? rpair : rsrc + kstride;
  };
  if (npairs > 0) load();
  for (int t = 0; t < T; ++t) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = tid + 256 * h, row = c >> 3, col = (c & 7) * 16;
      *(v4i *)(sL + row * GLDS + col) = gL[h];
      *(v4i *)(sR + row * GLDS + col) = gR[h];
    }
    __syncthreads();
    if (t + 1 < T) load();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      v4i a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = *(const v4i *)(sL + (wm * 64 + x * 32 + (lane & 31)) * GLDS + kk + 16 * (lane >> 5));
        b[x] = *(const v4i *)(sR + (wn * 64 + x * 32 + (lane & 31)) * GLDS + kk + 16 * (lane >> 5));
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
  if (mods) {   // residue products: the slot's value mod m_slot as INT8 (as the 256 kernel)
    auto Cq8 = gview_w((int8_t *)C + (size_t)slot * npad * npad);
    const double m = (double)mods[slot], rm = 1.0 / m;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = m0 + wm * 64 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int col = n0 + wn * 64 + y * 32 + (lane & 31);
          const double c = (double)acc[x][y][v];
          Cq8[(size_t)row * npad + col] = (int8_t)(int)(c - m * rint(c * rm));
        }
    return;
  }
  auto Cq = gview_w(C + (size_t)slot * npad * npad);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + wn * 64 + y * 32 + (lane & 31);
        Cq[(size_t)row * npad + col] = acc[x][y][v];
      }
}

__global__ __launch_bounds__(256, 2) void k_slice_gemm(const int8_t *__restrict__ Lp,
                                                       const int8_t *__restrict__ Rp,
                                                       size_t pstride, int npad, int kdim,
                                                       int kl, int kr, int d_min, DiagOrder order,
                                                       int32_t *__restrict__ C, RowBlocks rb,
                                                       int same, const int *__restrict__ mods,
                                                       const int *__restrict__ tab,
                                                       const int *__restrict__ dp,
                                                       const int *__restrict__ vblk) {
  int m0, n0, slot;
  if (tab) {   // block table: row tile | column tile << 8 | slot << 16 (128 x 128 tiles)
    if (dp) {
      if ((int)blockIdx.x >= dp[2]) return;
      kl = dp[0];
      kr = dp[1];
    }
    const int ent = tab[blockIdx.x];
    m0 = (ent & 0xff) * GBM;
    n0 = ((ent >> 8) & 0xff) * GBN;
    slot = ent >> 16;
  } else {
    const int tiles_n = npad / GBN;
    m0 = rb.m[blockIdx.x / tiles_n] * GBM;
    n0 = (blockIdx.x % tiles_n) * GBN;
    slot = order.q[blockIdx.y];
  }
  gemm128_item(Lp, Rp, pstride, npad, kdim, kl, kr, d_min, C, same, mods, vblk, m0, n0, slot);
}

constexpr int HBM_ = 256, HGM = 4;

// Block -> (row-block index, column offset) for the 256 x 256 kernel over a
// launch of tiles_m row blocks x tiles_n column blocks. Blocks are dispatched
// round-robin over the 8 XCDs (block id mod 8), and each XCD has its own L2, so
// the blocks one XCD runs at once should form a compact patch that shares
// operand panels. With tiles_n a multiple of 8 XCD x owns the column blocks x,
// 15 - x, 16 + x, ...; else with tiles_m a multiple of 8 it takes row blocks x, x + 8, ...;
// otherwise blocks walk groups of 4 row blocks.
__device__ __forceinline__ void tile_of_block(int bid, int tiles_m, int tiles_n, int &mi, int &n0) {
  if (tiles_n % 8 == 0) {
    // XCD x owns column blocks x, 15 - x, 16 + x, ... and walks them in groups of up to 8 row
    // blocks: its ~32 resident blocks form an 8 x 4 patch (as xcd_tile_order)
    const int xcd = bid & 7, local = bid >> 3;
    const int cb = tiles_n >> 3;
    const int rg = local / (8 * cb), rem = local - rg * 8 * cb;
    const int gs = min(8, tiles_m - rg * 8);
    const int c = rem / gs;
    mi = rg * 8 + rem % gs;
    n0 = (8 * c + ((c & 1) ? 7 - xcd : xcd)) * HBM_;
  } else if (tiles_m % 8 == 0) {
    const int xcd = bid & 7, local = bid >> 3;
    const int rows = tiles_m >> 3;
    mi = xcd + 8 * (local % rows);
    n0 = (local / rows) * HBM_;
  } else {
    const int group = bid / (HGM * tiles_n);
    const int first_m = group * HGM;
    const int gsz = min(tiles_m - first_m, HGM);
    const int inb = bid - group * HGM * tiles_n;
    mi = first_m + inb % gsz;
    n0 = (inb / gsz) * HBM_;
  }
}

// 256 x 256 tile kernel (npad >= 1024). 4 waves in a 2 x 2 arrangement, each
// 128 x 128 = 4 x 4 MFMA 32x32x32 blocks held in AGPRs. Operands move from
// global memory straight into a 4-stage LDS ring (global_load_lds_dwordx4:
// 64 lanes x 16 bytes land contiguously, 16 rows of 64 bytes per instruction);
// with K-blocked planes each instruction reads one contiguous kilobyte. Within a
// 64-byte row the 16-byte chunk c sits at chunk position c ^ ((row >> 2) & 3),
// so a fragment read (16 consecutive rows, one chunk) hits 16 distinct bank
// groups. Software pipeline: while the 32 MFMAs of stage t run from registers,
// the wave reads the fragments of stage t+1 from LDS into a second register set
// and issues the DMA of stage t+3, so the matrix cores are not left idle
// between stages; one barrier per stage.
constexpr int DBK = 64, DSTAGES = 4, DSTAGE_BYTES = 2 * 256 * DBK;

// Wait until at most N vector-memory operations of this wave are outstanding,
// then barrier. Also waits for this wave's LDS reads, so no wave still reads a slot
// that the DMA issued after the barrier overwrites. Written with the builtins (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4 left at 7, lgkmcnt 11:8 at 0) so
// that the compiler's own wait insertion knows what has completed here; the
// scheduling fences keep memory instructions on their side.
template <int N>
__device__ __forceinline__ void wait_vm_lds_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt has 6 bits");
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

// Four 16-byte-per-lane DMA loads of 16 rows (1 KB) each, 1 KB apart both in global memory and
// in LDS: the immediate offset of the instruction moves both addresses.
__device__ __forceinline__ void dma_rows4(const int8_t *g, int8_t *l) {
  typedef void __attribute__((address_space(3))) *lds_ptr;
  __builtin_amdgcn_global_load_lds((const void *)g, (lds_ptr)l, 16, 0, 0);
  __builtin_amdgcn_global_load_lds((const void *)g, (lds_ptr)l, 16, 1024, 0);
  __builtin_amdgcn_global_load_lds((const void *)g, (lds_ptr)l, 16, 2048, 0);
  __builtin_amdgcn_global_load_lds((const void *)g, (lds_ptr)l, 16, 3072, 0);
}

// F8: the planes hold FP8 E4M3 bytes of small integer digits (|digit| <= 15) instead of
// INT8 digits; one v_mfma_f32_32x32x64_f8f6f4 takes the two 32-deep halves of a stage that
// the INT8 form feeds to two v_mfma_i32_32x32x32_i8 (both operands see the same lane and byte
// order of k, so the sum over k is unchanged). The FP32 sums are integers below 2^24 (exact)
// and are stored as INT32 like the INT8 form's.
// One 256 x 256 output tile (rows m0.., columns n0..) of slot `slot` (body of k_slice_gemm256d
// and of the grouped persistent form).
template <bool F8>
__device__ __forceinline__ void gemm256_item(const int8_t *__restrict__ Lp,
                                             const int8_t *__restrict__ Rp, size_t pstride,
                                             int npad, int kdim, int kl, int kr, int d_min,
                                             int32_t *__restrict__ C, int same,
                                             const int *__restrict__ tcut,
                                             const int *__restrict__ mods,
                                             const int *__restrict__ vblk, int m0, int n0,
                                             int slot) {
  constexpr int S = DSTAGES;
  __shared__ __attribute__((aligned(1024))) int8_t ring[S * DSTAGE_BYTES];
  const int d = d_min + slot;
  // per-tile diagonal limit (tile = output column block m0 / 256, output row block n0 / 256):
  // the block's diagonal is not needed there, and nothing reads its slot
  if (tcut && d > tcut[(m0 / HBM_) * (npad / HBM_) + n0 / HBM_]) return;
  // vblk (same-plane products, per 256-row block of L: slot count, level): the block's
  // slots beyond its count are not needed; its R planes start at level * kCrtMax
  int roff = 0;
  if (vblk) {
    const int mb = m0 / HBM_;
    if (slot >= vblk[2 * mb]) return;
    roff = vblk[2 * mb + 1] * kCrtMax;
  }
  // same: slot q multiplies plane q + 1 of both operands (one pair); else the pairs of
  // diagonal d, planes (s, d - s)
  const int s_lo = same ? slot + 1 : max(1, d - kr), s_hi = same ? slot + 1 : min(kl, d - 1);
  const int rsum = same ? 2 * (slot + 1) : d;   // R plane of pair s: rsum - s
  const int npairs = s_hi - s_lo + 1;
  const int KT = kdim / DBK;
  const int T = npairs * KT;   // K-stages over all pairs of this diagonal
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  using Acc = std::conditional_t<F8, v16f, v16i>;
  Acc acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][c][v] = 0;

  // this lane's share of a stage: wave w fills rows [64w, 64w + 64) of both operands, 16 rows
  // per instruction; lane -> row 16i + lane/4, chunk position lane%4, which holds chunk
  // (lane%4) ^ ((row >> 2) & 3) of the row (the same for the four instructions, 16i being a
  // multiple of 4). The four instructions differ by 16 rows = 1 KB both in the plane and in the
  // ring, which their immediate offset carries, so one address serves all four.
  const int lrow = lane >> 2, lpos = lane & 3;
  const int loff = (wave * 64 + lrow) * DBK + 16 * (lpos ^ ((lrow >> 2) & 3));
  // issue stream: stages are issued in order; the next one is K-block ik of pair s_lo + ip,
  // whose K-blocks of this tile's rows start at lsrc / rsrc (K-blocks of a plane are
  // npad * 64 bytes apart; the next pair's L plane follows, its R plane precedes)
  const size_t kstride = (size_t)npad * DBK;
  const int8_t *lpair = Lp + (size_t)(s_lo - 1) * pstride + (size_t)m0 * DBK;
  const int8_t *rpair = Rp + (size_t)(roff + rsum - s_lo - 1) * pstride + (size_t)n0 * DBK;
  const int8_t *lsrc = lpair, *rsrc = rpair;
  int ik = 0;
  auto advance = [&]() {
    const bool wrap = ++ik == KT;
    ik = wrap ? 0 : ik;
    lpair = wrap ? lpair + pstride : lpair;
    rpair = wrap ? rpair - pstride : rpair;
    lsrc = wrap ? lpair : lsrc + kstride;
    rsrc = wrap ? rpair : rsrc + kstride;
  };
  auto issue = [&](int tt) {
    int8_t *st = ring + (tt % S) * DSTAGE_BYTES + wave * 64 * DBK;
    dma_rows4(lsrc + loff, st);
    dma_rows4(rsrc + loff, st + 256 * DBK);
    advance();
  };
  // fragment offsets within a stage: row r, 16-byte chunk c -> r*64 + 16*(c ^ ((r>>2)&3))
  int fa_off[2][4], fb_off[2][4];
  const int cgrp = lane >> 5;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int ra = wm * 128 + x * 32 + (lane & 31), rbr = wn * 128 + x * 32 + (lane & 31);
      const int c = 2 * ks + cgrp;
      fa_off[ks][x] = ra * DBK + 16 * (c ^ ((ra >> 2) & 3));
      fb_off[ks][x] = 256 * DBK + rbr * DBK + 16 * (c ^ ((rbr >> 2) & 3));
    }
  v4i fA[2][2][4], fB[2][2][4];   // [register set][k half][block]
  auto load_frags = [&](int tt, v4i (&fa)[2][4], v4i (&fb)[2][4]) {
    const int8_t *sb = ring + (tt % S) * DSTAGE_BYTES;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        fa[ks][x] = *(const v4i *)(sb + fa_off[ks][x]);
        fb[ks][x] = *(const v4i *)(sb + fb_off[ks][x]);
      }
  };
  // Wait until stage `need` has landed for every wave, given that stages up to
  // `last` have been issued (8 DMA instructions per stage and wave), then barrier.
  auto wait_stage = [&](int need, int last) {
    const int ahead = last - need;
    if (ahead >= 2) wait_vm_lds_barrier<16>();
    else if (ahead == 1) wait_vm_lds_barrier<8>();
    else wait_vm_lds_barrier<0>();
  };
  // prologue: stages 0..S-2 in flight, stage 0 landed, its fragments in set 0
  for (int q = 0; q < S - 1 && q < T; ++q) issue(q);
  wait_stage(0, min(T - 1, S - 2));
  load_frags(0, fA[0], fB[0]);

  // One stage: wait for stage tt+1 (which also guarantees that every wave has
  // read stage tt-1 from the slot the new DMA refills), issue the DMA of stage
  // tt+S-1, read stage tt+1 into the other register set, and run the MFMAs of
  // stage tt. Steady stages (tt+S-1 < T) are branch-free so the scheduler can
  // interleave the three instruction streams.
  // Steady INT8 stage in 8 chunks, fenced so they keep this order: chunk g reads its share of
  // the 16 fragments of stage tt+1 (3, 3, 3, 3, 2, 2, 0, 0 of the sequence A0 B0 A1 B1 ...),
  // runs 4 of the 32 MFMAs of stage tt and issues DMA instruction g of stage tt+S-1 (L rows
  // for g < 4, R rows after). With one wavefront per SIMD, issue is in program order, so
  // spreading the memory instructions over the MFMAs keeps the matrix core fed while they
  // issue, and the last reads land two chunks before the next stage's wait.
  auto chunk = [&](auto G, const v4i (&ca)[2][4], const v4i (&cb)[2][4], v4i (&na)[2][4],
                   v4i (&nb)[2][4], const int8_t *lg, const int8_t *rg, int8_t *dst,
                   const int8_t *sb) {
    constexpr int g = decltype(G)::value;
    constexpr int rlo = g < 4 ? 3 * g : g < 6 ? 12 + 2 * (g - 4) : 16;
    constexpr int rhi = g < 4 ? 3 * g + 3 : g < 6 ? 14 + 2 * (g - 4) : 16;
#pragma unroll
    for (int r = rlo; r < rhi; ++r) {
      const int f = r >> 1;
      if (r & 1) nb[f >> 2][f & 3] = *(const v4i *)(sb + fb_off[f >> 2][f & 3]);
      else na[f >> 2][f & 3] = *(const v4i *)(sb + fa_off[f >> 2][f & 3]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = 4 * g + j, ks = m >> 4, x = (m >> 2) & 3, y = m & 3;
      acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ca[ks][x], cb[ks][y], acc[x][y], 0, 0, 0);
    }
    typedef void __attribute__((address_space(3))) *lds_ptr;
    if constexpr (g < 4)
      __builtin_amdgcn_global_load_lds((const void *)lg, (lds_ptr)dst, 16, g * 1024, 0);
    else
      __builtin_amdgcn_global_load_lds((const void *)rg, (lds_ptr)(dst + 256 * DBK), 16,
                                       (g - 4) * 1024, 0);
    if constexpr (g == 7) advance();
    __builtin_amdgcn_sched_barrier(0);
  };
  auto stage = [&](auto steady, int tt, v4i (&ca)[2][4], v4i (&cb)[2][4], v4i (&na)[2][4],
                   v4i (&nb)[2][4]) {
    if constexpr (!F8 && decltype(steady)::value) {
      wait_vm_lds_barrier<8 * (S - 3)>();
      __builtin_amdgcn_sched_barrier(0);
      int8_t *dst = ring + ((tt + S - 1) % S) * DSTAGE_BYTES + wave * 64 * DBK;
      const int8_t *lg = lsrc + loff, *rg = rsrc + loff;
      const int8_t *sb = ring + ((tt + 1) % S) * DSTAGE_BYTES;
      chunk(std::integral_constant<int, 0>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 1>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 2>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 3>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 4>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 5>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 6>(), ca, cb, na, nb, lg, rg, dst, sb);
      chunk(std::integral_constant<int, 7>(), ca, cb, na, nb, lg, rg, dst, sb);
      return;
    }
    if constexpr (decltype(steady)::value) {
      wait_vm_lds_barrier<8 * (S - 3)>();
      issue(tt + S - 1);
      load_frags(tt + 1, na, nb);
    } else if (tt + 1 < T) {
      wait_stage(tt + 1, min(T - 1, tt + S - 2));
      if (tt + S - 1 < T) issue(tt + S - 1);
      load_frags(tt + 1, na, nb);
    }
    if constexpr (F8) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const v8i a8 = {ca[0][x][0], ca[0][x][1], ca[0][x][2], ca[0][x][3],
                          ca[1][x][0], ca[1][x][1], ca[1][x][2], ca[1][x][3]};
          const v8i b8 = {cb[0][y][0], cb[0][y][1], cb[0][y][2], cb[0][y][3],
                          cb[1][y][0], cb[1][y][1], cb[1][y][2], cb[1][y][3]};
          // formats 0, 0: E4M3 for both operands; zero scale operands select the unscaled form
          acc[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[x][y], 0, 0, 0,
                                                                      0, 0, 0);
        }
      if constexpr (decltype(steady)::value) {
        // per 2 MFMAs: one DMA instruction and two fragment reads
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            acc[x][y] =
                __builtin_amdgcn_mfma_i32_32x32x32_i8(ca[ks][x], cb[ks][y], acc[x][y], 0, 0, 0);
      if constexpr (decltype(steady)::value) {
        // per 4 MFMAs: one DMA instruction, two fragment reads and up to five scalar or vector
        // ALU instructions (addresses, the issue stream's pointers), so that a wave with one
        // wavefront per SIMD never issues a run of them while its matrix core idles
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x006, 3, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x006, 2, 0);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  using Steady = std::integral_constant<bool, true>;
  using Tail = std::integral_constant<bool, false>;
  const int t_steady = T - S + 1;   // stages tt < t_steady are steady
  int tt = 0;
  for (; tt + 1 < t_steady; tt += 2) {
    stage(Steady(), tt, fA[0], fB[0], fA[1], fB[1]);
    stage(Steady(), tt + 1, fA[1], fB[1], fA[0], fB[0]);
  }
  for (; tt < T; tt += 2) {   // tt is even here, so register set 0 holds stage tt
    stage(Tail(), tt, fA[0], fB[0], fA[1], fB[1]);
    if (tt + 1 < T) stage(Tail(), tt + 1, fA[1], fB[1], fA[0], fB[0]);
  }
  if (!F8 && mods) {   // residue products: store the slot's value mod m_slot (|r| <= 127) as INT8
    auto Cq8 = gview_w((int8_t *)C + (size_t)slot * npad * npad);
    const double m = (double)mods[slot], rm = 1.0 / m;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = m0 + wm * 128 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int col = n0 + wn * 128 + y * 32 + (lane & 31);
          const double c = (double)acc[x][y][v];
          Cq8[(size_t)row * npad + col] = (int8_t)(int)(c - m * rint(c * rm));
        }
    return;
  }
  auto Cq = gview_w(C + (size_t)slot * npad * npad);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 128 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + wn * 128 + y * 32 + (lane & 31);
        Cq[(size_t)row * npad + col] = (int32_t)acc[x][y][v];
      }
}

template <bool F8>
__global__ __launch_bounds__(256, 1) void k_slice_gemm256d(const int8_t *__restrict__ Lp,
                                                           const int8_t *__restrict__ Rp,
                                                           size_t pstride, int npad, int kdim,
                                                           int kl, int kr, int d_min,
                                                           DiagOrder order,
                                                           int32_t *__restrict__ C, RowBlocks rb,
                                                           int same, const int *__restrict__ tcut,
                                                           const int *__restrict__ tab,
                                                           const int *__restrict__ mods,
                                                           const int *__restrict__ vblk,
                                                           const int *__restrict__ dp) {
  int m0, n0, slot;
  if (dp) {   // device-planned table launch: sized for the largest table
    if ((int)blockIdx.x >= dp[2]) return;
    kl = dp[0];
    kr = dp[1];
  }
  if (tab) {   // block table: row block | column block << 8 | slot << 16
    const int ent = tab[blockIdx.x];
    m0 = (ent & 0xff) * HBM_;
    n0 = ((ent >> 8) & 0xff) * HBM_;
    slot = ent >> 16;
  } else {
    int mi;
    tile_of_block(blockIdx.x, rb.count, npad / HBM_, mi, n0);
    m0 = rb.m[mi] * HBM_;
    slot = order.q[blockIdx.y];
  }
  gemm256_item<F8>(Lp, Rp, pstride, npad, kdim, kl, kr, d_min, C, same, tcut, mods, vblk, m0, n0,
                   slot);
}

void launch_slice_gemm(const int8_t *Lp, const int8_t *Rp, size_t pstride, int npad, int kl,
                       int kr, int d_min, int ndiag, int32_t *C, const RowBlocks *rbp,
                       hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop, int kdim,
                       bool same_plane, const int *tcut, const int *mods, bool f8,
                       const int *vblk) {
  if (kdim <= 0) kdim = npad;
  // heaviest diagonals (most pairs) first, so the tail of the launch is light
  DiagOrder o;
  int cnt[kMaxDiag];
  for (int q = 0; q < ndiag; ++q) {
    int d = d_min + q;
    int lo = d - kr > 1 ? d - kr : 1, hi = kl < d - 1 ? kl : d - 1;
    cnt[q] = same_plane ? 1 : hi - lo + 1;
    o.q[q] = q;
  }
  for (int a = 1; a < ndiag; ++a)
    for (int b = a; b > 0 && cnt[o.q[b]] > cnt[o.q[b - 1]]; --b) {
      int t = o.q[b];
      o.q[b] = o.q[b - 1];
      o.q[b - 1] = t;
    }
  const int tr = gemm_tile_rows(npad);
  RowBlocks rb;
  if (rbp) {
    rb = *rbp;
  } else {
    rb.count = npad / tr;
    for (int i = 0; i < rb.count; ++i) rb.m[i] = i;
  }
  if (rb.count <= 0) return;
  const int tiles = rb.count * (npad / tr);
  if (f8)
    hipExtLaunchKernelGGL(k_slice_gemm256d<true>, dim3(tiles, ndiag), dim3(256), 0, s, ev_start,
                          ev_stop, 0, Lp, Rp, pstride, npad, kdim, kl, kr, d_min, o, C, rb,
                          (int)same_plane, tcut, (const int *)nullptr, (const int *)nullptr,
                          (const int *)nullptr, (const int *)nullptr);
  else if (npad >= 1024)
    hipExtLaunchKernelGGL(k_slice_gemm256d<false>, dim3(tiles, ndiag), dim3(256), 0, s, ev_start,
                          ev_stop, 0, Lp, Rp, pstride, npad, kdim, kl, kr, d_min, o, C, rb,
                          (int)same_plane, tcut, (const int *)nullptr, mods, vblk,
                          (const int *)nullptr);
  else
    hipExtLaunchKernelGGL(k_slice_gemm, dim3(tiles, ndiag), dim3(256), 0, s, ev_start, ev_stop, 0,
                          Lp, Rp, pstride, npad, kdim, kl, kr, d_min, o, C, rb, (int)same_plane,
                          mods, (const int *)nullptr, (const int *)nullptr, vblk);
}

// FP8 E4M3 (sign, 4 exponent bits with bias 7, 3 mantissa bits): a nonzero |d| <= 15 is
// 2^e (1 + m/8) with e = floor(log2 |d|) and m = 8 |d| / 2^e - 8, an integer since e <= 3.
__global__ void k_digits_e4m3(const int8_t *__restrict__ in, uint8_t *__restrict__ out,
                              size_t count, int *__restrict__ bad) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    const int d = in[i], a = d < 0 ? -d : d;
    if (a > 15) {
      atomicOr(bad, 1);
      out[i] = 0x7f;   // NaN
      continue;
    }
    int code = 0;
    if (a) {
      const int e = 31 - __clz(a);
      code = ((e + 7) << 3) | (((a << 3) >> e) - 8);
    }
    out[i] = (uint8_t)((d < 0 ? 0x80 : 0) | code);
  }
}

void launch_digits_e4m3(const int8_t *in, uint8_t *out, size_t count, int *bad, hipStream_t s) {
  const size_t blocks = std::min<size_t>((count + 255) / 256, 65536);
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_digits_e4m3, dim3((unsigned)blocks), dim3(256), 0, s, in, out, count, bad);
}

int gemm_tile_rows(int npad) { return npad >= 1024 ? HBM_ : GBM; }

void launch_slice_gemm_table(const int8_t *Lp, const int8_t *Rp, size_t pstride, int npad,
                             int kl, int kr, int d_min, const int *tab, int nblocks, int32_t *C,
                             hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop, int kdim,
                             const int *tcut, const int *dp) {
  if (kdim <= 0) kdim = npad;
  if (nblocks <= 0) return;
  DiagOrder o;
  RowBlocks rb;
  rb.count = 0;
  for (int q = 0; q < kMaxDiag; ++q) o.q[q] = q;
  if (npad >= 1024)
    hipExtLaunchKernelGGL(k_slice_gemm256d<false>, dim3(nblocks, 1), dim3(256), 0, s, ev_start,
                          ev_stop, 0, Lp, Rp, pstride, npad, kdim, kl, kr, d_min, o, C, rb, 0,
                          tcut, tab, (const int *)nullptr, (const int *)nullptr, dp);
  else
    hipExtLaunchKernelGGL(k_slice_gemm, dim3(nblocks, 1), dim3(256), 0, s, ev_start, ev_stop, 0,
                          Lp, Rp, pstride, npad, kdim, kl, kr, d_min, o, C, rb, 0,
                          (const int *)nullptr, tab, dp, (const int *)nullptr);
}

// Threads and entries per thread of the column epilogues (one block per output column):
// up to npad = 1024, 256 threads with npad / 256 entries each (rounded up to 1, 2 or 4), so a
// CU holds several columns' blocks at once and their latencies overlap; above it 1024 threads
// and npad / 1024 entries each. The single and grouped launches use the same shapes, so their
// reductions group the column's entries alike.
#define EPI_DISPATCH(npad, M)        \
  do {                               \
    if ((npad) <= 256) M(1, 256);    \
    else if ((npad) <= 512) M(2, 256);  \
    else if ((npad) <= 1024) M(4, 256); \
    else if ((npad) <= 2048) M(2, 1024); \
    else if ((npad) <= 4096) M(4, 1024); \
    else M(8, 1024);                 \
  } while (0)
#define EPI_DISPATCH_G(npad, M)      \
  do {                               \
    if ((npad) <= 256) M(1, 256);    \
    else if ((npad) <= 512) M(2, 256);  \
    else if ((npad) <= 1024) M(4, 256); \
    else if ((npad) <= 2048) M(2, 1024); \
    else M(4, 1024);                 \
  } while (0)

// Rows of a column epilogue's thread: EPT consecutive rows i = EPT tid + q (EPT divides 64,
// so they share one 64-row K-block), so the thread's entries of one slot are one vector load
// and its digits of one plane one vector store. A thread's rows are all below npad or none.
template <int EPT>
__device__ __forceinline__ int erow(int tid, int q) {
  return EPT * tid + q;
}
// EPT consecutive values at p (aligned to their total size), integers sign-extended from int8
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <int EPT>
__device__ __forceinline__ void load_i8v(const int8_t *__restrict__ p, int (&v)[EPT]) {
  if constexpr (EPT == 8) {
    const u32x2 w = *gview((const u32x2 *)p);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = (int)(int8_t)(w.x >> (8 * e));
      v[4 + e] = (int)(int8_t)(w.y >> (8 * e));
    }
  } else if constexpr (EPT == 4) {
    const uint32_t w = *gview((const uint32_t *)p);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (int)(int8_t)(w >> (8 * e));
  } else if constexpr (EPT == 2) {
    const uint32_t w = *gview((const uint16_t *)p);
    v[0] = (int)(int8_t)w;
    v[1] = (int)(int8_t)(w >> 8);
  } else {
    v[0] = *gview(p);
  }
}
template <int EPT>
__device__ __forceinline__ void load_i32v(const int32_t *__restrict__ p, int32_t (&v)[EPT]) {
  if constexpr (EPT >= 4) {
#pragma unroll
    for (int h = 0; h < EPT / 4; ++h) {
      const v4i w = gview((const v4i *)p)[h];
      v[4 * h] = w.x;
      v[4 * h + 1] = w.y;
      v[4 * h + 2] = w.z;
      v[4 * h + 3] = w.w;
    }
  } else if constexpr (EPT == 2) {
    const i32x2 w = *gview((const i32x2 *)p);
    v[0] = w.x;
    v[1] = w.y;
  } else {
    v[0] = *gview(p);
  }
}
template <int EPT>
__device__ __forceinline__ void load_f64v(const double *__restrict__ p, double (&v)[EPT]) {
  if constexpr (EPT >= 2) {
#pragma unroll
    for (int h = 0; h < EPT / 2; ++h) {
      const f64x2 w = gview((const f64x2 *)p)[h];
      v[2 * h] = w.x;
      v[2 * h + 1] = w.y;
    }
  } else {
    v[0] = *gview(p);
  }
}
// the low bytes of d[0..EPT) packed in order and stored at p (aligned to EPT bytes)
template <int EPT>
__device__ __forceinline__ void store_i8v(int8_t *__restrict__ p, const int (&d)[EPT]) {
  if constexpr (EPT == 8) {
    u32x2 w = {0u, 0u};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      w.x |= ((uint32_t)d[e] & 255u) << (8 * e);
      w.y |= ((uint32_t)d[4 + e] & 255u) << (8 * e);
    }
    *gview_w((u32x2 *)p) = w;
  } else if constexpr (EPT == 4) {
    uint32_t w = 0u;
#pragma unroll
    for (int e = 0; e < 4; ++e) w |= ((uint32_t)d[e] & 255u) << (8 * e);
    *gview_w((uint32_t *)p) = w;
  } else if constexpr (EPT == 2) {
    *gview_w((uint16_t *)p) = (uint16_t)(((uint32_t)d[0] & 255u) | (((uint32_t)d[1] & 255u) << 8));
  } else {
    *gview_w(p) = (int8_t)d[0];
  }
}

// Digit planes of one operand row j (an output column of a column epilogue): the values
// v (EPT per thread, rows erow(tid, q); zero beyond n) with column maximum ms,
// exponent exp_above(ms), written K-blocked for rows i < npad.
template <int EPT, int NT = kEpiThreads>
__device__ __forceinline__ void write_col_planes(const double (&v)[EPT], double ms, int j, int npad,
                                                 int8_t *__restrict__ planes, int k) {
  const size_t P = (size_t)npad * npad;
  const int i0 = erow<EPT>(threadIdx.x, 0);
  if (i0 >= npad) return;
  const int ee = exp_above(ms);
  // digits of the signed value: truncation toward zero gives each digit the value's sign and
  // the magnitude floor(|.|) would, and leaves a remainder of the same sign (all exact)
  double y[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) y[q] = ldexp(v[q], -ee);
  int8_t *dst = planes + kb_off(j, i0, npad);
  for (int t = 0; t < k; ++t) {
    int d[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const double t128 = y[q] * 128.0;
      const double dgt = trunc(t128);
      y[q] = t128 - dgt;
      d[q] = (int)dgt;
    }
    store_i8v<EPT>(dst + (size_t)t * P, d);
  }
}

// ---------------------------------------------------------------- V epilogue + column pass
// Reconstruction of P from its residues r_q = C_q mod m_q (symmetric), for the EPT rows of a
// thread: P / M = frac(sum_q r_q u_q) in [-1/2, 1/2), summed exactly in four 34-bit
// fixed-point limbs (u_q truncated to 136 bits, an error of at most 2^-124.2), carried into
// s0 + s1 + s2, then V = (P / M) M 2^(scale) as a double-word (vh, vl); with the double-word
// products by M the absolute error stays below 2^-115 M (the planner's floor).
template <int EPT, int NT = kEpiThreads>
__device__ __forceinline__ void crt_column(const int8_t *__restrict__ Ccol, size_t P, int n,
                                           int npad, int tid, const CrtRec &rec,
                                           const int (&scale)[EPT], double (&vh)[EPT],
                                           double (&vl)[EPT]) {
  const int i0 = erow<EPT>(tid, 0);
  // F = sum_q r_q u_q mod 1 in kCrtLimbs fixed-point limbs of 34 bits: |r_q| <= 127, so
  // r_q L[q][k] is an integer below 2^41 and at most 28 of them sum below 2^45.9: every limb
  // sum is exact. Truncating u_q to 136 bits moves F by at most 28 127 2^-136 = 2^-124.2.
  // A slot's EPT bytes per thread are one packed load (loadw); kD slots are in flight, in a
  // ring of packed words unpacked where they are used; terms in order of the moduli. The
  // ring's first fill does not wait for the record: the residue buffer holds at least
  // kCrtMax > kD slots, so its first kD slots exist whatever N is (those past N are unused).
  constexpr int kD = EPT >= 8 ? 6 : EPT >= 4 ? 8 : 12;
  static_assert(kD < kCrtMax, "the first ring fill reads slots below kCrtMax");
  // threads past the padded order read row 0 (no branch around the loads); all their rows
  // are >= n, so what they sum is discarded like the padding rows' results
  const int8_t *Crow = Ccol + (i0 < npad ? i0 : 0);
  auto loadw = [&](int s) -> uint2 {
    uint2 w = {0u, 0u};
    const int8_t *p = Crow + (size_t)s * P;
    if constexpr (EPT == 8) {
      const u32x2 v2 = *gview((const u32x2 *)p);
      w.x = v2.x;
      w.y = v2.y;
    }
    else if constexpr (EPT == 4) w.x = *gview((const uint32_t *)p);
    else if constexpr (EPT == 2) w.x = *gview((const uint16_t *)p);
    else w.x = (uint8_t)*gview(p);
    return w;
  };
  // The record's limbs, staged in LDS (every thread reads all of them); their loads go out
  // before the ring's, so that storing them waits for them alone.
  __shared__ double sL[kCrtMax * kCrtLimbs];
  constexpr int kLper = (kCrtMax * kCrtLimbs + NT - 1) / NT;
  double lv[kLper];
#pragma unroll
  for (int t = 0; t < kLper; ++t) {
    const int e = threadIdx.x + t * NT;
    lv[t] = e < kCrtMax * kCrtLimbs ? rec.L[e / kCrtLimbs][e % kCrtLimbs] : 0.0;
  }
  uint2 ring[kD];
#pragma unroll
  for (int u = 0; u < kD; ++u) ring[u] = loadw(u);
#pragma unroll
  for (int t = 0; t < kLper; ++t) {
    const int e = threadIdx.x + t * NT;
    if (e < kCrtMax * kCrtLimbs) sL[e] = lv[t];
  }
  const int N = rec.N;
  __syncthreads();
  double a[EPT][kCrtLimbs];
#pragma unroll
  for (int q = 0; q < EPT; ++q)
#pragma unroll
    for (int k = 0; k < kCrtLimbs; ++k) a[q][k] = 0.0;
  // All kCrtMax places of the sum are unrolled: the loads are unconditional (past the last
  // slot, slot N - 1 again, which hits the cache), so the memory-counter waits stay exact
  // with kD loads in flight; the terms themselves are skipped past N.
#pragma unroll
  for (int q = 0; q < kCrtMax; ++q) {
    const uint2 w = ring[q % kD];
    ring[q % kD] = loadw(max(min(q + kD, N - 1), 0));
    if (q < N) {
      double L[kCrtLimbs];
#pragma unroll
      for (int k = 0; k < kCrtLimbs; ++k) L[k] = sL[q * kCrtLimbs + k];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        // rows >= n carry the zero padding's residues; their results are discarded
        const uint32_t word = e < 4 ? w.x : w.y;
        const double rq = (double)(int)(int8_t)(word >> (8 * (e & 3)));
#pragma unroll
        for (int k = 0; k < kCrtLimbs; ++k) a[e][k] = fma(rq, L[k], a[e][k]);
      }
    }
  }
  static_assert(kCrtLimbs == 4 && kCrtLimbBits == 34, "limb scales below are written for 4 x 34");
  const double base = 0x1p34, rbase = 0x1p-34;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    // carries from the last limb up (exact: all values are integers below 2^53), then the
    // first limb mod 2^34: F in [0, 1) as limbs in [0, 2^34)
#pragma unroll
    for (int k = kCrtLimbs - 1; k > 0; --k) {
      const double cr = floor(a[q][k] * rbase);
      a[q][k] = fma(-cr, base, a[q][k]);
      a[q][k - 1] += cr;
    }
    a[q][0] = fma(-floor(a[q][0] * rbase), base, a[q][0]);
    // F = s0 + s1 + s2: s0 exact (34 bits), s1 + e the exact sum of the next two limbs
    double s0 = a[q][0] * 0x1p-34, s1, e;
    two_sum(a[q][1] * 0x1p-68, a[q][2] * 0x1p-102, s1, e);
    const double s2 = e + a[q][3] * 0x1p-136;
    // the symmetric representative: F in [-1/2, 1/2)
    if (s0 + s1 >= 0.5) s0 -= 1.0;
    // (s0 + s1 + s2) (M0 + M1 + M2): the terms down to 2^-99 M are exact products and are
    // summed as a double-word, so the absolute error stays near 2^-130 M
    double ph, pl, q1, q1e, q2, q2e, Lw, Le, tw, te;
    two_prod(s0, rec.M[0], ph, pl);
    two_prod(s0, rec.M[1], q1, q1e);
    two_prod(s1, rec.M[0], q2, q2e);
    two_sum(pl, q1, Lw, Le);
    two_sum(Lw, q2, tw, te);
    Lw = tw;
    Le += te + (q1e + q2e) + (s1 * rec.M[1] + s2 * rec.M[0] + s0 * rec.M[2]);
    double h2, l2;
    two_sum(ph, Lw, h2, l2);
    l2 += Le;
    fast_two_sum(h2, l2, h2, l2);
    vh[q] = ldexp(h2, scale[q]);
    vl[q] = ldexp(l2, scale[q]);
  }
}

template <int EPT, bool CRT, int NT = kEpiThreads>
__device__ __forceinline__ void epi_v_body(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag_all, const int *__restrict__ dcut,
    const int *__restrict__ eA, const int *__restrict__ eX, const double *__restrict__ X1, int n,
    double *lam, double *lam_lo, double *r, int *eR, double *resmax, int8_t *__restrict__ Rpl,
    int kr, int *flags, const CrtRec *__restrict__ recs, const int *__restrict__ vblk,
    const int *__restrict__ gate, int bx) {
  __shared__ double scratch[4 * (NT / 64)];
  if (gate && *gate == 0) return;
  const int j = bx, tid = threadIdx.x;
  const size_t P = (size_t)npad * npad;
  const int i0 = erow<EPT>(tid, 0);
  const bool live = i0 < npad;   // the thread's rows exist in the padded order
  if (j >= n) {
    double z[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) z[q] = 0.0;
    write_col_planes<EPT, NT>(z, 0.0, j, npad, Rpl, kr);
    return;
  }
  const int ej = eX[j];
  const int ndiag = dcut ? min(ndiag_all, dcut[j] - d_min + 1) : ndiag_all;
  const int32_t *Ccol = C + (size_t)j * npad + i0;
  const double *xcol = X1 + (size_t)j * n;
  double vh[EPT], vl[EPT];
  int eiq[EPT];
  {
    int ea[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) ea[q] = 0;
    if (live) load_i32v<EPT>(eA + i0, ea);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      vh[q] = vl[q] = 0.0;
      eiq[q] = (i0 + q < n) ? ea[q] + ej : 0;
    }
  }
  if constexpr (CRT) {
    // the record of this column's level (per 256-column block: slot count, level)
    const CrtRec &rec = recs[vblk ? vblk[2 * (j >> 8) + 1] : 0];
    int sc[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) sc[q] = eiq[q] + rec.sh;
    crt_column<EPT, NT>((const int8_t *)C + (size_t)j * npad, P, n, npad, tid, rec, sc, vh, vl);
  } else {
  // slice sum, smallest scale first; with few entries per thread the diagonals' values are
  // loaded kPD at a time, with many the next diagonal is loaded while this one is summed
  if constexpr (EPT >= 4) {
    int32_t cv[EPT], cn[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) cv[q] = 0;
    if (live && ndiag > 0) load_i32v<EPT>(Ccol + (size_t)(ndiag - 1) * P, cv);
#pragma unroll
    for (int q = 0; q < EPT; ++q)
      if (i0 + q >= n) cv[q] = 0;
#pragma unroll 1
    for (int qq = ndiag - 1; qq >= 0; --qq) {
      if (qq > 0) {
#pragma unroll
        for (int q = 0; q < EPT; ++q) cn[q] = 0;
        if (live) load_i32v<EPT>(Ccol + (size_t)(qq - 1) * P, cn);
#pragma unroll
        for (int q = 0; q < EPT; ++q)
          if (i0 + q >= n) cn[q] = 0;
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const double tv = ldexp((double)cv[q], eiq[q] - 7 * (d_min + qq));
        double s, e;
        two_sum(vh[q], tv, s, e);
        vh[q] = s;
        vl[q] += e;
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) cv[q] = cn[q];
    }
  } else {
  constexpr int kPD = 16 / EPT;
#pragma unroll 1
  for (int c0 = ndiag - 1; c0 >= 0; c0 -= kPD) {
    int32_t cv[kPD][EPT];
#pragma unroll
    for (int u = 0; u < kPD; ++u) {
      const int qq = c0 - u;
#pragma unroll
      for (int q = 0; q < EPT; ++q) cv[u][q] = 0;
      if (qq >= 0 && live) load_i32v<EPT>(Ccol + (size_t)qq * P, cv[u]);
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        if (i0 + q >= n) cv[u][q] = 0;
    }
#pragma unroll
    for (int u = 0; u < kPD; ++u) {
      const int qq = c0 - u;
      if (qq < 0) break;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const double tv = ldexp((double)cv[u][q], eiq[q] - 7 * (d_min + qq));
        double s, e;
        two_sum(vh[q], tv, s, e);
        vh[q] = s;
        vl[q] += e;
      }
    }
  }
  }
  }
  // the column of X^(1) is read where it is used (holding the thread's slice of it in
  // registers across the reductions costs spills)
  ddv sx = {0.0, 0.0}, sv = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = i0 + q;
    if (i < n) {
      fast_two_sum(vh[q], vl[q], vh[q], vl[q]);
      const double x = *gview(xcol + i);
      double p, pe;
      two_prod(x, x, p, pe);
      sx = dd_add_prod(sx, p, pe);
      two_prod(x, vh[q], p, pe);
      sv = dd_add_prod(sv, p, pe + x * vl[q]);
    }
  }
  block_dd_sum2<NT>(sx, sv, scratch);
  // r_j = 1 - x^T x,  lambda_j = x^T v / (1 - r_j)
  ddv rj = dd_add(ddv{1.0, 0.0}, ddv{-sx.h, -sx.l});
  ddv den = dd_add(ddv{1.0, 0.0}, ddv{-rj.h, -rj.l});
  const ddv ljd = dd_div_to_dd(sv, den);
  const double lj = ljd.h;
  // residual in pair arithmetic: (vh + vl) - x * (lambda_hi + lambda_lo)
  double rmax = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = i0 + q;
    if (i < n) {
      double p, pe, s, e;
      const double x = *gview(xcol + i);
      two_prod(x, lj, p, pe);
      two_sum(vh[q], -p, s, e);
      const double res = s + (((e + vl[q]) - pe) - x * ljd.l);
      vh[q] = res;
      rmax = fmax(rmax, fabs(res));
    } else {
      vh[q] = 0.0;
    }
  }
  rmax = block_max<NT>(rmax, scratch);
  const int er = exp_above(rmax);
  write_col_planes<EPT, NT>(vh, rmax, j, npad, Rpl, kr);
  if (tid == 0) {
    lam[j] = lj;
    lam_lo[j] = ljd.l;
    r[j] = rj.h;
    eR[j] = er;
    resmax[j] = rmax;
    if (!(fabs(lj) <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

template <int EPT, bool CRT, int NT>
__global__ __launch_bounds__(NT) void k_epi_v(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag_all, const int *__restrict__ dcut,
    const int *__restrict__ eA, const int *__restrict__ eX, const double *__restrict__ X1, int n,
    double *lam, double *lam_lo, double *r, int *eR, double *resmax, int8_t *__restrict__ Rpl,
    int kr, int *flags, const CrtRec *__restrict__ recs, const int *__restrict__ vblk,
    const int *__restrict__ gate) {
  epi_v_body<EPT, CRT, NT>(C, npad, d_min, ndiag_all, dcut, eA, eX, X1, n, lam, lam_lo, r, eR,
                           resmax, Rpl, kr, flags, recs, vblk, gate, blockIdx.x);
}

template <int EPT, int NT>
static void epi_v_t(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                    const int *eA, const int *eX, const double *X1, int n, double *lam, double *lam_lo, double *r,
                    int *eR, double *resmax, int8_t *Rpl, int kr, int *flags, hipStream_t s,
                    const int *gate) {
  hipLaunchKernelGGL((k_epi_v<EPT, false, NT>), dim3(npad), dim3(NT), 0, s, C, npad, d_min,
                     ndiag, dcut, eA, eX, X1, n, lam, lam_lo, r, eR, resmax, Rpl, kr, flags,
                     (const CrtRec *)nullptr, (const int *)nullptr, gate);
}

void launch_epi_v_crt(const int32_t *C, int npad, const CrtRec *recs, const int *vblk,
                      const int *eA, const int *eX, const double *X1, int n, double *lam,
                      double *lam_lo, double *r, int *eR, double *resmax, int8_t *Rpl, int kr,
                      int *flags, hipStream_t s, const int *gate) {
#define EPI_V_CRT(E, T)                                                                       \
  hipLaunchKernelGGL((k_epi_v<E, true, T>), dim3(npad), dim3(T), 0, s, C, npad, 2, 1,          \
                     (const int *)nullptr, eA, eX, X1, n, lam, lam_lo, r, eR, resmax, Rpl, kr,  \
                     flags, recs, vblk, gate)
  EPI_DISPATCH(npad, EPI_V_CRT);
#undef EPI_V_CRT
}

// Residue planes from digit planes: 4 bytes of every plane per thread, K planes (template,
// so no predicated work for absent planes). The weights are taken in the symmetric range
// (|w| <= 127), the digit sum (|sum| < 18 127 127 < 2^24) is reduced in FP32: its quotient
// by m_q is off by less than 2^-10 and never within 1 / (2 m_q) >= 2^-9 of a half-integer.
template <int K>
__global__ __launch_bounds__(256) void k_residues(const int8_t *__restrict__ planes,
                                                  size_t pstride, size_t count,
                                                  const ResWeights w, int8_t *__restrict__ res) {
  constexpr int G = (K + 3) / 4;   // groups of four planes
  const size_t e = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e >= count) return;
  unsigned v[4 * G];
#pragma unroll
  for (int t = 0; t < 4 * G; ++t)
    v[t] = (t < K) ? *(const unsigned *)(planes + (size_t)t * pstride + e) : 0u;
  // per element b and group g: the digits of planes 4g .. 4g + 3 as the bytes of one dword
  int dg[G][4];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      dg[g][b] = (int)(((v[4 * g] >> (8 * b)) & 0xffu) |
                       (((v[4 * g + 1] >> (8 * b)) & 0xffu) << 8) |
                       (((v[4 * g + 2] >> (8 * b)) & 0xffu) << 16) |
                       (((v[4 * g + 3] >> (8 * b)) & 0xffu) << 24));
  for (int q = 0; q < w.N; ++q) {
    const float m = (float)w.m[q], rm = w.rmf[q];
    unsigned packed = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      // sum_t d_t w_qt as signed byte dot products: |sum| <= 18 127^2 < 2^19
      int acc = 0;
#pragma unroll
      for (int g = 0; g < G; ++g) acc = __builtin_amdgcn_sdot4(dg[g][b], w.wp[q][g], acc, false);
      const float a = (float)acc;
      const int rr = (int)(a - m * rintf(a * rm));   // |rr| <= (m - 1) / 2 <= 127
      packed |= ((unsigned)(rr & 0xff)) << (8 * b);
    }
    *(unsigned *)(res + (size_t)q * pstride + e) = packed;
  }
}

template <int K>
static void residues_t(const int8_t *planes, size_t pstride, size_t count, const ResWeights &w,
                       int8_t *res, hipStream_t s) {
  const size_t threads = count / 4;
  hipLaunchKernelGGL(k_residues<K>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                     planes, pstride, count, w, res);
}

void launch_residues(const int8_t *planes, size_t pstride, size_t count, const ResWeights &w,
                     int8_t *res, hipStream_t s) {
  switch (w.k) {
#define RES_K(K) \
  case K: residues_t<K>(planes, pstride, count, w, res, s); break;
    RES_K(1) RES_K(2) RES_K(3) RES_K(4) RES_K(5) RES_K(6) RES_K(7) RES_K(8) RES_K(9)
    RES_K(10) RES_K(11) RES_K(12) RES_K(13) RES_K(14) RES_K(15) RES_K(16) RES_K(17) RES_K(18)
#undef RES_K
    default: break;
  }
}

void launch_epi_v(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                  const int *eA, const int *eX, const double *X1, int n, double *lam, double *lam_lo, double *r,
                  int *eR, double *resmax, int8_t *Rpl, int kr, int *flags, hipStream_t s,
                  const int *gate) {
#define EPI_V(E, T)                                                                          \
  epi_v_t<E, T>(C, npad, d_min, ndiag, dcut, eA, eX, X1, n, lam, lam_lo, r, eR, resmax, Rpl, kr, \
                flags, s, gate)
  EPI_DISPATCH(npad, EPI_V);
#undef EPI_V
}

// Slots of W entry (i, j) that hold diagonals to sum: up to the column's cutoff dcut[j] or,
// with a per-tile table (T = npad / 256 tiles a side), the cutoff of tile (j / 256, i / 256).
__device__ __forceinline__ int w_ndiag(const int *__restrict__ dcut, const int *__restrict__ tcut,
                                       int T, int ndiag_all, int d_min, int i, int j) {
  int dc = dcut ? dcut[j] : d_min + ndiag_all - 1;
  if (tcut) dc = min(dc, tcut[(j >> 8) * T + (i >> 8)]);
  return min(ndiag_all, dc - d_min + 1);
}

// Per-tile W cutoffs, one block per row block I (256 rows): sorts the eigenvalue estimates
// of its rows in LDS, then for every column j takes g = the distance from lambda_j to the
// nearest of them (other than lambda_j itself when j is in I) and the tile maximum over the
// column block J of eR_j - floor(log2 g); tcut[J T + I] = the last diagonal that keeps the
// tile's W error within theta delta g: ceil((max_{i in I} eX_i + cx + that) / 7), in
// [2, dmax] (+ dextra). Columns with a zero residual (mask[j] == 0) need nothing.
// With tcol and gcol (per column, optional), g is replaced by max(gcol_j, tcol_j g): a column
// whose own gap gcol_j is small takes its far tiles tcol_j <= 1 times tighter, never tighter
// than its own gap (the column-wide rule).
__device__ __forceinline__ void tile_cutoffs_body(const double *__restrict__ lam,
                                                      const int *__restrict__ eX,
                                                      const int *__restrict__ eR,
                                                      const double *__restrict__ resmax, int n,
                                                      int T, double cx, int dmax, int dextra,
                                                      const double *__restrict__ tcol,
                                                      const double *__restrict__ gcol,
                                                      int *__restrict__ tcut,
                                                      const double *__restrict__ cxp,
                                                      const int *__restrict__ dmaxp, int bx) {
  __shared__ double v[256];
  if (cxp) cx = *cxp;
  if (dmaxp) dmax = *dmaxp;
  __shared__ int tm[kMaxTileSide];
  __shared__ int exb;
  const int I = bx, tid = threadIdx.x;
  const int i0 = I * 256, cnt = min(256, n - i0);
  v[tid] = (tid < cnt) ? lam[i0 + tid] : INFINITY;
  if (tid < T) tm[tid] = INT_MIN;
  if (tid == 0) exb = -100000;
  __syncthreads();
  if (tid < cnt) atomicMax(&exb, eX[i0 + tid]);
  // bitonic sort of the 256 values (padding +inf at the end)
  for (int k = 2; k <= 256; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      const int p = tid ^ j;
      if (p > tid) {
        const double a = v[tid], b = v[p];
        const bool up = (tid & k) == 0;
        if ((a > b) == up) {
          v[tid] = b;
          v[p] = a;
        }
      }
    }
  __syncthreads();
  for (int j = tid; j < n; j += 256) {
    if (resmax[j] == 0.0) continue;
    const double x = lam[j];
    // first index with v[idx] >= x
    int lo = 0, hi = cnt;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (v[mid] < x) lo = mid + 1;
      else hi = mid;
    }
    // nearest entry at or above x, passing over column j's own value once when j is in I
    // (a second equal value is a tie: g = 0); the entry below, v[lo - 1] < x, is another
    int q = lo;
    if ((j / 256) == I && q < cnt && v[q] == x) ++q;
    double g = (q < cnt) ? v[q] - x : INFINITY;
    if (lo > 0) g = fmin(g, x - v[lo - 1]);
    if (tcol && g > 0.0 && g <= DBL_MAX) g = fmax(gcol[j], tcol[j] * g);
    const int val = (g > 0.0 && g <= DBL_MAX) ? eR[j] - ilogb(g) : (1 << 20);
    atomicMax(&tm[j / 256], val);
  }
  __syncthreads();
  if (tid < T) {
    const int val = tm[tid];
    int d = 2;
    if (val != INT_MIN && cnt > 0) {
      const double need = (exb + cx + (double)val) / 7.0;
      d = min(dmax, max(2, (int)ceil(need) + dextra));
    }
    tcut[tid * T + I] = d;
  }
}

__global__ __launch_bounds__(256) void k_tile_cutoffs(const double *__restrict__ lam,
                                                      const int *__restrict__ eX,
                                                      const int *__restrict__ eR,
                                                      const double *__restrict__ resmax, int n,
                                                      int T, double cx, int dmax, int dextra,
                                                      const double *__restrict__ tcol,
                                                      const double *__restrict__ gcol,
                                                      int *__restrict__ tcut,
                                                      const double *__restrict__ cxp,
                                                      const int *__restrict__ dmaxp) {
  tile_cutoffs_body(lam, eX, eR, resmax, n, T, cx, dmax, dextra, tcol, gcol, tcut, cxp, dmaxp, blockIdx.x);
}

void launch_tile_cutoffs(const double *lam, const int *eX, const int *eR, const double *resmax,
                         int n, int T, double cx, int dmax, int dextra, const double *tcol,
                         const double *gcol, int *tcut, hipStream_t s, const double *cxp,
                         const int *dmaxp) {
  hipLaunchKernelGGL(k_tile_cutoffs, dim3(T), dim3(256), 0, s, lam, eX, eR, resmax, n, T, cx,
                     dmax, dextra, tcol, gcol, tcut, cxp, dmaxp);
}

// ---------------------------------------------------------------- W epilogue -> E~
template <int EPT, int NT = kEpiThreads>
__device__ __forceinline__ void epi_w_body(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag_all, const int *__restrict__ dcut,
    const int *__restrict__ eX, const int *__restrict__ eR, const double *__restrict__ lam,
    const double *__restrict__ lam_lo, const double *__restrict__ r, int n, int *eE,
    double *emax, int8_t *__restrict__ Epl, int ke, int *flags, double tau, int *cpl_count,
    int *cpl_pairs, int cpl_cap, const int *__restrict__ tcut, int bx) {
  __shared__ double scratch[2 * (NT / 64)];
  const int j = bx, tid = threadIdx.x;
  const size_t P = (size_t)npad * npad;
  const int i0 = erow<EPT>(tid, 0);
  const bool live = i0 < npad;   // the thread's rows exist in the padded order
  if (j >= n) {
    double z[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) z[q] = 0.0;
    write_col_planes<EPT, NT>(z, 0.0, j, npad, Epl, ke);
    return;
  }
  const int ej = eR[j];
  const double lj = lam[j], ljl = lam_lo[j];
  const int32_t *Ccol = C + (size_t)j * npad + i0;
  const int T = npad >> 8;
  // the rows of a thread lie in one 256-row tile, so they share one diagonal count; the
  // diagonals past it were not computed for that tile and are neither loaded nor summed
  const int nd = live ? w_ndiag(dcut, tcut, T, ndiag_all, d_min, i0, j) : 0;
  // W_ij = 2^(eX_i + eR_j) sum_d C_d 2^(-7 d): the sum runs in units of 2^(eX_i + eR_j)
  // (power-of-two scalings, so the roundings are those of the scaled sum); rows >= n sum
  // whatever the padding holds (finite integers) and are not used
  double wq[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) wq[q] = 0.0;
  // as in the V epilogue: with few entries per thread the diagonals' values are loaded kPD
  // at a time; with many, kD diagonals are in flight in a ring (smallest scale first)
  if constexpr (EPT >= 4) {
    constexpr int kD = 3;
    int32_t ring[kD][EPT];
    auto loadd = [&](int qq, int32_t (&v)[EPT]) {
#pragma unroll
      for (int q = 0; q < EPT; ++q) v[q] = 0;
      if (qq >= 0) load_i32v<EPT>(Ccol + (size_t)qq * P, v);
    };
#pragma unroll
    for (int u = 0; u < kD; ++u) loadd(nd - 1 - u, ring[u]);
#pragma unroll 1
    for (int c0 = nd - 1; c0 >= 0; c0 -= kD) {
#pragma unroll
      for (int u = 0; u < kD; ++u) {
        const int qq = c0 - u;
        if (qq < 0) break;
        int32_t cv[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) cv[q] = ring[u][q];
        loadd(qq - kD, ring[u]);
        const double sc = ldexp(1.0, -7 * (d_min + qq));
#pragma unroll
        for (int q = 0; q < EPT; ++q) wq[q] = fma((double)cv[q], sc, wq[q]);
      }
    }
  } else {
  constexpr int kPD = 16 / EPT;
#pragma unroll 1
  for (int c0 = nd - 1; c0 >= 0; c0 -= kPD) {
    int32_t cv[kPD][EPT];
#pragma unroll
    for (int u = 0; u < kPD; ++u) {
      const int qq = c0 - u;
#pragma unroll
      for (int q = 0; q < EPT; ++q) cv[u][q] = 0;
      if (qq >= 0) load_i32v<EPT>(Ccol + (size_t)qq * P, cv[u]);
    }
#pragma unroll
    for (int u = 0; u < kPD; ++u) {
      const int qq = c0 - u;
      if (qq < 0) break;
      const double sc = ldexp(1.0, -7 * (d_min + qq));
#pragma unroll
      for (int q = 0; q < EPT; ++q) wq[q] = fma((double)cv[u][q], sc, wq[q]);
    }
  }
  }
  int exv[EPT];
  double ev[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) exv[q] = 0;
  if (live) load_i32v<EPT>(eX + i0, exv);   // values of rows >= n are not used
#pragma unroll
  for (int q = 0; q < EPT; ++q) wq[q] = ldexp(wq[q], exv[q] + ej);
  double ms = 0.0, mr = 0.0;
  int tie = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = i0 + q;
    ev[q] = 0.0;
    if (i < n) {
      const int ei = exv[q];
      const double w = wq[q];
      double e;
      if (i == j) {
        e = 0.5 * r[j];
      } else {
        const double den = dd_diff(lj, ljl, *gview(lam + i), *gview(lam_lo + i));
        if (den == 0.0) {
          tie = 1;
          e = 0.0;
        } else {
          e = w / den;
        }
        if (cpl_count && fabs(e) > tau) {   // a strong coupling: list the pair (i, j)
          const int q = atomicAdd(cpl_count, 1);
          if (q < cpl_cap) {
            cpl_pairs[2 * q] = i;
            cpl_pairs[2 * q + 1] = j;
          }
        }
      }
      mr = fmax(mr, fabs(e));
      const double es = ldexp(e, ei);
      ev[q] = es;
      ms = fmax(ms, fabs(es));
    }
  }
  if (tie) atomicOr(flags, FLAG_TIE);
  ms = block_max<NT>(ms, scratch);
  mr = block_max<NT>(mr, scratch);
  write_col_planes<EPT, NT>(ev, ms, j, npad, Epl, ke);
  if (tid == 0) {
    eE[j] = exp_above(ms);
    emax[j] = mr;
    if (!(mr <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

// At most 64 VGPRs (8 waves per SIMD): two 1024-thread blocks share a CU, so one block's
// loads and barriers overlap the other's arithmetic.
template <int EPT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_epi_w(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag_all, const int *__restrict__ dcut,
    const int *__restrict__ eX, const int *__restrict__ eR, const double *__restrict__ lam,
    const double *__restrict__ lam_lo, const double *__restrict__ r, int n, int *eE,
    double *emax, int8_t *__restrict__ Epl, int ke, int *flags, double tau, int *cpl_count,
    int *cpl_pairs, int cpl_cap, const int *__restrict__ tcut) {
  epi_w_body<EPT, NT>(C, npad, d_min, ndiag_all, dcut, eX, eR, lam, lam_lo, r, n, eE, emax, Epl,
                      ke, flags, tau, cpl_count, cpl_pairs, cpl_cap, tcut, blockIdx.x);
}

template <int EPT, int NT>
static void epi_w_t(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                    const int *eX, const int *eR, const double *lam, const double *lam_lo, const double *r, int n,
                    int *eE, double *emax, int8_t *Epl, int ke, int *flags, double tau,
                    int *cpl_count, int *cpl_pairs, int cpl_cap, const int *tcut,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_epi_w<EPT, NT>), dim3(npad), dim3(NT), 0, s, C, npad, d_min, ndiag, dcut,
                     eX, eR, lam, lam_lo, r, n, eE, emax, Epl, ke, flags, tau, cpl_count, cpl_pairs,
                     cpl_cap, tcut);
}

void launch_epi_w(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                  const int *eX, const int *eR, const double *lam, const double *lam_lo, const double *r, int n, int *eE,
                  double *emax, int8_t *Epl, int ke, int *flags, hipStream_t s, double tau,
                  int *cpl_count, int *cpl_pairs, int cpl_cap, const int *tcut) {
#define EPI_W(E, T)                                                                          \
  epi_w_t<E, T>(C, npad, d_min, ndiag, dcut, eX, eR, lam, lam_lo, r, n, eE, emax, Epl, ke, flags, \
                tau, cpl_count, cpl_pairs, cpl_cap, tcut, s)
  EPI_DISPATCH(npad, EPI_W);
#undef EPI_W
}

// ---------------------------------------------------------------- grouped correction
// Entry w_ij of W = X^(1)T Res, summed from the slots exactly as the W epilogue sums it
// (smallest scale first, FP64), so both see the same value.
__device__ __forceinline__ double w_entry(const int32_t *__restrict__ C, size_t P, int npad,
                                          int d_min, int ndiag, int scale, int i, int j) {
  const int32_t *Ccol = C + (size_t)j * npad + i;
  double w = 0.0;
  for (int qq = ndiag - 1; qq >= 0; --qq)
    w += ldexp((double)Ccol[(size_t)qq * P], scale - 7 * (d_min + qq));
  return w;
}

// One block per listed pair (a, b): the double-word dot product x_a^T x_b of two columns
// of X^(1) and the entry w_ab.
__global__ __launch_bounds__(256) void k_group_gram(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag_all, const int *__restrict__ dcut,
    const int *__restrict__ eX, const int *__restrict__ eR, const double *__restrict__ X1, int n,
    const int *__restrict__ pa, const int *__restrict__ pb, double *gh, double *gl, double *wab,
    const int *__restrict__ tcut) {
  __shared__ double scratch[2 * 4];
  const int q = blockIdx.x, a = pa[q], b = pb[q];
  const double *xa = X1 + (size_t)a * n, *xb = X1 + (size_t)b * n;
  ddv acc = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += 256) {
    double p, pe;
    two_prod(xa[i], xb[i], p, pe);
    acc = dd_add_prod(acc, p, pe);
  }
  acc = block_dd_sum<256>(acc, scratch);
  if (threadIdx.x == 0) {
    gh[q] = acc.h;
    gl[q] = acc.l;
    const int nd = w_ndiag(dcut, tcut, npad >> 8, ndiag_all, d_min, a, b);
    wab[q] = w_entry(C, (size_t)npad * npad, npad, d_min, nd, eX[a] + eR[b], a, b);
  }
}

void launch_group_gram(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                       const int *eX, const int *eR, const double *X1, int n, const int *pa,
                       const int *pb, int npairs, double *gh, double *gl, double *wab,
                       hipStream_t s, const int *tcut) {
  hipLaunchKernelGGL(k_group_gram, dim3(npairs), dim3(256), 0, s, C, npad, d_min, ndiag, dcut, eX,
                     eR, X1, n, pa, pb, gh, gl, wab, tcut);
}

// One block per group member: its new correction column, from the group's Ritz vectors
// Y (row-major k x k at Y + base) and Ritz values mu (per member):
//   e_{c_a, c_pos} = Y[a][pos] - [a == pos]                       (rows in the group)
//   e_{i, c_pos} = (sum_a w_{i c_a} Y[a][pos]) / (mu - lambda_i)    (other rows)
// then, as in the W epilogue, E' = 2^(eX_i) e, its exponent, maximum and digit planes.
template <int EPT>
__global__ __launch_bounds__(kEpiThreads) void k_group_fix(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag_all, const int *__restrict__ dcut,
    const int *__restrict__ eX, const int *__restrict__ eR, const double *__restrict__ lam,
    const double *__restrict__ lam_lo, int n, const int *__restrict__ gcol,
    const int *__restrict__ gfirst, const int *__restrict__ gk, const int *__restrict__ gpos,
    const int *__restrict__ gbase, const double *__restrict__ Y, const double *__restrict__ mu,
    const double *__restrict__ mu_lo, int *eE, double *emax, int8_t *__restrict__ Epl, int ke,
    int *flags, const int *__restrict__ tcut) {
  __shared__ double scratch[2 * (kEpiThreads / 64)];
  __shared__ int smem[kGroupMax], snd[kGroupMax], ser[kGroupMax];
  __shared__ double sy[kGroupMax];
  const int m = blockIdx.x, tid = threadIdx.x;
  const int j = gcol[m], k = gk[m], pos = gpos[m], first = gfirst[m];
  const double muj = mu[m], mujl = mu_lo[m];
  if (tid < k) {
    const int c = gcol[first + tid];
    smem[tid] = c;
    snd[tid] = dcut ? min(ndiag_all, dcut[c] - d_min + 1) : ndiag_all;
    ser[tid] = eR[c];
    sy[tid] = Y[gbase[m] + tid * k + pos];
  }
  __syncthreads();
  const size_t P = (size_t)npad * npad;
  double ev[EPT];
  double ms = 0.0, mr = 0.0;
  int tie = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = erow<EPT>(tid, q);
    ev[q] = 0.0;
    if (i < n) {
      int in = -1;
      for (int a = 0; a < k; ++a)
        if (smem[a] == i) in = a;
      double e;
      if (in >= 0) {
        e = (in == pos) ? sy[in] - 1.0 : sy[in];
      } else {
        double num = 0.0;
        const int ei = eX[i];
        for (int a = 0; a < k; ++a) {
          const int nd = tcut ? w_ndiag(dcut, tcut, npad >> 8, ndiag_all, d_min, i, smem[a])
                              : snd[a];
          num += w_entry(C, P, npad, d_min, nd, ei + ser[a], i, smem[a]) * sy[a];
        }
        const double den = dd_diff(muj, mujl, lam[i], lam_lo[i]);
        if (den == 0.0) {
          tie = 1;
          e = 0.0;
        } else {
          e = num / den;
        }
      }
      mr = fmax(mr, fabs(e));
      const double es = ldexp(e, eX[i]);
      ev[q] = es;
      ms = fmax(ms, fabs(es));
    }
  }
  if (tie) atomicOr(flags, FLAG_TIE);
  ms = block_max<kEpiThreads>(ms, scratch);
  mr = block_max<kEpiThreads>(mr, scratch);
  write_col_planes<EPT>(ev, ms, j, npad, Epl, ke);
  if (tid == 0) {
    eE[j] = exp_above(ms);
    emax[j] = mr;
    if (!(mr <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

template <int EPT>
static void group_fix_t(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                        const int *eX, const int *eR, const double *lam, const double *lam_lo, int n, const int *gcol,
                        const int *gfirst, const int *gk, const int *gpos, const int *gbase,
                        const double *Y, const double *mu, const double *mu_lo, int nmem, int *eE, double *emax,
                        int8_t *Epl, int ke, int *flags, const int *tcut, hipStream_t s) {
  hipLaunchKernelGGL(k_group_fix<EPT>, dim3(nmem), dim3(kEpiThreads), 0, s, C, npad, d_min, ndiag,
                     dcut, eX, eR, lam, lam_lo, n, gcol, gfirst, gk, gpos, gbase, Y, mu, mu_lo, eE, emax, Epl, ke,
                     flags, tcut);
}

void launch_group_fix(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                      const int *eX, const int *eR, const double *lam, const double *lam_lo, int n, const int *gcol,
                      const int *gfirst, const int *gk, const int *gpos, const int *gbase,
                      const double *Y, const double *mu, const double *mu_lo, int nmem, int *eE, double *emax,
                      int8_t *Epl, int ke, int *flags, hipStream_t s, const int *tcut) {
  const int ept = (npad + kEpiThreads - 1) / kEpiThreads;
  if (ept <= 1) group_fix_t<1>(C, npad, d_min, ndiag, dcut, eX, eR, lam, lam_lo, n, gcol, gfirst, gk, gpos, gbase, Y, mu, mu_lo, nmem, eE, emax, Epl, ke, flags, tcut, s);
  else if (ept <= 2) group_fix_t<2>(C, npad, d_min, ndiag, dcut, eX, eR, lam, lam_lo, n, gcol, gfirst, gk, gpos, gbase, Y, mu, mu_lo, nmem, eE, emax, Epl, ke, flags, tcut, s);
  else if (ept <= 4) group_fix_t<4>(C, npad, d_min, ndiag, dcut, eX, eR, lam, lam_lo, n, gcol, gfirst, gk, gpos, gbase, Y, mu, mu_lo, nmem, eE, emax, Epl, ke, flags, tcut, s);
  else group_fix_t<8>(C, npad, d_min, ndiag, dcut, eX, eR, lam, lam_lo, n, gcol, gfirst, gk, gpos, gbase, Y, mu, mu_lo, nmem, eE, emax, Epl, ke, flags, tcut, s);
}

// ---------------------------------------------------------------- update X <- X1 + X1 E~
__device__ __forceinline__ void epi_u_body(const int32_t *__restrict__ C, int npad, int d_min,
                                               int ndiag_all, const int *__restrict__ dcut,
                                               const int *__restrict__ eE,
                                               const double *__restrict__ X1, int n,
                                               double *__restrict__ X, int ldx,
                                               const int *__restrict__ colmap,
                                               const int *__restrict__ errflags, int bx, int by) {
  const int i = bx * 256 + threadIdx.x, j = by;
  if (i >= n) return;
  if (errflags && (*errflags & kFlagsError)) return;
  const size_t P = (size_t)npad * npad;
  const int32_t *Ccol = C + (size_t)j * npad;
  const int ej = eE[j];
  const int ndiag = dcut ? min(ndiag_all, dcut[j] - d_min + 1) : ndiag_all;
  // the diagonals' values loaded 16 at a time, added smallest scale first
  double u = 0.0;
#pragma unroll 1
  for (int c0 = ndiag - 1; c0 >= 0; c0 -= 16) {
    int32_t cv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) cv[k] = c0 - k >= 0 ? Ccol[(size_t)(c0 - k) * P + i] : 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (c0 - k < 0) break;
      u += ldexp((double)cv[k], ej - 7 * (d_min + c0 - k));
    }
  }
  X[(size_t)(colmap ? colmap[j] : j) * ldx + i] = X1[(size_t)j * n + i] + u;
}

__global__ __launch_bounds__(256) void k_epi_u(const int32_t *__restrict__ C, int npad, int d_min,
                                               int ndiag_all, const int *__restrict__ dcut,
                                               const int *__restrict__ eE,
                                               const double *__restrict__ X1, int n,
                                               double *__restrict__ X, int ldx,
                                               const int *__restrict__ colmap,
                                               const int *__restrict__ errflags) {
  epi_u_body(C, npad, d_min, ndiag_all, dcut, eE, X1, n, X, ldx, colmap, errflags, blockIdx.x, blockIdx.y);
}

void launch_epi_u(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                  const int *eE, const double *X1, int n, double *X, int ldx, hipStream_t s,
                  const int *colmap, const int *errflags) {
  hipLaunchKernelGGL(k_epi_u, dim3((n + 255) / 256, n), dim3(256), 0, s, C, npad, d_min, ndiag, dcut,
                     eE, X1, n, X, ldx, colmap, errflags);
}

__device__ __forceinline__ void scatter_body(const double *__restrict__ v, const int *__restrict__ colmap, int n,
                          double *__restrict__ out, const int *__restrict__ errflags, int bx) {
  if (errflags && (*errflags & kFlagsError)) return;
  const int p = bx * 256 + threadIdx.x;
  if (p < n) out[colmap ? colmap[p] : p] = v[p];
}

__global__ void k_scatter(const double *__restrict__ v, const int *__restrict__ colmap, int n,
                          double *__restrict__ out, const int *__restrict__ errflags) {
  scatter_body(v, colmap, n, out, errflags, blockIdx.x);
}

void launch_scatter(const double *v, const int *colmap, int n, double *out, hipStream_t s,
                    const int *errflags) {
  hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, v, colmap, n, out,
                     errflags);
}


// ================================================================ complex Hermitian case
// Complex matrices are interleaved (real, imaginary) and column-major: element (i, j) at
// 2 (i + j ld). A complex operand row is "realified": its digit plane holds K = 2 npad
// entries, the real parts at k < npad and the imaginary parts at npad + k, so that one
// real slice GEMM of reduction length 2 npad forms the real (or imaginary) part of a
// complex product. Both parts of a column share one exponent (that of the larger part).

__global__ __launch_bounds__(256) void k_colstats_c(const double *__restrict__ M, int ld,
                                                    int rows, int cols, int *e, int *c,
                                                    double *mx, int *flags,
                                                    const int *__restrict__ colmap) {
  __shared__ double scratch[4];
  const int j = blockIdx.x;
  if (j >= cols) {
    if (threadIdx.x == 0) {
      e[j] = 0;
      c[j] = 0;
      if (mx) mx[j] = 0.0;
    }
    return;
  }
  const double2 *col = (const double2 *)(M + 2 * (size_t)(colmap ? colmap[j] : j) * ld);
  double m = 0.0;
  int bad = 0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    const double2 z = col[i];
    const double a = fabs(z.x), b = fabs(z.y);
    if (!(a <= DBL_MAX) || !(b <= DBL_MAX)) bad = 1;
    else m = fmax(m, fmax(a, b));
  }
  if (bad) atomicOr(flags, FLAG_NONFINITE);
  m = block_max<256>(m, scratch);
  if (threadIdx.x == 0) {
    int ee = exp_above(m);
    e[j] = ee;
    c[j] = ceil_log2(m);
    if (mx) mx[j] = m;
    if (m != 0.0 && (ee < -400 || ee > 400)) atomicOr(flags, FLAG_RANGE);
  }
}

void launch_colstats_c(const double *M, int ld, int rows, int cols, int cols_pad, int *e, int *c,
                       double *mx, int *flags, hipStream_t s, const int *colmap) {
  hipLaunchKernelGGL(k_colstats_c, dim3(cols_pad), dim3(256), 0, s, M, ld, rows, cols, e, c, mx,
                     flags, colmap);
}

// Digits 1..kk of a (sign-magnitude, base 128 below 2^ej) into dig; returns the value of
// the first k of them.
__device__ __forceinline__ double digits_of(double a, int ej, int kk, int k,
                                            int (&dig)[kMaxPlanesSplit]) {
  double y = ldexp(fabs(a), -ej);
  const int sg = (a < 0.0) ? -1 : 1;
  double val = 0.0;
#pragma unroll
  for (int t = 0; t < kMaxPlanesSplit; ++t) {
    dig[t] = 0;
    if (t < kk) {
      double t128 = y * 128.0;
      double d = floor(t128);
      y = t128 - d;
      dig[t] = sg * (int)d;
      if (t < k) val += ldexp(d, ej - 7 * (t + 1));
    }
  }
  return (a < 0.0) ? -val : val;
}

// Digit planes of a complex matrix M (rows x cols, ld) with column exponents e, 64 x 64
// tiles of the padded rpad x cpad area (zero digits outside):
//   planes (k planes, stride pstride): row j = column j realified,
//     (j, i) = digit of Re M_ij, (j, rpad + i) = digit of Im M_ij (K-blocked, cpad rows);
//   planes2 (optional): the realified column of i M: (j, i) = -Im M_ij, (j, rpad + i) = Re M_ij;
//   trunc (optional, complex, ld ldt): the value of the first k digits of both parts;
//   planesT (optional, kT planes): row i = row i of M with its imaginary parts negated,
//     (i, j) = Re M_ij, (i, cpad + j) = -Im M_ij (K-blocked, rpad rows).
// colmap (may be null): column j is read from column colmap[j] of M.
template <bool WITH_T>
__global__ __launch_bounds__(256) void k_split_c(const double *__restrict__ M, int ld, int rows,
                                                 int cols, const int *__restrict__ e, int k,
                                                 int8_t *__restrict__ planes,
                                                 int8_t *__restrict__ planes2, size_t pstride,
                                                 int rpad, int cpad, double *__restrict__ trunc,
                                                 int ldt, int8_t *__restrict__ planesT,
                                                 size_t pstrideT, int kT,
                                                 const int *__restrict__ colmap) {
  constexpr int TP = kMaxPlanesT * 64 * kTStride;   // one part's transpose tile
  __shared__ __attribute__((aligned(16))) int8_t sT[WITH_T ? 2 * TP : 16];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int ig = threadIdx.x & 15, jl = threadIdx.x >> 4;
  const int kk = (WITH_T && kT > k) ? kT : k;
  const double2 *Mz = (const double2 *)M;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const int jj = jl + 16 * q, j = j0 + jj;
    const int ej = (j < cols) ? e[j] : 0;
    const size_t mcol = (j < cols) ? (size_t)(colmap ? colmap[j] : j) * ld : 0;
    unsigned pr[kMaxPlanesSplit], pi[kMaxPlanesSplit], pn[kMaxPlanesSplit];
#pragma unroll
    for (int t = 0; t < kMaxPlanesSplit; ++t) pr[t] = pi[t] = pn[t] = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ii = 4 * ig + u, i = i0 + ii;
      double2 z = {0.0, 0.0};
      if (i < rows && j < cols) z = Mz[mcol + i];
      int dr[kMaxPlanesSplit], di[kMaxPlanesSplit];
      const double vr = digits_of(z.x, ej, kk, k, dr);
      const double vi = digits_of(z.y, ej, kk, k, di);
#pragma unroll
      for (int t = 0; t < kMaxPlanesSplit; ++t) {
        if (t < k) {
          pr[t] |= ((unsigned)(dr[t] & 0xff)) << (8 * u);
          pi[t] |= ((unsigned)(di[t] & 0xff)) << (8 * u);
          pn[t] |= ((unsigned)((-di[t]) & 0xff)) << (8 * u);
        }
        if (WITH_T && t < kT) {
          sT[(t * 64 + ii) * kTStride + jj] = (int8_t)dr[t];
          sT[TP + (t * 64 + ii) * kTStride + jj] = (int8_t)(-di[t]);
        }
      }
      if (trunc && i < rows && j < cols) {
        trunc[2 * ((size_t)j * ldt + i)] = vr;
        trunc[2 * ((size_t)j * ldt + i) + 1] = vi;
      }
    }
#pragma unroll
    for (int t = 0; t < kMaxPlanesSplit; ++t)
      if (t < k) {
        int8_t *pl = planes + (size_t)t * pstride;
        *(unsigned *)(pl + kb_off(j, i0 + 4 * ig, cpad)) = pr[t];
        *(unsigned *)(pl + kb_off(j, rpad + i0 + 4 * ig, cpad)) = pi[t];
        if (planes2) {
          int8_t *p2 = planes2 + (size_t)t * pstride;
          *(unsigned *)(p2 + kb_off(j, i0 + 4 * ig, cpad)) = pn[t];
          *(unsigned *)(p2 + kb_off(j, rpad + i0 + 4 * ig, cpad)) = pr[t];
        }
      }
  }
  if (WITH_T) {
    __syncthreads();
    const int ii = threadIdx.x >> 2, jq = (threadIdx.x & 3) * 16;
    for (int t = 0; t < kT; ++t) {
      int8_t *pt = planesT + (size_t)t * pstrideT;
      const v4i wr = *(const v4i *)(sT + (t * 64 + ii) * kTStride + jq);
      const v4i wn = *(const v4i *)(sT + TP + (t * 64 + ii) * kTStride + jq);
      *(v4i *)(pt + kb_off(i0 + ii, j0 + jq, rpad)) = wr;
      *(v4i *)(pt + kb_off(i0 + ii, cpad + j0 + jq, rpad)) = wn;
    }
  }
}

void launch_split_c(const double *M, int ld, int rows, int cols, const int *e, int k,
                    int8_t *planes, int8_t *planes2, size_t pstride, int rpad, int cpad,
                    double *trunc, int ldt, int8_t *planesT, size_t pstrideT, int kT,
                    hipStream_t s, const int *colmap) {
  dim3 grid(rpad / 64, cpad / 64);
  if (planesT && kT > 0)
    hipLaunchKernelGGL(k_split_c<true>, grid, dim3(256), 0, s, M, ld, rows, cols, e, k, planes,
                       planes2, pstride, rpad, cpad, trunc, ldt, planesT, pstrideT, kT, colmap);
  else
    hipLaunchKernelGGL(k_split_c<false>, grid, dim3(256), 0, s, M, ld, rows, cols, e, k, planes,
                       planes2, pstride, rpad, cpad, trunc, ldt, (int8_t *)nullptr, (size_t)0, 0,
                       colmap);
}

// Realified digit planes of one complex operand row j (an output column of a column
// epilogue) with exponent ee: planes gets (re; im), planes2 (im; -re), the realified
// column of -i v. Plane stride 2 npad^2; rows i >= n hold zero digits.
template <int EPT>
__device__ __forceinline__ void write_col_planes_c(const double (&re)[EPT], const double (&im)[EPT],
                                                   int ee, int j, int n, int npad,
                                                   int8_t *__restrict__ planes,
                                                   int8_t *__restrict__ planes2, int k) {
  const size_t P2 = 2 * (size_t)npad * npad;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = threadIdx.x + kEpiThreads * q;
    if (i < npad) {
      const double ar = (i < n) ? re[q] : 0.0, ai = (i < n) ? im[q] : 0.0;
      double yr = ldexp(fabs(ar), -ee), yi = ldexp(fabs(ai), -ee);
      const int sr = (ar < 0.0) ? -1 : 1, si = (ai < 0.0) ? -1 : 1;
      const size_t o1 = kb_off(j, i, npad), o2 = kb_off(j, npad + i, npad);
      for (int t = 0; t < k; ++t) {
        double t128 = yr * 128.0;
        double d = floor(t128);
        yr = t128 - d;
        const int dr = sr * (int)d;
        t128 = yi * 128.0;
        d = floor(t128);
        yi = t128 - d;
        const int di = si * (int)d;
        planes[t * P2 + o1] = (int8_t)dr;
        planes[t * P2 + o2] = (int8_t)di;
        planes2[t * P2 + o1] = (int8_t)di;
        planes2[t * P2 + o2] = (int8_t)(-dr);
      }
    }
  }
}

// V epilogue and column pass, complex: V = Vr + i Vi from the slots of the two products,
// r_j = 1 - x_j^H x_j, lambda_j = Re(x_j^H v_j) / (1 - r_j) (double-word), the residual
// V - x_j lambda_j of both parts (pair arithmetic), its exponent and maximum over both
// parts, and the realified planes of Res (Rpl) and of -i Res (Rpl2).
template <int EPT>
__global__ __launch_bounds__(kEpiThreads) void k_epi_v_c(
    const int32_t *__restrict__ Cr, const int32_t *__restrict__ Ci, int npad, int d_min,
    int ndiag_all, const int *__restrict__ dcut, const int *__restrict__ eA,
    const int *__restrict__ eX, const double *__restrict__ X1, int n, double *lam,
    double *lam_lo, double *r, int *eR, double *resmax, int8_t *__restrict__ Rpl,
    int8_t *__restrict__ Rpl2, int kr, int *flags) {
  __shared__ double scratch[4 * (kEpiThreads / 64)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const size_t P = (size_t)npad * npad;
  double rr[EPT], ri[EPT];
  if (j >= n) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) rr[q] = ri[q] = 0.0;
    write_col_planes_c<EPT>(rr, ri, 0, j, 0, npad, Rpl, Rpl2, kr);
    return;
  }
  const int ej = eX[j];
  const int ndiag = dcut ? min(ndiag_all, dcut[j] - d_min + 1) : ndiag_all;
  const size_t coff = (size_t)j * npad;
  const double2 *xcol = (const double2 *)X1 + (size_t)j * n;
  double vrh[EPT], vrl[EPT], vih[EPT], vil[EPT];
  int eiq[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    vrh[q] = vrl[q] = vih[q] = vil[q] = 0.0;
    eiq[q] = (i < n) ? eA[i] + ej : 0;
  }
#pragma unroll 1
  for (int qq = ndiag - 1; qq >= 0; --qq) {
    const int32_t *Cqr = Cr + coff + (size_t)qq * P, *Cqi = Ci + coff + (size_t)qq * P;
    int32_t cr[EPT], ci[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int i = tid + kEpiThreads * q;
      cr[q] = (i < n) ? Cqr[i] : 0;
      ci[q] = (i < n) ? Cqi[i] : 0;
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int sc = eiq[q] - 7 * (d_min + qq);
      double s_, e_;
      two_sum(vrh[q], ldexp((double)cr[q], sc), s_, e_);
      vrh[q] = s_;
      vrl[q] += e_;
      two_sum(vih[q], ldexp((double)ci[q], sc), s_, e_);
      vih[q] = s_;
      vil[q] += e_;
    }
  }
  ddv sx = {0.0, 0.0}, sv = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    if (i < n) {
      fast_two_sum(vrh[q], vrl[q], vrh[q], vrl[q]);
      fast_two_sum(vih[q], vil[q], vih[q], vil[q]);
      const double2 x = xcol[i];
      double p, pe;
      two_prod(x.x, x.x, p, pe);
      sx = dd_add_prod(sx, p, pe);
      two_prod(x.y, x.y, p, pe);
      sx = dd_add_prod(sx, p, pe);
      two_prod(x.x, vrh[q], p, pe);
      sv = dd_add_prod(sv, p, pe + x.x * vrl[q]);
      two_prod(x.y, vih[q], p, pe);
      sv = dd_add_prod(sv, p, pe + x.y * vil[q]);
    }
  }
  block_dd_sum2<kEpiThreads>(sx, sv, scratch);
  ddv rj = dd_add(ddv{1.0, 0.0}, ddv{-sx.h, -sx.l});
  ddv den = dd_add(ddv{1.0, 0.0}, ddv{-rj.h, -rj.l});
  const ddv ljd = dd_div_to_dd(sv, den);
  const double lj = ljd.h;
  double rmax = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    rr[q] = ri[q] = 0.0;
    if (i < n) {
      const double2 x = xcol[i];
      double p, pe, s_, e_;
      two_prod(x.x, lj, p, pe);
      two_sum(vrh[q], -p, s_, e_);
      rr[q] = s_ + (((e_ + vrl[q]) - pe) - x.x * ljd.l);
      two_prod(x.y, lj, p, pe);
      two_sum(vih[q], -p, s_, e_);
      ri[q] = s_ + (((e_ + vil[q]) - pe) - x.y * ljd.l);
      rmax = fmax(rmax, fmax(fabs(rr[q]), fabs(ri[q])));
    }
  }
  rmax = block_max<kEpiThreads>(rmax, scratch);
  const int er = exp_above(rmax);
  write_col_planes_c<EPT>(rr, ri, er, j, n, npad, Rpl, Rpl2, kr);
  if (tid == 0) {
    lam[j] = lj;
    lam_lo[j] = ljd.l;
    r[j] = rj.h;
    eR[j] = er;
    resmax[j] = rmax;
    if (!(fabs(lj) <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

void launch_epi_v_c(const int32_t *Cr, const int32_t *Ci, int npad, int d_min, int ndiag,
                    const int *dcut, const int *eA, const int *eX, const double *X1, int n,
                    double *lam, double *lam_lo, double *r, int *eR, double *resmax,
                    int8_t *Rpl, int8_t *Rpl2, int kr, int *flags, hipStream_t s) {
  const int ept = (npad + kEpiThreads - 1) / kEpiThreads;
#define EPI_V_C(E)                                                                          \
  hipLaunchKernelGGL(k_epi_v_c<E>, dim3(npad), dim3(kEpiThreads), 0, s, Cr, Ci, npad, d_min,  \
                     ndiag, dcut, eA, eX, X1, n, lam, lam_lo, r, eR, resmax, Rpl, Rpl2, kr,   \
                     flags)
  if (ept <= 1) EPI_V_C(1);
  else if (ept <= 2) EPI_V_C(2);
  else EPI_V_C(4);
#undef EPI_V_C
}

// W epilogue, complex: W = Wr + i Wi, e_ij = w_ij / (lambda_j - lambda_i) (both parts, the
// difference of the double-word eigenvalues), e_jj = r_j / 2, E'_ij = 2^eX_i e_ij; emax_j =
// max_i |e_ij| (modulus), eE_j the exponent of the larger part of column j of E', and the
// realified planes of E' (Epl) and of -i E' (Epl2).
template <int EPT>
__global__ __launch_bounds__(kEpiThreads) void k_epi_w_c(
    const int32_t *__restrict__ Cr, const int32_t *__restrict__ Ci, int npad, int d_min,
    int ndiag_all, const int *__restrict__ dcut, const int *__restrict__ eX,
    const int *__restrict__ eR, const double *__restrict__ lam,
    const double *__restrict__ lam_lo, const double *__restrict__ r, int n, int *eE,
    double *emax, int8_t *__restrict__ Epl, int8_t *__restrict__ Epl2, int ke, int *flags) {
  __shared__ double scratch[2 * (kEpiThreads / 64)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const size_t P = (size_t)npad * npad;
  double er_[EPT], ei_[EPT];
  if (j >= n) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) er_[q] = ei_[q] = 0.0;
    write_col_planes_c<EPT>(er_, ei_, 0, j, 0, npad, Epl, Epl2, ke);
    return;
  }
  const int ej = eR[j];
  const double lj = lam[j], ljl = lam_lo[j];
  const int ndiag = dcut ? min(ndiag_all, dcut[j] - d_min + 1) : ndiag_all;
  const size_t coff = (size_t)j * npad;
  double wr[EPT], wi[EPT];
  int eiq[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    wr[q] = wi[q] = 0.0;
    eiq[q] = (i < n) ? eX[i] + ej : 0;
  }
#pragma unroll 1
  for (int qq = ndiag - 1; qq >= 0; --qq) {
    const int32_t *Cqr = Cr + coff + (size_t)qq * P, *Cqi = Ci + coff + (size_t)qq * P;
    int32_t cr[EPT], ci[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int i = tid + kEpiThreads * q;
      cr[q] = (i < n) ? Cqr[i] : 0;
      ci[q] = (i < n) ? Cqi[i] : 0;
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int sc = eiq[q] - 7 * (d_min + qq);
      wr[q] += ldexp((double)cr[q], sc);
      wi[q] += ldexp((double)ci[q], sc);
    }
  }
  double ms = 0.0, mr = 0.0;
  int tie = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    er_[q] = ei_[q] = 0.0;
    if (i < n) {
      double a, b;
      if (i == j) {
        a = 0.5 * r[j];
        b = 0.0;
      } else {
        const double den = dd_diff(lj, ljl, lam[i], lam_lo[i]);
        if (den == 0.0) {
          tie = 1;
          a = b = 0.0;
        } else {
          a = wr[q] / den;
          b = wi[q] / den;
        }
      }
      mr = fmax(mr, sqrt(a * a + b * b));
      er_[q] = ldexp(a, eX[i]);
      ei_[q] = ldexp(b, eX[i]);
      ms = fmax(ms, fmax(fabs(er_[q]), fabs(ei_[q])));
    }
  }
  if (tie) atomicOr(flags, FLAG_TIE);
  ms = block_max<kEpiThreads>(ms, scratch);
  mr = block_max<kEpiThreads>(mr, scratch);
  const int ee = exp_above(ms);
  write_col_planes_c<EPT>(er_, ei_, ee, j, n, npad, Epl, Epl2, ke);
  if (tid == 0) {
    eE[j] = ee;
    emax[j] = mr;
    if (!(mr <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

void launch_epi_w_c(const int32_t *Cr, const int32_t *Ci, int npad, int d_min, int ndiag,
                    const int *dcut, const int *eX, const int *eR, const double *lam,
                    const double *lam_lo, const double *r, int n, int *eE, double *emax,
                    int8_t *Epl, int8_t *Epl2, int ke, int *flags, hipStream_t s) {
  const int ept = (npad + kEpiThreads - 1) / kEpiThreads;
#define EPI_W_C(E)                                                                          \
  hipLaunchKernelGGL(k_epi_w_c<E>, dim3(npad), dim3(kEpiThreads), 0, s, Cr, Ci, npad, d_min,  \
                     ndiag, dcut, eX, eR, lam, lam_lo, r, n, eE, emax, Epl, Epl2, ke, flags)
  if (ept <= 1) EPI_W_C(1);
  else if (ept <= 2) EPI_W_C(2);
  else EPI_W_C(4);
#undef EPI_W_C
}

// Update, complex: X_ij = X1_ij + U_ij for both parts, U from the slots of the two products
// scaled by 2^(eE_j - 7d); column j goes to column colmap[j] of X (colmap may be null).
__global__ __launch_bounds__(256) void k_epi_u_c(const int32_t *__restrict__ Cr,
                                                 const int32_t *__restrict__ Ci, int npad,
                                                 int d_min, int ndiag_all,
                                                 const int *__restrict__ dcut,
                                                 const int *__restrict__ eE,
                                                 const double *__restrict__ X1, int n,
                                                 double *__restrict__ X, int ldx,
                                                 const int *__restrict__ colmap) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const size_t P = (size_t)npad * npad;
  const size_t coff = (size_t)j * npad + i;
  const int ej = eE[j];
  const int ndiag = dcut ? min(ndiag_all, dcut[j] - d_min + 1) : ndiag_all;
  double ur = 0.0, ui = 0.0;
  for (int qq = ndiag - 1; qq >= 0; --qq) {
    const int sc = ej - 7 * (d_min + qq);
    ur += ldexp((double)Cr[coff + (size_t)qq * P], sc);
    ui += ldexp((double)Ci[coff + (size_t)qq * P], sc);
  }
  const double2 x1 = ((const double2 *)X1)[(size_t)j * n + i];
  double2 out;
  out.x = x1.x + ur;
  out.y = x1.y + ui;
  ((double2 *)X)[(size_t)(colmap ? colmap[j] : j) * ldx + i] = out;
}

void launch_epi_u_c(const int32_t *Cr, const int32_t *Ci, int npad, int d_min, int ndiag,
                    const int *dcut, const int *eE, const double *X1, int n, double *X, int ldx,
                    hipStream_t s, const int *colmap) {
  hipLaunchKernelGGL(k_epi_u_c, dim3((n + 255) / 256, n), dim3(256), 0, s, Cr, Ci, npad, d_min,
                     ndiag, dcut, eE, X1, n, X, ldx, colmap);
}

// ================================================================ grouped batches
// A batch of independent solves runs as one launch per step and size class (problems of equal
// npad, consecutive in gp): block b of such a launch serves problem first + b / bpp with the
// local block index b % bpp, as the single-problem launch would. The products run as
// persistent kernels over a work list of (problem, tile, slot) items built on the device from
// each problem's plan. A problem whose solve has stopped (DevState::skip) does nothing.

__global__ __launch_bounds__(256) void k_colstats_g(const GProb *__restrict__ gp, int first,
                                                    int bpp, int of_x) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  const int j = blockIdx.x % bpp;
  if (!of_x) {
    colstats_body(q.A, q.lda, q.n, q.n, q.w.eA, q.w.cA, q.w.mxA, q.w.flags, nullptr, q.w.ssA, j);
  } else {
    if (q.pb.st->skip) return;
    colstats_body(q.X, q.ldx, q.n, q.n, q.w.eX, q.w.cX, q.w.mxX, q.w.flags, q.w.colmap, q.w.ssX,
                  j);
  }
}

// WITH_T false: the planes of A (once per solve); true: X^(1), its planes in both layouts.
template <bool WITH_T>
__global__ __launch_bounds__(256) void k_split_g(const GProb *__restrict__ gp, int first, int gx) {
  const int bpp = gx * gx;
  const GProb &q = gp[first + blockIdx.x / bpp];
  const int lb = blockIdx.x % bpp, bx = lb % gx, by = lb / gx;
  if constexpr (!WITH_T) {
    split_cols_body<false>(q.A, q.lda, q.n, q.n, q.w.eA, q.ka, q.w.AP, q.P, q.npad, q.npad,
                           nullptr, 0, nullptr, 0, 0, nullptr, nullptr, bx, by);
  } else {
    if (q.pb.st->skip) return;
    split_cols_body<true>(q.X, q.ldx, q.n, q.n, q.w.eX, kKxMax, q.w.XP, q.P, q.npad, q.npad,
                          q.w.X1, q.n, q.w.XPT, q.P, kKxMax, q.w.colmap, &q.pb.st->kx, bx, by);
  }
}

template <int EPT, bool CRT, int NT>
__global__ __launch_bounds__(NT) void k_epi_v_g(const GProb *__restrict__ gp, int first,
                                                         int bpp) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  const int j = blockIdx.x % bpp;
  DevState *st = q.pb.st;
  if (st->skip) return;
  if constexpr (CRT)
    epi_v_body<EPT, true, NT>(q.w.Cs, q.npad, 2, 1, nullptr, q.w.eA, q.w.eX, q.w.X1, q.n, q.w.lam,
                          q.w.lam_lo, q.w.r, q.w.eR, q.w.resmax, q.w.RP, kKrMax, q.w.flags,
                          st->recs, q.w.vblk, &st->vres, j);
  else
    epi_v_body<EPT, false, NT>(q.w.Cs, q.npad, 2, kMaxDiag - 1, q.w.dcut[0], q.w.eA, q.w.eX, q.w.X1,
                           q.n, q.w.lam, q.w.lam_lo, q.w.r, q.w.eR, q.w.resmax, q.w.RP, kKrMax,
                           q.w.flags, nullptr, nullptr, &st->vslice, j);
}

__global__ __launch_bounds__(256) void k_tile_cutoffs_g(const GProb *__restrict__ gp, int first,
                                                        int bpp) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  DevState *st = q.pb.st;
  if (st->skip) return;
  tile_cutoffs_body(q.w.lam, q.w.eX, q.w.eR, q.w.resmax, q.n, q.npad / 256, 0.0, 2, q.pp.d_extra,
                    q.w.wtol, q.w.wtol + q.npad, q.w.tcut, &st->cx, &st->dmax_w,
                    blockIdx.x % bpp);
}

template <int EPT, int NT>
__global__ __launch_bounds__(NT) void k_epi_w_g(const GProb *__restrict__ gp, int first,
                                                         int bpp) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  if (q.pb.st->skip) return;
  epi_w_body<EPT, NT>(q.w.Cs, q.npad, 2, kMaxDiag - 1, q.w.dcut[1], q.w.eX, q.w.eR, q.w.lam,
                  q.w.lam_lo, q.w.r, q.n, q.w.eE, q.w.emax, q.w.EP, kKeMax, q.w.flags, 0.0,
                  nullptr, nullptr, 0, q.npad >= 1024 ? q.w.tcut : nullptr, blockIdx.x % bpp);
}

__global__ __launch_bounds__(256) void k_epi_u_g(const GProb *__restrict__ gp, int first,
                                                 int gx, int bpp) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  const int lb = blockIdx.x % bpp, bx = lb % gx, by = lb / gx;
  if (by >= q.n || q.pb.st->skip) return;
  epi_u_body(q.w.Cs, q.npad, 2, kMaxDiag - 1, q.w.dcut[2], q.w.eE, q.w.X1, q.n, q.X, q.ldx,
             q.w.colmap, q.w.flags, bx, by);
}

__global__ __launch_bounds__(256) void k_scatter_g(const GProb *__restrict__ gp, int first,
                                                   int bpp) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  if (q.pb.st->skip) return;
  scatter_body(q.w.lam, q.w.colmap, q.n, q.D, q.w.flags, blockIdx.x % bpp);
}

// Work items of one product over the problems gp[first .. first + count) (tile rows `tile`
// each): item = {problem, row tile | column tile << 8 | slot << 16}. which: 0 V by residues
// (the slots below each 256-row block's modulus count, when V goes by residues), 1 V by slices,
// 2 W, 3 X^(1) E~ (each problem's block table). One block; also resets the item counter.
// A problem planned on 256-row tiles (npad >= 1024) and run on the 128-row tile splits each
// block-table entry into its four 128-row quarters (split = 4); the slot values do not depend on
// the tile, so the choice never changes a result.
__device__ __forceinline__ int tab_split(const GProb &q, int tile) {
  const int tr = q.npad >= 1024 ? 256 : 128;
  return (tr / tile) * (tr / tile);
}
__device__ __forceinline__ int items_of(const GProb &q, int which, int tile) {
  const DevState &st = *q.pb.st;
  if (st.skip) return 0;
  if (which == 0) {
    if (!st.vres) return 0;
    const int TT = q.npad / tile;
    int c = 0;
    for (int mi = 0; mi < TT; ++mi) c += q.w.vblk[2 * ((mi * tile) >> 8)];
    return c * TT;
  }
  return (which == 1 ? st.gemm_v : which == 2 ? st.gemm_w : st.gemm_u)[2] * tab_split(q, tile);
}

__global__ __launch_bounds__(1024) void k_worklist_g(const GProb *__restrict__ gp, int first,
                                                     int count, int which, int tile,
                                                     int2 *__restrict__ items,
                                                     int *__restrict__ total,
                                                     int *__restrict__ ctr) {
  __shared__ int off[1025];
  __shared__ int wsum[16];
  int base_off = 0;
  for (int base = 0; base < count; base += 1024) {
    const int k = base + (int)threadIdx.x;
    const int c = k < count ? items_of(gp[first + k], which, tile) : 0;
    // block-wide exclusive scan of c
    int v = c;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(v, o);
      if (lane >= o) v += t;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < wv; ++q) before += wsum[q];
    off[threadIdx.x] = base_off + before + v - c;
    if (threadIdx.x == 1023) off[1024] = base_off + before + v;
    __syncthreads();
    const int chunk = min(1024, count - base);
    for (int kk = wv; kk < chunk; kk += 16) {   // one problem per wavefront at a time
      const GProb &q = gp[first + base + kk];
      const int o0 = off[kk], cnt = off[kk + 1] - o0;
      const int g = first + base + kk;
      if (which == 0) {
        const int TT = q.npad / tile;
        for (int e = lane; e < cnt; e += 64) {
          const int ni = e % TT;
          int r = e / TT, mi = 0;
          for (; mi < TT; ++mi) {
            const int cm = q.w.vblk[2 * ((mi * tile) >> 8)];
            if (r < cm) break;
            r -= cm;
          }
          items[o0 + e] = make_int2(g, mi | (ni << 8) | (r << 16));
        }
      } else {
        const int *tab = q.w.tab[which - 1];
        if (tab_split(q, tile) == 1) {
          for (int e = lane; e < cnt; e += 64) items[o0 + e] = make_int2(g, tab[e]);
        } else {
          for (int e = lane; e < cnt; e += 64) {
            const int ent = tab[e >> 2], sub = e & 3;
            const int r = 2 * (ent & 0xff) + (sub & 1), c = 2 * ((ent >> 8) & 0xff) + (sub >> 1);
            items[o0 + e] = make_int2(g, r | (c << 8) | ((ent >> 16) << 16));
          }
        }
      }
    }
    base_off = off[1024];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *total = base_off;
    *ctr = 0;
  }
}

// The products of a grouped batch: persistent blocks take items from the list in order (one
// atomic counter) until it is exhausted.
template <int TILE, int WHICH>
__global__ __launch_bounds__(256, TILE == 256 ? 1 : 3) void k_gemm_g(
    const GProb *__restrict__ gp, const int2 *__restrict__ items, const int *__restrict__ total,
    int *__restrict__ ctr) {
  __shared__ int s_w;
  const int tot = *total;
  for (;;) {
    if (threadIdx.x == 0) s_w = atomicAdd(ctr, 1);
    __syncthreads();
    // uniform values (scalar registers), so the item's loop control stays scalar
    const int w = __builtin_amdgcn_readfirstlane(s_w);
    __syncthreads();   // every wave has read s_w and left the previous item's LDS
    if (w >= tot) return;
    const int2 it = items[w];
    const GProb &q = gp[__builtin_amdgcn_readfirstlane(it.x)];
    const DevState &st = *q.pb.st;
    const int ent = __builtin_amdgcn_readfirstlane(it.y);
    const int m0 = (ent & 0xff) * TILE, n0 = ((ent >> 8) & 0xff) * TILE, slot = ent >> 16;
    const int8_t *Lp, *Rp;
    int kl, kr, same = 0;
    const int *mods = nullptr, *vblk = nullptr, *tcut = nullptr;
    if constexpr (WHICH == 0) {
      Lp = q.w.XRES;
      Rp = q.w.ARES;
      kl = kr = kCrtMax;
      same = 1;
      mods = q.w.mods;
      vblk = q.w.vblk;
    } else if constexpr (WHICH == 1) {
      Lp = q.w.XP;
      Rp = q.w.AP;
      kl = st.gemm_v[0];
      kr = st.gemm_v[1];
    } else if constexpr (WHICH == 2) {
      Lp = q.w.RP;
      Rp = q.w.XP;
      kl = st.gemm_w[0];
      kr = st.gemm_w[1];
      if (q.npad >= 1024) tcut = q.w.tcut;
    } else {
      Lp = q.w.EP;
      Rp = q.w.XPT;
      kl = st.gemm_u[0];
      kr = st.gemm_u[1];
    }
    if constexpr (TILE == 256) {
      gemm256_item<false>(Lp, Rp, q.P, q.npad, q.npad, kl, kr, 2, q.w.Cs, same, tcut, mods, vblk,
                          m0, n0, slot);
    } else {
      // a quarter of a 256-row tile obeys that tile's W cutoff
      if (tcut && 2 + slot > tcut[(m0 >> 8) * (q.npad >> 8) + (n0 >> 8)]) continue;
      gemm128_item(Lp, Rp, q.P, q.npad, q.npad, kl, kr, 2, q.w.Cs, same, mods, vblk, m0, n0,
                   slot);
    }
  }
}

__global__ void k_fill_hash_i8(int8_t *__restrict__ p, size_t n, unsigned seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)i * 2654435761u ^ seed;   // multiplicative hash, then xorshift mixing
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = (int8_t)((int)(h % 255u) - 127);
  }
}
void launch_fill_hash_i8(int8_t *p, size_t n, unsigned seed, hipStream_t s) {
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fill_hash_i8, dim3((unsigned)blocks), dim3(256), 0, s, p, n, seed);
}

void launch_colstats_g(const GProb *gp, int first, int count, int npad, bool of_x, hipStream_t s) {
  hipLaunchKernelGGL(k_colstats_g, dim3(count * npad), dim3(256), 0, s, gp, first, npad,
                     of_x ? 1 : 0);
}
void launch_split_g(const GProb *gp, int first, int count, int npad, bool of_x, hipStream_t s) {
  const int gx = npad / 64;
  if (of_x)
    hipLaunchKernelGGL(k_split_g<true>, dim3(count * gx * gx), dim3(256), 0, s, gp, first, gx);
  else
    hipLaunchKernelGGL(k_split_g<false>, dim3(count * gx * gx), dim3(256), 0, s, gp, first, gx);
}
void launch_epi_v_g(const GProb *gp, int first, int count, int npad, bool crt, hipStream_t s) {
  const dim3 grid(count * npad);
#define EPI_V_G(E, T)                                                                            \
  do {                                                                                           \
    if (crt) hipLaunchKernelGGL((k_epi_v_g<E, true, T>), grid, dim3(T), 0, s, gp, first, npad);  \
    else hipLaunchKernelGGL((k_epi_v_g<E, false, T>), grid, dim3(T), 0, s, gp, first, npad);     \
  } while (0)
  // grouped batches hold npad <= kGroupMaxNpad (4 entries per thread at most)
  EPI_DISPATCH_G(npad, EPI_V_G);
#undef EPI_V_G
}
void launch_tile_cutoffs_g(const GProb *gp, int first, int count, int npad, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_cutoffs_g, dim3(count * (npad / 256)), dim3(256), 0, s, gp, first,
                     npad / 256);
}
void launch_epi_w_g(const GProb *gp, int first, int count, int npad, hipStream_t s) {
  const dim3 grid(count * npad);
#define EPI_W_G(E, T) hipLaunchKernelGGL((k_epi_w_g<E, T>), grid, dim3(T), 0, s, gp, first, npad)
  EPI_DISPATCH_G(npad, EPI_W_G);
#undef EPI_W_G
}
void launch_epi_u_g(const GProb *gp, int first, int count, int npad, hipStream_t s) {
  const int gx = npad / 256;
  hipLaunchKernelGGL(k_epi_u_g, dim3(count * gx * npad), dim3(256), 0, s, gp, first, gx,
                     gx * npad);
}
void launch_scatter_g(const GProb *gp, int first, int count, int npad, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_g, dim3(count * (npad / 256)), dim3(256), 0, s, gp, first,
                     npad / 256);
}
void launch_worklist_g(const GProb *gp, int first, int count, int which, int tile, int2 *items,
                       int *total, int *ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_worklist_g, dim3(1), dim3(1024), 0, s, gp, first, count, which, tile,
                     items, total, ctr);
}
template <int TILE>
static void gemm_g_t(const GProb *gp, int blocks, const int2 *items, const int *total, int *ctr,
                     int which, hipStream_t s) {
  const dim3 g(blocks), b(256);
  switch (which) {
    case 0: hipLaunchKernelGGL((k_gemm_g<TILE, 0>), g, b, 0, s, gp, items, total, ctr); break;
    case 1: hipLaunchKernelGGL((k_gemm_g<TILE, 1>), g, b, 0, s, gp, items, total, ctr); break;
    case 2: hipLaunchKernelGGL((k_gemm_g<TILE, 2>), g, b, 0, s, gp, items, total, ctr); break;
    default: hipLaunchKernelGGL((k_gemm_g<TILE, 3>), g, b, 0, s, gp, items, total, ctr); break;
  }
}
void launch_gemm_g(const GProb *gp, int tile, int blocks, const int2 *items, const int *total,
                   int *ctr, int which, hipStream_t s) {
  if (blocks <= 0) return;
  if (tile == 256) gemm_g_t<256>(gp, blocks, items, total, ctr, which, s);
  else gemm_g_t<128>(gp, blocks, items, total, ctr, which, s);
}

}  // namespace refeig
