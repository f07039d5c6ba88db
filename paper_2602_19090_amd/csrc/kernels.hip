// gfx950 (MI355X) kernels for Ozaki-scheme eigenvector refinement.
//
// Data layout (npad = n rounded up to 256, P = npad * npad):
//   digit planes   int8, plane-major; in plane t, element (row m, k) at m*npad + k
//                  so every GEMM operand row is K-contiguous (the "TN" form).
//   slot C_d       int32 n x n per pair diagonal d, element (i, j) at j*npad + i,
//                  i.e. column-major, so the column epilogues read columns
//                  contiguously.
//
// Every floating-point expression in this file is compiled with
// -ffp-contract=off: the error-free transformations (TwoSum, the exact product
// via fma) must not be contracted or reassociated.
#include "kernels.h"

#include <float.h>

namespace refeig {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

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
  double m = scratch[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) m = fmax(m, scratch[q]);
  return m;
}
// Block-wide double-word sum in a fixed order (deterministic).
template <int NT>
__device__ __forceinline__ ddv block_dd_sum(ddv v, double *scratch) {
  v = wave_dd_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    scratch[2 * w] = v.h;
    scratch[2 * w + 1] = v.l;
  }
  __syncthreads();
  ddv s = {scratch[0], scratch[1]};
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) s = dd_add(s, ddv{scratch[2 * q], scratch[2 * q + 1]});
  return s;
}

// ---------------------------------------------------------------- column statistics
__global__ __launch_bounds__(256) void k_colstats(const double *__restrict__ M, int ld, int rows,
                                                  int cols, int *e, int *c, double *mx,
                                                  int *flags) {
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
  const double *col = M + (size_t)j * ld;
  double m = 0.0;
  int bad = 0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    double a = fabs(col[i]);
    if (!(a <= DBL_MAX)) bad = 1;
    else m = fmax(m, a);
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

void launch_colstats(const double *M, int ld, int rows, int cols, int cols_pad, int *e, int *c,
                     double *mx, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_colstats, dim3(cols_pad), dim3(256), 0, s, M, ld, rows, cols, e, c, mx,
                     flags);
}

// ---------------------------------------------------------------- digit planes
constexpr int kMaxPlanesSplit = 18;
constexpr int kMaxPlanesT = 9;
constexpr int kTStride = 80;  // LDS row stride of the transpose tile (16-byte aligned)

template <bool WITH_T>
__global__ __launch_bounds__(256) void k_split_cols(const double *__restrict__ M, int ld, int rows,
                                                    int cols, const int *__restrict__ e, int k,
                                                    int8_t *__restrict__ planes, size_t pstride,
                                                    int rpad, int cpad, double *__restrict__ trunc,
                                                    int ldt, int8_t *__restrict__ planesT,
                                                    size_t pstrideT, int kT) {
  __shared__ __attribute__((aligned(16))) int8_t sT[WITH_T ? kMaxPlanesT * 64 * kTStride : 16];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int ig = threadIdx.x & 15, jl = threadIdx.x >> 4;
  const int kk = (WITH_T && kT > k) ? kT : k;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const int jj = jl + 16 * q, j = j0 + jj;
    const int ej = (j < cols) ? e[j] : 0;
    unsigned packed[kMaxPlanesSplit];
#pragma unroll
    for (int t = 0; t < kMaxPlanesSplit; ++t) packed[t] = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ii = 4 * ig + u, i = i0 + ii;
      const double a = (i < rows && j < cols) ? M[(size_t)j * ld + i] : 0.0;
      double y = ldexp(fabs(a), -ej);
      const int sg = (a < 0.0) ? -1 : 1;
      double val = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxPlanesSplit; ++t) {
        if (t < kk) {
          double t128 = y * 128.0;
          double d = floor(t128);
          y = t128 - d;
          int dig = sg * (int)d;
          if (t < k) {
            packed[t] |= ((unsigned)(dig & 0xff)) << (8 * u);
            val += ldexp(d, ej - 7 * (t + 1));
          }
          if (WITH_T && t < kT) sT[(t * 64 + ii) * kTStride + jj] = (int8_t)dig;
        }
      }
      if (trunc && i < rows && j < cols) trunc[(size_t)j * ldt + i] = (a < 0.0) ? -val : val;
    }
#pragma unroll
    for (int t = 0; t < kMaxPlanesSplit; ++t)
      if (t < k)
        *(unsigned *)(planes + (size_t)t * pstride + (size_t)j * rpad + i0 + 4 * ig) = packed[t];
  }
  if (WITH_T) {
    __syncthreads();
    const int ii = threadIdx.x >> 2, jq = (threadIdx.x & 3) * 16;
    for (int t = 0; t < kT; ++t) {
      v4i w = *(const v4i *)(sT + (t * 64 + ii) * kTStride + jq);
      *(v4i *)(planesT + (size_t)t * pstrideT + (size_t)(i0 + ii) * cpad + j0 + jq) = w;
    }
  }
}

void launch_split_cols(const double *M, int ld, int rows, int cols, const int *e, int k,
                       int8_t *planes, size_t pstride, int rpad, int cpad, double *trunc, int ldt,
                       int8_t *planesT, size_t pstrideT, int kT, hipStream_t s) {
  dim3 grid(rpad / 64, cpad / 64);
  if (planesT && kT > 0)
    hipLaunchKernelGGL(k_split_cols<true>, grid, dim3(256), 0, s, M, ld, rows, cols, e, k, planes,
                       pstride, rpad, cpad, trunc, ldt, planesT, pstrideT, kT);
  else
    hipLaunchKernelGGL(k_split_cols<false>, grid, dim3(256), 0, s, M, ld, rows, cols, e, k, planes,
                       pstride, rpad, cpad, trunc, ldt, (int8_t *)nullptr, (size_t)0, 0);
}

// ---------------------------------------------------------------- INT8 slice GEMM
// One block computes one 128 x 128 tile of one diagonal slot:
//   C_d[m][p] = sum over pairs (s, d - s) of sum_k L_s[m][k] R_{d-s}[p][k].
// 4 waves in a 2 x 2 arrangement, each 64 x 64 = 2 x 2 MFMA 32x32x32 blocks.
// K advances 128 bytes per LDS stage; the next stage is prefetched into
// registers while the current one feeds the matrix cores.
constexpr int GBM = 128, GBN = 128, GBK = 128, GLDS = GBK + 16;

__global__ __launch_bounds__(256, 2) void k_slice_gemm(const int8_t *__restrict__ Lp,
                                                       const int8_t *__restrict__ Rp,
                                                       size_t pstride, int npad, int kl, int kr,
                                                       int d_min, DiagOrder order,
                                                       int32_t *__restrict__ C) {
  __shared__ __attribute__((aligned(16))) int8_t sL[GBM * GLDS];
  __shared__ __attribute__((aligned(16))) int8_t sR[GBN * GLDS];
  const int tiles_n = npad / GBN;
  const int m0 = (blockIdx.x / tiles_n) * GBM;
  const int n0 = (blockIdx.x % tiles_n) * GBN;
  const int slot = order.q[blockIdx.y];
  const int d = d_min + slot;
  const int s_lo = max(1, d - kr), s_hi = min(kl, d - 1);
  const int npairs = s_hi - s_lo + 1;
  const int KT = npad / GBK;
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
  auto load = [&](int t) {
    const int p = t / KT, k0 = (t - p * KT) * GBK;
    const int s = s_lo + p;
    const int8_t *Lb = Lp + (size_t)(s - 1) * pstride + (size_t)m0 * npad + k0;
    const int8_t *Rb = Rp + (size_t)(d - s - 1) * pstride + (size_t)n0 * npad + k0;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = tid + 256 * h, row = c >> 3, col = (c & 7) * 16;
      gL[h] = *(const v4i *)(Lb + (size_t)row * npad + col);
      gR[h] = *(const v4i *)(Rb + (size_t)row * npad + col);
    }
  };
  if (npairs > 0) load(0);
  for (int t = 0; t < T; ++t) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = tid + 256 * h, row = c >> 3, col = (c & 7) * 16;
      *(v4i *)(sL + row * GLDS + col) = gL[h];
      *(v4i *)(sR + row * GLDS + col) = gR[h];
    }
    __syncthreads();
    if (t + 1 < T) load(t + 1);
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
  int32_t *Cq = C + (size_t)slot * npad * npad;
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

// Large-tile variant: one block computes a 256 x 256 tile with 4 waves, each
// owning 128 x 128 (4 x 4 MFMA 32x32x32 blocks, 256 accumulator registers held
// in the AGPR half of the register file). Each fragment read from LDS feeds 4
// MFMAs. K advances 128 bytes per stage through two LDS buffers (147 KB of the
// 160 KB): while the matrix cores consume stage t, stage t+1 goes from
// registers into the other buffer and the global loads of stage t+2 are in
// flight, with one barrier per stage.
// Tile order: the blocks of one XCD (block id mod 8) get a contiguous range of
// tiles, walked in groups of 4 tile-rows, so the ~32 blocks an XCD runs at once
// cover a 4 x 8 patch and share its L and R panels in that XCD's L2.
constexpr int HBM_ = 256, HBK = 128, HLDS = HBK + 16, HGM = 4;

__global__ __launch_bounds__(256, 1) void k_slice_gemm256(const int8_t *__restrict__ Lp,
                                                          const int8_t *__restrict__ Rp,
                                                          size_t pstride, int npad, int kl, int kr,
                                                          int d_min, DiagOrder order,
                                                          int32_t *__restrict__ C) {
  __shared__ __attribute__((aligned(16))) int8_t sL[2][HBM_ * HLDS];
  __shared__ __attribute__((aligned(16))) int8_t sR[2][HBM_ * HLDS];
  const int tiles_n = npad / HBM_;
  const int G = gridDim.x;
  int b = blockIdx.x;
  if ((G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3);
  const int group = b / (HGM * tiles_n);
  const int first_m = group * HGM;
  const int gsz = min(tiles_n - first_m, HGM);
  const int inb = b - group * HGM * tiles_n;
  const int m0 = (first_m + inb % gsz) * HBM_;
  const int n0 = (inb / gsz) * HBM_;
  const int slot = order.q[blockIdx.y];
  const int d = d_min + slot;
  const int s_lo = max(1, d - kr), s_hi = min(kl, d - 1);
  const int npairs = s_hi - s_lo + 1;
  const int KT = npad / HBK;
  const int T = npairs * KT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  v16i acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][c][v] = 0;

  // global -> register staging: 256 rows x 128 bytes per operand = 2048 chunks
  // of 16 bytes, 8 per thread; 8 consecutive threads read one 128-byte row.
  v4i gL[8], gR[8];
  auto load = [&](int tt) {
    const int p = tt / KT, k0 = (tt - p * KT) * HBK;
    const int s = s_lo + p;
    const int8_t *Lb = Lp + (size_t)(s - 1) * pstride + (size_t)m0 * npad + k0;
    const int8_t *Rb = Rp + (size_t)(d - s - 1) * pstride + (size_t)n0 * npad + k0;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int c = tid + 256 * h, row = c >> 3, col = (c & 7) * 16;
      gL[h] = *(const v4i *)(Lb + (size_t)row * npad + col);
      gR[h] = *(const v4i *)(Rb + (size_t)row * npad + col);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int c = tid + 256 * h, row = c >> 3, col = (c & 7) * 16;
      *(v4i *)(&sL[buf][row * HLDS + col]) = gL[h];
      *(v4i *)(&sR[buf][row * HLDS + col]) = gR[h];
    }
  };
  if (T > 0) {
    load(0);
    stash(0);
    if (T > 1) load(1);
  }
  // Fragment addresses: lane l reads 16 bytes of row (l mod 32) of each 32-row
  // block at K offset 16 (l / 32) within the 32-byte MFMA step.
  const int fa_off = (wm * 128 + (lane & 31)) * HLDS + 16 * (lane >> 5);
  const int fb_off = (wn * 128 + (lane & 31)) * HLDS + 16 * (lane >> 5);
  for (int tt = 0; tt < T; ++tt) {
    const int cur = tt & 1;
    __syncthreads();                 // stage tt visible; buffer cur^1 no longer read
    const int8_t *bL = sL[cur], *bR = sR[cur];
    v4i fa[2][4], fb[2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      fa[0][x] = *(const v4i *)(bL + fa_off + x * 32 * HLDS);
      fb[0][x] = *(const v4i *)(bR + fb_off + x * 32 * HLDS);
    }
#pragma unroll
    for (int ks = 0; ks < HBK / 32; ++ks) {
      const int c = ks & 1;
      if (ks + 1 < HBK / 32) {       // next step's fragments, in flight during the MFMAs
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          fa[c ^ 1][x] = *(const v4i *)(bL + fa_off + x * 32 * HLDS + (ks + 1) * 32);
          fb[c ^ 1][x] = *(const v4i *)(bR + fb_off + x * 32 * HLDS + (ks + 1) * 32);
        }
      }
      if (ks == 1 && tt + 1 < T) stash(cur ^ 1);              // LDS writes of stage tt+1
      if (ks == 2 && tt + 2 < T) load(tt + 2);                // global loads of stage tt+2
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[c][x], fb[c][y], acc[x][y], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  int32_t *Cq = C + (size_t)slot * npad * npad;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 128 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + wn * 128 + y * 32 + (lane & 31);
        Cq[(size_t)row * npad + col] = acc[x][y][v];
      }
}

void launch_slice_gemm(const int8_t *Lp, const int8_t *Rp, size_t pstride, int npad, int kl,
                       int kr, int d_min, int ndiag, int32_t *C, hipStream_t s) {
  // heaviest diagonals (most pairs) first, so the tail of the launch is light
  DiagOrder o;
  int cnt[kMaxDiag];
  for (int q = 0; q < ndiag; ++q) {
    int d = d_min + q;
    int lo = d - kr > 1 ? d - kr : 1, hi = kl < d - 1 ? kl : d - 1;
    cnt[q] = hi - lo + 1;
    o.q[q] = q;
  }
  for (int a = 1; a < ndiag; ++a)
    for (int b = a; b > 0 && cnt[o.q[b]] > cnt[o.q[b - 1]]; --b) {
      int t = o.q[b];
      o.q[b] = o.q[b - 1];
      o.q[b - 1] = t;
    }
  if (npad >= 1024) {
    const int tiles = (npad / HBM_) * (npad / HBM_);
    hipLaunchKernelGGL(k_slice_gemm256, dim3(tiles, ndiag), dim3(256), 0, s, Lp, Rp, pstride,
                       npad, kl, kr, d_min, o, C);
  } else {
    const int tiles = (npad / GBM) * (npad / GBN);
    hipLaunchKernelGGL(k_slice_gemm, dim3(tiles, ndiag), dim3(256), 0, s, Lp, Rp, pstride, npad,
                       kl, kr, d_min, o, C);
  }
}

// ---------------------------------------------------------------- V epilogue + column pass
template <int EPT>
__global__ __launch_bounds__(kEpiThreads) void k_epi_v(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag, const int *__restrict__ eA,
    const int *__restrict__ eX, const double *__restrict__ X1, int n, double *lam, double *r,
    int *eR, double *resmax, int8_t *__restrict__ Rpl, int kr, int *flags) {
  __shared__ double scratch[2 * (kEpiThreads / 64)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const size_t P = (size_t)npad * npad;
  int8_t *Rcol = Rpl + (size_t)j * npad;
  if (j >= n) {
    for (int q = 0; q < EPT; ++q) {
      const int i = tid + kEpiThreads * q;
      if (i < npad)
        for (int t = 0; t < kr; ++t) Rcol[t * P + i] = 0;
    }
    return;
  }
  const int ej = eX[j];
  const int32_t *Ccol = C + (size_t)j * npad;
  const double *xcol = X1 + (size_t)j * n;
  double vh[EPT], vl[EPT];
  ddv sx = {0.0, 0.0}, sv = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    vh[q] = vl[q] = 0.0;
    if (i < n) {
      const int ei = eA[i];
      double h = 0.0, l = 0.0;
#pragma unroll 1
      for (int qq = ndiag - 1; qq >= 0; --qq) {
        const double tv = ldexp((double)Ccol[(size_t)qq * P + i], ei + ej - 7 * (d_min + qq));
        double s, e;
        two_sum(h, tv, s, e);
        h = s;
        l += e;
      }
      fast_two_sum(h, l, vh[q], vl[q]);
      const double x = xcol[i];
      double p, pe;
      two_prod(x, x, p, pe);
      sx = dd_add_prod(sx, p, pe);
      two_prod(x, vh[q], p, pe);
      sv = dd_add_prod(sv, p, pe + x * vl[q]);
    }
  }
  sx = block_dd_sum<kEpiThreads>(sx, scratch);
  sv = block_dd_sum<kEpiThreads>(sv, scratch);
  // r_j = 1 - x^T x,  lambda_j = x^T v / (1 - r_j)
  ddv rj = dd_add(ddv{1.0, 0.0}, ddv{-sx.h, -sx.l});
  ddv den = dd_add(ddv{1.0, 0.0}, ddv{-rj.h, -rj.l});
  const double lj = dd_div_to_d(sv, den);
  // residual in pair arithmetic: (vh + vl) - x * lambda
  double rmax = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    if (i < n) {
      double p, pe, s, e;
      two_prod(xcol[i], lj, p, pe);
      two_sum(vh[q], -p, s, e);
      const double res = s + ((e + vl[q]) - pe);
      vh[q] = res;
      rmax = fmax(rmax, fabs(res));
    }
  }
  rmax = block_max<kEpiThreads>(rmax, scratch);
  const int er = exp_above(rmax);
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    if (i < npad) {
      const double a = (i < n) ? vh[q] : 0.0;
      double y = ldexp(fabs(a), -er);
      const int sg = (a < 0.0) ? -1 : 1;
      for (int t = 0; t < kr; ++t) {
        double t128 = y * 128.0;
        double dgt = floor(t128);
        y = t128 - dgt;
        Rcol[t * P + i] = (int8_t)(sg * (int)dgt);
      }
    }
  }
  if (tid == 0) {
    lam[j] = lj;
    r[j] = rj.h;
    eR[j] = er;
    resmax[j] = rmax;
    if (!(fabs(lj) <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

template <int EPT>
static void epi_v_t(const int32_t *C, int npad, int d_min, int ndiag, const int *eA, const int *eX,
                    const double *X1, int n, double *lam, double *r, int *eR, double *resmax,
                    int8_t *Rpl, int kr, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_epi_v<EPT>, dim3(npad), dim3(kEpiThreads), 0, s, C, npad, d_min, ndiag, eA,
                     eX, X1, n, lam, r, eR, resmax, Rpl, kr, flags);
}

void launch_epi_v(const int32_t *C, int npad, int d_min, int ndiag, const int *eA, const int *eX,
                  const double *X1, int n, double *lam, double *r, int *eR, double *resmax,
                  int8_t *Rpl, int kr, int *flags, hipStream_t s) {
  const int ept = (npad + kEpiThreads - 1) / kEpiThreads;
  if (ept <= 1) epi_v_t<1>(C, npad, d_min, ndiag, eA, eX, X1, n, lam, r, eR, resmax, Rpl, kr, flags, s);
  else if (ept <= 2) epi_v_t<2>(C, npad, d_min, ndiag, eA, eX, X1, n, lam, r, eR, resmax, Rpl, kr, flags, s);
  else if (ept <= 4) epi_v_t<4>(C, npad, d_min, ndiag, eA, eX, X1, n, lam, r, eR, resmax, Rpl, kr, flags, s);
  else epi_v_t<8>(C, npad, d_min, ndiag, eA, eX, X1, n, lam, r, eR, resmax, Rpl, kr, flags, s);
}

// ---------------------------------------------------------------- W epilogue -> E~
template <int EPT>
__global__ __launch_bounds__(kEpiThreads) void k_epi_w(
    const int32_t *__restrict__ C, int npad, int d_min, int ndiag, const int *__restrict__ eX,
    const int *__restrict__ eR, const double *__restrict__ lam, const double *__restrict__ r,
    int n, int *eE, double *emax, int8_t *__restrict__ Epl, int ke, int *flags) {
  __shared__ double scratch[2 * (kEpiThreads / 64)];
  const int j = blockIdx.x, tid = threadIdx.x;
  const size_t P = (size_t)npad * npad;
  int8_t *Ecol = Epl + (size_t)j * npad;
  if (j >= n) {
    for (int q = 0; q < EPT; ++q) {
      const int i = tid + kEpiThreads * q;
      if (i < npad)
        for (int t = 0; t < ke; ++t) Ecol[t * P + i] = 0;
    }
    return;
  }
  const int ej = eR[j];
  const double lj = lam[j];
  const int32_t *Ccol = C + (size_t)j * npad;
  double ev[EPT];
  double ms = 0.0, mr = 0.0;
  int tie = 0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    ev[q] = 0.0;
    if (i < n) {
      const int ei = eX[i];
      double w = 0.0;
#pragma unroll 1
      for (int qq = ndiag - 1; qq >= 0; --qq)
        w += ldexp((double)Ccol[(size_t)qq * P + i], ei + ej - 7 * (d_min + qq));
      double e;
      if (i == j) {
        e = 0.5 * r[j];
      } else {
        const double den = lj - lam[i];
        if (den == 0.0) {
          tie = 1;
          e = 0.0;
        } else {
          e = w / den;
        }
      }
      mr = fmax(mr, fabs(e));
      const double es = ldexp(e, ei);
      ev[q] = es;
      ms = fmax(ms, fabs(es));
    }
  }
  if (tie) atomicOr(flags, FLAG_TIE);
  ms = block_max<kEpiThreads>(ms, scratch);
  mr = block_max<kEpiThreads>(mr, scratch);
  const int ee = exp_above(ms);
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int i = tid + kEpiThreads * q;
    if (i < npad) {
      const double a = ev[q];
      double y = ldexp(fabs(a), -ee);
      const int sg = (a < 0.0) ? -1 : 1;
      for (int t = 0; t < ke; ++t) {
        double t128 = y * 128.0;
        double dgt = floor(t128);
        y = t128 - dgt;
        Ecol[t * P + i] = (int8_t)(sg * (int)dgt);
      }
    }
  }
  if (tid == 0) {
    eE[j] = ee;
    emax[j] = mr;
    if (!(mr <= DBL_MAX)) atomicOr(flags, FLAG_NONFINITE);
  }
}

template <int EPT>
static void epi_w_t(const int32_t *C, int npad, int d_min, int ndiag, const int *eX, const int *eR,
                    const double *lam, const double *r, int n, int *eE, double *emax,
                    int8_t *Epl, int ke, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_epi_w<EPT>, dim3(npad), dim3(kEpiThreads), 0, s, C, npad, d_min, ndiag, eX,
                     eR, lam, r, n, eE, emax, Epl, ke, flags);
}

void launch_epi_w(const int32_t *C, int npad, int d_min, int ndiag, const int *eX, const int *eR,
                  const double *lam, const double *r, int n, int *eE, double *emax,
                  int8_t *Epl, int ke, int *flags, hipStream_t s) {
  const int ept = (npad + kEpiThreads - 1) / kEpiThreads;
  if (ept <= 1) epi_w_t<1>(C, npad, d_min, ndiag, eX, eR, lam, r, n, eE, emax, Epl, ke, flags, s);
  else if (ept <= 2) epi_w_t<2>(C, npad, d_min, ndiag, eX, eR, lam, r, n, eE, emax, Epl, ke, flags, s);
  else if (ept <= 4) epi_w_t<4>(C, npad, d_min, ndiag, eX, eR, lam, r, n, eE, emax, Epl, ke, flags, s);
  else epi_w_t<8>(C, npad, d_min, ndiag, eX, eR, lam, r, n, eE, emax, Epl, ke, flags, s);
}

// ---------------------------------------------------------------- update X <- X1 + X1 E~
__global__ __launch_bounds__(256) void k_epi_u(const int32_t *__restrict__ C, int npad, int d_min,
                                               int ndiag, const int *__restrict__ eE,
                                               const double *__restrict__ X1, int n,
                                               double *__restrict__ X, int ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const size_t P = (size_t)npad * npad;
  const int32_t *Ccol = C + (size_t)j * npad;
  const int ej = eE[j];
  double u = 0.0;
  for (int qq = ndiag - 1; qq >= 0; --qq)
    u += ldexp((double)Ccol[(size_t)qq * P + i], ej - 7 * (d_min + qq));
  X[(size_t)j * ldx + i] = X1[(size_t)j * n + i] + u;
}

void launch_epi_u(const int32_t *C, int npad, int d_min, int ndiag, const int *eE,
                  const double *X1, int n, double *X, int ldx, hipStream_t s) {
  hipLaunchKernelGGL(k_epi_u, dim3((n + 255) / 256, n), dim3(256), 0, s, C, npad, d_min, ndiag, eE,
                     X1, n, X, ldx);
}

}  // namespace refeig
