// Planning arithmetic of an iteration, shared by the host orchestrator and the device
// planning kernels: beta of Sec. 4.1, the digit counts of X^(1) and A, the modulus counts
// and reconstruction constants of V by residues, the pair-diagonal cutoffs of the three
// products, and the block order of a tabled launch. Both sides run the same code (plain
// IEEE operations, no library transcendental), so they plan an iteration identically.
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>

#include "kernels.h"

namespace refeig {

#define RF_HD __host__ __device__ inline

constexpr int kKxMaxP = 9;    // digit planes of X^(1) at most
constexpr int kKrMaxP = 12;   // digit planes of the residual and of E~

// The odd, pairwise coprime moduli <= 255, largest first (from 255 down, each one coprime
// to all taken before it).
RF_HD int modulus(int q) {
  switch (q) {
    case 0: return 255;  case 1: return 253;  case 2: return 251;  case 3: return 247;
    case 4: return 241;  case 5: return 239;  case 6: return 233;  case 7: return 229;
    case 8: return 227;  case 9: return 223;  case 10: return 217; case 11: return 211;
    case 12: return 199; case 13: return 197; case 14: return 193; case 15: return 191;
    case 16: return 181; case 17: return 179; case 18: return 173; case 19: return 167;
    case 20: return 163; case 21: return 157; case 22: return 151; case 23: return 149;
    case 24: return 139; case 25: return 137; case 26: return 131; default: return 127;
  }
}

// log2(x) for finite x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)), log2 m = 2 atanh(s) /
// ln 2, s = (m - 1) / (m + 1), |s| < 0.172, by its series to s^25 (absolute error below
// 1e-18). Only the four basic operations, in a fixed order.
RF_HD double plan_log2(double x) {
  int e = 0;
  double m = frexp(x, &e);   // m in [0.5, 1)
  if (m < 0.70710678118654752) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
  double p = 1.0 / 25.0;
  p = p * s2 + 1.0 / 23.0;
  p = p * s2 + 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  p = p * s2 + 1.0;
  const double ln_m = 2.0 * s * p;
  return (double)e + ln_m * 1.4426950408889634;
}

// Slice pairs (s, d - s), 1 <= s <= kl, 1 <= d - s <= kr, on pair diagonal d.
RF_HD int npairs_of(int d, int kl, int kr) {
  const int lo = d - kr > 1 ? d - kr : 1, hi = kl < d - 1 ? kl : d - 1;
  return hi >= lo ? hi - lo + 1 : 0;
}

// ---- beta of Sec. 4.1 (floor form) and the digit count of X^(1).
// S = sum_j 2^(2 c_j) over the nonzero columns, from a histogram of 2 c_j (index 2 c_j +
// kBetaBias), summed from the smallest power up: exact for any realistic spread.
constexpr int kBetaBias = 1024, kBetaBins = 2048;
RF_HD double pow2_sum(const int *hist) {
  double S = 0.0;
  for (int b = 0; b < kBetaBins; ++b)
    if (hist[b]) S += (double)hist[b] * ldexp(1.0, b - kBetaBias);
  return S;
}
// beta = floor(log2((1/(0.75u)) sqrt(xi delta g / (L S)))), evaluated as q = ((xi delta) g) /
// (L S), t = sqrt(q) / (0.75 2^-53), beta = exponent(t) - 1 (exact floor of log2 t);
// kx = ceil((54 - beta + extra) / 7), extra = max_j (e_j - c_j): the X^(1) grid
// 2^(c_j + beta - 54) is the rounding bound u ufp(tau_j) of eq. (minamihata).
RF_HD void beta_core(double xi, double delta, double g, double L, double S, int extra,
                     int *beta, int *kx) {
  const double q = ((xi * delta) * g) / (L * S);
  const double t = sqrt(q) / (0.75 * ldexp(1.0, -53));
  int ex = 0;
  (void)frexp(t, &ex);
  *beta = ex - 1;
  const int num = 54 - *beta + extra;
  int k = num <= 0 ? 1 : (num + 6) / 7;
  if (k < 1) k = 1;
  if (k > kKxMaxP) k = kKxMaxP;
  *kx = k;
}

// ---- pair-diagonal cutoffs (Sec. 4.1's sqrt(n) relaxation in the growth terms)
// V by slices, column j: the smallest D with 7D >= eA_max + eX_j + 7 + log2(1.5 kx) + lgrowth
// - log2(theta delta g_j), plus d_extra, at least 2.
RF_HD int cut_v(int eA_max, double lgrowth, int kx, int eXj, double theta, double delta, double g,
                int dextra) {
  const double c0 = (double)eA_max + 7.0 + plan_log2(1.5 * kx) + lgrowth;
  const double need = (c0 + (double)eXj - plan_log2(theta * delta * g)) / 7.0;
  const int d = (int)ceil(need) + dextra;
  return d > 2 ? d : 2;
}
// V by residues, column j: digits of A, ka1 >= (eA_max + lgrowth + eX_j - log2(theta delta
// g_j)) / 7 (truncating A costs sqrt(n) 2^(eA_max + eX_j - 7 ka1)), plus d_extra.
RF_HD int cut_ka(int eA_max, double lgrowth, int eXj, double theta, double delta, double g,
                 int dextra) {
  const double nd = ((double)eA_max + lgrowth + (double)eXj - plan_log2(theta * delta * g)) / 7.0;
  return (int)ceil(nd) + dextra;
}
// W = X^(1)T Res, column j (eR_j the residual column's exponent); the column-independent
// part c0 = cut_w_c0(...) may be formed once per iteration.
RF_HD double cut_w_c0(int eXmax, int kx, double lsqn) {
  return (double)eXmax + 7.0 + plan_log2(1.5 * kx) + lsqn;
}
RF_HD int cut_w_from(double c0, int eRj, double theta, double delta, double g, int dextra) {
  const double need = (c0 + (double)eRj - plan_log2(theta * delta * g)) / 7.0;
  const int d = (int)ceil(need) + dextra;
  return d > 2 ? d : 2;
}
RF_HD int cut_w(int eXmax, int kx, double lsqn, int eRj, double theta, double delta, double g,
                int dextra) {
  return cut_w_from(cut_w_c0(eXmax, kx, lsqn), eRj, theta, delta, g, dextra);
}
// The per-tile W cutoff's constant: 7 + log2(1.5 kx) + lsqn - log2(theta delta).
RF_HD double cx_tile(int kx, double lsqn, double theta, double delta) {
  return 7.0 + plan_log2(1.5 * kx) + lsqn - plan_log2(theta * delta);
}
// X^(1) E~, column j (eE_j the exponent of E~'s column, t_j its noise tightening).
RF_HD double cut_u_c0(int kx, double lsqn, double theta, double delta) {
  return 7.0 + plan_log2(1.008 * kx) + lsqn - plan_log2(theta * delta);
}
RF_HD int cut_u_from(double c0, int eEj, double tj, int dextra) {
  const double need = (c0 + (double)eEj - plan_log2(tj)) / 7.0;
  const int d = (int)ceil(need) + dextra;
  return d > 2 ? d : 2;
}
RF_HD int cut_u(int kx, double lsqn, int eEj, double theta, double delta, double tj,
                int dextra) {
  return cut_u_from(cut_u_c0(kx, lsqn, theta, delta), eEj, tj, dextra);
}
// Noise tightening of column j (the reading of the paper's cut bound for loose targets):
// t_j = min(1, sqrt(delta_int g_j / (4 L)) / (theta delta_k)).
RF_HD double w_tight(double delta_int, double g, double L, double theta, double delta_k) {
  const double t = sqrt(delta_int * g / (4.0 * L)) / (theta * delta_k);
  return t < 1.0 ? t : 1.0;
}

// ---- V by residues: modulus counts, reconstruction constants, residue weights.
// The smallest N with sum_{q < N} log2 m_q > need_bits, or -1 above kCrtMax.
RF_HD int crt_count(double need_bits) {
  double bits = 0.0;
  int N = 0;
  while (N < kCrtMax && bits <= need_bits) bits += plan_log2((double)modulus(N++));
  return bits > need_bits ? N : -1;
}
// The same with lg[q] = plan_log2(modulus(q)) given (the same sums in the same order).
RF_HD int crt_count_lg(double need_bits, const double *lg) {
  double bits = 0.0;
  int N = 0;
  while (N < kCrtMax && bits <= need_bits) bits += lg[N++];
  return bits > need_bits ? N : -1;
}
// Bits the moduli must exceed for ka1 digits of A, kx of X^(1), reduction length npad and
// the Cauchy-Schwarz headroom hbits (log2 of a bound on ||a_i|| 2^-eA_i ||x_j|| 2^-eX_j;
// < 0: unknown): prod m_q > 4 2^hb 128^(ka1 + kx), hb = min(hbits, log2 npad).
RF_HD double crt_need_bits(int npad, int ka1, int kx, double hbits) {
  const double lnp = plan_log2((double)npad);
  const double hb = (hbits >= 0.0 && hbits < lnp) ? hbits : lnp;
  return 2.0 + hb + 7.0 * (double)(ka1 + kx);
}

RF_HD int inv_mod_i(int a, int m) {   // a^-1 mod m (gcd(a, m) = 1)
  int t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
  while (nr) {
    const int q = r / nr, tt = t - q * nt, rr = r - q * nr;
    t = nt;
    nt = tt;
    r = nr;
    nr = rr;
  }
  return t < 0 ? t + m : t;
}

// Weights of k digit planes for N moduli: w_qt = 128^(k-1-t) mod m_q in the symmetric range,
// also packed four planes to a dword (byte i of wp[q][g] is w[q][4g + i]). The rows are
// independent: res_weights_row fills modulus slot q (parallel callers give each q its own
// thread), res_weights_build fills all of them.
RF_HD void res_weights_row(int k, int N, int q, ResWeights &rw) {
  const int m = q < N ? modulus(q) : 1;
  rw.m[q] = m;
  rw.rmf[q] = 1.0f / (float)m;
  for (int t = 0; t < kCrtPlanes; ++t) rw.w[q][t] = 0;
  if (q < N) {
    unsigned pw = 1;   // < 255: products stay below 2^15
    for (int t = k - 1; t >= 0; --t) {
      rw.w[q][t] = (int)pw > m / 2 ? (int)pw - m : (int)pw;
      pw = pw * 128u % (unsigned)m;
    }
  }
  for (int g = 0; g < (kCrtPlanes + 3) / 4; ++g) {
    unsigned v = 0u;
    for (int i = 0; i < 4 && 4 * g + i < kCrtPlanes; ++i)
      v |= ((unsigned)rw.w[q][4 * g + i] & 0xffu) << (8 * i);
    rw.wp[q][g] = (int)v;
  }
}
RF_HD void res_weights_build(int k, int N, ResWeights &rw) {
  rw.N = N;
  rw.k = k;
  for (int q = 0; q < kCrtMax; ++q) res_weights_row(k, N, q, rw);
}

// Reconstruction record of N moduli for ka1 digits of A and kx of X^(1): V = P 2^(eA_i +
// eX_j + sh), sh = -7 (ka1 + kx); M = prod m_q (double-word); per modulus u_q = y_q / m_q
// (triple-double, y_q = (M / m_q)^-1 mod m_q) and its kCrtLimbs limbs of kCrtLimbBits bits
// (long division, exact in 64-bit integers): P / M = sum_q r_q u_q mod 1.
// crt_rec_head fills the shared fields; after it, crt_rec_modulus (one q < kCrtMax each)
// writes disjoint fields and may run in parallel; crt_rec_build runs them in order.
RF_HD void crt_rec_head(int N, int ka1, int kx, CrtRec &rec) {
  rec.N = N;
  rec.sh = -7 * (ka1 + kx);
  double a0 = 1.0, a1 = 0.0;
  for (int q = 0; q < N; ++q) {
    const double md = (double)modulus(q);
    const double p0 = a0 * md, e0 = fma(a0, md, -p0);
    const double sl = e0 + a1 * md;
    a0 = p0 + sl;
    a1 = sl - (a0 - p0);
  }
  rec.M[0] = a0;
  rec.M[1] = a1;
  rec.M[2] = 0.0;
}
RF_HD void crt_rec_modulus(int q, CrtRec &rec) {
  const int N = rec.N;
  rec.m[q] = q < N ? modulus(q) : 1;
  rec.rm[q] = q < N ? 1.0 / (double)rec.m[q] : 0.0;
  rec.u[q][0] = rec.u[q][1] = rec.u[q][2] = 0.0;
  for (int k = 0; k < kCrtLimbs; ++k) rec.L[q][k] = 0.0;
  if (q >= N) return;
  const int m = modulus(q);
  unsigned Mq = 1;   // (M / m_q) mod m_q; products below 2^16
  for (int l = 0; l < N; ++l)
    if (l != q) Mq = Mq * ((unsigned)modulus(l) % (unsigned)m) % (unsigned)m;
  const int yi = inv_mod_i((int)Mq, m);
  const double y = (double)yi, md = (double)m;
  const double u0 = y / md, r0 = fma(-u0, md, y);
  const double u1 = r0 / md, r1 = fma(-u1, md, r0);
  rec.u[q][0] = u0;
  rec.u[q][1] = u1;
  rec.u[q][2] = r1 / md;
  unsigned long long rem = (unsigned long long)yi;   // < m < 2^8: num < 2^(8 + limb bits)
  for (int k = 0; k < kCrtLimbs; ++k) {
    const unsigned long long num = rem << kCrtLimbBits;
    rec.L[q][k] = (double)(num / (unsigned)m);
    rem = num % (unsigned)m;
  }
}
RF_HD void crt_rec_build(int N, int ka1, int kx, CrtRec &rec) {
  crt_rec_head(N, ka1, kx, rec);
  for (int q = 0; q < kCrtMax; ++q) crt_rec_modulus(q, rec);
}

// Block -> (row block, column block) of a launch over tiles_m row blocks x tiles_n column
// blocks: blocks go round-robin to the 8 XCDs (id mod 8), each with its own L2; with tiles_n
// a multiple of 8 XCD x owns one column block of each group of 8, x in even groups and 7 - x
// in odd ones (x, 15 - x, 16 + x, ...: its R operand stays in its L2), and walks them in
// groups of up to 8 row blocks. Spread rather than contiguous column sets keep the XCDs' work
// even when the work per tile drifts along the columns (per-tile cutoffs do).
RF_HD void xcd_tile_order(int bid, int tiles_m, int tiles_n, int &mi, int &nb) {
  if (tiles_n % 8 == 0) {
    const int xcd = bid & 7, local = bid >> 3, cb = tiles_n >> 3;
    const int rg = local / (8 * cb), rem = local - rg * 8 * cb;
    const int left = tiles_m - rg * 8;
    const int gs = left < 8 ? left : 8;
    const int c = rem / gs;
    mi = rg * 8 + rem % gs;
    nb = 8 * c + ((c & 1) ? 7 - xcd : xcd);
  } else if (tiles_m % 8 == 0) {
    const int xcd = bid & 7, local = bid >> 3, rows = tiles_m >> 3;
    mi = xcd + 8 * (local % rows);
    nb = local / rows;
  } else {
    const int group = bid / (4 * tiles_n), first_m = group * 4;
    const int left = tiles_m - first_m;
    const int gsz = left < 4 ? left : 4, inb = bid - group * 4 * tiles_n;
    mi = first_m + inb % gsz;
    nb = inb / gsz;
  }
}

#undef RF_HD

}  // namespace refeig
