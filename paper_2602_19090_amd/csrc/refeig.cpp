// Host orchestrator and C ABI of the eigenvector-refinement library.
//
// One call of refine_eigvecs runs, per iteration (Algorithm 1 with the first
// slice X^(1) of Sec. 3, products by the Ozaki scheme on INT8 digit planes):
//   working column order (by gap), folded into the reads and writes of X and D
//   colstats(X) -> beta (Sec. 4.1), kx          [host reads n exponents]
//   split X -> X^(1), its digit planes (both layouts)
//   V = A X^(1)          per-diagonal slice GEMMs + fused column pass
//                        (r, lambda, residual V - X^(1) D^, residual planes)
//                                               [host reads lambda, exponents]
//   W = X^(1)T Res       slice GEMMs + E~ epilogue (E~ planes)
//                                               [host reads column maxima]
//   (opt-in) grouped correction: Rayleigh-Ritz on strongly coupled columns
//   X <- X^(1) + X^(1) E~ slice GEMMs + update epilogue
// The A planes are built once per call. How many pair diagonals each product
// keeps is decided on the host from the target error and the eigenvalue gaps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <unordered_set>
#include <unordered_map>
#include <queue>
#include <map>
#include <fstream>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <thread>
#include <time.h>
#include <vector>

#include <rocblas/rocblas.h>

#include "../../include/refeig.h"
#include "kernels.h"
#include "plain.h"
#include "plan.h"
#include "devplan.h"
#include "work.h"

using namespace refeig;

namespace {

constexpr int kKaMaxLimit = 18;

#define HIPCHK(x)                                                        \
  do {                                                                   \
    hipError_t err__ = (x);                                              \
    if (err__ != hipSuccess) {                                           \
      fprintf(stderr, "refeig: %s failed: %s\n", #x, hipGetErrorString(err__)); \
      return REFEIG_E_HIP;                                               \
    }                                                                    \
  } while (0)

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }


int nslots(int ka, bool crt = false) {
  return std::max(std::max(ka, kKrMax + kKxMax), crt ? kCrtMax : 0);
}

constexpr int kGroupColsMax = 1024;   // group members corrected per iteration (at most)
constexpr int kCouplingsMax = 1 << 16; // strong couplings listed per iteration (at most)

// Carves the workspace; returns the bytes needed (base may be null).
size_t carve(int n, int ka, char *base, Work *w, bool crt = false) {
  Work t;
  t.n = n;
  t.npad = round_up(n, kTile);
  t.ka = ka;
  t.P = (size_t)t.npad * t.npad;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  t.AP = (int8_t *)take(t.P * ka);
  t.XP = (int8_t *)take(t.P * kKxMax);
  t.XPT = (int8_t *)take(t.P * kKxMax);
  t.RP = (int8_t *)take(t.P * kKrMax);
  t.EP = (int8_t *)take(t.P * kKeMax);
  t.Cs = (int32_t *)take(t.P * 4 * (size_t)nslots(ka, crt));
  if (crt) {
    t.ARES = (int8_t *)take(t.P * kCrtMax * kVLevels);   // level l at planes l kCrtMax
    t.XRES = (int8_t *)take(t.P * kCrtMax);
  }
  t.X1 = (double *)take(sizeof(double) * (size_t)n * n);
  const size_t vi = sizeof(int) * t.npad, vd = sizeof(double) * t.npad;
  t.eA = (int *)take(vi);
  t.cA = (int *)take(vi);
  t.eX = (int *)take(vi);
  t.cX = (int *)take(vi);
  t.eR = (int *)take(vi);
  t.eE = (int *)take(vi);
  t.flags = (int *)take(256);
  for (int q = 0; q < 3; ++q) t.dcut[q] = (int *)take(vi);
  t.colmap = (int *)take(vi);
  t.tcut = (int *)take(sizeof(int) * (kMaxN / 256) * (kMaxN / 256));
  t.mods = (int *)take(sizeof(int) * kCrtMax);
  t.recs = (CrtRec *)take(sizeof(CrtRec) * kVLevels);
  t.vblk = (int *)take(sizeof(int) * 2 * (kMaxN / 256));
  t.ssA = (double *)take(vd);
  t.ssX = (double *)take(vd);
  t.wtol = (double *)take(2 * vd);
  for (int q = 0; q < 3; ++q)
    t.tab[q] = (int *)take(sizeof(int) * (kMaxN / 256) * (kMaxN / 256) * kMaxDiag);
  t.cpl = (int *)take(sizeof(int) * (2 * (size_t)kCouplingsMax + 64));
  const size_t npr = (size_t)kGroupColsMax * kGroupMax;
  t.g_pa = (int *)take(sizeof(int) * npr);
  t.g_pb = (int *)take(sizeof(int) * npr);
  t.g_gh = (double *)take(sizeof(double) * npr);
  t.g_gl = (double *)take(sizeof(double) * npr);
  t.g_w = (double *)take(sizeof(double) * npr);
  t.g_Y = (double *)take(sizeof(double) * npr);
  t.g_col = (int *)take(sizeof(int) * kGroupColsMax);
  t.g_first = (int *)take(sizeof(int) * kGroupColsMax);
  t.g_k = (int *)take(sizeof(int) * kGroupColsMax);
  t.g_pos = (int *)take(sizeof(int) * kGroupColsMax);
  t.g_base = (int *)take(sizeof(int) * kGroupColsMax);
  t.g_mu = (double *)take(sizeof(double) * kGroupColsMax);
  t.g_mul = (double *)take(sizeof(double) * kGroupColsMax);
  t.mxA = (double *)take(vd);
  t.mxX = (double *)take(vd);
  t.lam = (double *)take(vd);
  t.lam_lo = (double *)take(vd);
  t.r = (double *)take(vd);
  t.resmax = (double *)take(vd);
  t.emax = (double *)take(vd);
  t.dst = (DevState *)take(sizeof(DevState));
  t.gapsw = (double *)take(vd);
  t.skey = (double *)take(vd);
  t.sidx = (int *)take(vi);
  if (w) *w = t;
  return off;
}

// ---- FP64 plain form: workspace
constexpr int kPlainKaMax = 8, kPlainKxMax = 4;
struct PlainWork {
  double *SA, *SX, *X1, *P, *Vh, *Vl, *Res, *E;
  int *eX, *cX, *flags;
  double *mxX, *lam, *r;
  unsigned long long *colmax;
};
size_t carve_plain(int n, char *base, PlainWork *w) {
  PlainWork t;
  size_t off = 0;
  const size_t nn = (size_t)n * n * sizeof(double);
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  t.SA = (double *)take(nn * kPlainKaMax);
  t.SX = (double *)take(nn * kPlainKxMax);
  t.X1 = (double *)take(nn);
  t.P = (double *)take(nn);
  t.Vh = (double *)take(nn);
  t.Vl = (double *)take(nn);
  t.Res = (double *)take(nn);
  t.E = (double *)take(nn);
  const int npad = round_up(n, kTile);
  t.eX = (int *)take(sizeof(int) * npad);
  t.cX = (int *)take(sizeof(int) * npad);
  t.flags = (int *)take(256);
  t.mxX = (double *)take(sizeof(double) * npad);
  t.lam = (double *)take(sizeof(double) * npad);
  t.r = (double *)take(sizeof(double) * npad);
  t.colmax = (unsigned long long *)take(sizeof(unsigned long long) * npad);
  if (w) *w = t;
  return off;
}

// ---- complex Hermitian case: workspace. Digit planes are realified (K = 2 npad, plane
// stride 2 npad^2); each complex product keeps the slots of its real and imaginary parts.
constexpr int kMaxNHerm = 4096;   // the complex column epilogues hold 4 values per thread
struct HermWork {
  int npad = 0;
  size_t P = 0;
  int8_t *AP1, *AP2, *XP, *XT, *RP1, *RP2, *EP1, *EP2;
  int32_t *Cr, *Ci;
  double *X1;
  int *eA, *cA, *eX, *cX, *eR, *eE, *flags, *colmap;
  int *dcut[3];
  double *mxA, *mxX, *lam, *lam_lo, *r, *resmax, *emax;
};
size_t carve_herm(int n, int ka, char *base, HermWork *w) {
  HermWork t;
  t.npad = round_up(n, kTile);
  t.P = (size_t)t.npad * t.npad;
  const size_t P2 = 2 * t.P;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  t.AP1 = (int8_t *)take(P2 * ka);
  t.AP2 = (int8_t *)take(P2 * ka);
  t.XP = (int8_t *)take(P2 * kKxMax);
  t.XT = (int8_t *)take(P2 * kKxMax);
  t.RP1 = (int8_t *)take(P2 * kKrMax);
  t.RP2 = (int8_t *)take(P2 * kKrMax);
  t.EP1 = (int8_t *)take(P2 * kKeMax);
  t.EP2 = (int8_t *)take(P2 * kKeMax);
  t.Cr = (int32_t *)take(t.P * 4 * (size_t)nslots(ka));
  t.Ci = (int32_t *)take(t.P * 4 * (size_t)nslots(ka));
  t.X1 = (double *)take(sizeof(double) * 2 * (size_t)n * n);
  const size_t vi = sizeof(int) * t.npad, vd = sizeof(double) * t.npad;
  t.eA = (int *)take(vi);
  t.cA = (int *)take(vi);
  t.eX = (int *)take(vi);
  t.cX = (int *)take(vi);
  t.eR = (int *)take(vi);
  t.eE = (int *)take(vi);
  t.flags = (int *)take(256);
  t.colmap = (int *)take(vi);
  for (int q = 0; q < 3; ++q) t.dcut[q] = (int *)take(vi);
  t.mxA = (double *)take(vd);
  t.mxX = (double *)take(vd);
  t.lam = (double *)take(vd);
  t.lam_lo = (double *)take(vd);
  t.r = (double *)take(vd);
  t.resmax = (double *)take(vd);
  t.emax = (double *)take(vd);
  if (w) *w = t;
  return off;
}

// Residue weights of k digit planes for N odd moduli m_q <= 255: w_qt = 128^(k-1-t) mod m_q
// in the symmetric range (|w| <= 127), also packed four planes to a dword for the dot4
// products of the residue kernel.
void res_weights(int k, int N, const int *mods, ResWeights &rw) {
  rw.N = N;
  rw.k = k;
  for (int q = 0; q < N; ++q) {
    const int m = mods[q];
    rw.m[q] = m;
    rw.rmf[q] = 1.0f / (float)m;
    for (int t = 0; t < kCrtPlanes; ++t) rw.w[q][t] = 0;
    // 128^(k-1-t) mod m, from the least significant digit up, in the symmetric range
    auto sym = [m](long long v) { return (int)(v > m / 2 ? v - m : v); };
    long long pw = 1;
    for (int t = k - 1; t >= 0; --t) {
      rw.w[q][t] = sym(pw);
      pw = pw * 128 % m;
    }
    for (int g = 0; g < (kCrtPlanes + 3) / 4; ++g) {
      unsigned v = 0u;
      for (int i = 0; i < 4 && 4 * g + i < kCrtPlanes; ++i)
        v |= ((unsigned)rw.w[q][4 * g + i] & 0xffu) << (8 * i);
      rw.wp[q][g] = (int)v;
    }
  }
}

// Plans V = P 2^(eA_i + eX_j - 7 (ka1 + kx)) with P = A~ X~ (ka1 digits of A, kx of X^(1),
// reduction length npad): enough moduli that prod m_q > 4 2^hbits 128^(ka1 + kx) (so
// |P| < M / 4), the digit weights of both residue passes and the reconstruction record.
// False when more than kCrtMax moduli would be needed.
// hbits (optional): log2 of a bound on ||a_i|| 2^-eA_i times ||x_j|| 2^-eX_j over all rows
// and columns (Cauchy-Schwarz: |P_ij| <= ||A~_i|| ||X~_j|| <= 2^(hbits + 7 (ka1 + kx)));
// log2(npad) (the bound for any input) when absent or larger.
bool crt_plan(int npad, int ka1, int kx, ResWeights &wA, ResWeights &wX, CrtRec &rec,
              double hbits = -1.0) {
  const int N = crt_count(crt_need_bits(npad, ka1, kx, hbits));
  if (N < 0 || ka1 > kCrtPlanes || kx > kCrtPlanes) return false;
  res_weights_build(ka1, N, wA);
  res_weights_build(kx, N, wX);
  crt_rec_build(N, ka1, kx, rec);
  return true;
}

int ka_of(const refeig_opts *o) {
  int ka = (o && o->ka_max > 0) ? o->ka_max : kKaMaxLimit;
  return std::min(ka, kKaMaxLimit);
}


// Per-column pair cutoffs -> per GEMM tile (max over its columns, the block
// computes those diagonals anyway), expanded back to every column and uploaded
// for the epilogues; tiles with equal cutoffs are grouped for one launch each.
// *pairs_eff = kept slice products in units of one n x n x n product.
struct CutPlan {
  int dmax = 2;
  double pairs_eff = 0.0;
  std::vector<std::pair<int, RowBlocks>> groups;  // (last diagonal, row blocks)
};
bool plan_cutoffs(const std::vector<int> &dcol, int n, int npad, int kl, int kr, int dmax_allowed,
                  int *dev, std::vector<int> &host, hipStream_t s, CutPlan &plan) {
  const int tr = gemm_tile_rows(npad);
  host.assign(npad, 2);
  plan = CutPlan();
  std::vector<int> dtile;
  for (int t0 = 0; t0 < npad; t0 += tr) {
    int dt = 2;
    for (int j = t0; j < std::min(t0 + tr, n); ++j) dt = std::max(dt, dcol[j]);
    dt = std::min(dt, dmax_allowed);
    for (int j = t0; j < t0 + tr; ++j) host[j] = dt;
    dtile.push_back(dt);
    plan.dmax = std::max(plan.dmax, dt);
    int pr = 0;
    for (int d = 2; d <= dt; ++d) pr += npairs_of(d, kl, kr);
    plan.pairs_eff += pr * (double)tr / npad;
  }
  for (int dv = plan.dmax; dv >= 2; --dv) {
    RowBlocks rb;
    rb.count = 0;
    for (int t = 0; t < (int)dtile.size(); ++t)
      if (dtile[t] == dv) rb.m[rb.count++] = t;
    if (rb.count) plan.groups.emplace_back(dv, rb);
  }
  return hipMemcpyAsync(dev, host.data(), sizeof(int) * npad, hipMemcpyHostToDevice, s) ==
         hipSuccess;
}

// One launch per group; ev_start is taken by the first dispatch, ev_stop by the last.
// Block order of the 256 x 256 kernel within one (group, diagonal): a launch-local block
// id -> (index into the group's row blocks, column block). Blocks go round-robin to the 8
// XCDs (id mod 8), each with its own L2; with tiles_n a multiple of 8 XCD x owns the column
// blocks x, 15 - x, 16 + x, ... and walks them in groups of up to 8 row blocks (the kernel's
// own order without a table).

// One launch per product (npad >= 1024): the blocks of every group and diagonal in one table,
// the diagonals with the most pairs first, so blocks of all groups share the chip and the
// launch ends on light blocks (with per-tile cutoffs many blocks exit at once, and one launch
// per group would end on its few heavy blocks). Uploaded to dev; returns the block count (0:
// npad < 1024, one launch per group).
int prepare_table(const CutPlan &plan, int npad, int kl, int kr, std::vector<int> &tab, int *dev,
                  hipStream_t s) {
  if (npad < 1024 || !dev) return 0;
  const int tiles_n = npad / 256;
  std::vector<std::pair<int, std::pair<int, int>>> combos;   // (-pairs, (group, slot))
  for (int g = 0; g < (int)plan.groups.size(); ++g)
    for (int q = 0; q + 2 <= plan.groups[g].first; ++q)
      combos.push_back({-npairs_of(2 + q, kl, kr), {g, q}});
  std::stable_sort(combos.begin(), combos.end(),
                   [](const auto &a, const auto &b) { return a.first < b.first; });
  tab.clear();
  for (const auto &c : combos) {
    const RowBlocks &rb = plan.groups[c.second.first].second;
    const int q = c.second.second;
    for (int b = 0; b < rb.count * tiles_n; ++b) {
      int mi, nb;
      xcd_tile_order(b, rb.count, tiles_n, mi, nb);
      tab.push_back(rb.m[mi] | (nb << 8) | (q << 16));
    }
  }
  if (tab.empty()) return 0;
  if (hipMemcpyAsync(dev, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return -1;
  return (int)tab.size();
}

void launch_plan(const CutPlan &plan, const int8_t *Lp, const int8_t *Rp, size_t P, int npad,
                 int kl, int kr, int32_t *C, hipStream_t s, hipEvent_t ev_start,
                 hipEvent_t ev_stop, int kdim = 0, const int *tcut = nullptr,
                 const int *tab = nullptr, int nblocks = 0) {
  if (tab && nblocks > 0) {
    launch_slice_gemm_table(Lp, Rp, P, npad, kl, kr, 2, tab, nblocks, C, s, ev_start, ev_stop,
                            kdim, tcut);
    return;
  }
  const size_t ng = plan.groups.size();
  for (size_t q = 0; q < ng; ++q)
    launch_slice_gemm(Lp, Rp, P, npad, kl, kr, 2, plan.groups[q].first - 1, C,
                      &plan.groups[q].second, s, q == 0 ? ev_start : nullptr,
                      q + 1 == ng ? ev_stop : nullptr, kdim, false, tcut);
}

// ---------------------------------------------------------------- grouped correction (host)
// Double-word arithmetic for the small Rayleigh-Ritz problems (k <= kGroupMax).
struct HD {
  double h, l;
};
inline HD hd(double a) { return {a, 0.0}; }
inline HD hd_two_sum(double a, double b) {
  double s = a + b, z = s - a;
  return {s, (a - (s - z)) + (b - z)};
}
inline HD hd_norm(double h, double l) {
  double s = h + l;
  return {s, l - (s - h)};
}
inline HD hd_add(HD a, HD b) {
  HD s = hd_two_sum(a.h, b.h);
  HD t = hd_two_sum(a.l, b.l);
  s.l += t.h;
  s = hd_norm(s.h, s.l);
  s.l += t.l;
  return hd_norm(s.h, s.l);
}
inline HD hd_neg(HD a) { return {-a.h, -a.l}; }
inline HD hd_sub(HD a, HD b) { return hd_add(a, hd_neg(b)); }
inline HD hd_mul(HD a, HD b) {
  double p = a.h * b.h;
  double e = std::fma(a.h, b.h, -p);
  e += a.h * b.l + a.l * b.h;
  return hd_norm(p, e);
}
inline HD hd_div(HD a, HD b) {
  double q1 = a.h / b.h;
  HD r = hd_sub(a, hd_mul(b, hd(q1)));
  double q2 = r.h / b.h;
  r = hd_sub(r, hd_mul(b, hd(q2)));
  double q3 = r.h / b.h;
  return hd_add(hd_norm(q1, q2), hd(q3));
}
inline HD hd_sqrt(HD a) {
  if (!(a.h > 0.0)) return hd(0.0);
  double x = std::sqrt(a.h);
  HD r = hd_sub(a, hd_mul(hd(x), hd(x)));
  return hd_norm(x, r.h / (2.0 * x));
}

// Ritz pairs of one group: G (k x k, double-word Gram matrix of the members' columns),
// Wg (k x k, w_ab), lamg (current double-word eigenvalue estimates). T = W + G diag(lambda),
// symmetrised; T y = mu G y through the Cholesky factor of G and Jacobi rotations (FP64,
// then double-word). Each member keeps the Ritz vector with its largest entry (greedily, first
// indices on ties), signed so that entry is positive. Y row-major, Y[a][b] = entry a of
// member b's vector. Returns false if G is not positive definite.
bool group_ritz(int k, const std::vector<HD> &G, const std::vector<double> &Wg,
                const std::vector<HD> &lamg, double *Y, double *mu, double *mu_lo) {
  std::vector<HD> T(k * k), L(k * k, hd(0.0)), M(k * k), Q(k * k), Z(k * k);
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) T[a * k + b] = hd_add(hd(Wg[a * k + b]), hd_mul(G[a * k + b], lamg[b]));
  for (int a = 0; a < k; ++a)
    for (int b = a + 1; b < k; ++b) {
      HD m = hd_add(T[a * k + b], T[b * k + a]);
      m = {0.5 * m.h, 0.5 * m.l};
      T[a * k + b] = T[b * k + a] = m;
    }
  for (int a = 0; a < k; ++a) {
    HD d = G[a * k + a];
    for (int c = 0; c < a; ++c) d = hd_sub(d, hd_mul(L[a * k + c], L[a * k + c]));
    if (!(d.h > 0.0)) return false;
    L[a * k + a] = hd_sqrt(d);
    for (int b = a + 1; b < k; ++b) {
      HD v = G[b * k + a];
      for (int c = 0; c < a; ++c) v = hd_sub(v, hd_mul(L[b * k + c], L[a * k + c]));
      L[b * k + a] = hd_div(v, L[a * k + a]);
    }
  }
  // Z = L^-1 T, then M = Z L^-T
  for (int b = 0; b < k; ++b)
    for (int a = 0; a < k; ++a) {
      HD v = T[a * k + b];
      for (int c = 0; c < a; ++c) v = hd_sub(v, hd_mul(L[a * k + c], Z[c * k + b]));
      Z[a * k + b] = hd_div(v, L[a * k + a]);
    }
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      HD v = Z[a * k + b];
      for (int c = 0; c < b; ++c) v = hd_sub(v, hd_mul(M[a * k + c], L[b * k + c]));
      M[a * k + b] = hd_div(v, L[b * k + b]);
    }
  for (int a = 0; a < k; ++a)
    for (int b = a + 1; b < k; ++b) {
      HD m = hd_add(M[a * k + b], M[b * k + a]);
      m = {0.5 * m.h, 0.5 * m.l};
      M[a * k + b] = M[b * k + a] = m;
    }
  // Eigenvectors of M. Cyclic Jacobi in FP64 on the high parts first; its basis Qf is made
  // orthonormal to double-word accuracy by one Newton-Schulz step, Q1 = Qf (3I - Qf^T Qf) / 2;
  // then double-word Jacobi sweeps on the nearly diagonal Q1^T M Q1 finish the job (one or two
  // sweeps), and Q = Q1 Qd.
  std::vector<double> Mf(k * k), Qf(k * k);
  for (int q = 0; q < k * k; ++q) Mf[q] = M[q].h;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) Qf[a * k + b] = a == b ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double dmax = 0.0, off = 0.0;
    for (int a = 0; a < k; ++a) dmax = std::max(dmax, std::fabs(Mf[a * k + a]));
    for (int a = 0; a < k; ++a)
      for (int b = a + 1; b < k; ++b) off = std::max(off, std::fabs(Mf[a * k + b]));
    if (off == 0.0 || off <= 1e-17 * dmax) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = Mf[p * k + q];
        if (apq == 0.0) continue;
        const double th = (Mf[q * k + q] - Mf[p * k + p]) / (2.0 * apq);
        const double at = std::fabs(th);
        double t = at > 1e150 ? 0.5 / at : 1.0 / (at + std::sqrt(at * at + 1.0));
        if (th < 0.0) t = -t;
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < k; ++r) {
          const double mp = Mf[r * k + p], mq = Mf[r * k + q];
          Mf[r * k + p] = c * mp - sn * mq;
          Mf[r * k + q] = sn * mp + c * mq;
        }
        for (int r = 0; r < k; ++r) {
          const double mp = Mf[p * k + r], mq = Mf[q * k + r];
          Mf[p * k + r] = c * mp - sn * mq;
          Mf[q * k + r] = sn * mp + c * mq;
        }
        for (int r = 0; r < k; ++r) {
          const double qp = Qf[r * k + p], qq = Qf[r * k + q];
          Qf[r * k + p] = c * qp - sn * qq;
          Qf[r * k + q] = sn * qp + c * qq;
        }
      }
  }
  auto dd_matmul = [&](const std::vector<HD> &A_, bool transA, const std::vector<HD> &B_,
                       std::vector<HD> &C_) {
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        HD acc = hd(0.0);
        for (int c = 0; c < k; ++c)
          acc = hd_add(acc, hd_mul(transA ? A_[c * k + a] : A_[a * k + c], B_[c * k + b]));
        C_[a * k + b] = acc;
      }
  };
  std::vector<HD> Q0(k * k), N(k * k), Q1(k * k), Mt(k * k);
  for (int q = 0; q < k * k; ++q) Q0[q] = hd(Qf[q]);
  dd_matmul(Q0, true, Q0, N);                          // N = Qf^T Qf
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      HD v = hd_neg(N[a * k + b]);
      if (a == b) v = hd_add(v, hd(3.0));
      N[a * k + b] = {0.5 * v.h, 0.5 * v.l};         // (3I - N) / 2
    }
  dd_matmul(Q0, false, N, Q1);                         // Q1 = Qf (3I - N) / 2
  dd_matmul(M, false, Q1, Z);                          // Z = M Q1
  dd_matmul(Q1, true, Z, Mt);                          // Mt = Q1^T M Q1
  for (int a = 0; a < k; ++a)
    for (int b = a + 1; b < k; ++b) {
      HD m = hd_add(Mt[a * k + b], Mt[b * k + a]);
      m = {0.5 * m.h, 0.5 * m.l};
      Mt[a * k + b] = Mt[b * k + a] = m;
    }
  std::vector<HD> Qd(k * k);
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) Qd[a * k + b] = hd(a == b ? 1.0 : 0.0);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double dmax = 0.0, off = 0.0;
    for (int a = 0; a < k; ++a) dmax = std::max(dmax, std::fabs(Mt[a * k + a].h));
    for (int a = 0; a < k; ++a)
      for (int b = a + 1; b < k; ++b) off = std::max(off, std::fabs(Mt[a * k + b].h));
    if (off == 0.0 || off <= 1e-32 * dmax) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const HD apq = Mt[p * k + q];
        if (apq.h == 0.0) continue;
        const HD th = hd_div(hd_sub(Mt[q * k + q], Mt[p * k + p]), {2.0 * apq.h, 2.0 * apq.l});
        const HD at = th.h < 0.0 ? hd_neg(th) : th;
        HD t = at.h > 1e30 ? hd_div(hd(0.5), at)
                           : hd_div(hd(1.0), hd_add(at, hd_sqrt(hd_add(hd_mul(at, at), hd(1.0)))));
        if (th.h < 0.0) t = hd_neg(t);
        const HD c = hd_div(hd(1.0), hd_sqrt(hd_add(hd_mul(t, t), hd(1.0))));
        const HD sn = hd_mul(t, c);
        for (int r = 0; r < k; ++r) {
          const HD mp = Mt[r * k + p], mq = Mt[r * k + q];
          Mt[r * k + p] = hd_sub(hd_mul(c, mp), hd_mul(sn, mq));
          Mt[r * k + q] = hd_add(hd_mul(sn, mp), hd_mul(c, mq));
        }
        for (int r = 0; r < k; ++r) {
          const HD mp = Mt[p * k + r], mq = Mt[q * k + r];
          Mt[p * k + r] = hd_sub(hd_mul(c, mp), hd_mul(sn, mq));
          Mt[q * k + r] = hd_add(hd_mul(sn, mp), hd_mul(c, mq));
        }
        for (int r = 0; r < k; ++r) {
          const HD qp = Qd[r * k + p], qq = Qd[r * k + q];
          Qd[r * k + p] = hd_sub(hd_mul(c, qp), hd_mul(sn, qq));
          Qd[r * k + q] = hd_add(hd_mul(sn, qp), hd_mul(c, qq));
        }
      }
  }
  dd_matmul(Q1, false, Qd, Q);                         // Q = Q1 Qd
  M = Mt;                                              // Ritz values on the diagonal
  // Ritz vectors V = L^-T Q (columns), by back substitution
  std::vector<HD> V(k * k);
  for (int b = 0; b < k; ++b)
    for (int a = k - 1; a >= 0; --a) {
      HD v = Q[a * k + b];
      for (int c = a + 1; c < k; ++c) v = hd_sub(v, hd_mul(L[c * k + a], V[c * k + b]));
      V[a * k + b] = hd_div(v, L[a * k + a]);
    }
  std::vector<char> used_v(k, 0), used_c(k, 0);
  for (int step = 0; step < k; ++step) {
    int ba = -1, bv = -1;
    double best = -1.0;
    for (int a = 0; a < k; ++a) {
      if (used_c[a]) continue;
      for (int v = 0; v < k; ++v) {
        if (used_v[v]) continue;
        const double x = std::fabs(V[a * k + v].h);
        if (x > best) {
          best = x;
          ba = a;
          bv = v;
        }
      }
    }
    used_c[ba] = used_v[bv] = 1;
    mu[ba] = M[bv * k + bv].h;
    mu_lo[ba] = M[bv * k + bv].l;
    const double sg = V[ba * k + bv].h < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < k; ++r) Y[r * k + ba] = sg * V[r * k + bv].h;
  }
  return true;
}

int uf_root(std::vector<int> &par, int a) {
  while (par[a] != a) {
    par[a] = par[par[a]];
    a = par[a];
  }
  return a;
}

// xi of beta: the option, else min(k^2, n) under the sparse rule (Sec. 4.3), else n
// (the dense rule of Sec. 4.1).
double xi_of(const refeig_opts &o, int n) {
  if (o.xi > 0.0) return o.xi;
  if (o.sparse_k > 0) return std::min((double)o.sparse_k * o.sparse_k, (double)n);
  return (double)n;
}
// log2 of the statistical error growth of a product with A: sqrt(n) for dense A,
// min(k, sqrt(n)) under the sparse rule.
double lgrowth_of(const refeig_opts &o, int n) {
  const double sq = std::sqrt((double)n);
  return plan_log2(o.sparse_k > 0 ? std::min((double)o.sparse_k, sq) : sq);
}

// beta of Sec. 4.1 (floor form): beta = floor(log2((1/(0.75u)) sqrt(xi delta g / (L S)))),
// evaluated as q = ((xi*delta)*g)/(L*S), t = sqrt(q)/(0.75*2^-53), beta = exponent(t) - 1.
// kx = ceil((54 - beta + max_j(e_j - c_j)) / 7): the X^(1) grid 2^(c_j+beta-54) is the
// rounding bound u*ufp(tau_j) of eq. (minamihata).
void beta_rule(int n, double xi, double delta, double g, double L, const std::vector<int> &e,
               const std::vector<int> &c, const std::vector<double> &mx, int *beta, int *kx) {
  std::vector<int> hist(kBetaBins, 0);
  int extra = 0;
  for (int j = 0; j < n; ++j) {
    if (mx[j] == 0.0) continue;
    const int b = std::min(kBetaBins - 1, std::max(0, 2 * c[j] + kBetaBias));
    ++hist[b];
    extra = std::max(extra, e[j] - c[j]);
  }
  beta_core(xi, delta, g, L, pow2_sum(hist.data()), extra, beta, kx);
}

// Working column order: by gap, widest first; ties (two columns share a gap) go by
// eigenvalue, so the order does not depend on where the caller put the columns.
void working_order(const std::vector<double> &lam, const std::vector<double> &gaps,
                   std::vector<int> &order) {
  const int n = (int)lam.size();
  order.resize(n);
  for (int p = 0; p < n; ++p) order[p] = p;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return gaps[a] != gaps[b] ? gaps[a] > gaps[b] : lam[a] < lam[b];
  });
}

// Per-column distance to the nearest other eigenvalue estimate.
void column_gaps(const std::vector<double> &lam, std::vector<double> &g, double *gmin,
                 double *lmax) {
  const int n = (int)lam.size();
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  g.assign(n, INFINITY);
  double m = INFINITY, L = 0.0;
  for (int p = 0; p + 1 < n; ++p) {
    double d = lam[idx[p + 1]] - lam[idx[p]];
    g[idx[p]] = std::min(g[idx[p]], d);
    g[idx[p + 1]] = std::min(g[idx[p + 1]], d);
    m = std::min(m, d);
  }
  for (int i = 0; i < n; ++i) L = std::max(L, std::fabs(lam[i]));
  if (n == 1) {
    g[0] = 1.0;
    m = 1.0;
  }
  *gmin = m;
  *lmax = L;
}

// ---- FP64 plain form: the same iteration with FP64-slice products on DGEMM.
// V = sum over kept pairs of A_row^(r) X^(s), every product exact in FP64 because
// both slices carry b = 53 - alpha bits with 2 alpha >= 53 + log2 n (Sec. 2.3,
// eq. alp_beta with alpha = beta); W and X^(1) E~ are single DGEMMs.
int refine_plain(const double *A, int lda, double *X, int ldx, double *D, int n, double target,
                 const refeig_opts &o, void *work, size_t work_bytes, hipStream_t s,
                 refeig_report *rep) {
  const int verbose = o.verbose;
  const size_t need = carve_plain(n, nullptr, nullptr);
  bool own = false;
  if (!work) {
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMalloc(&work, need));
    own = true;
  } else if (work_bytes < need) {
    return REFEIG_E_NOMEM;
  }
  PlainWork w;
  carve_plain(n, (char *)work, &w);
  const int npad = round_up(n, kTile);
  const size_t nn = (size_t)n * n;
  const double delta_int = target / o.delta_safety;
  const double xi = xi_of(o, n);
  const double lgrowth_a = lgrowth_of(o, n);   // error growth of products of A's planes
  const int alpha = (int)std::ceil((53.0 + plan_log2((double)n)) / 2.0);
  const int b = 53 - alpha;  // bits per FP64 slice
  auto t_start = std::chrono::steady_clock::now();
  rocblas_handle hb = nullptr;
  std::vector<int> eX(npad), cX(npad), eA(npad), cA(npad);
  std::vector<double> mxX(npad), mxA(npad), lam(n), lam_prev(n), gaps;
  std::vector<unsigned long long> cm(npad);
  int hflags = 0, status = REFEIG_OK;
  hipEvent_t ev[4];
  for (auto &e : ev) HIPCHK(hipEventCreate(&e));
  auto cleanup = [&](int st) {
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (hb) (void)rocblas_destroy_handle(hb);
    if (own) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(work);
    }
    if (rep) {
      rep->status = st;
      rep->ms_total =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
              .count();
    }
    return st;
  };
#define PSTEP(x)                                                                            \
  do {                                                                                      \
    hipError_t err__ = (x);                                                                 \
    if (err__ != hipSuccess) {                                                              \
      fprintf(stderr, "refeig: %s failed: %s\n", #x, hipGetErrorString(err__));             \
      return cleanup(REFEIG_E_HIP);                                                         \
    }                                                                                       \
  } while (0)
#define BSTEP(x)                                                                            \
  do {                                                                                      \
    if ((x) != rocblas_status_success) {                                                    \
      fprintf(stderr, "refeig: %s failed\n", #x);                                           \
      return cleanup(REFEIG_E_HIP);                                                         \
    }                                                                                       \
  } while (0)
  BSTEP(rocblas_create_handle(&hb));
  BSTEP(rocblas_set_stream(hb, s));
  const double one = 1.0, zero = 0.0;

  PSTEP(hipMemcpyAsync(lam_prev.data(), D, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  PSTEP(hipMemsetAsync(w.flags, 0, sizeof(int), s));
  // A: its columns are its rows (symmetric); kPlainKaMax FP64 slices per column
  launch_colstats(A, lda, n, n, npad, w.eX, w.cX, w.mxX, w.flags, s);
  PSTEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  PSTEP(hipMemcpyAsync(eA.data(), w.eX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
  PSTEP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(lam_prev[i])) return cleanup(REFEIG_E_NONFINITE);
  if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
  if (hflags & FLAG_RANGE) return cleanup(REFEIG_E_RANGE);
  int eA_max = -100000;
  for (int i = 0; i < n; ++i) eA_max = std::max(eA_max, eA[i]);
  launch_sigma_split_cols(A, lda, n, alpha, kPlainKaMax, w.SA, s);

  const int iters = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  double eps_prev = INFINITY;
  for (int it = 0; it < iters; ++it) {
    PSTEP(hipEventRecord(ev[0], s));
    launch_colstats(X, ldx, n, n, npad, w.eX, w.cX, w.mxX, w.flags, s);
    PSTEP(hipMemcpyAsync(eX.data(), w.eX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    PSTEP(hipMemcpyAsync(cX.data(), w.cX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    PSTEP(hipMemcpyAsync(mxX.data(), w.mxX, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    PSTEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    PSTEP(hipStreamSynchronize(s));
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    double gmin, lmax;
    column_gaps(lam_prev, gaps, &gmin, &lmax);
    if (!(gmin > 0.0)) return cleanup(REFEIG_E_GAP);
    int beta, kx_unused;
    beta_rule(n, xi, delta_int, gmin, lmax, eX, cX, mxX, &beta, &kx_unused);
    launch_x1_rn(X, ldx, n, w.cX, w.mxX, beta, w.X1, s);
    const int kx = std::min(kPlainKxMax, std::max(1, (54 - beta + b - 1) / b));
    launch_sigma_split_cols(w.X1, n, n, alpha, kx, w.SX, s);
    int eXmax = -100000;
    for (int j = 0; j < n; ++j) eXmax = std::max(eXmax, eX[j]);
    int dv = 2;
    for (int j = 0; j < n; ++j) {
      if (mxX[j] == 0.0) continue;
      double need_bits = eA_max + eX[j] + b + plan_log2(1.5 * kx) + lgrowth_a -
                         plan_log2(o.theta * delta_int * gaps[j]);
      dv = std::max(dv, (int)std::ceil(need_bits / b));
    }
    dv = std::min(dv + o.d_extra, kPlainKaMax + kx);
    // V: pairs (r, s) with r + s <= dv, summed from the smallest weight up
    PSTEP(hipEventRecord(ev[1], s));
    int pv = 0;
    for (int d = dv; d >= 2; --d)
      for (int sx = 1; sx <= kx; ++sx) {
        const int ra = d - sx;
        if (ra < 1 || ra > kPlainKaMax) continue;
        BSTEP(rocblas_dgemm(hb, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &one,
                            w.SA + (size_t)(ra - 1) * nn, n, w.SX + (size_t)(sx - 1) * nn, n,
                            &zero, w.P, n));
        launch_dd_accum(w.P, w.Vh, w.Vl, nn, pv == 0, s);
        ++pv;
      }
    PSTEP(hipEventRecord(ev[2], s));
    launch_colpass_dd(w.Vh, w.Vl, w.X1, n, w.lam, w.r, w.Res, w.flags, s);
    // W = X1^T Res, E~, U = X1 E~, X = X1 + U
    BSTEP(rocblas_dgemm(hb, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &one,
                        w.X1, n, w.Res, n, &zero, w.P, n));
    PSTEP(hipMemsetAsync(w.colmax, 0, sizeof(unsigned long long) * npad, s));
    launch_etilde(w.P, w.lam, w.r, n, w.E, w.colmax, w.flags, s);
    BSTEP(rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, w.X1, n,
                        w.E, n, &zero, w.P, n));
    launch_update(w.X1, w.P, n, X, ldx, s);
    PSTEP(hipMemcpyAsync(D, w.lam, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    PSTEP(hipMemcpyAsync(lam.data(), w.lam, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    PSTEP(hipMemcpyAsync(cm.data(), w.colmax, sizeof(unsigned long long) * n,
                         hipMemcpyDeviceToHost, s));
    PSTEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    PSTEP(hipEventRecord(ev[3], s));
    PSTEP(hipGetLastError());
    PSTEP(hipStreamSynchronize(s));
    if (hflags & 2) return cleanup(REFEIG_E_GAP);
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    double eps = 0.0;
    for (int j = 0; j < n; ++j) {
      double v;
      std::memcpy(&v, &cm[j], sizeof(v));
      eps = std::max(eps, v);
    }
    float t_it = 0, tv = 0;
    (void)hipEventElapsedTime(&t_it, ev[0], ev[3]);
    (void)hipEventElapsedTime(&tv, ev[1], ev[2]);
    column_gaps(lam, gaps, &gmin, &lmax);
    if (rep && it < REFEIG_MAX_ITERS) {
      rep->beta[it] = beta;
      rep->kx[it] = kx;
      rep->dv[it] = dv;
      rep->dw[it] = 0;
      rep->du[it] = 0;
      rep->pairs[it] = pv + 2;
      rep->pairs_p[it][0] = pv;
      rep->pairs_p[it][1] = 1;
      rep->pairs_p[it][2] = 1;
      rep->pairs_f[it][0] = pv;
      rep->pairs_f[it][1] = 1;
      rep->pairs_f[it][2] = 1;
      rep->ms_p[it][0] = tv;
      rep->eps[it] = eps;
      rep->ms_iter[it] = t_it;
      rep->ms_gemm[it] = tv;
      rep->iters = it + 1;
      rep->min_gap = gmin;
      rep->max_abs_lambda = lmax;
    }
    if (verbose)
      fprintf(stderr, "refeig plain it %d: beta %d slices A %d X %d (b=%d) dv %d dgemm %d eps %.3e "
                      "ms %.2f (V %.2f)\n", it + 1, beta, kPlainKaMax, kx, b, dv, pv + 2, eps, t_it, tv);
    lam_prev = lam;
    if (o.fixed_iters > 0) continue;
    const double xi_stop = (o.stop_rule == 1) ? 1.0 : xi;
    if (eps <= delta_int || eps * eps * lmax / (xi_stop * gmin) <= delta_int) break;
    if (it >= 1 && eps > 0.5 * eps_prev) {
      // no quadratic decrease: the floor that the products' truncation leaves. When that
      // floor is within the target the iterate has converged to it, else it has stagnated.
      if (eps > target) status = REFEIG_NOT_CONVERGED;
      break;
    }
    eps_prev = eps;
    if (it + 1 == iters) status = REFEIG_NOT_CONVERGED;
  }
  return cleanup(status);
#undef PSTEP
#undef BSTEP
}

// ---------------------------------------------------------------- complex Hermitian case
// Algorithm 1 with the X^(1) cut for A = A^H (the extension Sec. 5 names as future work):
// the same iteration as the real INT8 loop, with complex operands realified so that every
// complex product is two real slice GEMMs of reduction length 2 npad:
//   V = A X^(1):   Re V = (Re a_i ; Im a_i) . (Re x_j ; Im x_j),
//                  Im V = (-Im a_i ; Re a_i) . (Re x_j ; Im x_j)      (a_i: column i of A)
//   W = X^(1)H R:  Re W = (Re x_i ; Im x_i) . (Re r_j ; Im r_j),
//                  Im W = (Re x_i ; Im x_i) . (Im r_j ; -Re r_j)
//   U = X^(1) E':  Re U = (Re X_i. ; -Im X_i.) . (Re e'_j ; Im e'_j),
//                  Im U = (Re X_i. ; -Im X_i.) . (Im e'_j ; -Re e'_j)
// Options beyond the paper's method (grouping, schedule, sparse rule, FP64 form) are not
// offered here.
int refine_herm(const double *A, int lda, double *X, int ldx, double *D, int n, double target,
                const refeig_opts &o, void *work, size_t work_bytes, hipStream_t s,
                refeig_report *rep) {
  const int ka_max = ka_of(&o);
  const size_t need = carve_herm(n, ka_max, nullptr, nullptr);
  bool own = false;
  if (!work) {
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMalloc(&work, need));
    own = true;
  } else if (work_bytes < need) {
    return REFEIG_E_NOMEM;
  }
  HermWork w;
  carve_herm(n, ka_max, (char *)work, &w);
  const int npad = w.npad;
  const size_t P2 = 2 * w.P;
  const int K2 = 2 * npad;
  const double delta = target / o.delta_safety;
  const double xi = xi_of(o, n);
  const double theta = o.theta;
  const double lsq2n = 0.5 * plan_log2(2.0 * n);   // statistical growth over 2n real terms
  auto t_start = std::chrono::steady_clock::now();

  int status = REFEIG_OK;
  std::vector<int> eX(npad), cX(npad), eR(npad), eE(npad), eA(npad);
  std::vector<double> mxX(npad), lam(n), lam_prev(n), resmax(npad), emax(npad), gaps, gaps_nat;
  std::vector<int> cmap(n), dhost;
  int hflags = 0;
  hipEvent_t ev[8];
  for (auto &e : ev) HIPCHK(hipEventCreate(&e));
  auto cleanup = [&](int st) {
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (own) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(work);
    }
    if (rep) {
      rep->status = st;
      rep->ms_total =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
              .count();
    }
    return st;
  };
#define STEP(x)                                   \
  do {                                            \
    hipError_t err__ = (x);                       \
    if (err__ != hipSuccess) {                    \
      fprintf(stderr, "refeig: %s failed: %s\n", #x, hipGetErrorString(err__)); \
      return cleanup(REFEIG_E_HIP);               \
    }                                             \
  } while (0)

  STEP(hipMemcpyAsync(lam_prev.data(), D, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  STEP(hipMemsetAsync(w.flags, 0, sizeof(int), s));
  // A: column exponents over both parts (column i realified = operand row i) and the planes
  // of (Re a_i ; Im a_i) and (-Im a_i ; Re a_i), once
  launch_colstats_c(A, lda, n, n, npad, w.eA, w.cA, w.mxA, w.flags, s);
  STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  STEP(hipMemcpyAsync(eA.data(), w.eA, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
  STEP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(lam_prev[i])) return cleanup(REFEIG_E_NONFINITE);
  if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
  if (hflags & FLAG_RANGE) return cleanup(REFEIG_E_RANGE);
  int eA_max = -100000;
  for (int i = 0; i < n; ++i) eA_max = std::max(eA_max, eA[i]);
  launch_split_c(A, lda, n, n, w.eA, ka_max, w.AP1, w.AP2, P2, npad, npad, nullptr, 0, nullptr,
                 0, 0, s);
  STEP(hipGetLastError());

  const int iters = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  double eps_prev = INFINITY;
  for (int it = 0; it < iters; ++it) {
    STEP(hipEventRecord(ev[0], s));
    double gmin, lmax;
    column_gaps(lam_prev, gaps_nat, &gmin, &lmax);
    if (!(gmin > 0.0)) return cleanup(REFEIG_E_GAP);
    working_order(lam_prev, gaps_nat, cmap);
    STEP(hipMemcpyAsync(w.colmap, cmap.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    launch_colstats_c(X, ldx, n, n, npad, w.eX, w.cX, w.mxX, w.flags, s, w.colmap);
    STEP(hipMemcpyAsync(eX.data(), w.eX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(cX.data(), w.cX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(mxX.data(), w.mxX, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    STEP(hipStreamSynchronize(s));
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    if (hflags & FLAG_RANGE) return cleanup(REFEIG_E_RANGE);
    gaps.resize(n);
    for (int p = 0; p < n; ++p) gaps[p] = gaps_nat[cmap[p]];
    int beta, kx;
    beta_rule(n, xi, delta, gmin, lmax, eX, cX, mxX, &beta, &kx);
    if (o.kx_force > 0) kx = o.kx_force;
    // X^(1): column planes (Re x_j ; Im x_j) and row planes (Re X_i. ; -Im X_i.)
    launch_split_c(X, ldx, n, n, w.eX, kx, w.XP, nullptr, P2, npad, npad, w.X1, n, w.XT, P2, kx,
                   s, w.colmap);
    // ---- V = A X^(1)
    int eXmax = -100000;
    for (int j = 0; j < n; ++j) eXmax = std::max(eXmax, eX[j]);
    std::vector<int> dcol(npad, 2);
    {
      const double c0 = eA_max + 7 + plan_log2(1.5 * kx) + lsq2n;
      for (int j = 0; j < n; ++j) {
        if (mxX[j] == 0.0) continue;
        double nd = (c0 + eX[j] - plan_log2(theta * delta * gaps[j])) / 7.0;
        dcol[j] = std::max(2, (int)std::ceil(nd) + o.d_extra);
      }
    }
    CutPlan plan;
    if (!plan_cutoffs(dcol, n, npad, kx, ka_max, std::min(ka_max + 1, kx + ka_max), w.dcut[0],
                      dhost, s, plan))
      return cleanup(REFEIG_E_HIP);
    const int dv = plan.dmax;
    const double pv = plan.pairs_eff;
    launch_plan(plan, w.XP, w.AP1, P2, npad, kx, ka_max, w.Cr, s, ev[1], nullptr, K2);
    launch_plan(plan, w.XP, w.AP2, P2, npad, kx, ka_max, w.Ci, s, nullptr, ev[2], K2);
    launch_epi_v_c(w.Cr, w.Ci, npad, 2, dv - 1, w.dcut[0], w.eA, w.eX, w.X1, n, w.lam, w.lam_lo,
                   w.r, w.eR, w.resmax, w.RP1, w.RP2, kKrMax, w.flags, s);
    STEP(hipMemcpyAsync(lam.data(), w.lam, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(eR.data(), w.eR, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(resmax.data(), w.resmax, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    STEP(hipStreamSynchronize(s));
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    // ---- W = X^(1)H Res -> E~
    column_gaps(lam, gaps, &gmin, &lmax);
    if (!(gmin > 0.0)) return cleanup(REFEIG_E_GAP);
    {
      const double c0 = eXmax + 7 + plan_log2(1.5 * kx) + lsq2n;
      std::fill(dcol.begin(), dcol.end(), 2);
      for (int j = 0; j < n; ++j) {
        if (resmax[j] == 0.0) continue;
        double nd = (c0 + eR[j] - plan_log2(theta * delta * gaps[j])) / 7.0;
        dcol[j] = std::max(2, (int)std::ceil(nd) + o.d_extra);
      }
    }
    if (!plan_cutoffs(dcol, n, npad, kKrMax, kx, std::min(kKrMax + 1, kKrMax + kx), w.dcut[1],
                      dhost, s, plan))
      return cleanup(REFEIG_E_HIP);
    const int dw = plan.dmax;
    const double pw = plan.pairs_eff;
    launch_plan(plan, w.RP1, w.XP, P2, npad, kKrMax, kx, w.Cr, s, ev[3], nullptr, K2);
    launch_plan(plan, w.RP2, w.XP, P2, npad, kKrMax, kx, w.Ci, s, nullptr, ev[4], K2);
    launch_epi_w_c(w.Cr, w.Ci, npad, 2, dw - 1, w.dcut[1], w.eX, w.eR, w.lam, w.lam_lo, w.r, n,
                   w.eE, w.emax, w.EP1, w.EP2, kKeMax, w.flags, s);
    STEP(hipMemcpyAsync(eE.data(), w.eE, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(emax.data(), w.emax, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    STEP(hipStreamSynchronize(s));
    if (hflags & FLAG_TIE) return cleanup(REFEIG_E_GAP);
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    double eps = 0.0;
    for (int j = 0; j < n; ++j) eps = std::max(eps, emax[j]);
    // ---- X <- X^(1) + X^(1) E~ (each column t_j times tighter for noise stability, as in
    // the real path; W here already keeps each column within theta delta g_j)
    {
      const double c0 = 7 + plan_log2(1.008 * kx) + lsq2n - plan_log2(theta * delta);
      std::fill(dcol.begin(), dcol.end(), 2);
      for (int j = 0; j < n; ++j) {
        if (emax[j] == 0.0) continue;
        const double t = std::sqrt(delta * gaps[j] / (4.0 * lmax)) / (theta * delta);
        const double need = (c0 + eE[j] - plan_log2(std::min(1.0, t))) / 7.0;
        dcol[j] = std::max(2, (int)std::ceil(need) + o.d_extra);
      }
    }
    if (!plan_cutoffs(dcol, n, npad, kKeMax, kx, std::min(kKeMax + 1, kKeMax + kx), w.dcut[2],
                      dhost, s, plan))
      return cleanup(REFEIG_E_HIP);
    const int du = plan.dmax;
    const double pu = plan.pairs_eff;
    launch_plan(plan, w.EP1, w.XT, P2, npad, kKeMax, kx, w.Cr, s, ev[5], nullptr, K2);
    launch_plan(plan, w.EP2, w.XT, P2, npad, kKeMax, kx, w.Ci, s, nullptr, ev[6], K2);
    launch_epi_u_c(w.Cr, w.Ci, npad, 2, du - 1, w.dcut[2], w.eE, w.X1, n, X, ldx, s, w.colmap);
    launch_scatter(w.lam, w.colmap, n, D, s);
    STEP(hipEventRecord(ev[7], s));
    STEP(hipGetLastError());
    STEP(hipEventSynchronize(ev[7]));
    float t_it = 0, g1 = 0, g2 = 0, g3 = 0;
    (void)hipEventElapsedTime(&t_it, ev[0], ev[7]);
    (void)hipEventElapsedTime(&g1, ev[1], ev[2]);
    (void)hipEventElapsedTime(&g2, ev[3], ev[4]);
    (void)hipEventElapsedTime(&g3, ev[5], ev[6]);
    if (rep && it < REFEIG_MAX_ITERS) {
      // pair counts per real slice GEMM of reduction 2n; each product runs two of them
      rep->beta[it] = beta;
      rep->kx[it] = kx;
      rep->dv[it] = dv;
      rep->dw[it] = dw;
      rep->du[it] = du;
      rep->pairs[it] = (int)std::lround(2 * (pv + pw + pu));
      rep->eps[it] = eps;
      rep->ms_iter[it] = t_it;
      rep->ms_gemm[it] = g1 + g2 + g3;
      rep->pairs_f[it][0] = 2 * pv;
      rep->pairs_f[it][1] = 2 * pw;
      rep->pairs_f[it][2] = 2 * pu;
      rep->pairs_p[it][0] = (int)std::lround(2 * pv);
      rep->pairs_p[it][1] = (int)std::lround(2 * pw);
      rep->pairs_p[it][2] = (int)std::lround(2 * pu);
      rep->ms_p[it][0] = g1;
      rep->ms_p[it][1] = g2;
      rep->ms_p[it][2] = g3;
      rep->delta_it[it] = delta;
      rep->iters = it + 1;
      rep->min_gap = gmin;
      rep->max_abs_lambda = lmax;
    }
    if (o.verbose)
      fprintf(stderr,
              "refeig herm it %d: beta %d kx %d dv %d dw %d du %d eps %.3e gap %.3e ms %.2f "
              "(gemm %.2f)\n",
              it + 1, beta, kx, dv, dw, du, eps, gmin, t_it, g1 + g2 + g3);
    for (int p = 0; p < n; ++p) lam_prev[cmap[p]] = lam[p];
    if (o.fixed_iters > 0) {
      eps_prev = eps;
      continue;
    }
    const double xi_stop = (o.stop_rule == 1) ? 1.0 : xi;
    if (eps <= delta || eps * eps * lmax / (xi_stop * gmin) <= delta) break;
    if (it >= 1 && eps > 0.5 * eps_prev) {
      // no quadratic decrease: the floor that the products' truncation leaves. When that
      // floor is within the target the iterate has converged to it, else it has stagnated.
      if (eps > target) status = REFEIG_NOT_CONVERGED;
      break;
    }
    eps_prev = eps;
    if (it + 1 == iters) status = REFEIG_NOT_CONVERGED;
  }
  return cleanup(status);
#undef STEP
}

// ---- device-planned solve: every decision of an iteration is made by the planning kernels
// (devplan.hip) from values already on the device, so the host only enqueues.

// Timing events, reused across calls (a call takes a set and returns it).
struct EventPool {
  std::mutex mu;
  std::vector<hipEvent_t> free_;
  std::vector<hipEvent_t> take(size_t k) {
    std::vector<hipEvent_t> out;
    {
      std::lock_guard<std::mutex> lk(mu);
      while (out.size() < k && !free_.empty()) {
        out.push_back(free_.back());
        free_.pop_back();
      }
    }
    while (out.size() < k) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) break;
      out.push_back(e);
    }
    return out;
  }
  void give(std::vector<hipEvent_t> &ev) {
    std::lock_guard<std::mutex> lk(mu);
    for (auto e : ev) free_.push_back(e);
    ev.clear();
  }
};
EventPool &event_pool() {
  static EventPool *p = new EventPool();   // never destroyed: events live with the process
  return *p;
}

constexpr int kEvPerIter = 18;   // as the host-planned solve: iteration, products, phases

void fill_report_from_device(const DevState &st, int flags, int iters_enqueued,
                             refeig_report *rep) {
  const int k = std::min(st.iters_done, REFEIG_MAX_ITERS);
  rep->iters = k;
  for (int it = 0; it < k; ++it) {
    const DevIter &r = st.rep[it];
    rep->beta[it] = r.beta;
    rep->kx[it] = r.kx;
    rep->dv[it] = r.dv;
    rep->dw[it] = r.dw;
    rep->du[it] = r.du;
    rep->eps[it] = r.eps;
    rep->pairs_f[it][0] = r.pv;
    rep->pairs_f[it][1] = r.pw;
    rep->pairs_f[it][2] = r.pu;
    rep->pairs_p[it][0] = (int)std::lround(r.pv);
    rep->pairs_p[it][1] = (int)std::lround(r.pw);
    rep->pairs_p[it][2] = (int)std::lround(r.pu);
    rep->pairs[it] = (int)std::lround(r.pv + r.pw + r.pu);
    rep->launches_p[it][0] = r.lv;
    rep->launches_p[it][1] = r.lw;
    rep->launches_p[it][2] = r.lu;
    rep->vres[it] = r.vres;
    rep->delta_it[it] = r.delta;
    rep->min_gap = r.gmin;
    rep->max_abs_lambda = r.lmax;
  }
  (void)flags;
  (void)iters_enqueued;
}

int status_of(const DevState &st, int flags) {
  if (flags & FLAG_NONFINITE) return REFEIG_E_NONFINITE;
  if (flags & FLAG_RANGE) return REFEIG_E_RANGE;
  if (flags & (FLAG_GAP | FLAG_TIE)) return REFEIG_E_GAP;
  return st.stop_status;
}

// Scalars and device pointers the planning kernels of one solve read (iteration 0).
PlanParams plan_params(int n, int npad, const refeig_opts &o, double target) {
  PlanParams pp;
  pp.n = n;
  pp.npad = npad;
  pp.it = 0;
  pp.iters = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  pp.fixed = o.fixed_iters > 0 ? 1 : 0;
  pp.kx_force = o.kx_force;
  pp.ka_max = ka_of(&o);
  pp.d_extra = o.d_extra;
  pp.vmode = o.vmode;
  pp.stop_rule = o.stop_rule;
  pp.crt = o.vmode == 1 ? 1 : 0;
  pp.theta = o.theta;
  pp.delta_int = target / o.delta_safety;
  pp.delta_k = pp.delta_int;
  pp.xi = xi_of(o, n);
  pp.xi_stop = o.stop_rule == 1 ? 1.0 : pp.xi;
  pp.lgrowth_a = lgrowth_of(o, n);
  pp.lsqn = 0.5 * plan_log2((double)n);
  pp.target = target;
  return pp;
}
PlanBufs plan_bufs(const Work &w, const double *D) {
  PlanBufs pb;
  pb.st = w.dst;
  pb.D = D;
  pb.colmap = w.colmap;
  pb.gapsw = w.gapsw;
  pb.eA = w.eA;
  pb.mxA = w.mxA;
  pb.ssA = w.ssA;
  pb.eX = w.eX;
  pb.cX = w.cX;
  pb.mxX = w.mxX;
  pb.ssX = w.ssX;
  pb.lam = w.lam;
  pb.eR = w.eR;
  pb.resmax = w.resmax;
  pb.eE = w.eE;
  pb.emax = w.emax;
  pb.wtol = w.wtol;
  for (int q = 0; q < 3; ++q) {
    pb.dcut[q] = w.dcut[q];
    pb.tab[q] = w.tab[q];
  }
  pb.vblk = w.vblk;
  pb.tcut = w.npad >= 1024 ? w.tcut : nullptr;
  pb.flags = w.flags;
  pb.mods = w.mods;
  pb.skey = w.skey;
  pb.sidx = w.sidx;
  return pb;
}

// The solve with device planning (INT8 path, no grouping, no schedule). `work` holds at least
// carve(n, ka_max, crt) bytes. enqueue_only: no wait and no event (fixed_iters > 0).
int refine_device(const double *A, int lda, double *X, int ldx, double *D, int n, double target,
                  const refeig_opts &o, void *work, hipStream_t s, refeig_report *rep,
                  bool enqueue_only) {
  const int ka_max = ka_of(&o);
  const bool crt = o.vmode == 1;
  Work w;
  carve(n, ka_max, (char *)work, &w, crt);
  const int npad = w.npad;
  const size_t P = w.P;
  const int iters = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  PlanParams pp = plan_params(n, npad, o, target);
  const PlanBufs pb = plan_bufs(w, D);
  DevState *st = w.dst;
  const int tr = gemm_tile_rows(npad), TT = npad / tr;
  // launch sizes of the tabled products: the largest tables the cutoffs allow
  const int maxv = TT * TT * ka_max;
  const int maxw = TT * TT * kKrMax, maxu = TT * TT * kKeMax;
  const int T256 = npad / 256;
  std::vector<hipEvent_t> ev;
  if (!enqueue_only) ev = event_pool().take((size_t)kEvPerIter * iters);
  const bool timed = !enqueue_only && ev.size() == (size_t)kEvPerIter * iters;
  auto E = [&](int it, int q) -> hipEvent_t { return timed ? ev[(size_t)it * kEvPerIter + q] : nullptr; };
  auto rec = [&](int it, int q) {
    if (timed) (void)hipEventRecord(E(it, q), s);
  };
  auto t_start = std::chrono::steady_clock::now();
  // A: column exponents (= row exponents, A is symmetric) and its digit planes, once
  launch_fill_int(w.flags, 1, 0, s);
  launch_colstats(A, lda, n, n, npad, w.eA, w.cA, w.mxA, w.flags, s, nullptr, w.ssA);
  launch_dp_init(pp, pb, s);
  launch_split_cols(A, lda, n, n, w.eA, ka_max, w.AP, P, npad, npad, nullptr, 0, nullptr, 0, 0, s);
  int it = 0, host_status = REFEIG_OK;
  DevState hst;
  int hflags = 0;
  for (; it < iters; ++it) {
    pp.it = it;
    rec(it, 0);
    launch_dp_order(pp, pb, s);
    rec(it, 8);
    launch_colstats(X, ldx, n, n, npad, w.eX, w.cX, w.mxX, w.flags, s, w.colmap, w.ssX);
    rec(it, 9);
    launch_dp_vplan(pp, pb, s);
    rec(it, 10);
    launch_split_cols(X, ldx, n, n, w.eX, kKxMax, w.XP, P, npad, npad, w.X1, n, w.XPT, P, kKxMax,
                      s, w.colmap, &st->kx);
    rec(it, 11);
    rec(it, 12);
    if (crt) {
      for (int l = 0; l < kVLevels; ++l)
        launch_residues_dev(w.AP, P, P, &st->wA[l], w.ARES + (size_t)l * kCrtMax * P,
                            &st->ares_dirty[l], s);
      launch_residues_dev(w.XP, P, P, &st->wX, w.XRES, &st->vres, s);
      // one launch for all moduli: slots beyond a block's count (0 when V goes by slices) exit
      launch_slice_gemm(w.XRES, w.ARES, P, npad, kCrtMax, kCrtMax, 2, kCrtMax, w.Cs, nullptr, s,
                        E(it, 1), E(it, 2), 0, true, nullptr, w.mods, false, w.vblk);
      launch_epi_v_crt(w.Cs, npad, st->recs, w.vblk, w.eA, w.eX, w.X1, n, w.lam, w.lam_lo, w.r,
                       w.eR, w.resmax, w.RP, kKrMax, w.flags, s, &st->vres);
    }
    // V by slices (vmode 0, or where the reconstruction floor rules residues out): the table
    // is empty otherwise
    launch_slice_gemm_table(w.XP, w.AP, P, npad, kKxMax, ka_max, 2, w.tab[0], maxv, w.Cs, s,
                            crt ? nullptr : E(it, 1), crt ? nullptr : E(it, 2), 0, nullptr,
                            st->gemm_v);
    launch_epi_v(w.Cs, npad, 2, kMaxDiag - 1, w.dcut[0], w.eA, w.eX, w.X1, n, w.lam, w.lam_lo, w.r,
                 w.eR, w.resmax, w.RP, kKrMax, w.flags, s, &st->vslice);
    rec(it, 13);
    rec(it, 14);
    launch_dp_wplan(pp, pb, s);
    if (npad >= 1024)
      launch_tile_cutoffs(w.lam, w.eX, w.eR, w.resmax, n, T256, 0.0, 2, o.d_extra, w.wtol,
                          w.wtol + npad, w.tcut, s, &st->cx, &st->dmax_w);
    launch_slice_gemm_table(w.RP, w.XP, P, npad, kKrMax, kKxMax, 2, w.tab[1], maxw, w.Cs, s,
                            E(it, 3), E(it, 4), 0, npad >= 1024 ? w.tcut : nullptr, st->gemm_w);
    launch_epi_w(w.Cs, npad, 2, kMaxDiag - 1, w.dcut[1], w.eX, w.eR, w.lam, w.lam_lo, w.r, n, w.eE,
                 w.emax, w.EP, kKeMax, w.flags, s, 0.0, nullptr, nullptr, 0,
                 npad >= 1024 ? w.tcut : nullptr);
    rec(it, 15);
    launch_dp_uplan(pp, pb, s);
    rec(it, 16);
    launch_slice_gemm_table(w.EP, w.XPT, P, npad, kKeMax, kKxMax, 2, w.tab[2], maxu, w.Cs, s,
                            E(it, 5), E(it, 6), 0, nullptr, st->gemm_u);
    launch_epi_u(w.Cs, npad, 2, kMaxDiag - 1, w.dcut[2], w.eE, w.X1, n, X, ldx, s, w.colmap,
                 w.flags);
    launch_scatter(w.lam, w.colmap, n, D, s, w.flags);
    rec(it, 17);
    rec(it, 7);
    if (hipGetLastError() != hipSuccess) {
      host_status = REFEIG_E_HIP;
      break;
    }
    if (!pp.fixed) {   // the stop test's decision (one small read per iteration)
      if (hipMemcpyAsync(&hst.done, &st->done, sizeof(int), hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        host_status = REFEIG_E_HIP;
        break;
      }
      if (hst.done) {
        ++it;
        break;
      }
    }
  }
  if (enqueue_only) return host_status;
  if (host_status == REFEIG_OK) {
    if (hipMemcpyAsync(&hst, st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      host_status = REFEIG_E_HIP;
  }
  int status = host_status;
  if (status == REFEIG_OK) status = status_of(hst, hflags);
  if (rep && host_status == REFEIG_OK) {
    fill_report_from_device(hst, hflags, it, rep);
    if (timed)
      for (int k = 0; k < std::min(hst.iters_done, REFEIG_MAX_ITERS); ++k) {
        float t = 0, g1 = 0, g2 = 0, g3 = 0;
        (void)hipEventElapsedTime(&t, E(k, 0), E(k, 7));
        (void)hipEventElapsedTime(&g1, E(k, 1), E(k, 2));
        (void)hipEventElapsedTime(&g2, E(k, 3), E(k, 4));
        (void)hipEventElapsedTime(&g3, E(k, 5), E(k, 6));
        rep->ms_iter[k] = t;
        rep->ms_p[k][0] = g1;
        rep->ms_p[k][1] = g2;
        rep->ms_p[k][2] = g3;
        rep->ms_gemm[k] = g1 + g2 + g3;
        for (int q = 0; q < 5; ++q) {
          float ph = 0;
          (void)hipEventElapsedTime(&ph, E(k, 8 + 2 * q), E(k, 9 + 2 * q));
          rep->ms_phase[k][q] = ph;
        }
      }
  }
  if (!ev.empty()) event_pool().give(ev);
  if (rep) {
    rep->status = status;
    rep->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
            .count();
  }
  return status;
}

// ---- grouped batches: the solves of a batch advance together, one launch per step and size
// class, the products as persistent kernels over a device-built work list of (problem, tile,
// slot) items. Every problem's arithmetic is that of its single call (the same kernels' bodies
// on the same plan), so its result is bit for bit the same.
bool grouped_batch(const refeig_opts &o) {
  return o.mode == REFEIG_OZAKI_INT8 && o.plan == 0 && o.group_tau == 0.0 && o.schedule == 0 &&
         !o.enqueue_only;
}

// Workspaces of the problems run together: 16 GiB, or REFEIG_GROUP_CHUNK_MIB from the
// environment (read at each call; the workspace query and the solve must see the same value).
size_t group_chunk_bytes() {
  const char *e = std::getenv("REFEIG_GROUP_CHUNK_MIB");
  if (e) {
    const long long m = std::atoll(e);
    if (m > 0) return (size_t)m << 20;
  }
  return 16ull << 30;
}

size_t ws_rounded(int n, const refeig_opts &o) {
  return (carve(n, ka_of(&o), nullptr, nullptr, o.vmode == 1) + 255) / 256 * 256;
}
// Work items a problem's products can ask for at most (tiles x slots).
size_t item_cap(int n) {   // on the 128-row tile, which bounds the 256-row one as well
  const int tt = round_up(n, kTile) / 128;
  return (size_t)tt * tt * std::max(kCrtMax, kMaxDiag);
}
size_t stage_stride() { return (sizeof(DevState) + sizeof(int) + 255) / 256 * 256; }

// The batch's own area (descriptors, work lists, counters, the state staging) for count
// problems with icap items, then the region the problems' workspaces are carved from.
struct GroupArea {
  GProb *gp;
  int2 *items;
  int *cnt;     // [0..1] total, counter of the 256-tile list; [2..3] of the 128-tile one; [4]
  char *stage;
};
size_t group_area(int count, size_t icap, char *base, GroupArea *ga) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  GroupArea g;
  g.gp = (GProb *)take(sizeof(GProb) * (size_t)count);
  g.items = (int2 *)take(sizeof(int2) * icap);
  g.cnt = (int *)take(sizeof(int) * 8);
  g.stage = take(stage_stride() * (size_t)count);
  if (ga) *ga = g;
  return off;
}

size_t grouped_bytes(int count, const int *n, const refeig_opts &o) {
  size_t icap = 0, sum = 0, mx = 0;
  for (int i = 0; i < count; ++i) {
    const size_t w = ws_rounded(n[i], o);
    sum += w;
    mx = std::max(mx, w);
    if (round_up(n[i], kTile) <= kGroupMaxNpad) icap += item_cap(n[i]);
  }
  return group_area(count, icap, nullptr, nullptr) +
         std::min(sum, std::max(group_chunk_bytes(), mx));
}

// ---- product tile of grouped batches: the 256-row tile or, split in four, the 128-row one for
// padded orders from 1024 (below 1024 the plan itself is on 128-row tiles). Either gives the
// same results; the choice is timed once per padded order on synthetic planes and kept in an
// on-disk cache (one JSON object, "<arch>:<npad>": tile), REFEIG_TUNE_CACHE naming the file
// (else $XDG_CACHE_HOME/refeig/tiles.json, else $HOME/.cache/refeig/tiles.json).
// REFEIG_TUNE=0 takes the cached choice or the 256-row default without timing anything.
std::mutex g_tile_mu;
std::map<std::string, int> g_tile;   // "<cache file>|<arch>:<npad>" -> tile, this process

std::string tile_cache_path() {
  const char *e = std::getenv("REFEIG_TUNE_CACHE");
  if (e && *e) return e;
  const char *x = std::getenv("XDG_CACHE_HOME");
  const char *h = std::getenv("HOME");
  std::string base = (x && *x) ? std::string(x) : (h && *h) ? std::string(h) + "/.cache" : "/tmp";
  return base + "/refeig/tiles.json";
}
std::map<std::string, int> read_tile_cache(const std::string &path) {
  std::map<std::string, int> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while ((i = t.find('"', i)) != std::string::npos) {   // "key": value pairs
    const size_t j = t.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = t.substr(i + 1, j - i - 1);
    size_t k = t.find(':', j);
    if (k == std::string::npos) break;
    const int v = std::atoi(t.c_str() + k + 1);
    if (v == 128 || v == 256) out[key] = v;
    i = j + 1;
  }
  return out;
}
void write_tile_cache(const std::string &path, const std::map<std::string, int> &m) {
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
    (void)mkdir(path.substr(0, p).c_str(), 0755);
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{";
    bool first = true;
    for (const auto &kv : m) {
      f << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": " << kv.second;
      first = false;
    }
    f << "\n}\n";
  }
  (void)std::rename(tmp.c_str(), path.c_str());
}
std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> known;   // device -> architecture name
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lk(mu);
  auto it = known.find(d);
  if (it != known.end()) return it->second;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, d) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  return known[d] = a.substr(0, a.find(':'));
}
std::string tile_key(int npad) {
  return tile_cache_path() + "|" + device_arch() + ":" + std::to_string(npad);
}
int gtile_of(int npad) {
  if (npad < 1024) return 128;
  const char *f = std::getenv("REFEIG_TILE");   // 128 or 256: a fixed choice (A/B, tests)
  if (f && (std::atoi(f) == 128 || std::atoi(f) == 256)) return std::atoi(f);
  const std::string key = tile_key(npad);
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tile.find(key);
  return it == g_tile.end() ? 256 : it->second;
}

// Time the W-type product of two synthetic problems of order npad (12 x 8 digit planes, all
// tiles, slots 0..11) on both tiles; scratch: device memory the solve has not started to use.
// Returns the faster tile, or 0 when the scratch is too small or a call failed.
int time_tiles(int npad, char *scratch, size_t bytes, hipStream_t s) {
  const size_t P = (size_t)npad * npad;
  const int TT = npad / 256, nslot = 12, G = 2;
  const int ntab = TT * TT * nslot;
  size_t off = 0;
  auto take = [&](size_t b) {
    char *p = scratch + off;
    off += (b + 255) / 256 * 256;
    return p;
  };
  int8_t *Lp = (int8_t *)take(P * 12), *Rp = (int8_t *)take(P * 8);
  int32_t *Cs[G];
  for (int g = 0; g < G; ++g) Cs[g] = (int32_t *)take(P * 4 * nslot);
  int *tab = (int *)take(sizeof(int) * ntab);
  int *tcut = (int *)take(sizeof(int) * TT * TT);
  DevState *st = (DevState *)take(sizeof(DevState) * G);
  GProb *gp = (GProb *)take(sizeof(GProb) * G);
  int2 *items = (int2 *)take(sizeof(int2) * (size_t)ntab * 4 * G);
  int *cnt = (int *)take(sizeof(int) * 4);
  if (off > bytes) return 0;
  std::vector<int> htab(ntab), htc(TT * TT, kMaxDiag + 1);
  for (int q = 0, e = 0; q < nslot; ++q)
    for (int r = 0; r < TT; ++r)
      for (int c = 0; c < TT; ++c) htab[e++] = r | (c << 8) | (q << 16);
  std::vector<DevState> hst(G);
  std::memset(hst.data(), 0, sizeof(DevState) * G);
  for (auto &d : hst) {
    d.gemm_w[0] = kKrMax;
    d.gemm_w[1] = 8;
    d.gemm_w[2] = ntab;
  }
  std::vector<GProb> hp(G);
  std::memset((void *)hp.data(), 0, sizeof(GProb) * G);
  for (int g = 0; g < G; ++g) {
    GProb &q = hp[g];
    q.n = q.npad = npad;
    q.P = P;
    q.w.RP = Lp;
    q.w.XP = Rp;
    q.w.Cs = Cs[g];
    q.w.tab[1] = tab;
    q.w.tcut = tcut;
    q.pb.st = st + g;
  }
  launch_fill_hash_i8(Lp, P * 12, 0x9e3779b9u, s);
  launch_fill_hash_i8(Rp, P * 8, 0x7f4a7c15u, s);
  if (hipMemcpyAsync(tab, htab.data(), sizeof(int) * ntab, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(tcut, htc.data(), sizeof(int) * TT * TT, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(st, hst.data(), sizeof(DevState) * G, hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 0;
  float best[2] = {1e30f, 1e30f};
  const int tiles[2] = {256, 128};
  bool ok = true;
  for (int v = 0; v < 2 && ok; ++v) {
    for (auto &q : hp) q.gtile = tiles[v];
    ok = hipMemcpyAsync(gp, hp.data(), sizeof(GProb) * G, hipMemcpyHostToDevice, s) ==
         hipSuccess;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      launch_worklist_g(gp, 0, G, 2, tiles[v], items, cnt, cnt + 1, s);
      ok = hipEventRecord(e0, s) == hipSuccess;
      launch_gemm_g(gp, tiles[v], tiles[v] == 256 ? 256 : 768, items, cnt, cnt + 1, 2, s);
      float ms = 0.0f;
      ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      if (ok) best[v] = std::min(best[v], ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok || hipStreamSynchronize(s) != hipSuccess) return 0;
  return best[1] < best[0] ? 128 : 256;
}

// The tile of every padded order from 1024 in npads: from this process's choices, else the
// cache, else timed (REFEIG_TUNE != 0) and stored in the cache.
void ensure_tiles(const std::vector<int> &npads, char *scratch, size_t bytes, hipStream_t s) {
  std::vector<int> need;
  {
    std::vector<std::pair<int, std::string>> keys;
    for (int np : npads)
      if (np >= 1024) keys.emplace_back(np, tile_key(np));
    std::lock_guard<std::mutex> lk(g_tile_mu);
    for (const auto &k : keys)
      if (!g_tile.count(k.second) && std::find(need.begin(), need.end(), k.first) == need.end())
        need.push_back(k.first);
  }
  const char *f = std::getenv("REFEIG_TILE");
  if (need.empty() || (f && (std::atoi(f) == 128 || std::atoi(f) == 256))) return;
  const char *tune = std::getenv("REFEIG_TUNE");
  const bool timing = !(tune && std::atoi(tune) == 0);
  const std::string path = tile_cache_path(), arch = device_arch();
  std::map<std::string, int> cache = read_tile_cache(path);
  bool dirty = false;
  for (int np : need) {
    const std::string key = arch + ":" + std::to_string(np);
    int t = 256;
    auto it = cache.find(key);
    if (it != cache.end()) {
      t = it->second;
    } else if (timing) {
      const int r = time_tiles(np, scratch, bytes, s);
      if (r) {
        t = r;
        cache[key] = r;
        dirty = true;
      }
    }
    const std::string pk = tile_key(np);
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile[pk] = t;
  }
  if (dirty) write_tile_cache(path, cache);
}

// One chunk of a grouped batch: problems ids (npad descending, all <= kGroupMaxNpad), their
// workspaces carved from `region`. prepare_chunk fills the host descriptors and the launch
// shapes, enqueue_chunk enqueues the solve (with fixed iterations it never waits, so it can be
// captured), collect_chunk gathers the planning states and fills statuses and reports.
struct ChunkPlan {
  struct Cls {
    int first, count, npad;
  };
  std::vector<int> ids;
  std::vector<GProb> hp;   // host copy of the descriptors (uploaded to ga.gp)
  std::vector<Cls> cls;
  int G = 0, g256 = 0, blocks256 = 0, blocks128 = 0;
  size_t cap256 = 0;
};

void prepare_chunk(ChunkPlan &cp, const std::vector<int> &ids, const int *n,
                   const double *const *A, const int *lda, double *const *X, const int *ldx,
                   double *const *D, const double *target, const refeig_opts &o, char *region) {
  cp.ids = ids;
  cp.G = (int)ids.size();
  const int ka_max = ka_of(&o);
  const bool crt = o.vmode == 1;
  cp.hp.assign(cp.G, GProb());
  size_t off = 0;
  for (int k = 0; k < cp.G; ++k) {
    const int i = ids[k];
    GProb &q = cp.hp[k];
    carve(n[i], ka_max, region + off, &q.w, crt);
    off += ws_rounded(n[i], o);
    q.A = A[i];
    q.X = X[i];
    q.D = D[i];
    q.lda = lda[i];
    q.ldx = ldx[i];
    q.n = n[i];
    q.npad = q.w.npad;
    q.ka = ka_max;
    q.P = q.w.P;
    q.pp = plan_params(n[i], q.npad, o, target[i]);
    q.pb = plan_bufs(q.w, D[i]);
    q.gtile = gtile_of(q.npad);
  }
  cp.cls.clear();
  for (int k = 0; k < cp.G; ++k) {
    if (cp.cls.empty() || cp.cls.back().npad != cp.hp[k].npad)
      cp.cls.push_back({k, 0, cp.hp[k].npad});
    ++cp.cls.back().count;
  }
  size_t cap128 = 0;
  cp.g256 = 0;
  cp.cap256 = 0;
  for (int k = 0; k < cp.G; ++k) {
    if (cp.hp[k].gtile == 256) {
      ++cp.g256;
      cp.cap256 += item_cap(cp.hp[k].n);
    } else {
      cap128 += item_cap(cp.hp[k].n);
    }
  }
  cp.blocks256 = (int)std::min<size_t>(256, cp.cap256);
  cp.blocks128 = (int)std::min<size_t>(768, cap128);   // three blocks per CU
}

// Enqueues iterations it0 .. it1 - 1 (it0 == 0 also enqueues the once-per-solve steps); with
// gather, the planning states are gathered into ga.stage at the end.
void enqueue_chunk(const ChunkPlan &cp, const GroupArea &ga, const refeig_opts &o, int it0,
                   int it1, bool gather, hipStream_t s) {
  const GProb *gp = ga.gp;
  const int G = cp.G, g256 = cp.g256;
  int2 *items256 = ga.items, *items128 = ga.items + cp.cap256;
  auto products = [&](int which) {
    if (g256) {
      launch_worklist_g(gp, 0, g256, which, 256, items256, ga.cnt, ga.cnt + 1, s);
      launch_gemm_g(gp, 256, cp.blocks256, items256, ga.cnt, ga.cnt + 1, which, s);
    }
    if (G > g256) {
      launch_worklist_g(gp, g256, G - g256, which, 128, items128, ga.cnt + 2, ga.cnt + 3, s);
      launch_gemm_g(gp, 128, cp.blocks128, items128, ga.cnt + 2, ga.cnt + 3, which, s);
    }
  };
  // The planning kernels take one block per problem whatever its order, so each runs as one
  // launch over the whole batch; the other steps are one launch per size class.
  if (it0 == 0) {   // once per solve: A's column statistics, the planning state, A's planes
    launch_flags_clear_g(gp, G, s);
    for (const auto &c : cp.cls) launch_colstats_g(gp, c.first, c.count, c.npad, false, s);
    launch_dp_init_g(gp, 0, G, s);
    for (const auto &c : cp.cls) launch_split_g(gp, c.first, c.count, c.npad, false, s);
  }
  for (int it = it0; it < it1; ++it) {
    launch_dp_order_g(gp, 0, G, it, s);
    for (const auto &c : cp.cls) launch_colstats_g(gp, c.first, c.count, c.npad, true, s);
    launch_dp_vplan_g(gp, 0, G, it, s);
    for (const auto &c : cp.cls) launch_split_g(gp, c.first, c.count, c.npad, true, s);
    if (o.vmode == 1) {
      for (const auto &c : cp.cls)
        for (int l = 0; l <= kVLevels; ++l)
          launch_residues_g(gp, c.first, c.count, (size_t)c.npad * c.npad, l, s);
      products(0);
      for (const auto &c : cp.cls) launch_epi_v_g(gp, c.first, c.count, c.npad, true, s);
    }
    products(1);
    for (const auto &c : cp.cls) launch_epi_v_g(gp, c.first, c.count, c.npad, false, s);
    launch_dp_wplan_g(gp, 0, G, it, s);
    for (const auto &c : cp.cls)
      if (c.npad >= 1024) launch_tile_cutoffs_g(gp, c.first, c.count, c.npad, s);
    products(2);
    for (const auto &c : cp.cls) launch_epi_w_g(gp, c.first, c.count, c.npad, s);
    launch_dp_uplan_g(gp, 0, G, it, s);
    products(3);
    for (const auto &c : cp.cls) launch_epi_u_g(gp, c.first, c.count, c.npad, s);
    for (const auto &c : cp.cls) launch_scatter_g(gp, c.first, c.count, c.npad, s);
  }
  if (gather) launch_gather_state_g(gp, G, ga.stage, stage_stride(), s);
}

// Statuses and reports from ga.stage (filled by enqueue_chunk's gather; the caller has waited).
int collect_chunk(const ChunkPlan &cp, const GroupArea &ga, double ms, refeig_report *reports,
                  int *status) {
  const size_t stride = stage_stride();
  std::vector<char> stage(stride * cp.G);
  if (hipMemcpy(stage.data(), ga.stage, stride * cp.G, hipMemcpyDeviceToHost) != hipSuccess)
    return REFEIG_E_HIP;
  for (int k = 0; k < cp.G; ++k) {
    DevState hst;
    int hflags = 0;
    std::memcpy(&hst, stage.data() + stride * k, sizeof(DevState));
    std::memcpy(&hflags, stage.data() + stride * k + sizeof(DevState), sizeof(int));
    const int st = status_of(hst, hflags);
    status[cp.ids[k]] = st;
    if (reports) {
      refeig_report *r = &reports[cp.ids[k]];
      std::memset(r, 0, sizeof(*r));
      fill_report_from_device(hst, hflags, 0, r);
      r->status = st;
      r->ms_total = ms;   // the chunk's wall time (its solves run together)
    }
  }
  return REFEIG_OK;
}

int run_chunk(const std::vector<int> &ids, const int *n, const double *const *A, const int *lda,
              double *const *X, const int *ldx, double *const *D, const double *target,
              const refeig_opts &o, const GroupArea &ga, char *region, hipStream_t s,
              refeig_report *reports, std::vector<int> &status) {
  auto t_start = std::chrono::steady_clock::now();
  ChunkPlan cp;
  prepare_chunk(cp, ids, n, A, lda, X, ldx, D, target, o, region);
  auto fail = [&](int st) {
    (void)hipStreamSynchronize(s);   // nothing in flight reads cp.hp after this returns
    for (int k = 0; k < cp.G; ++k) status[ids[k]] = st;
    return st;
  };
  if (hipMemcpyAsync(ga.gp, cp.hp.data(), sizeof(GProb) * cp.G, hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return fail(REFEIG_E_HIP);
  const int iters = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  if (o.fixed_iters > 0) {
    enqueue_chunk(cp, ga, o, 0, iters, true, s);
    if (hipGetLastError() != hipSuccess) return fail(REFEIG_E_HIP);
  } else {
    for (int it = 0; it < iters; ++it) {
      enqueue_chunk(cp, ga, o, it, it + 1, false, s);
      if (hipGetLastError() != hipSuccess) return fail(REFEIG_E_HIP);
      if (it + 1 < iters) {   // stop once every solve has stopped
        int running = 0;
        launch_count_running_g(ga.gp, cp.G, ga.cnt + 4, s);
        if (hipMemcpyAsync(&running, ga.cnt + 4, sizeof(int), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return fail(REFEIG_E_HIP);
        if (running == 0) break;
      }
    }
    launch_gather_state_g(ga.gp, cp.G, ga.stage, stage_stride(), s);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(REFEIG_E_HIP);
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
          .count();
  const int st = collect_chunk(cp, ga, ms, reports, status.data());
  return st == REFEIG_OK ? REFEIG_OK : fail(st);
}

bool opts_valid(const refeig_opts &o) {
  return o.delta_safety >= 1.0 && o.theta > 0.0 && o.theta <= 1.0 && o.max_iter >= 1 &&
         o.group_tau >= 0.0 && o.kx_force >= 0 && o.kx_force <= kKxMax && o.sparse_k >= 0 &&
         o.schedule >= 0 && o.schedule <= 1 && o.vmode >= 0 && o.vmode <= 1 &&
         o.max_iter <= REFEIG_MAX_ITERS && o.fixed_iters <= REFEIG_MAX_ITERS;
}

int refine_grouped(int count, const int *n, const double *const *A, const int *lda,
                   double *const *X, const int *ldx, double *const *D, const double *target,
                   const refeig_opts &o, char *work, size_t work_bytes, hipStream_t s,
                   refeig_report *reports) {
  std::vector<int> status(count, REFEIG_E_ARG);
  if (reports) std::memset(reports, 0, sizeof(refeig_report) * count);
  const bool ok_opts = opts_valid(o);
  // problems run together (valid, npad <= kGroupMaxNpad) by npad descending, and the rest
  std::vector<int> grouped, alone;
  size_t icap = 0;
  for (int i = 0; i < count; ++i) {
    const bool valid = ok_opts && A[i] && X[i] && D[i] && n[i] >= 1 && n[i] <= kMaxN &&
                       lda[i] >= n[i] && ldx[i] >= n[i] && target[i] > 0.0;
    if (!valid) continue;
    if (round_up(n[i], kTile) <= kGroupMaxNpad) {
      grouped.push_back(i);
      icap += item_cap(n[i]);
    } else {
      alone.push_back(i);
    }
  }
  GroupArea ga;
  const size_t area = group_area(count, icap, work, &ga);
  char *region = work + area;
  const size_t room = std::min(work_bytes - area, std::max(group_chunk_bytes(), [&] {
                                 size_t mx = 0;
                                 for (int i = 0; i < count; ++i)
                                   if (n[i] >= 1 && n[i] <= kMaxN)
                                     mx = std::max(mx, ws_rounded(n[i], o));
                                 return mx;
                               }()));
  // product tiles (the region is free until the first chunk), then the problems ordered with
  // the 256-row tile's first, each tile group by npad descending
  {
    std::vector<int> npads;
    for (int i : grouped) npads.push_back(round_up(n[i], kTile));
    ensure_tiles(npads, region, room, s);
  }
  std::stable_sort(grouped.begin(), grouped.end(), [&](int a, int b) {
    const int pa = round_up(n[a], kTile), pb = round_up(n[b], kTile);
    const int ta = gtile_of(pa), tb = gtile_of(pb);
    return ta != tb ? ta > tb : pa > pb;
  });
  // chunks of consecutive problems whose workspaces fit in the region together
  size_t k = 0;
  while (k < grouped.size()) {
    std::vector<int> ids;
    size_t used = 0;
    while (k < grouped.size() && (ids.empty() || used + ws_rounded(n[grouped[k]], o) <= room)) {
      used += ws_rounded(n[grouped[k]], o);
      ids.push_back(grouped[k++]);
    }
    if (used > room) return REFEIG_E_NOMEM;
    run_chunk(ids, n, A, lda, X, ldx, D, target, o, ga, region, s, reports, status);
  }
  for (int i : alone)
    status[i] = refine_eigvecs(A[i], lda[i], X[i], ldx[i], D[i], n[i], target[i], &o, region,
                               room, (refeig_stream_t)s, reports ? &reports[i] : nullptr);
  int worst = REFEIG_OK;
  for (int i = 0; i < count; ++i) {
    if (reports && status[i] == REFEIG_E_ARG) reports[i].status = REFEIG_E_ARG;
    if (status[i] < 0) return status[i];
    if (status[i] != REFEIG_OK) worst = status[i];
  }
  return worst;
}

}  // namespace

extern "C" {

int refeig_default_opts(refeig_opts *o) {
  if (!o) return REFEIG_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->mode = REFEIG_OZAKI_INT8;
  o->max_iter = 8;
  o->fixed_iters = 0;
  o->stop_rule = 0;
  o->delta_safety = 8.0;
  o->xi = 0.0;
  o->theta = 0.25;
  o->ka_max = kKaMaxLimit;
  o->d_extra = 0;
  o->verbose = 0;
  o->vmode = 1;
  return REFEIG_OK;
}

int refeig_workspace_bytes(int n, const refeig_opts *o, size_t *bytes) {
  if (n < 1 || n > kMaxN || !bytes) return REFEIG_E_ARG;
  *bytes = (o && o->mode == REFEIG_FP64_PLAIN) ? carve_plain(n, nullptr, nullptr)
                                               : carve(n, ka_of(o), nullptr, nullptr,
                                                       !o || o->vmode == 1);
  return REFEIG_OK;
}

int refeig_herm_workspace_bytes(int n, const refeig_opts *o, size_t *bytes) {
  if (n < 1 || n > kMaxNHerm || !bytes) return REFEIG_E_ARG;
  *bytes = carve_herm(n, ka_of(o), nullptr, nullptr);
  return REFEIG_OK;
}

int refine_eigvecs_herm(const double *A, int lda, double *X, int ldx, double *D, int n,
                        double target, const refeig_opts *opts, void *work, size_t work_bytes,
                        refeig_stream_t stream, refeig_report *rep) {
  refeig_opts o;
  if (opts) o = *opts;
  else refeig_default_opts(&o);
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (!A || !X || !D || n < 1 || n > kMaxNHerm || lda < n || ldx < n || !(target > 0.0) ||
      !(o.delta_safety >= 1.0) || !(o.theta > 0.0 && o.theta <= 1.0) || o.max_iter < 1 ||
      o.kx_force < 0 || o.kx_force > kKxMax || o.max_iter > REFEIG_MAX_ITERS ||
      o.fixed_iters > REFEIG_MAX_ITERS || o.mode != REFEIG_OZAKI_INT8 || o.group_tau != 0.0 ||
      o.schedule != 0 || o.sparse_k != 0 || o.vmode < 0 || o.vmode > 1)
    return REFEIG_E_ARG;
  return refine_herm(A, lda, X, ldx, D, n, target, o, work, work_bytes, (hipStream_t)stream,
                     rep);
}

const char *refeig_strerror(int s) {
  switch (s) {
    case REFEIG_OK: return "ok";
    case REFEIG_NOT_CONVERGED: return "not converged (stagnation or iteration limit)";
    case REFEIG_E_ARG: return "invalid argument";
    case REFEIG_E_NONFINITE: return "non-finite value in A, X or D";
    case REFEIG_E_GAP: return "two eigenvalue estimates coincide";
    case REFEIG_E_RANGE: return "row/column maximum outside [2^-400, 2^400]";
    case REFEIG_E_NOMEM: return "workspace too small or allocation failed";
    case REFEIG_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int refeig_split_cols(const double *M, int ld, int rows, int cols, int k, int *exps,
                      int8_t *planes, double *trunc, refeig_stream_t stream) {
  return refeig_split_cols_ex(M, ld, rows, cols, k, nullptr, exps, planes, trunc, 0, nullptr,
                              stream);
}

int refeig_split_cols_ex(const double *M, int ld, int rows, int cols, int k, const int *colmap,
                         int *exps, int8_t *planes, double *trunc, int kT, int8_t *planesT,
                         refeig_stream_t stream) {
  if (!M || !exps || !planes || rows < 1 || cols < 1 || ld < rows || k < 1 || k > 18 ||
      kT < 0 || kT > kKxMax || (kT > 0) != (planesT != nullptr))
    return REFEIG_E_ARG;
  if (colmap)
    for (int j = 0; j < cols; ++j)
      if (colmap[j] < 0 || colmap[j] >= cols) return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int rpad = round_up(rows, kTile), cpad = round_up(cols, kTile);
  // exponents are produced for the padded column range; copy the first cols out
  int *cbuf = nullptr;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMalloc((void **)&cbuf, sizeof(int) * (3 * (size_t)cpad + 64)));
  int *e_int = cbuf, *c_int = cbuf + cpad, *dmap = cbuf + 2 * cpad, *flags = cbuf + 3 * cpad;
  hipError_t err = hipSuccess;
  if (colmap)
    err = hipMemcpyAsync(dmap, colmap, sizeof(int) * cols, hipMemcpyHostToDevice, s);
  if (err == hipSuccess) err = hipMemsetAsync(flags, 0, sizeof(int), s);
  int hf = 0;
  if (err == hipSuccess) {
    launch_colstats(M, ld, rows, cols, cpad, e_int, c_int, nullptr, flags, s,
                    colmap ? dmap : nullptr);
    launch_split_cols(M, ld, rows, cols, e_int, k, planes, (size_t)rpad * cpad, rpad, cpad,
                      trunc, rows, planesT, (size_t)rpad * cpad, kT, s, colmap ? dmap : nullptr);
    err = hipGetLastError();
  }
  if (err == hipSuccess)
    err = hipMemcpyAsync(exps, e_int, sizeof(int) * cols, hipMemcpyDeviceToDevice, s);
  if (err == hipSuccess) err = hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  (void)hipFree(cbuf);
  if (err != hipSuccess) {
    fprintf(stderr, "refeig: refeig_split_cols_ex: %s\n", hipGetErrorString(err));
    return REFEIG_E_HIP;
  }
  if (hf & FLAG_NONFINITE) return REFEIG_E_NONFINITE;
  if (hf & FLAG_RANGE) return REFEIG_E_RANGE;
  return REFEIG_OK;
}

int refeig_residue_planes(const int8_t *planes, size_t plane_stride, size_t count, int k,
                          int nmod, const int *moduli, int8_t *res, refeig_stream_t stream) {
  if (!planes || !res || !moduli || k < 1 || k > kCrtPlanes || nmod < 1 || nmod > kCrtMax ||
      count == 0 || count % 4 != 0 || plane_stride < count || plane_stride % 4 != 0)
    return REFEIG_E_ARG;
  for (int q = 0; q < nmod; ++q)
    if (moduli[q] < 3 || moduli[q] > 255 || moduli[q] % 2 == 0) return REFEIG_E_ARG;
  ResWeights w;
  res_weights(k, nmod, moduli, w);
  hipStream_t s = (hipStream_t)stream;
  launch_residues(planes, plane_stride, count, w, res, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return REFEIG_OK;
}

int refeig_residue_gemm(const int8_t *Lp, const int8_t *Rp, size_t plane_stride, int npad,
                        int nmod, const int *moduli, const int *vblk, int8_t *C,
                        refeig_stream_t stream) {
  if (!Lp || !Rp || !C || !moduli || npad < kTile || npad % kTile || nmod < 1 ||
      nmod > kCrtMax || plane_stride < (size_t)npad * npad || (vblk && npad < 1024))
    return REFEIG_E_ARG;
  for (int q = 0; q < nmod; ++q)
    if (moduli[q] < 3 || moduli[q] > 255 || moduli[q] % 2 == 0) return REFEIG_E_ARG;
  const int nb = npad / kTile;
  if (vblk)
    for (int b = 0; b < nb; ++b)
      if (vblk[2 * b] < 0 || vblk[2 * b] > nmod || vblk[2 * b + 1] < 0 ||
          vblk[2 * b + 1] >= kVLevels)
        return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int *buf = nullptr;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMalloc((void **)&buf, sizeof(int) * (kCrtMax + 2 * (size_t)nb)));
  hipError_t err = hipMemcpyAsync(buf, moduli, sizeof(int) * nmod, hipMemcpyHostToDevice, s);
  if (err == hipSuccess && vblk)
    err = hipMemcpyAsync(buf + kCrtMax, vblk, sizeof(int) * 2 * nb, hipMemcpyHostToDevice, s);
  if (err == hipSuccess) {
    launch_slice_gemm(Lp, Rp, plane_stride, npad, nmod, nmod, 2, nmod, (int32_t *)C, nullptr, s,
                      nullptr, nullptr, 0, true, nullptr, buf, false,
                      vblk ? buf + kCrtMax : nullptr);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (err != hipSuccess) {
    fprintf(stderr, "refeig: refeig_residue_gemm: %s\n", hipGetErrorString(err));
    return REFEIG_E_HIP;
  }
  return REFEIG_OK;
}

int refeig_slice_gemm(const int8_t *Lp, const int8_t *Rp, size_t plane_stride, int npad, int kl,
                      int kr, int d_min, int ndiag, int32_t *C, refeig_stream_t stream) {
  if (!Lp || !Rp || !C || npad < kTile || npad % kTile || kl < 1 || kr < 1 || d_min < 2 ||
      ndiag < 1 || ndiag > kMaxDiag || d_min + ndiag - 1 > kl + kr)
    return REFEIG_E_ARG;
  for (int q = 0; q < ndiag; ++q)
    if ((double)npairs_of(d_min + q, kl, kr) * npad * 127.0 * 127.0 >= 2147483648.0)
      return REFEIG_E_ARG;
  if (plane_stride < (size_t)npad * npad) return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  launch_slice_gemm(Lp, Rp, plane_stride, npad, kl, kr, d_min, ndiag, C, nullptr, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return REFEIG_OK;
}

int refeig_digits_to_e4m3(const int8_t *digits, uint8_t *codes, size_t count,
                          refeig_stream_t stream) {
  if (count == 0) return REFEIG_OK;
  if (!digits || !codes) return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int *bad = nullptr, hbad = 0;
  HIPCHK(hipMalloc((void **)&bad, sizeof(int)));
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
  if (e == hipSuccess) {
    launch_digits_e4m3(digits, codes, count, bad, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(bad);
  if (e != hipSuccess) return REFEIG_E_HIP;
  return hbad ? REFEIG_E_ARG : REFEIG_OK;
}

int refeig_slice_gemm_fp8(const uint8_t *Lp8, const uint8_t *Rp8, size_t plane_stride, int npad,
                          int kl, int kr, int d_min, int ndiag, int32_t *C,
                          refeig_stream_t stream) {
  if (!Lp8 || !Rp8 || !C || npad < 1024 || npad % kTile || kl < 1 || kr < 1 || d_min < 2 ||
      ndiag < 1 || ndiag > kMaxDiag || d_min + ndiag - 1 > kl + kr)
    return REFEIG_E_ARG;
  for (int q = 0; q < ndiag; ++q)
    if ((double)npairs_of(d_min + q, kl, kr) * npad * 15.0 * 15.0 >= 16777216.0)
      return REFEIG_E_ARG;
  if (plane_stride < (size_t)npad * npad) return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  launch_slice_gemm((const int8_t *)Lp8, (const int8_t *)Rp8, plane_stride, npad, kl, kr, d_min,
                    ndiag, C, nullptr, s, nullptr, nullptr, 0, false, nullptr, nullptr, true);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return REFEIG_OK;
}

int refine_eigvecs(const double *A, int lda, double *X, int ldx, double *D, int n,
                   double target, const refeig_opts *o_in, void *work, size_t work_bytes,
                   refeig_stream_t stream, refeig_report *rep) {
  refeig_opts o;
  if (o_in) o = *o_in;
  else refeig_default_opts(&o);
  const int verbose = o.verbose;
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (!A || !X || !D || n < 1 || n > kMaxN || lda < n || ldx < n || !(target > 0.0) ||
      !(o.delta_safety >= 1.0) || !(o.theta > 0.0 && o.theta <= 1.0) || o.max_iter < 1 ||
      !(o.group_tau >= 0.0) || o.kx_force < 0 || o.kx_force > kKxMax || o.sparse_k < 0 ||
      o.schedule < 0 || o.schedule > 1 || o.vmode < 0 || o.vmode > 1 ||
      o.max_iter > REFEIG_MAX_ITERS || o.fixed_iters > REFEIG_MAX_ITERS)
    return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (o.mode == REFEIG_FP64_PLAIN && !o.enqueue_only)
    return refine_plain(A, lda, X, ldx, D, n, target, o, work, work_bytes, s, rep);
  if (o.mode != REFEIG_OZAKI_INT8 || o.plan < 0 || o.plan > 1) return REFEIG_E_ARG;
  // device planning unless the options need the host (grouped correction, schedule)
  const bool dev_plan = o.plan == 0 && o.group_tau == 0.0 && o.schedule == 0;
  if (o.enqueue_only && !(dev_plan && o.fixed_iters > 0 && work)) return REFEIG_E_ARG;
  const int ka_max = ka_of(&o);
  const bool crt = o.vmode == 1;
  const size_t need = carve(n, ka_max, nullptr, nullptr, crt);
  bool own = false;
  if (!work) {
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMalloc(&work, need));
    own = true;
  } else if (work_bytes < need) {
    return REFEIG_E_NOMEM;
  }
  if (dev_plan) {
    const int st = refine_device(A, lda, X, ldx, D, n, target, o, work, s, rep,
                                 o.enqueue_only != 0);
    if (own) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(work);
    }
    return st;
  }
  Work w;
  carve(n, ka_max, (char *)work, &w, crt);
  const int npad = w.npad;
  const size_t P = w.P;
  const double delta_int = target / o.delta_safety;
  const double xi = xi_of(o, n);
  const double theta = o.theta;
  const double lsqn = 0.5 * plan_log2((double)n);
  const double lgrowth_a = lgrowth_of(o, n);   // error growth of products of A's planes
  auto t_start = std::chrono::steady_clock::now();

  int status = REFEIG_OK;
  std::vector<int> eX(npad), cX(npad), eR(npad), eE(npad), eA(npad), cA(npad);
  std::vector<double> mxX(npad), mxA(npad), lam(n), lam_prev(n), resmax(npad), emax(npad), gaps,
      wtolh(2 * (size_t)npad, 0.0);
  // host sources of the residue product's uploads, alive until the function returns
  std::vector<CrtRec> rec(kVLevels);
  std::vector<int> vb(2 * (size_t)(npad / 256));
  std::vector<double> gaps_nat;
  std::vector<int> cmap(n), cpl, tcut, htab[3];
  int hflags = 0;
  // ev[0] / ev[7]: iteration start / end; ev[1..6]: the three slice products; ev[8..17]:
  // the phases (column statistics, split, V, W, update) for the report
  hipEvent_t ev[18];
  for (auto &e : ev) HIPCHK(hipEventCreate(&e));

  auto cleanup = [&](int st) {
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (own) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(work);
    }
    if (rep) {
      rep->status = st;
      rep->ms_total =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
              .count();
    }
    return st;
  };
#define STEP(x)                                   \
  do {                                            \
    hipError_t err__ = (x);                       \
    if (err__ != hipSuccess) {                    \
      fprintf(stderr, "refeig: %s failed: %s\n", #x, hipGetErrorString(err__)); \
      return cleanup(REFEIG_E_HIP);               \
    }                                             \
  } while (0)

  // D on entry: the eigenvalue estimates that set beta of the first iteration
  STEP(hipMemcpyAsync(lam_prev.data(), D, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  STEP(hipMemsetAsync(w.flags, 0, sizeof(int), s));
  // A: column exponents (= row exponents, A is symmetric) and its digit planes, once
  launch_colstats(A, lda, n, n, npad, w.eA, w.cA, w.mxA, w.flags, s, nullptr, crt ? w.ssA : nullptr);
  STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  STEP(hipMemcpyAsync(eA.data(), w.eA, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
  std::vector<double> ssA(crt ? npad : 0), mxAh(crt ? npad : 0), ssX(crt ? npad : 0);
  if (crt) {
    STEP(hipMemcpyAsync(ssA.data(), w.ssA, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(mxAh.data(), w.mxA, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
  }
  STEP(hipStreamSynchronize(s));
  // max_i ||a_i|| 2^-eA_i (A symmetric: rows = columns) for the residue product's bound
  double hA = 0.0;
  for (int i = 0; crt && i < n; ++i)
    if (mxAh[i] != 0.0) hA = std::max(hA, std::ldexp(std::sqrt(ssA[i]), -eA[i]));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(lam_prev[i])) return cleanup(REFEIG_E_NONFINITE);
  if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
  if (hflags & FLAG_RANGE) return cleanup(REFEIG_E_RANGE);
  int eA_max = -100000;
  for (int i = 0; i < n; ++i) eA_max = std::max(eA_max, eA[i]);
  launch_split_cols(A, lda, n, n, w.eA, ka_max, w.AP, P, npad, npad, nullptr, 0, nullptr, 0, 0,
                    s);
  STEP(hipGetLastError());

  const int iters = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  double eps_prev = INFINITY;
  int ares_ka[kVLevels], ares_n[kVLevels];   // digit and modulus counts of A's residues per level
  for (int l = 0; l < kVLevels; ++l) ares_ka[l] = ares_n[l] = -1;
  int it = 0;
  for (; it < iters; ++it) {
    STEP(hipEventRecord(ev[0], s));
    // ---- working column order: widest gap first. The iteration is equivariant under a
    // column permutation (each column keeps its own arithmetic), and a GEMM block spans
    // 256 columns and computes the pair diagonals its neediest column requires, so columns
    // that need similar diagonal counts (set by their gaps) are placed together. Column p
    // of every working array is column cmap[p] of X and D.
    double gmin, lmax;
    column_gaps(lam_prev, gaps_nat, &gmin, &lmax);
    if (!(gmin > 0.0)) return cleanup(REFEIG_E_GAP);
    working_order(lam_prev, gaps_nat, cmap);
    STEP(hipMemcpyAsync(w.colmap, cmap.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    // ---- beta and kx from the previous eigenvalue estimates and column maxima of X
    STEP(hipEventRecord(ev[8], s));
    launch_colstats(X, ldx, n, n, npad, w.eX, w.cX, w.mxX, w.flags, s, w.colmap,
                    crt ? w.ssX : nullptr);
    STEP(hipEventRecord(ev[9], s));
    STEP(hipMemcpyAsync(eX.data(), w.eX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(cX.data(), w.cX, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(mxX.data(), w.mxX, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    if (crt) STEP(hipMemcpyAsync(ssX.data(), w.ssX, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    STEP(hipStreamSynchronize(s));
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    if (hflags & FLAG_RANGE) return cleanup(REFEIG_E_RANGE);
    gaps.resize(n);
    for (int p = 0; p < n; ++p) gaps[p] = gaps_nat[cmap[p]];
    int beta, kx;
    // accuracy this iteration's products aim at: the internal delta, or, with the adaptive
    // schedule (an extension beyond the paper), a looser level while the previous correction
    // e was large. This iteration's output error is then about e^4 and the next one's about
    // e^8 (quadratic convergence). Loose products leave an error nu = theta delta_k in every
    // entry of X; the next iteration turns it into about nu^2 max|lambda| / gap (the same
    // amplification that bounds the X^(1) cut of Sec. 4.1), kept at a tenth of that
    // iteration's own output error, or of delta when that one is the last.
    double delta_k = delta_int;
    if (o.schedule == 1 && it > 0 && std::isfinite(eps_prev)) {
      const double e4 = std::pow(eps_prev, 4.0);
      const double direct = 0.01 * e4;
      const double noise = (0.1 / theta) * std::sqrt(std::max(e4 * e4, delta_int) * gmin / lmax);
      delta_k = std::max(delta_int, std::min(direct, noise));
    }
    beta_rule(n, xi, delta_k, gmin, lmax, eX, cX, mxX, &beta, &kx);
    if (o.kx_force > 0) kx = o.kx_force;
    // ---- X^(1) and its planes (both layouts)
    STEP(hipEventRecord(ev[10], s));
    launch_split_cols(X, ldx, n, n, w.eX, kx, w.XP, P, npad, npad, w.X1, n, w.XPT, P, kx, s,
                      w.colmap);
    STEP(hipEventRecord(ev[11], s));
    // ---- V = A X^(1): per column j keep pair diagonals d <= dv(j)
    int eXmax = -100000;
    for (int j = 0; j < n; ++j) eXmax = std::max(eXmax, eX[j]);
    std::vector<int> dcol(npad, 2), dhost;
    for (int j = 0; j < n; ++j)
      if (mxX[j] != 0.0)
        dcol[j] = cut_v(eA_max, lgrowth_a, kx, eX[j], theta, delta_k, gaps[j], o.d_extra);
    const int dv_allowed = std::min(ka_max + 1, kx + ka_max);
    const int ka = ka_max;
    CutPlan plan;
    STEP(hipEventRecord(ev[12], s));
    int dv = 2, lv = 0;
    double pv = 0.0;
    bool by_res = false;
    if (crt) {
      // V by residues. The digits of A that column j needs follow from the truncation bound
      // sqrt(n) 2^(eA_max + eX_j - 7 ka1) <= theta delta gap_j (X^(1) enters exactly). Each
      // 256-column block takes the count of its neediest column, rounded up to one of at most
      // kVLevels levels spaced two digits apart below the largest; a level's product needs
      // fewer moduli (its P is smaller), so its blocks skip the GEMM slots beyond its count.
      const int nb = npad / 256;
      std::vector<int> kab(nb, 1);
      for (int j = 0; j < n; ++j) {
        if (mxX[j] == 0.0) continue;
        kab[j / 256] = std::max(kab[j / 256], cut_ka(eA_max, lgrowth_a, eX[j], theta, delta_k,
                                                     gaps[j], o.d_extra));
      }
      int ka_top = 1;
      for (int b = 0; b < nb; ++b) ka_top = std::max(ka_top, kab[b] = std::min(kab[b], ka_max));
      const bool levels = npad >= 1024;   // the 256-tile GEMM reads the block table
      std::vector<int> lvb(nb, 0);
      int ka_l[kVLevels] = {0};
      for (int b = 0; b < nb; ++b) {
        lvb[b] = levels ? std::min(kVLevels - 1, (ka_top - kab[b]) / 2) : 0;
        ka_l[lvb[b]] = std::max(ka_l[lvb[b]], kab[b]);
      }
      // Cauchy-Schwarz headroom: max ||x_j|| 2^-eX_j (X^(1) is X truncated, never larger)
      double hX = 0.0;
      for (int j = 0; j < n; ++j)
        if (mxX[j] != 0.0) hX = std::max(hX, std::ldexp(std::sqrt(ssX[j]), -eX[j]));
      const double hbits =
          (hA > 0.0 && hX > 0.0) ? plan_log2(hA * hX * (1.0 + 1e-6)) : -1.0;
      ResWeights wA[kVLevels], wX, wXl;   // X's weights: level 0's (the most moduli)
      bool ok = true;
      for (int l = 0; l < kVLevels && ok; ++l)
        if (ka_l[l] > 0) ok = crt_plan(npad, ka_l[l], kx, wA[l], l == 0 ? wX : wXl, rec[l],
                                       hbits);
      // The reconstruction resolves P to within 2^-115 M (the 34-bit limbs of at most 28
      // terms lose at most 2^-124.2 M, the double-word products by M the rest), so V_ij carries up to 2^(eA_max + eX_j + sh - 115) M of it. Where that is not
      // well inside column j's share theta delta gap_j, this iteration forms V by slices.
      for (int j = 0; ok && j < n; ++j) {
        if (mxX[j] == 0.0) continue;
        const CrtRec &rl = rec[lvb[j / 256]];
        const double fl = std::ldexp(rl.M[0], eA_max + eX[j] + rl.sh - 115);
        if (!(fl <= 0.25 * theta * delta_k * gaps[j])) ok = false;
      }
      if (ok) {
        by_res = true;
        // A's residues depend only on the digit count and the moduli: reused while they repeat
        for (int l = 0; l < kVLevels; ++l) {
          if (ka_l[l] == 0 || (ka_l[l] == ares_ka[l] && rec[l].N == ares_n[l])) continue;
          launch_residues(w.AP, P, P, wA[l], w.ARES + (size_t)l * kCrtMax * P, s);
          ares_ka[l] = ka_l[l];
          ares_n[l] = rec[l].N;
        }
        // level 0 has the most moduli; the other levels use a prefix of them
        launch_residues(w.XP, P, P, wX, w.XRES, s);
        double nsum = 0.0;
        for (int b = 0; b < nb; ++b) {
          vb[2 * b] = rec[lvb[b]].N;
          vb[2 * b + 1] = lvb[b];
          nsum += rec[lvb[b]].N;
        }
        STEP(hipMemcpyAsync(w.mods, rec[0].m, sizeof(int) * rec[0].N, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.recs, rec.data(), sizeof(CrtRec) * kVLevels, hipMemcpyHostToDevice,
                            s));
        STEP(hipMemcpyAsync(w.vblk, vb.data(), sizeof(int) * 2 * nb, hipMemcpyHostToDevice, s));
        // one launch: slot q = residue planes q of X^(1) and of A at the block's level,
        // stored mod m_q as INT8
        launch_slice_gemm(w.XRES, w.ARES, P, npad, rec[0].N, rec[0].N, 2, rec[0].N, w.Cs,
                          nullptr, s, ev[1], ev[2], 0, true, nullptr, w.mods, false,
                          levels ? w.vblk : nullptr);
        launch_epi_v_crt(w.Cs, npad, w.recs, levels ? w.vblk : nullptr, w.eA, w.eX, w.X1, n,
                         w.lam, w.lam_lo, w.r, w.eR, w.resmax, w.RP, kKrMax, w.flags, s);
        dv = ka_top + kx;
        pv = nsum / nb;   // products of n x n x n
        lv = 1;
      }
    }
    if (!by_res) {
      if (!plan_cutoffs(dcol, n, npad, kx, ka, dv_allowed, w.dcut[0], dhost, s, plan))
        return cleanup(REFEIG_E_HIP);
      dv = plan.dmax;
      pv = plan.pairs_eff;
      lv = (int)plan.groups.size();
      const int nbv = prepare_table(plan, npad, kx, ka, htab[0], w.tab[0], s);
      if (nbv < 0) return cleanup(REFEIG_E_HIP);
      if (nbv > 0) lv = 1;
      launch_plan(plan, w.XP, w.AP, P, npad, kx, ka, w.Cs, s, ev[1], ev[2], 0, nullptr, w.tab[0],
                  nbv);
      launch_epi_v(w.Cs, npad, 2, dv - 1, w.dcut[0], w.eA, w.eX, w.X1, n, w.lam, w.lam_lo, w.r,
                   w.eR, w.resmax, w.RP, kKrMax, w.flags, s);
    }
    STEP(hipEventRecord(ev[13], s));
    STEP(hipMemcpyAsync(lam.data(), w.lam, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(eR.data(), w.eR, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(resmax.data(), w.resmax, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    STEP(hipStreamSynchronize(s));
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    // ---- W = X^(1)T Res -> E~
    column_gaps(lam, gaps, &gmin, &lmax);
    if (!(gmin > 0.0)) return cleanup(REFEIG_E_GAP);
    std::fill(dcol.begin(), dcol.end(), 2);
    for (int j = 0; j < n; ++j)
      if (resmax[j] != 0.0)
        dcol[j] = cut_w(eXmax, kx, lsqn, eR[j], theta, delta_k, gaps[j], o.d_extra);
    // Noise stability: the W tiles far from column j's eigenvalue, and the product X^(1) E~,
    // leave an error of about nu_j = theta delta t_j along every eigenvector in column j of
    // the new X; the next iteration turns it into about nu_j^2 max|lambda| / g_j (the
    // amplification that bounds the X^(1) cut of Sec. 4.1), kept at a quarter of the
    // internal delta. t_j = 1 unless g_j is tiny next to max|lambda| and delta is loose.
    bool tight = false;
    for (int j = 0; j < n; ++j) {
      wtolh[j] = w_tight(delta_int, gaps[j], lmax, theta, delta_k);
      wtolh[npad + j] = gaps[j];
      tight = tight || wtolh[j] < 1.0;
    }
    const int kR = kKrMax, kxw = kx;
    const int dw_allowed = std::min(kKrMax + 1, kR + kxw);
    // Per-tile cutoffs (256 x 256 tiles, npad >= 1024): entry (i, j) needs its error within
    // theta delta |lambda_j - lambda_i|, so tile (column block J, row block I) keeps the
    // diagonals its columns need against the nearest eigenvalue in row block I (the column's
    // own gap in its own block). Never more than the column cutoff above.
    const int *tcut_dev = nullptr;
    double pw_tiles = -1.0;
    const int T = npad / 256;
    STEP(hipEventRecord(ev[14], s));
    if (npad >= 1024) {
      // on the device (nothing for the host to wait for); the pair count of the report is
      // read back after the iteration
      const double cx = cx_tile(kx, lsqn, theta, delta_k);
      if (tight)
        STEP(hipMemcpyAsync(w.wtol, wtolh.data(), sizeof(double) * 2 * npad,
                            hipMemcpyHostToDevice, s));
      launch_tile_cutoffs(w.lam, w.eX, w.eR, w.resmax, n, T, cx, dw_allowed, o.d_extra,
                          tight ? w.wtol : nullptr, tight ? w.wtol + npad : nullptr, w.tcut, s);
      STEP(hipGetLastError());
      tcut_dev = w.tcut;
      pw_tiles = 0.0;
    }
    if (!plan_cutoffs(dcol, n, npad, kR, kxw, dw_allowed, w.dcut[1], dhost, s, plan))
      return cleanup(REFEIG_E_HIP);
    const int dw = plan.dmax;
    const double pw = pw_tiles >= 0.0 ? pw_tiles : plan.pairs_eff;
    const std::vector<int> whost = dhost;   // per-column last diagonal of the W launches
    int lw = (int)plan.groups.size();
    const int nbw = prepare_table(plan, npad, kR, kxw, htab[1], w.tab[1], s);
    if (nbw < 0) return cleanup(REFEIG_E_HIP);
    if (nbw > 0) lw = 1;
    launch_plan(plan, w.RP, w.XP, P, npad, kR, kxw, w.Cs, s, ev[3], ev[4], 0, tcut_dev, w.tab[1],
                nbw);
    const bool grouping = o.group_tau > 0.0;
    if (grouping) STEP(hipMemsetAsync(w.cpl, 0, sizeof(int), s));
    launch_epi_w(w.Cs, npad, 2, dw - 1, w.dcut[1], w.eX, w.eR, w.lam, w.lam_lo, w.r, n, w.eE,
                 w.emax, w.EP, kKeMax, w.flags, s, o.group_tau, grouping ? w.cpl : nullptr,
                 w.cpl + 64, kCouplingsMax, tcut_dev);
    STEP(hipEventRecord(ev[15], s));
    STEP(hipMemcpyAsync(eE.data(), w.eE, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(emax.data(), w.emax, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
    STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    int ncpl = 0;
    if (grouping) STEP(hipMemcpyAsync(&ncpl, w.cpl, sizeof(int), hipMemcpyDeviceToHost, s));
    STEP(hipStreamSynchronize(s));
    if (grouping && ncpl > 0 && ncpl <= kCouplingsMax) {
      cpl.resize(2 * (size_t)ncpl);
      STEP(hipMemcpyAsync(cpl.data(), w.cpl + 64, sizeof(int) * 2 * ncpl, hipMemcpyDeviceToHost,
                          s));
      STEP(hipStreamSynchronize(s));
    }
    if (hflags & FLAG_TIE) return cleanup(REFEIG_E_GAP);
    if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
    // ---- grouped correction (opt-in; not part of the paper's method): every pair (i, j)
    // whose first-order correction |e_ij| exceeds group_tau links columns i and j; each
    // linked group gets the Rayleigh-Ritz solution on its span instead of the first-order
    // entries. (More couplings than the list holds: no grouping in this iteration.)
    int ngroups = 0;
    if (grouping && ncpl > 0 && ncpl <= kCouplingsMax) {
      std::vector<int> par(n);
      for (int j = 0; j < n; ++j) par[j] = j;
      for (int q = 0; q < ncpl; ++q) {
        int a = uf_root(par, cpl[2 * q]), b = uf_root(par, cpl[2 * q + 1]);
        if (a != b) par[std::max(a, b)] = std::min(a, b);
      }
      std::vector<std::vector<int>> comp(n);
      for (int j = 0; j < n; ++j) comp[uf_root(par, j)].push_back(j);
      std::vector<int> gcol, gfirst, gk, gpos, gbase, pa, pb;
      std::vector<int> gstart;   // first member slot of each group
      int ybase = 0;
      for (int root = 0; root < n; ++root) {
        const int k = (int)comp[root].size();
        if (k < 2 || k > kGroupMax || (int)gcol.size() + k > kGroupColsMax) continue;
        const int first = (int)gcol.size();
        gstart.push_back(first);
        for (int a = 0; a < k; ++a) {
          gcol.push_back(comp[root][a]);
          gfirst.push_back(first);
          gk.push_back(k);
          gpos.push_back(a);
          gbase.push_back(ybase);
          for (int b = 0; b < k; ++b) {
            pa.push_back(comp[root][a]);
            pb.push_back(comp[root][b]);
          }
        }
        ybase += k * k;
      }
      ngroups = (int)gstart.size();
      if (verbose) {
        int linked = 0, biggest = 0, skipped = 0;
        for (int root = 0; root < n; ++root) {
          const int k = (int)comp[root].size();
          if (k < 2) continue;
          linked += k;
          biggest = std::max(biggest, k);
        }
        for (int root = 0; root < n; ++root)
          if ((int)comp[root].size() > kGroupMax) ++skipped;
        fprintf(stderr, "refeig it %d: %d groups (%d linked columns, largest %d, %d too large)\n",
                it + 1, ngroups, linked, biggest, skipped);
      }
      if (ngroups > 0) {
        const int nmem = (int)gcol.size(), npr = (int)pa.size();
        STEP(hipMemcpyAsync(w.g_pa, pa.data(), sizeof(int) * npr, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_pb, pb.data(), sizeof(int) * npr, hipMemcpyHostToDevice, s));
        launch_group_gram(w.Cs, npad, 2, dw - 1, w.dcut[1], w.eX, w.eR, w.X1, n, w.g_pa, w.g_pb,
                          npr, w.g_gh, w.g_gl, w.g_w, s, tcut_dev);
        std::vector<double> gh(npr), gl(npr), gw(npr), Yh(npr), muh(nmem), mul(nmem), laml(n);
        STEP(hipMemcpyAsync(laml.data(), w.lam_lo, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        STEP(hipMemcpyAsync(gh.data(), w.g_gh, sizeof(double) * npr, hipMemcpyDeviceToHost, s));
        STEP(hipMemcpyAsync(gl.data(), w.g_gl, sizeof(double) * npr, hipMemcpyDeviceToHost, s));
        STEP(hipMemcpyAsync(gw.data(), w.g_w, sizeof(double) * npr, hipMemcpyDeviceToHost, s));
        STEP(hipStreamSynchronize(s));
        for (int g = 0; g < ngroups; ++g) {
          const int first = gstart[g], k = gk[first], base = gbase[first];
          std::vector<HD> G(k * k);
          std::vector<double> Wg(k * k);
          std::vector<HD> lamg(k);
          for (int q = 0; q < k * k; ++q) {
            G[q] = {gh[base + q], gl[base + q]};
            Wg[q] = gw[base + q];
          }
          for (int a = 0; a < k; ++a) lamg[a] = {lam[gcol[first + a]], laml[gcol[first + a]]};
          if (!group_ritz(k, G, Wg, lamg, Yh.data() + base, muh.data() + first,
                          mul.data() + first))
            return cleanup(REFEIG_E_GAP);
        }
        STEP(hipMemcpyAsync(w.g_Y, Yh.data(), sizeof(double) * npr, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_mu, muh.data(), sizeof(double) * nmem, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_mul, mul.data(), sizeof(double) * nmem, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_col, gcol.data(), sizeof(int) * nmem, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_first, gfirst.data(), sizeof(int) * nmem, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_k, gk.data(), sizeof(int) * nmem, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_pos, gpos.data(), sizeof(int) * nmem, hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(w.g_base, gbase.data(), sizeof(int) * nmem, hipMemcpyHostToDevice, s));
        launch_group_fix(w.Cs, npad, 2, dw - 1, w.dcut[1], w.eX, w.eR, w.lam, w.lam_lo, n,
                         w.g_col, w.g_first, w.g_k, w.g_pos, w.g_base, w.g_Y, w.g_mu, w.g_mul,
                         nmem, w.eE, w.emax, w.EP, kKeMax, w.flags, s, tcut_dev);
        STEP(hipMemcpyAsync(eE.data(), w.eE, sizeof(int) * npad, hipMemcpyDeviceToHost, s));
        STEP(hipMemcpyAsync(emax.data(), w.emax, sizeof(double) * npad, hipMemcpyDeviceToHost, s));
        STEP(hipMemcpyAsync(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        STEP(hipStreamSynchronize(s));
        if (hflags & FLAG_TIE) return cleanup(REFEIG_E_GAP);
        if (hflags & FLAG_NONFINITE) return cleanup(REFEIG_E_NONFINITE);
      }
    }
    double eps = 0.0;
    for (int j = 0; j < n; ++j) eps = std::max(eps, emax[j]);
    // ---- X <- X^(1) + X^(1) E~
    std::fill(dcol.begin(), dcol.end(), 2);
    for (int j = 0; j < n; ++j)
      if (emax[j] != 0.0) dcol[j] = cut_u(kx, lsqn, eE[j], theta, delta_k, wtolh[j], o.d_extra);
    const int kE = kKeMax, kxu = kx;
    if (!plan_cutoffs(dcol, n, npad, kE, kxu, std::min(kKeMax + 1, kE + kxu), w.dcut[2], dhost, s,
                      plan))
      return cleanup(REFEIG_E_HIP);
    const int du = plan.dmax;
    const double pu = plan.pairs_eff;
    int lu = (int)plan.groups.size();
    const int nbu = prepare_table(plan, npad, kE, kxu, htab[2], w.tab[2], s);
    if (nbu < 0) return cleanup(REFEIG_E_HIP);
    if (nbu > 0) lu = 1;
    STEP(hipEventRecord(ev[16], s));
    launch_plan(plan, w.EP, w.XPT, P, npad, kE, kxu, w.Cs, s, ev[5], ev[6], 0, nullptr, w.tab[2],
                nbu);
    launch_epi_u(w.Cs, npad, 2, du - 1, w.dcut[2], w.eE, w.X1, n, X, ldx, s, w.colmap);
    launch_scatter(w.lam, w.colmap, n, D, s);
    STEP(hipEventRecord(ev[17], s));
    STEP(hipEventRecord(ev[7], s));
    STEP(hipGetLastError());
    STEP(hipEventSynchronize(ev[7]));
    double pw_it = pw;
    if (tcut_dev) {   // W pairs actually computed under the per-tile cutoffs
      tcut.resize((size_t)T * T);
      STEP(hipMemcpy(tcut.data(), w.tcut, sizeof(int) * T * T, hipMemcpyDeviceToHost));
      pw_it = 0.0;
      for (int q = 0; q < T * T; ++q) {
        const int dl = std::min(tcut[q], whost[(size_t)(q / T) * 256]);   // the block's launch
        for (int d = 2; d <= dl; ++d) pw_it += npairs_of(d, kR, kxw);
      }
      pw_it /= (double)T * T;
      if (verbose && nbw > 0) {   // blocks of the W table that ran (not above their tile cutoff)
        int live = 0;
        std::vector<int> by_pairs(kKrMax + 2, 0), by_pairs_all(kKrMax + 2, 0);
        for (int e : htab[1]) {
          const int J = e & 0xff, I = (e >> 8) & 0xff, d = 2 + (e >> 16);
          const int np = npairs_of(d, kR, kxw);
          ++by_pairs_all[np];
          if (d <= tcut[(size_t)J * T + I]) {
            ++live;
            ++by_pairs[np];
          }
        }
        fprintf(stderr, "refeig it %d: W table %d blocks, %d live; live blocks by pairs:", it + 1,
                nbw, live);
        for (int q = 1; q <= kKrMax; ++q)
          if (by_pairs_all[q]) fprintf(stderr, " %d:%d/%d", q, by_pairs[q], by_pairs_all[q]);
        // live pair work by XCD (blocks go to XCDs round robin by index)
        double xw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (size_t e = 0; e < htab[1].size(); ++e) {
          const int v = htab[1][e], J = v & 0xff, I = (v >> 8) & 0xff, d = 2 + (v >> 16);
          if (d <= tcut[(size_t)J * T + I]) xw[e % 8] += npairs_of(d, kR, kxw);
        }
        fprintf(stderr, "; live pair-blocks by XCD:");
        for (int x = 0; x < 8; ++x) fprintf(stderr, " %.0f", xw[x]);
        fprintf(stderr, "\n");
      }
    }
    float t_it = 0, g1 = 0, g2 = 0, g3 = 0;
    (void)hipEventElapsedTime(&t_it, ev[0], ev[7]);
    (void)hipEventElapsedTime(&g1, ev[1], ev[2]);
    (void)hipEventElapsedTime(&g2, ev[3], ev[4]);
    (void)hipEventElapsedTime(&g3, ev[5], ev[6]);
    float ph[5] = {0, 0, 0, 0, 0};
    for (int q = 0; q < 5; ++q) (void)hipEventElapsedTime(&ph[q], ev[8 + 2 * q], ev[9 + 2 * q]);
    if (rep && it < REFEIG_MAX_ITERS) {
      rep->beta[it] = beta;
      rep->kx[it] = kx;
      rep->dv[it] = dv;
      rep->dw[it] = dw;
      rep->du[it] = du;
      rep->pairs[it] = (int)std::lround(pv + pw_it + pu);
      rep->eps[it] = eps;
      rep->ms_iter[it] = t_it;
      rep->ms_gemm[it] = g1 + g2 + g3;
      rep->pairs_p[it][0] = (int)std::lround(pv);
      rep->pairs_p[it][1] = (int)std::lround(pw_it);
      rep->pairs_p[it][2] = (int)std::lround(pu);
      rep->pairs_f[it][0] = pv;
      rep->pairs_f[it][1] = pw_it;
      rep->pairs_f[it][2] = pu;
      rep->ms_p[it][0] = g1;
      rep->ms_p[it][1] = g2;
      rep->ms_p[it][2] = g3;
      rep->launches_p[it][0] = lv;
      rep->launches_p[it][1] = lw;
      rep->launches_p[it][2] = lu;
      rep->groups[it] = ngroups;
      rep->delta_it[it] = delta_k;
      rep->vres[it] = by_res ? 1 : 0;
      for (int q = 0; q < 5; ++q) rep->ms_phase[it][q] = ph[q];
      rep->iters = it + 1;
      rep->min_gap = gmin;
      rep->max_abs_lambda = lmax;
    }
    if (verbose)
      fprintf(stderr,
              "refeig it %d: beta %d kx %d dv %d dw %d du %d pairs %d eps %.3e gap %.3e "
              "ms %.2f (gemm %.2f)\n",
              it + 1, beta, kx, dv, dw, du, (int)std::lround(pv + pw_it + pu), eps, gmin, t_it,
              g1 + g2 + g3);
    for (int p = 0; p < n; ++p) lam_prev[cmap[p]] = lam[p];
    if (o.fixed_iters > 0) {
      eps_prev = eps;
      continue;
    }
    // The correction eps = max|E~| estimates the error of X^(1) (Sec. 3.2: X = X^(1)(I + E)),
    // which never falls below the truncation grid that beta sets. The forward error after
    // the update is modelled by eq. (assume2): eps^2 max|lambda| / (xi gap); stop once that
    // is within the internal delta (xi from the options; strict mode takes xi = 1).
    const double xi_stop = (o.stop_rule == 1) ? 1.0 : xi;
    if (eps <= delta_int || eps * eps * lmax / (xi_stop * gmin) <= delta_int) break;
    if (it >= 1 && eps > 0.5 * eps_prev) {
      // no quadratic decrease: the floor that the products' truncation leaves. When that
      // floor is within the target the iterate has converged to it, else it has stagnated.
      if (eps > target) status = REFEIG_NOT_CONVERGED;
      break;
    }
    eps_prev = eps;
    if (it + 1 == iters) status = REFEIG_NOT_CONVERGED;
  }
  return cleanup(status);
#undef STEP
}

int refeig_read_report(const void *work, int n, const refeig_opts *o_in, int *status,
                       refeig_report *report) {
  refeig_opts o;
  if (o_in) o = *o_in;
  else refeig_default_opts(&o);
  if (!work || !status || n < 1 || n > kMaxN) return REFEIG_E_ARG;
  Work w;
  carve(n, ka_of(&o), (char *)work, &w, o.vmode == 1);
  DevState hst;
  int hflags = 0;
  HIPCHK(hipMemcpy(&hst, w.dst, sizeof(DevState), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&hflags, w.flags, sizeof(int), hipMemcpyDeviceToHost));
  *status = status_of(hst, hflags);
  if (report) {
    std::memset(report, 0, sizeof(*report));
    fill_report_from_device(hst, hflags, hst.iters_done, report);
    report->status = *status;
  }
  return REFEIG_OK;
}

int refeig_tile_cache_lookup(const char *arch, int npad, int *tile) {
  if (!arch || !tile || npad < 1) return REFEIG_E_ARG;
  if (npad < 1024) {
    *tile = 128;
    return REFEIG_OK;
  }
  const auto m = read_tile_cache(tile_cache_path());
  const auto it = m.find(std::string(arch) + ":" + std::to_string(npad));
  *tile = it == m.end() ? 256 : it->second;
  return it == m.end() ? REFEIG_NOT_CONVERGED : REFEIG_OK;
}

int refeig_row_nonzeros(const double *A, int lda, int n, refeig_stream_t stream, int *k) {
  if (!A || !k || n < 1 || lda < n) return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int *d = nullptr;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMalloc((void **)&d, sizeof(int)));
  HIPCHK(hipMemsetAsync(d, 0, sizeof(int), s));
  launch_row_nonzeros(A, lda, n, d, s);
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipFree(d));
  *k = h;
  return REFEIG_OK;
}

int refeig_host_beta(int n, const double *lam, const int *e, const int *c, const double *mx,
                     double target, const refeig_opts *o_in, int *beta, int *kx) {
  if (n < 1 || !lam || !e || !c || !mx || !beta || !kx || !(target > 0.0)) return REFEIG_E_ARG;
  refeig_opts o;
  if (o_in) o = *o_in;
  else refeig_default_opts(&o);
  std::vector<double> l(lam, lam + n), g, m(mx, mx + n);
  std::vector<int> ev(e, e + n), cv(c, c + n);
  double gmin, lmax;
  column_gaps(l, g, &gmin, &lmax);
  if (!(gmin > 0.0)) return REFEIG_E_GAP;
  const double xi = xi_of(o, n);
  beta_rule(n, xi, target / o.delta_safety, gmin, lmax, ev, cv, m, beta, kx);
  return REFEIG_OK;
}

int refeig_host_crt_plan(int npad, int ka1, int kx, int *N, int *moduli, int *wA, int *wX,
                         double *U, double *L, double *M) {
  if (npad < 1 || ka1 < 1 || kx < 1 || !N || !moduli || !wA || !wX || !U || !L || !M)
    return REFEIG_E_ARG;
  ResWeights a, x;
  CrtRec rec;
  if (!crt_plan(npad, ka1, kx, a, x, rec)) return REFEIG_E_ARG;
  *N = rec.N;
  for (int q = 0; q < rec.N; ++q) {
    moduli[q] = rec.m[q];
    for (int t = 0; t < kCrtPlanes; ++t) {
      wA[q * kCrtPlanes + t] = a.w[q][t];
      wX[q * kCrtPlanes + t] = x.w[q][t];
    }
  }
  for (int q = 0; q < rec.N; ++q)
    for (int c = 0; c < 3; ++c) U[3 * q + c] = rec.u[q][c];
  for (int q = 0; q < rec.N; ++q)
    for (int k = 0; k < kCrtLimbs; ++k) L[kCrtLimbs * q + k] = rec.L[q][k];
  for (int c = 0; c < 3; ++c) M[c] = rec.M[c];
  return REFEIG_OK;
}

int refeig_host_column_order(int n, const double *lam, int *order) {
  if (n < 1 || !lam || !order) return REFEIG_E_ARG;
  std::vector<double> l(lam, lam + n), g;
  double gmin, lmax;
  column_gaps(l, g, &gmin, &lmax);
  std::vector<int> cm(n);
  working_order(l, g, cm);
  for (int p = 0; p < n; ++p) order[p] = cm[p];
  return REFEIG_OK;
}

int refeig_host_group_ritz(int k, const double *G_hi, const double *G_lo, const double *W,
                           const double *lam_hi, const double *lam_lo, double *Y, double *mu_hi,
                           double *mu_lo) {
  if (k < 2 || k > kGroupMax || !G_hi || !G_lo || !W || !lam_hi || !lam_lo || !Y || !mu_hi ||
      !mu_lo)
    return REFEIG_E_ARG;
  std::vector<HD> G(k * k), lg(k);
  std::vector<double> Wg(W, W + k * k);
  for (int q = 0; q < k * k; ++q) G[q] = {G_hi[q], G_lo[q]};
  for (int a = 0; a < k; ++a) lg[a] = {lam_hi[a], lam_lo[a]};
  return group_ritz(k, G, Wg, lg, Y, mu_hi, mu_lo) ? REFEIG_OK : REFEIG_E_GAP;
}

int refeig_batched_workspace_bytes(int count, const int *n, const refeig_opts *o, size_t *bytes) {
  if (count < 1 || !n || !bytes) return REFEIG_E_ARG;
  refeig_opts opts;
  if (o) opts = *o;
  else refeig_default_opts(&opts);
  int nmax = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kMaxN) return REFEIG_E_ARG;
    nmax = std::max(nmax, n[i]);
  }
  if (grouped_batch(opts)) {
    *bytes = grouped_bytes(count, n, opts);
    return *bytes ? REFEIG_OK : REFEIG_E_ARG;
  }
  size_t one = 0;
  const int st = refeig_workspace_bytes(nmax, o, &one);
  if (st != REFEIG_OK) return st;
  *bytes = (size_t)std::min(count, REFEIG_BATCH_LANES) * ((one + 255) / 256 * 256);
  return REFEIG_OK;
}

int refine_eigvecs_batched(int count, const int *n, const double *const *A, const int *lda,
                           double *const *X, const int *ldx, double *const *D,
                           const double *target, const refeig_opts *o, void *work,
                           size_t work_bytes, refeig_stream_t stream, refeig_report *reports) {
  if (count < 1 || !n || !A || !lda || !X || !ldx || !D || !target) return REFEIG_E_ARG;
  size_t need = 0;
  int st = refeig_batched_workspace_bytes(count, n, o, &need);
  if (st != REFEIG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  bool own = false;
  if (!work) {
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMalloc(&work, need));
    own = true;
  } else if (work_bytes < need) {
    return REFEIG_E_NOMEM;
  }
  refeig_opts opts;
  if (o) opts = *o;
  else refeig_default_opts(&opts);
  if (grouped_batch(opts)) {
    const int st = refine_grouped(count, n, A, lda, X, ldx, D, target, opts, (char *)work, need,
                                  s, reports);
    if (own) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(work);
    }
    return st;
  }
  const int lanes = std::min(count, REFEIG_BATCH_LANES);
  const size_t slice = need / lanes;
  // lanes: own streams (default priority), joined to the caller's stream by events
  std::vector<hipStream_t> ls(lanes, nullptr);
  std::vector<hipEvent_t> le(lanes + 1, nullptr);
  bool ok = hipEventCreateWithFlags(&le[lanes], hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(le[lanes], s) == hipSuccess;
  for (int l = 0; l < lanes && ok; ++l)
    ok = hipStreamCreateWithFlags(&ls[l], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&le[l], hipEventDisableTiming) == hipSuccess &&
         hipStreamWaitEvent(ls[l], le[lanes], 0) == hipSuccess;
  std::vector<int> status(count, REFEIG_E_HIP);
  if (ok) {
    // each lane takes the next unstarted problem until none is left
    std::atomic<int> next{0};
    auto run_lane = [&](int l) {
      char *wl = (char *)work + (size_t)l * slice;
      for (int i = next++; i < count; i = next++)
        status[i] = refine_eigvecs(A[i], lda[i], X[i], ldx[i], D[i], n[i], target[i], o, wl,
                                   slice, (refeig_stream_t)ls[l], reports ? &reports[i] : nullptr);
    };
    std::vector<std::thread> th;
    for (int l = 1; l < lanes; ++l) th.emplace_back(run_lane, l);
    run_lane(0);
    for (auto &t : th) t.join();
    for (int l = 0; l < lanes; ++l)
      ok = ok && hipEventRecord(le[l], ls[l]) == hipSuccess &&
           hipStreamWaitEvent(s, le[l], 0) == hipSuccess;
  }
  for (int l = 0; l < lanes; ++l) {
    if (ls[l]) (void)hipStreamSynchronize(ls[l]);
    if (ls[l]) (void)hipStreamDestroy(ls[l]);
    if (le[l]) (void)hipEventDestroy(le[l]);
  }
  if (le[lanes]) (void)hipEventDestroy(le[lanes]);
  if (own) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(work);
  }
  if (!ok) return REFEIG_E_HIP;
  int worst = REFEIG_OK;
  for (int i = 0; i < count; ++i) {
    if (status[i] < 0) return status[i];
    if (status[i] != REFEIG_OK) worst = status[i];
  }
  return worst;
}


// ---- a grouped batch captured once in a HIP graph and replayed
struct refeig_batch {
  int count = 0;
  refeig_opts o;
  ChunkPlan cp;
  GroupArea ga;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;
  bool launched = false;
};

static int batch_need(int count, const int *n, const refeig_opts &o, size_t *icap, size_t *sum) {
  if (count < 1 || !n) return REFEIG_E_ARG;
  if (!grouped_batch(o) || o.fixed_iters < 1 || !opts_valid(o)) return REFEIG_E_ARG;
  *icap = 0;
  *sum = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kMaxN || round_up(n[i], kTile) > kGroupMaxNpad) return REFEIG_E_ARG;
    *icap += item_cap(n[i]);
    *sum += ws_rounded(n[i], o);
  }
  return REFEIG_OK;
}

int refeig_batch_workspace_bytes(int count, const int *n, const refeig_opts *o_in,
                                 size_t *bytes) {
  refeig_opts o;
  if (o_in) o = *o_in;
  else refeig_default_opts(&o);
  size_t icap = 0, sum = 0;
  if (!bytes) return REFEIG_E_ARG;
  const int st = batch_need(count, n, o, &icap, &sum);
  if (st != REFEIG_OK) return st;
  *bytes = group_area(count, icap, nullptr, nullptr) + sum;
  return REFEIG_OK;
}

int refeig_batch_create(int count, const int *n, const double *const *A, const int *lda,
                        double *const *X, const int *ldx, double *const *D,
                        const double *target, const refeig_opts *o_in, void *work,
                        size_t work_bytes, refeig_batch **out) {
  if (!out) return REFEIG_E_ARG;
  *out = nullptr;
  refeig_opts o;
  if (o_in) o = *o_in;
  else refeig_default_opts(&o);
  size_t icap = 0, sum = 0;
  int st = batch_need(count, n, o, &icap, &sum);
  if (st != REFEIG_OK) return st;
  if (!A || !lda || !X || !ldx || !D || !target || !work) return REFEIG_E_ARG;
  for (int i = 0; i < count; ++i)
    if (!A[i] || !X[i] || !D[i] || lda[i] < n[i] || ldx[i] < n[i] || !(target[i] > 0.0))
      return REFEIG_E_ARG;
  const size_t area = group_area(count, icap, nullptr, nullptr);
  if (work_bytes < area + sum) return REFEIG_E_NOMEM;
  std::vector<int> ids(count), npads(count);
  for (int i = 0; i < count; ++i) {
    ids[i] = i;
    npads[i] = round_up(n[i], kTile);
  }
  ensure_tiles(npads, (char *)work + area, work_bytes - area, nullptr);
  std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
    const int ta = gtile_of(npads[a]), tb = gtile_of(npads[b]);
    return ta != tb ? ta > tb : npads[a] > npads[b];
  });
  auto *b = new refeig_batch();
  b->count = count;
  b->o = o;
  group_area(count, icap, (char *)work, &b->ga);
  prepare_chunk(b->cp, ids, n, A, lda, X, ldx, D, target, o, (char *)work + area);
  hipStream_t cs = nullptr;
  bool ok = hipMemcpy(b->ga.gp, b->cp.hp.data(), sizeof(GProb) * b->cp.G,
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
            hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    enqueue_chunk(b->cp, b->ga, o, 0, o.fixed_iters, true, cs);
    ok = hipStreamEndCapture(cs, &b->graph) == hipSuccess &&
         hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok) {
    refeig_batch_destroy(b);
    return REFEIG_E_HIP;
  }
  *out = b;
  return REFEIG_OK;
}

int refeig_batch_launch(refeig_batch *b, refeig_stream_t stream) {
  if (!b || !b->exec) return REFEIG_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipGraphLaunch(b->exec, s));
  b->last = s;
  b->launched = true;
  return REFEIG_OK;
}

int refeig_batch_results(refeig_batch *b, int *status, refeig_report *reports) {
  if (!b || !status || !b->launched) return REFEIG_E_ARG;
  HIPCHK(hipStreamSynchronize(b->last));
  std::vector<int> st(b->count, REFEIG_E_HIP);
  const int r = collect_chunk(b->cp, b->ga, 0.0, reports, st.data());
  if (r != REFEIG_OK) return r;
  int worst = REFEIG_OK;
  for (int i = 0; i < b->count; ++i) {
    status[i] = st[i];
    if (st[i] < 0 && worst >= 0) worst = st[i];
    else if (st[i] != REFEIG_OK && worst == REFEIG_OK) worst = st[i];
  }
  return worst;
}

int refeig_batch_destroy(refeig_batch *b) {
  if (!b) return REFEIG_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return REFEIG_OK;
}

}  // extern "C"

namespace {

// ---- HBM-footprint admission of the serving loop (the server below and its host-only
// simulation share it). A request holds its workspace, refeig_workspace_bytes(n) rounded to
// 256 bytes, in the server's arena from its start until it completes.
struct Arena {
  std::map<size_t, size_t> free_;   // offset -> length of each free run
  explicit Arena(size_t size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {   // first fit
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        const size_t o = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[o + bytes] = rest;
        *off = o;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Pending {
  int ticket;
  size_t bytes;
  int passed;   // later requests that started before this one
};

// When a lane is free: the oldest pending request whose workspace fits in the arena starts.
// A request that does not fit may be passed by later ones that do, at most kBypassMax
// times; after that nothing starts before it (no starvation of large requests). Returns the
// queue index (and the arena offset) or -1.
constexpr int kBypassMax = 4;
int admit(std::deque<Pending> &q, Arena &ar, size_t *off) {
  for (size_t i = 0; i < q.size(); ++i) {
    if (ar.alloc(q[i].bytes, off)) {
      for (size_t k = 0; k < i; ++k) ++q[k].passed;
      return (int)i;
    }
    if (q[i].passed >= kBypassMax) return -1;
  }
  return -1;
}

size_t request_bytes(int n, const refeig_opts *o) {
  size_t b = 0;
  if (refeig_workspace_bytes(n, o, &b) != REFEIG_OK) return 0;
  return (b + 255) / 256 * 256;
}

}  // namespace

struct refeig_server {
  struct Req {
    const double *A;
    double *X, *D;
    int lda, ldx, n;
    double target;
    size_t bytes;
    hipEvent_t ready;   // recorded on the caller's stream at submission
  };
  struct Done {
    int status = REFEIG_E_HIP;
    refeig_report rep;
    double t_done = 0.0;
  };
  int device = 0, lanes = 0;
  size_t budget = 0;
  refeig_opts opts;
  void *base = nullptr;
  Arena arena{0};
  std::vector<hipStream_t> streams;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::unordered_map<int, Req> reqs;      // submitted, not yet started
  std::unordered_map<int, Done> results;  // finished, not yet waited for
  std::unordered_set<int> live;           // submitted, not yet waited for
  int next_ticket = 0;
  bool stop = false;

  static double now() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
  }
  void lane(int l) {
    (void)hipSetDevice(device);
    for (;;) {
      int t = -1;
      size_t off = 0;
      Req r;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (!queue.empty()) {
            const int i = admit(queue, arena, &off);
            if (i >= 0) {
              t = queue[i].ticket;
              queue.erase(queue.begin() + i);
              r = reqs[t];
              reqs.erase(t);
              break;
            }
          } else if (stop) {
            return;
          }
          cv_work.wait(lk);
        }
      }
      // the caller's writes of A, X and D (on its stream) come first
      refeig_report rep;
      int st = REFEIG_E_HIP;
      if (hipStreamWaitEvent(streams[l], r.ready, 0) == hipSuccess)
        st = refine_eigvecs(r.A, r.lda, r.X, r.ldx, r.D, r.n, r.target, &opts,
                            (char *)base + off, r.bytes, (refeig_stream_t)streams[l], &rep);
      // refine_eigvecs returns after its last kernel has finished (it waits for it)
      (void)hipEventDestroy(r.ready);
      const double td = now();
      {
        std::lock_guard<std::mutex> lk(mu);
        arena.release(off, r.bytes);
        Done &d = results[t];
        d.status = st;
        d.rep = rep;
        d.t_done = td;
      }
      cv_done.notify_all();
      cv_work.notify_all();   // freed memory may admit waiting requests
    }
  }
};

extern "C" {

int refeig_server_create(int lanes, size_t budget_bytes, const refeig_opts *o,
                         refeig_server **server) {
  if (!server || lanes < 1 || lanes > 64 || budget_bytes < 256) return REFEIG_E_ARG;
  *server = nullptr;
  refeig_server *sv = new refeig_server();
  if (o) sv->opts = *o;
  else refeig_default_opts(&sv->opts);
  sv->lanes = lanes;
  sv->budget = budget_bytes / 256 * 256;
  sv->arena = Arena(sv->budget);
  if (hipGetDevice(&sv->device) != hipSuccess || hipMalloc(&sv->base, sv->budget) != hipSuccess) {
    delete sv;
    return REFEIG_E_NOMEM;
  }
  sv->streams.assign(lanes, nullptr);
  for (int l = 0; l < lanes; ++l)
    if (hipStreamCreateWithFlags(&sv->streams[l], hipStreamNonBlocking) != hipSuccess) {
      for (int k = 0; k < l; ++k) (void)hipStreamDestroy(sv->streams[k]);
      (void)hipFree(sv->base);
      delete sv;
      return REFEIG_E_HIP;
    }
  for (int l = 0; l < lanes; ++l) sv->threads.emplace_back(&refeig_server::lane, sv, l);
  *server = sv;
  return REFEIG_OK;
}

int refeig_server_submit(refeig_server *sv, const double *A, int lda, double *X, int ldx,
                         double *D, int n, double target_fwd_err, refeig_stream_t stream,
                         int *ticket) {
  if (!sv || !A || !X || !D || !ticket || n < 1 || n > kMaxN || lda < n || ldx < n ||
      !(target_fwd_err > 0.0))
    return REFEIG_E_ARG;
  const size_t bytes = request_bytes(n, &sv->opts);
  if (bytes == 0) return REFEIG_E_ARG;
  if (bytes > sv->budget) return REFEIG_E_NOMEM;   // would never fit
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return REFEIG_E_HIP;
  if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return REFEIG_E_HIP;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      (void)hipEventDestroy(ev);
      return REFEIG_E_ARG;
    }
    *ticket = sv->next_ticket++;
    sv->reqs[*ticket] = {A, X, D, lda, ldx, n, target_fwd_err, bytes, ev};
    sv->queue.push_back({*ticket, bytes, 0});
    sv->live.insert(*ticket);
  }
  sv->cv_work.notify_one();
  return REFEIG_OK;
}

int refeig_server_wait(refeig_server *sv, int ticket, int *status, refeig_report *report,
                       double *t_done) {
  if (!sv || !status) return REFEIG_E_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (!sv->live.count(ticket)) return REFEIG_E_ARG;
  sv->cv_done.wait(lk, [&] { return sv->results.count(ticket) > 0; });
  const refeig_server::Done &d = sv->results[ticket];
  *status = d.status;
  if (report) *report = d.rep;
  if (t_done) *t_done = d.t_done;
  sv->results.erase(ticket);
  sv->live.erase(ticket);
  return REFEIG_OK;
}

int refeig_server_destroy(refeig_server *sv) {
  if (!sv) return REFEIG_E_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto &t : sv->threads) t.join();
  for (auto st : sv->streams)
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  (void)hipFree(sv->base);
  delete sv;
  return REFEIG_OK;
}

int refeig_server_request_bytes(int n, const refeig_opts *o, size_t *bytes) {
  if (!bytes || n < 1 || n > kMaxN) return REFEIG_E_ARG;
  refeig_opts d;
  if (!o) {
    refeig_default_opts(&d);
    o = &d;
  }
  *bytes = request_bytes(n, o);
  return *bytes ? REFEIG_OK : REFEIG_E_ARG;
}

int refeig_host_admission_sim(int count, const double *t_arr, const size_t *bytes,
                              const double *dur, int lanes, size_t budget, double *t_start,
                              size_t *offset) {
  if (count < 0 || lanes < 1 || (count > 0 && (!t_arr || !bytes || !dur || !t_start)))
    return REFEIG_E_ARG;
  for (int i = 0; i < count; ++i)
    if (!(dur[i] >= 0.0) || (i > 0 && t_arr[i] < t_arr[i - 1])) return REFEIG_E_ARG;
  budget = budget / 256 * 256;
  Arena ar(budget);
  std::deque<Pending> q;
  struct Run {
    double t_end;
    int req;
    size_t off;
    bool operator>(const Run &o) const { return t_end > o.t_end || (t_end == o.t_end && req > o.req); }
  };
  std::priority_queue<Run, std::vector<Run>, std::greater<Run>> running;
  std::vector<size_t> rb(count);
  int next = 0, busy = 0;
  double now = 0.0;
  for (int i = 0; i < count; ++i) {
    t_start[i] = -1.0;
    if (offset) offset[i] = 0;
    rb[i] = (bytes[i] + 255) / 256 * 256;
  }
  while (next < count || !running.empty()) {
    // next event: a completion first when it is not later than the next arrival
    if (!running.empty() && (next >= count || running.top().t_end <= t_arr[next])) {
      const Run r = running.top();
      running.pop();
      now = r.t_end;
      ar.release(r.off, rb[r.req]);
      --busy;
    } else {
      now = t_arr[next];
      if (rb[next] <= budget) q.push_back({next, rb[next], 0});
      ++next;
    }
    size_t off = 0;
    while (busy < lanes && !q.empty()) {
      const int i = admit(q, ar, &off);
      if (i < 0) break;
      const int rq = q[i].ticket;
      q.erase(q.begin() + i);
      t_start[rq] = now;
      if (offset) offset[rq] = off;
      running.push({now + dur[rq], rq, off});
      ++busy;
    }
  }
  return REFEIG_OK;
}

}  // extern "C"
