// Device-side planning of the refinement iteration (see devplan.h). Every kernel here is a
// single block of 1024 threads except the residue kernel; the arithmetic of the decisions is
// the shared code of plan.h, so the plan matches the host orchestrator's.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cstdint>

#include "../../include/refeig.h"
#include "devplan.h"
#include "plan.h"
#include "work.h"

namespace refeig {

namespace {

constexpr int kPT = 1024;   // threads of a planning kernel

// Block-wide reductions (every thread gets the result). s: shared scratch of >= 16 entries.
__device__ double blk_max_d(double v, double *s) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = s[0];
  for (int q = 1; q < kPT / 64; ++q) m = fmax(m, s[q]);
  __syncthreads();
  return m;
}
__device__ double blk_min_d(double v, double *s) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = s[0];
  for (int q = 1; q < kPT / 64; ++q) m = fmin(m, s[q]);
  __syncthreads();
  return m;
}
__device__ int blk_max_i(int v, int *s) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  int m = s[0];
  for (int q = 1; q < kPT / 64; ++q) m = max(m, s[q]);
  __syncthreads();
  return m;
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Bitonic sort of N2 (a power of two, <= kDevSortMax) entries (key, aux) ascending by (key,
// aux), in LDS. Entry i belongs to thread i mod kPT (R = N2 / kPT entries per thread, at
// least 1). The exchanges at distance j < 64 pair lanes of one wavefront and run in registers
// (shuffles, no barrier); the longer ones go through LDS, each thread loading all its pairs
// before it compares and stores them, so the R independent exchanges overlap.
template <typename K, int R>
__device__ void bitonic_r(K *key, int *aux, int N2) {
  const int lane = threadIdx.x & 63;
  for (int k = 2; k <= N2; k <<= 1) {
    int j = k >> 1;
    for (; j >= 64; j >>= 1) {
      __syncthreads();
      K a[R], bv[R];
      int ia[R], ib[R];
      bool act[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + r * kPT, l = i ^ j;
        act[r] = i < N2 && l > i;
        if (act[r]) {
          a[r] = key[i];
          bv[r] = key[l];
          ia[r] = aux[i];
          ib[r] = aux[l];
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + r * kPT, l = i ^ j;
        if (act[r]) {
          const bool up = (i & k) == 0;
          const bool gt = (a[r] > bv[r]) || (a[r] == bv[r] && ia[r] > ib[r]);
          if (gt == up) {
            key[i] = bv[r];
            key[l] = a[r];
            aux[i] = ib[r];
            aux[l] = ia[r];
          }
        }
      }
    }
    __syncthreads();
    K a[R];
    int ia[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = threadIdx.x + r * kPT;
      a[r] = i < N2 ? key[i] : K(0);
      ia[r] = i < N2 ? aux[i] : 0;
    }
    for (int jj = j; jj > 0; jj >>= 1) {
      const bool low = (lane & jj) == 0;   // this entry is the pair's lower index
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + r * kPT;
        const bool up = (i & k) == 0;
        const K b = __shfl_xor(a[r], jj);
        const int ib = __shfl_xor(ia[r], jj);
        // the pair (lower, upper) is out of order when lower > upper
        const bool gt = low ? ((a[r] > b) || (a[r] == b && ia[r] > ib))
                            : ((b > a[r]) || (b == a[r] && ib > ia[r]));
        if (gt == up) {
          a[r] = b;
          ia[r] = ib;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = threadIdx.x + r * kPT;
      if (i < N2) {
        key[i] = a[r];
        aux[i] = ia[r];
      }
    }
  }
  __syncthreads();
}
template <typename K>
__device__ void bitonic(K *key, int *aux, int N2) {
  static_assert(kDevSortMax == 8 * kPT, "entries per thread: 1, 2, 4 or 8");
  if (N2 <= kPT) bitonic_r<K, 1>(key, aux, N2);
  else if (N2 <= 2 * kPT) bitonic_r<K, 2>(key, aux, N2);
  else if (N2 <= 4 * kPT) bitonic_r<K, 4>(key, aux, N2);
  else bitonic_r<K, 8>(key, aux, N2);
}

// Block table of a tabled slice-GEMM launch from each tile's last diagonal dt[J] (LDS, ntile
// tiles per side, 2 <= dt[J] <= kMaxDiag + 1): groups of tiles with equal dt, largest first;
// (group, slot) combinations ordered by pair count, most first (stable); within one, the XCD
// XCD order of xcd_tile_order. Entry = row tile | column tile << 8 | slot << 16. Returns the
// entry count. The slots are ranked once by pair count (descending, stable); a run of slots
// with equal counts is taken group by group, and in a group the slots q with q + 2 <= dt (a
// prefix of the run, which holds ascending q): block (run r, group g) holds those
// combinations' entries, and the blocks follow each other run by run, group by group.
constexpr int kTabRuns = kMaxDiag;   // runs and groups a block index is formed from
struct TabScratch {
  int vcnt[kMaxDiag + 2], gidx[kMaxDiag + 2];
  int gval[kMaxDiag + 2], gcnt[kMaxDiag + 2], goff[kMaxDiag + 2];
  int rows[64];
  int ng, nrun;
  int np[kMaxDiag], qs[kMaxDiag], rstart[kMaxDiag + 1];
  int boff[kTabRuns * kTabRuns + 1];
  int wsum[kPT / 64];
};
__device__ int build_table(const int *dt, int ntile, int kl, int kr, int *tab, TabScratch &ts) {
  const int tid = threadIdx.x;
  if (tid < kMaxDiag + 2) ts.vcnt[tid] = 0;
  __syncthreads();
  if (tid < ntile) atomicAdd(&ts.vcnt[dt[tid]], 1);
  if (tid >= 64 && tid < 64 + kMaxDiag) ts.np[tid - 64] = npairs_of(2 + (tid - 64), kl, kr);
  __syncthreads();
  if (tid == 0) {   // groups, largest dt first
    int ng = 0, nr = 0;
    for (int v = kMaxDiag + 1; v >= 2; --v)
      if (ts.vcnt[v]) {
        ts.gval[ng] = v;
        ts.gcnt[ng] = ts.vcnt[v];
        ts.goff[ng] = nr;
        ts.gidx[v] = ng;
        nr += ts.vcnt[v];
        ++ng;
      }
    ts.ng = ng;
  }
  if (tid >= 64 && tid < 64 + kMaxDiag) {   // rank of slot q: more pairs first, then q
    const int q = tid - 64, v = ts.np[q];
    int rk = 0;
    for (int k = 0; k < kMaxDiag; ++k) rk += (ts.np[k] > v || (ts.np[k] == v && k < q)) ? 1 : 0;
    ts.qs[rk] = q;
  }
  __syncthreads();
  if (tid < ntile) {   // tile J's place in its group (ascending J)
    const int v = dt[tid];
    int rk = 0;
    for (int J = 0; J < tid; ++J) rk += dt[J] == v ? 1 : 0;
    ts.rows[ts.goff[ts.gidx[v]] + rk] = tid;
  }
  if (tid == 64) {   // runs of equal pair counts (those with pairs)
    int nrun = 0;
    for (int k = 0; k < kMaxDiag; ++k) {
      if (ts.np[ts.qs[k]] < 1) break;
      if (k == 0 || ts.np[ts.qs[k]] != ts.np[ts.qs[k - 1]]) ts.rstart[nrun++] = k;
    }
    int end = 0;
    while (end < kMaxDiag && ts.np[ts.qs[end]] >= 1) ++end;
    ts.rstart[nrun] = end;
    ts.nrun = nrun;
  }
  __syncthreads();
  // block (r, g) = thread r kTabRuns + g: its entry count, then an exclusive scan in that order
  int sz = 0;
  {
    const int r = tid / kTabRuns, g = tid % kTabRuns;
    if (r < ts.nrun && g < ts.ng) {
      int c = 0;
      for (int k = ts.rstart[r]; k < ts.rstart[r + 1]; ++k) c += ts.qs[k] + 2 <= ts.gval[g] ? 1 : 0;
      sz = c * ts.gcnt[g] * ntile;
    }
  }
  static_assert(kTabRuns * kTabRuns == kPT, "one thread per (run, group) block");
  const int lane = tid & 63, wv = tid >> 6;
  int v = sz;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane == 63) ts.wsum[wv] = v;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wv; ++w) before += ts.wsum[w];
  ts.boff[tid] = before + v - sz;
  if (tid == kPT - 1) ts.boff[kPT] = before + v;
  __syncthreads();
  const int total = ts.boff[kPT];
  for (int e = tid; e < total; e += kPT) {
    int lo = 0, hi = kPT - 1;   // the last block starting at or before e (it holds e)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ts.boff[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int r = lo / kTabRuns, g = lo % kTabRuns;
    const int per = ts.gcnt[g] * ntile, local = e - ts.boff[lo];
    const int k = local / per, within = local - k * per;
    const int q = ts.qs[ts.rstart[r] + k];
    int mi, nb;
    xcd_tile_order(within, ts.gcnt[g], ntile, mi, nb);
    tab[e] = ts.rows[ts.goff[g] + mi] | (nb << 8) | (q << 16);
  }
  __syncthreads();
  return total;
}

// Per-tile last diagonal from per-column cutoffs: dt = min(max(2, max over the tile's
// columns < n), dallowed); every column of the tile (padding included) gets dt in dcut.
// Returns the largest dt and the pair work in n x n x n products (tiles of tr rows).
__device__ int tile_cutoffs_from_columns(int *dtile, const int *dcol_lds, int n, int npad, int tr,
                                         int dallowed, int kl, int kr, int *dcut, double *pairs,
                                         int *ired) {
  const int nt = npad / tr;
  for (int J = threadIdx.x; J < nt; J += kPT) {
    int d = 2;
    for (int j = J * tr; j < min((J + 1) * tr, n); ++j) d = max(d, dcol_lds[j]);
    dtile[J] = min(d, dallowed);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < npad; j += kPT) dcut[j] = dtile[j / tr];
  int dm = 2;
  for (int J = threadIdx.x; J < nt; J += kPT) dm = max(dm, dtile[J]);
  dm = blk_max_i(dm, ired);
  if (threadIdx.x == 0) {
    double pe = 0.0;
    for (int J = 0; J < nt; ++J) {
      int pr = 0;
      for (int d = 2; d <= dtile[J]; ++d) pr += npairs_of(d, kl, kr);
      pe += pr * (double)tr / npad;
    }
    *pairs = pe;
  }
  __syncthreads();
  return dm;
}

}  // namespace

// ---------------------------------------------------------------- once per solve
__device__ __forceinline__ void dp_init_body(PlanParams p, PlanBufs b) {
  __shared__ double red[16];
  __shared__ int ired[16];
  int em = -100000;
  double h = 0.0;
  for (int i = threadIdx.x; i < p.n; i += kPT) {
    em = max(em, b.eA[i]);
    if (b.mxA[i] != 0.0) h = fmax(h, ldexp(sqrt(b.ssA[i]), -b.eA[i]));
  }
  em = blk_max_i(em, ired);
  h = blk_max_d(h, red);
  if (threadIdx.x < kCrtMax) b.mods[threadIdx.x] = modulus(threadIdx.x);
  if (threadIdx.x == 0) {
    DevState &st = *b.st;
    st.eA_max = em;
    st.hA = h;
    st.done = 0;
    st.skip = 0;
    st.stop_status = 0;
    st.iters_done = 0;
    st.eps_prev = INFINITY;
    for (int l = 0; l < kVLevels; ++l) {
      st.ares_ka[l] = st.ares_n[l] = -1;
      st.ares_dirty[l] = 0;
    }
  }
}

__global__ __launch_bounds__(kPT) void k_dp_init(PlanParams p, PlanBufs b) {
  dp_init_body(p, b);
}

// ---------------------------------------------------------------- working column order
// From the entry estimates D (natural order): gaps, the smallest gap and max |lambda|, and the
// working order (gap descending, ties by eigenvalue ascending): colmap, gapsw.
__device__ __forceinline__ void dp_order_body(PlanParams p, PlanBufs b) {
  __shared__ double key[kDevSortMax];    // eigenvalues, then the gap keys (as 64-bit ints)
  __shared__ int idx[kDevSortMax];       // sorted position -> column
  __shared__ int rk[kDevSortMax];        // second sort: rank in eigenvalue order
  __shared__ double red[16];
  const int n = p.n, N2 = pow2_at_least(n);
  // after the first iteration, D holds the last W plan's Rayleigh quotients, already sorted
  // (unless an error stopped the update; ties, gap 0, are an error either way)
  __shared__ int s_reuse;
  if (threadIdx.x == 0) s_reuse = p.it > 0 && !(*b.flags & kFlagsError);
  __syncthreads();
  if (s_reuse) {
    for (int i = threadIdx.x; i < N2; i += kPT) {
      key[i] = i < n ? b.skey[i] : INFINITY;
      idx[i] = i < n ? b.sidx[i] : i;
    }
    __syncthreads();
  } else {
    int bad = 0;
    for (int i = threadIdx.x; i < N2; i += kPT) {
      double v = i < n ? b.D[i] : INFINITY;
      if (i < n && !(fabs(v) <= DBL_MAX)) {
        bad = 1;
        v = 0.0;
      }
      key[i] = v;
      idx[i] = i;
    }
    if (bad) atomicOr(b.flags, FLAG_NONFINITE);
    bitonic<double>(key, idx, N2);
  }
  double lmax;
  // gaps in eigenvalue order, kept in registers of the thread that owns the position (at
  // most kDevSortMax / kPT per thread)
  double gl[kDevSortMax / kPT];
  double gm = INFINITY, lm = 0.0;
#pragma unroll
  for (int q = 0; q < kDevSortMax / kPT; ++q) {
    const int pp = threadIdx.x + q * kPT;
    gl[q] = INFINITY;
    if (pp < n) {
      const double dl = pp > 0 ? key[pp] - key[pp - 1] : INFINITY;
      const double dr = pp + 1 < n ? key[pp + 1] - key[pp] : INFINITY;
      gl[q] = fmin(dl, dr);
      gm = fmin(gm, dr);
      lm = fmax(lm, fabs(key[pp]));
    }
  }
  gm = blk_min_d(gm, red);
  lmax = blk_max_d(lm, red);
  if (n == 1) {
    gl[0] = 1.0;
    gm = 1.0;
  }
  if (!(gm > 0.0) && threadIdx.x == 0) atomicOr(b.flags, FLAG_GAP);
  __syncthreads();
  // second sort: keys ~bits(g) ascending = g descending, ties by eigenvalue rank
  unsigned long long *k2 = (unsigned long long *)key;
  auto fill_k2 = [&]() {
#pragma unroll
    for (int q = 0; q < kDevSortMax / kPT; ++q) {
      const int pp = threadIdx.x + q * kPT;
      if (pp < N2) {
        k2[pp] = pp < n ? ~(unsigned long long)__double_as_longlong(gl[q]) : ~0ull;
        rk[pp] = pp;
      }
    }
  };
  fill_k2();
  // After the first iteration the gaps usually keep the previous working order (b.colmap,
  // not yet rewritten): put the keys in that order and sort only if (key, rank) is not
  // strictly ascending there. The comparator orders by (key, rank), so the sorted order is
  // unique and both ways give the same keys and ranks.
  __shared__ int s_sorted;
  if (threadIdx.x == 0) s_sorted = s_reuse;
  __syncthreads();
  if (s_sorted) {
    constexpr int kE = kDevSortMax / kPT;
    int rq[kE];
    unsigned long long kq[kE];
    for (int r = threadIdx.x; r < n; r += kPT) rk[idx[r]] = r;   // column -> rank
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      const int pp = threadIdx.x + q * kPT;
      rq[q] = pp < n ? rk[b.colmap[pp]] : pp;
      kq[q] = pp < n ? k2[rq[q]] : ~0ull;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      const int pp = threadIdx.x + q * kPT;
      if (pp < N2) {
        k2[pp] = kq[q];
        rk[pp] = rq[q];
      }
    }
    __syncthreads();
    int bad = 0;
    for (int pp = threadIdx.x; pp + 1 < n; pp += kPT)
      bad |= !(k2[pp] < k2[pp + 1] || (k2[pp] == k2[pp + 1] && rk[pp] < rk[pp + 1]));
    if (bad) s_sorted = 0;   // every writer writes the same value
    __syncthreads();
    if (!s_sorted) fill_k2();
  }
  if (!s_sorted) bitonic<unsigned long long>(k2, rk, N2);
  for (int q = threadIdx.x; q < p.npad; q += kPT) {
    if (q < n) {
      const int r = rk[q];
      b.colmap[q] = idx[r];
      b.gapsw[q] = __longlong_as_double((long long)~k2[q]);
    } else {
      b.colmap[q] = q;
      b.gapsw[q] = 0.0;
    }
  }
  if (threadIdx.x == 0) {
    b.st->gmin = gm;
    b.st->lmax = lmax;
  }
}

__global__ __launch_bounds__(kPT) void k_dp_order(PlanParams p, PlanBufs b) {
  dp_order_body(p, b);
}

// ---------------------------------------------------------------- beta, kx and the V plan
__device__ __forceinline__ void dp_vplan_body(PlanParams p, PlanBufs b) {
  __shared__ int hist[kBetaBins];
  __shared__ int dcol[kDevSortMax];
  __shared__ int dtile[64];
  __shared__ int kab[kDevSortMax / 256], lvb[kDevSortMax / 256];
  __shared__ double red[16];
  __shared__ int ired[16];
  __shared__ int s_ok, s_kx;
  __shared__ TabScratch ts;
  DevState &st = *b.st;
  DevIter &rep = st.rep[p.it < 32 ? p.it : 31];
  const int n = p.n, npad = p.npad;
  for (int q = threadIdx.x; q < kBetaBins; q += kPT) hist[q] = 0;
  __syncthreads();
  int extra = 0, exm = -100000;
  double hx = 0.0;
  for (int j = threadIdx.x; j < n; j += kPT) {
    exm = max(exm, b.eX[j]);
    if (b.mxX[j] == 0.0) continue;
    atomicAdd(&hist[min(kBetaBins - 1, max(0, 2 * b.cX[j] + kBetaBias))], 1);
    extra = max(extra, b.eX[j] - b.cX[j]);
    hx = fmax(hx, ldexp(sqrt(b.ssX[j]), -b.eX[j]));
  }
  extra = blk_max_i(extra, ired);
  exm = blk_max_i(exm, ired);
  hx = blk_max_d(hx, red);
  // the histogram's nonzero bins as bit masks, so the sum below visits only those (in the
  // ascending order of pow2_sum)
  __shared__ unsigned long long nzm[kBetaBins / 64];
  if (threadIdx.x < kBetaBins / 64) {
    unsigned long long m = 0ull;
    for (int k = 0; k < 64; ++k)
      if (hist[64 * threadIdx.x + k]) m |= 1ull << k;
    nzm[threadIdx.x] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0;
    for (int w = 0; w < kBetaBins / 64; ++w)
      for (unsigned long long m = nzm[w]; m; m &= m - 1) {
        const int bb = 64 * w + __ffsll((long long)m) - 1;
        S += (double)hist[bb] * ldexp(1.0, bb - kBetaBias);
      }
    int beta = 0, kx = 1;
    beta_core(p.xi, p.delta_k, st.gmin, st.lmax, S, extra, &beta, &kx);
    if (p.kx_force > 0) kx = p.kx_force;
    st.beta = beta;
    st.kx = kx;
    st.eXmax = exm;
    st.hX = hx;
    s_kx = kx;
    rep.beta = beta;
    rep.kx = kx;
    rep.delta = p.delta_k;
  }
  __syncthreads();
  const int kx = s_kx;
  const int eA_max = st.eA_max;
  const int nb = npad / 256;
  // ---- V by residues: A's digits per 256-column block, levels, moduli, floor check
  if (threadIdx.x == 0) s_ok = 0;
  __syncthreads();
  if (p.crt) {
    __shared__ double lgm[kCrtMax];   // log2 of each modulus
    for (int q = threadIdx.x; q < nb; q += kPT) kab[q] = 1;
    if (threadIdx.x >= 64 && threadIdx.x < 64 + kCrtMax)
      lgm[threadIdx.x - 64] = plan_log2((double)modulus(threadIdx.x - 64));
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kPT)
      if (b.mxX[j] != 0.0)
        atomicMax(&kab[j / 256], cut_ka(eA_max, p.lgrowth_a, b.eX[j], p.theta, p.delta_k,
                                        b.gapsw[j], p.d_extra));
    __syncthreads();
    if (threadIdx.x == 0) {
      int ka_top = 1;
      for (int q = 0; q < nb; ++q) {
        kab[q] = min(kab[q], p.ka_max);
        ka_top = max(ka_top, kab[q]);
      }
      const bool levels = npad >= 1024;
      int ka_l[kVLevels] = {0, 0, 0, 0};
      for (int q = 0; q < nb; ++q) {
        lvb[q] = levels ? min(kVLevels - 1, (ka_top - kab[q]) / 2) : 0;
        ka_l[lvb[q]] = max(ka_l[lvb[q]], kab[q]);
      }
      const double hbits = (st.hA > 0.0 && st.hX > 0.0) ? plan_log2(st.hA * st.hX * (1.0 + 1e-6))
                                                        : -1.0;
      int ok = 1;
      for (int l = 0; l < kVLevels; ++l) {
        st.ka_l[l] = ka_l[l];
        st.N_l[l] = 0;
        if (ka_l[l] > 0) {
          const int N = crt_count_lg(crt_need_bits(npad, ka_l[l], kx, hbits), lgm);
          if (N < 0 || ka_l[l] > kCrtPlanes || kx > kCrtPlanes) ok = 0;
          else st.N_l[l] = N;
        }
      }
      st.ka_top = ka_top;
      s_ok = ok;
    }
    __syncthreads();
    if (s_ok && threadIdx.x < kVLevels && st.ka_l[threadIdx.x] > 0)
      crt_rec_head(st.N_l[threadIdx.x], st.ka_l[threadIdx.x], kx, st.recs[threadIdx.x]);
    __syncthreads();
    if (s_ok) {   // the per-modulus fields, one thread each
      for (int i = threadIdx.x; i < kVLevels * kCrtMax; i += kPT) {
        const int l = i / kCrtMax, r = i - l * kCrtMax;
        if (st.ka_l[l] <= 0) continue;
        crt_rec_modulus(r, st.recs[l]);
      }
    }
    __syncthreads();
    if (s_ok) {   // reconstruction floor against each column's share of delta
      int fail = 0;
      for (int j = threadIdx.x; j < n; j += kPT) {
        if (b.mxX[j] == 0.0) continue;
        const CrtRec &rl = st.recs[lvb[j / 256]];
        const double fl = ldexp(rl.M[0], eA_max + b.eX[j] + rl.sh - 115);
        if (!(fl <= 0.25 * p.theta * p.delta_k * b.gapsw[j])) fail = 1;
      }
      if (fail) atomicAnd(&s_ok, 0);
    }
    __syncthreads();
  }
  const int vres = s_ok;
  if (vres) {
    // weights of X^(1)'s digits and of A's at each level whose digit or modulus count changed,
    // one thread per modulus slot
    __shared__ int s_dirty[kVLevels];
    if (threadIdx.x < kVLevels) {
      const int l = threadIdx.x;
      const int ka = st.ka_l[l], N = st.N_l[l];
      s_dirty[l] = ka > 0 && (ka != st.ares_ka[l] || N != st.ares_n[l]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (kVLevels + 1) * kCrtMax; i += kPT) {
      const int l = i / kCrtMax - 1, q = i - (l + 1) * kCrtMax;
      if (l < 0) res_weights_row(kx, st.N_l[0], q, st.wX);
      else if (s_dirty[l]) res_weights_row(st.ka_l[l], st.N_l[l], q, st.wA[l]);
    }
    if (threadIdx.x == 0) {
      st.wX.N = st.N_l[0];
      st.wX.k = kx;
    }
    if (threadIdx.x < kVLevels) {
      const int l = threadIdx.x;
      if (s_dirty[l]) {
        st.wA[l].N = st.N_l[l];
        st.wA[l].k = st.ka_l[l];
        st.ares_ka[l] = st.ka_l[l];
        st.ares_n[l] = st.N_l[l];
      }
      st.ares_dirty[l] = s_dirty[l];
    }
    for (int q = threadIdx.x; q < nb; q += kPT) {
      b.vblk[2 * q] = st.N_l[lvb[q]];
      b.vblk[2 * q + 1] = lvb[q];
    }
    if (threadIdx.x == 0) {
      double nsum = 0.0;
      for (int q = 0; q < nb; ++q) nsum += st.N_l[lvb[q]];
      rep.pv = nsum / nb;
      rep.dv = st.ka_top + kx;
      rep.lv = 1;
      st.gemm_v[0] = kx;
      st.gemm_v[1] = p.ka_max;
      st.gemm_v[2] = 0;   // no slice table
    }
  } else {
    for (int q = threadIdx.x; q < nb; q += kPT) {
      b.vblk[2 * q] = 0;
      b.vblk[2 * q + 1] = 0;
    }
    if (threadIdx.x < kVLevels) st.ares_dirty[threadIdx.x] = 0;
    // ---- V by slices: per-column cutoffs, per-tile maxima, the block table
    for (int j = threadIdx.x; j < npad; j += kPT)
      dcol[j] = (j < n && b.mxX[j] != 0.0)
                    ? cut_v(eA_max, p.lgrowth_a, kx, b.eX[j], p.theta, p.delta_k, b.gapsw[j],
                            p.d_extra)
                    : 2;
    __syncthreads();
    const int tr = npad >= 1024 ? 256 : 128;
    const int dallowed = min(p.ka_max + 1, kx + p.ka_max);
    double pairs = 0.0;
    const int dv = tile_cutoffs_from_columns(dtile, dcol, n, npad, tr, dallowed, kx, p.ka_max,
                                             b.dcut[0], &pairs, ired);
    const int cnt = build_table(dtile, npad / tr, kx, p.ka_max, b.tab[0], ts);
    if (threadIdx.x == 0) {
      st.gemm_v[0] = kx;
      st.gemm_v[1] = p.ka_max;
      st.gemm_v[2] = cnt;
      rep.pv = pairs;
      rep.dv = dv;
      rep.lv = 1;
    }
  }
  if (threadIdx.x == 0) {
    st.vres = vres;
    st.vslice = 1 - vres;
    rep.vres = vres;
  }
}

__global__ __launch_bounds__(kPT) void k_dp_vplan(PlanParams p, PlanBufs b) {
  dp_vplan_body(p, b);
}

// ---------------------------------------------------------------- the W plan
__device__ __forceinline__ void dp_wplan_body(PlanParams p, PlanBufs b) {
  __shared__ double key[kDevSortMax];
  __shared__ int idx[kDevSortMax];
  __shared__ int dcol[kDevSortMax];
  __shared__ int dtile[64];
  __shared__ double red[16];
  __shared__ int ired[16];
  __shared__ TabScratch ts;
  DevState &st = *b.st;
  DevIter &rep = st.rep[p.it < 32 ? p.it : 31];
  const int n = p.n, npad = p.npad, N2 = pow2_at_least(n), kx = st.kx;
  // After the first iteration the quotients usually keep the previous iteration's order: take
  // them in that order (its columns, through the inverse of this iteration's working order,
  // held in dcol until the cutoffs below) and sort only if they are not strictly ascending
  // there. Distinct keys have one sorted order, so both ways give the same key and idx.
  __shared__ int s_sorted;
  if (threadIdx.x == 0) s_sorted = p.it > 0 && !(*b.flags & kFlagsError);
  __syncthreads();
  if (s_sorted) {
    for (int q = threadIdx.x; q < n; q += kPT) dcol[b.colmap[q]] = q;
    __syncthreads();
    for (int r = threadIdx.x; r < N2; r += kPT) {
      if (r < n) {
        const int pw = dcol[b.sidx[r]];
        key[r] = b.lam[pw];
        idx[r] = pw;
      } else {
        key[r] = INFINITY;
        idx[r] = r;
      }
    }
    __syncthreads();
    int bad = 0;
    for (int r = threadIdx.x; r + 1 < n; r += kPT) bad |= !(key[r] < key[r + 1]);
    if (bad) s_sorted = 0;   // every writer writes the same value
    __syncthreads();
  }
  if (!s_sorted) {
    for (int i = threadIdx.x; i < N2; i += kPT) {
      key[i] = i < n ? b.lam[i] : INFINITY;
      idx[i] = i;
    }
    bitonic<double>(key, idx, N2);
  }
  // the sorted quotients and their columns: after this iteration D holds exactly these values
  // (the update scatters them), so the next iteration's order needs no sort of D
  for (int pp = threadIdx.x; pp < n; pp += kPT) {
    b.skey[pp] = key[pp];
    b.sidx[pp] = b.colmap[idx[pp]];
  }
  // gaps of the Rayleigh quotients, to their working positions (held in wtol[npad + j])
  double gm = INFINITY, lm = 0.0;
  for (int pp = threadIdx.x; pp < n; pp += kPT) {
    const double dl = pp > 0 ? key[pp] - key[pp - 1] : INFINITY;
    const double dr = pp + 1 < n ? key[pp + 1] - key[pp] : INFINITY;
    b.wtol[npad + idx[pp]] = fmin(dl, dr);
    gm = fmin(gm, dr);
    lm = fmax(lm, fabs(key[pp]));
  }
  gm = blk_min_d(gm, red);
  lm = blk_max_d(lm, red);
  if (n == 1) {
    if (threadIdx.x == 0) b.wtol[npad] = 1.0;
    gm = 1.0;
  }
  if (!(gm > 0.0) && threadIdx.x == 0) atomicOr(b.flags, FLAG_GAP);
  __syncthreads();
  const double cw0 = cut_w_c0(st.eXmax, kx, p.lsqn);
  for (int j = threadIdx.x; j < npad; j += kPT) {
    if (j < n) {
      const double g = b.wtol[npad + j];
      b.wtol[j] = w_tight(p.delta_int, g, lm, p.theta, p.delta_k);
      dcol[j] = b.resmax[j] != 0.0
                    ? cut_w_from(cw0, b.eR[j], p.theta, p.delta_k, g, p.d_extra)
                    : 2;
    } else {
      dcol[j] = 2;
    }
  }
  __syncthreads();
  const int tr = npad >= 1024 ? 256 : 128;
  const int dallowed = min(kKrMaxP + 1, kKrMaxP + kx);
  double pairs = 0.0;
  const int dw = tile_cutoffs_from_columns(dtile, dcol, n, npad, tr, dallowed, kKrMaxP, kx,
                                           b.dcut[1], &pairs, ired);
  const int cnt = build_table(dtile, npad / tr, kKrMaxP, kx, b.tab[1], ts);
  if (threadIdx.x == 0) {
    st.gmin_w = gm;
    st.lmax_w = lm;
    st.cx = cx_tile(kx, p.lsqn, p.theta, p.delta_k);
    st.dmax_w = dallowed;
    st.gemm_w[0] = kKrMaxP;
    st.gemm_w[1] = kx;
    st.gemm_w[2] = cnt;
    rep.dw = dw;
    rep.pw = pairs;   // replaced by the pairs under the tile cutoffs when they apply
    rep.lw = 1;
    rep.gmin = gm;
    rep.lmax = lm;
  }
}

__global__ __launch_bounds__(kPT) void k_dp_wplan(PlanParams p, PlanBufs b) {
  dp_wplan_body(p, b);
}

// ---------------------------------------------------------------- the X^(1) E~ plan, stop test
__device__ __forceinline__ void dp_uplan_body(PlanParams p, PlanBufs b) {
  __shared__ int dcol[kDevSortMax];
  __shared__ int dtile[64];
  __shared__ double red[16];
  __shared__ int ired[16];
  __shared__ TabScratch ts;
  DevState &st = *b.st;
  DevIter &rep = st.rep[p.it < 32 ? p.it : 31];
  const int n = p.n, npad = p.npad, kx = st.kx;
  double eps = 0.0;
  const double cu0 = cut_u_c0(kx, p.lsqn, p.theta, p.delta_k);
  for (int j = threadIdx.x; j < npad; j += kPT) {
    if (j < n) {
      eps = fmax(eps, b.emax[j]);
      dcol[j] = b.emax[j] != 0.0 ? cut_u_from(cu0, b.eE[j], b.wtol[j], p.d_extra) : 2;
    } else {
      dcol[j] = 2;
    }
  }
  eps = blk_max_d(eps, red);
  __syncthreads();
  const int tr = npad >= 1024 ? 256 : 128;
  const int dallowed = min(kKrMaxP + 1, kKrMaxP + kx);
  double pairs = 0.0;
  const int du = tile_cutoffs_from_columns(dtile, dcol, n, npad, tr, dallowed, kKrMaxP, kx,
                                           b.dcut[2], &pairs, ired);
  const int cnt = build_table(dtile, npad / tr, kKrMaxP, kx, b.tab[2], ts);
  // W pairs computed under the per-tile cutoffs (the tile's diagonal, at most its launch's)
  double pw = -1.0;
  if (npad >= 1024 && b.tcut) {
    const int T = npad / 256;
    double acc = 0.0;
    for (int q = threadIdx.x; q < T * T; q += kPT) {
      const int dl = min(b.tcut[q], b.dcut[1][(q / T) * 256]);
      int pr = 0;
      for (int d = 2; d <= dl; ++d) pr += npairs_of(d, kKrMaxP, kx);
      acc += pr;
    }
    // a sum of small integers: exact in any order
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kPT / 64; ++w) t += red[w];
      pw = t / ((double)T * T);
    }
  }
  if (threadIdx.x == 0) {
    st.gemm_u[0] = kKrMaxP;
    st.gemm_u[1] = kx;
    st.gemm_u[2] = cnt;
    rep.du = du;
    rep.pu = pairs;
    rep.lu = 1;
    rep.eps = eps;
    if (pw >= 0.0) rep.pw = pw;
    const bool err = (*b.flags & kFlagsError) != 0;
    if (!err) st.iters_done = p.it + 1;
    if (err) {
      st.done = 1;
    } else if (!p.fixed) {
      // the stop test: eps = max |E~| estimates the error of X^(1); the post-update error
      // modelled by eq. (assume2) is eps^2 max|lambda| / (xi gap)
      if (eps <= p.delta_int || eps * eps * st.lmax_w / (p.xi_stop * st.gmin_w) <= p.delta_int) {
        st.done = 1;
      } else if (p.it >= 1 && eps > 0.5 * st.eps_prev) {
        // no quadratic decrease: the floor that the products' truncation leaves
        st.done = 1;
        if (eps > p.target) st.stop_status = REFEIG_NOT_CONVERGED;
      } else if (p.it + 1 == p.iters) {
        st.done = 1;
        st.stop_status = REFEIG_NOT_CONVERGED;
      }
    }
    st.eps_prev = eps;
  }
}

__global__ __launch_bounds__(kPT) void k_dp_uplan(PlanParams p, PlanBufs b) {
  dp_uplan_body(p, b);
}

// ---------------------------------------------------------------- residue planes
// G: groups of four digit planes (K <= 4 G), a template so that the loads and the byte dot
// products of absent groups are not issued.
template <int G>
__device__ __forceinline__ void residues_dev_loop(const int8_t *__restrict__ planes,
                                                  size_t pstride, size_t count, int K, int N,
                                                  const int (*swp)[(kCrtPlanes + 3) / 4],
                                                  const int *snm, const int *sm22, const float *srm,
                                                  int8_t *__restrict__ res, int bid, int nblk) {
  for (size_t e = ((size_t)bid * 256 + threadIdx.x) * 4; e < count;
       e += (size_t)nblk * 256 * 4) {
    unsigned v[4 * G];
#pragma unroll
    for (int t = 0; t < 4 * G; ++t)
      v[t] = (t < K) ? *(const unsigned *)(planes + (size_t)t * pstride + e) : 0u;
    int dg[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        dg[g][bb] = (int)(((v[4 * g] >> (8 * bb)) & 0xffu) |
                          (((v[4 * g + 1] >> (8 * bb)) & 0xffu) << 8) |
                          (((v[4 * g + 2] >> (8 * bb)) & 0xffu) << 16) |
                          (((v[4 * g + 3] >> (8 * bb)) & 0xffu) << 24));
    int8_t *out = res + e;
    for (int q = 0; q < N; ++q, out += pstride) {
      const int nm = snm[q], m22 = sm22[q];
      const float rm = srm[q];
      int rr[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        int acc = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) acc = __builtin_amdgcn_sdot4(dg[g][bb], swp[q][g], acc, false);
        // |acc| <= 18 127^2 < 2^19, so acc rm_q is within 2^-13 of acc / m_q, which is at
        // least 1 / (2 m_q) > 2^-9 from a half-integer (m_q odd): acc rm_q + 1.5 2^23 rounded
        // once is the float 1.5 2^23 + q with q = rint(acc / m_q). The low 24 bits of its
        // pattern are 2^22 + q (bit 23 clear), so acc - m_q q = (acc + m_q 2^22) -
        // m_q (2^22 + q) is one signed 24-bit multiply-add
        const int bits = __float_as_int(fmaf((float)acc, rm, 0x1.8p23f));
        rr[bb] = __mul24(bits, nm) + (acc + m22);
      }
      // the low bytes of the four residues, in order
      const unsigned lo = __builtin_amdgcn_perm((unsigned)rr[1], (unsigned)rr[0], 0x0c0c0400u);
      const unsigned hi = __builtin_amdgcn_perm((unsigned)rr[3], (unsigned)rr[2], 0x04000c0cu);
      *(unsigned *)out = lo | hi;
    }
  }
}

__device__ __forceinline__ void residues_dev_body(const int8_t *__restrict__ planes,
                                                  size_t pstride, size_t count,
                                                  const ResWeights *__restrict__ w,
                                                  int8_t *__restrict__ res,
                                                  const int *__restrict__ gate, int bid, int nblk) {
  if (gate && *gate == 0) return;
  constexpr int G = (kCrtPlanes + 3) / 4;
  __shared__ int swp[kCrtMax][G];
  __shared__ int snm[kCrtMax], sm22[kCrtMax];   // -m_q and m_q 2^22
  __shared__ float srm[kCrtMax];
  const int K = w->k, N = w->N;
  for (int q = threadIdx.x; q < kCrtMax * G; q += 256) swp[q / G][q % G] = w->wp[q / G][q % G];
  for (int q = threadIdx.x; q < kCrtMax; q += 256) {
    snm[q] = -w->m[q];
    sm22[q] = w->m[q] << 22;
    srm[q] = w->rmf[q];
  }
  __syncthreads();
  static_assert(G == 5, "digit planes up to 18: groups 1..5");
  switch ((K + 3) / 4) {
    case 1: residues_dev_loop<1>(planes, pstride, count, K, N, swp, snm, sm22, srm, res, bid, nblk); break;
    case 2: residues_dev_loop<2>(planes, pstride, count, K, N, swp, snm, sm22, srm, res, bid, nblk); break;
    case 3: residues_dev_loop<3>(planes, pstride, count, K, N, swp, snm, sm22, srm, res, bid, nblk); break;
    case 4: residues_dev_loop<4>(planes, pstride, count, K, N, swp, snm, sm22, srm, res, bid, nblk); break;
    default: residues_dev_loop<5>(planes, pstride, count, K, N, swp, snm, sm22, srm, res, bid, nblk); break;
  }
}

__global__ __launch_bounds__(256) void k_residues_dev(const int8_t *__restrict__ planes,
                                                      size_t pstride, size_t count,
                                                      const ResWeights *__restrict__ w,
                                                      int8_t *__restrict__ res,
                                                      const int *__restrict__ gate) {
  residues_dev_body(planes, pstride, count, w, res, gate, blockIdx.x, gridDim.x);
}

__global__ void k_fill_int(int *p, int n, int v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- grouped batches
// The planning kernels over problems gp[first .. first + gridDim.x), one block each, the
// iteration as an argument. Iteration it of a problem whose stop test has ended its solve is
// skipped (DevState::skip, set by the order kernel; with fixed iterations every one runs, as
// in a single call).
__global__ __launch_bounds__(kPT) void k_dp_init_g(const GProb *__restrict__ gp, int first) {
  const GProb &q = gp[first + blockIdx.x];
  dp_init_body(q.pp, q.pb);
}
__device__ __forceinline__ PlanParams params_at(const GProb &q, int it) {
  PlanParams p = q.pp;
  p.it = it;
  return p;
}
__global__ __launch_bounds__(kPT) void k_dp_order_g(const GProb *__restrict__ gp, int first,
                                                    int it) {
  const GProb &q = gp[first + blockIdx.x];
  DevState &st = *q.pb.st;
  const int stop = !q.pp.fixed && st.done;
  if (threadIdx.x == 0) st.skip = stop;
  if (stop) return;
  dp_order_body(params_at(q, it), q.pb);
}
__global__ __launch_bounds__(kPT) void k_dp_vplan_g(const GProb *__restrict__ gp, int first,
                                                    int it) {
  const GProb &q = gp[first + blockIdx.x];
  if (q.pb.st->skip) return;
  dp_vplan_body(params_at(q, it), q.pb);
}
__global__ __launch_bounds__(kPT) void k_dp_wplan_g(const GProb *__restrict__ gp, int first,
                                                    int it) {
  const GProb &q = gp[first + blockIdx.x];
  if (q.pb.st->skip) return;
  dp_wplan_body(params_at(q, it), q.pb);
}
__global__ __launch_bounds__(kPT) void k_dp_uplan_g(const GProb *__restrict__ gp, int first,
                                                    int it) {
  const GProb &q = gp[first + blockIdx.x];
  if (q.pb.st->skip) return;
  dp_uplan_body(params_at(q, it), q.pb);
}

// Residue planes: which < kVLevels, A's digits at that level; which == kVLevels, X^(1)'s.
__global__ __launch_bounds__(256) void k_residues_g(const GProb *__restrict__ gp, int first,
                                                    int bpp, int which) {
  const GProb &q = gp[first + blockIdx.x / bpp];
  DevState *st = q.pb.st;
  if (st->skip) return;
  const int lb = blockIdx.x % bpp;
  if (which < kVLevels)
    residues_dev_body(q.w.AP, q.P, q.P, &st->wA[which], q.w.ARES + (size_t)which * kCrtMax * q.P,
                      &st->ares_dirty[which], lb, bpp);
  else
    residues_dev_body(q.w.XP, q.P, q.P, &st->wX, q.w.XRES, &st->vres, lb, bpp);
}

__global__ void k_flags_clear_g(const GProb *__restrict__ gp, int count) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g < count) gp[g].w.flags[0] = 0;
}

// Problems whose solve still runs (not done), into *out.
__global__ __launch_bounds__(256) void k_count_running_g(const GProb *__restrict__ gp, int count,
                                                         int *__restrict__ out) {
  __shared__ int ws[4];
  int c = 0;
  for (int g = threadIdx.x; g < count; g += 256) c += gp[g].pb.st->done ? 0 : 1;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *out = ws[0] + ws[1] + ws[2] + ws[3];
}

// Each problem's planning state and error flags, gathered for one copy to the host: problem
// g at out + g stride (the DevState, then the flags word).
__global__ __launch_bounds__(256) void k_gather_state_g(const GProb *__restrict__ gp,
                                                        char *__restrict__ out, size_t stride) {
  const GProb &q = gp[blockIdx.x];
  const int *src = (const int *)q.pb.st;
  int *dst = (int *)(out + (size_t)blockIdx.x * stride);
  constexpr int W = (int)(sizeof(DevState) / sizeof(int));
  for (int i = threadIdx.x; i < W; i += 256) dst[i] = src[i];
  if (threadIdx.x == 0) dst[W] = q.w.flags[0];
}

void launch_dp_init_g(const GProb *gp, int first, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_init_g, dim3(count), dim3(kPT), 0, s, gp, first);
}
void launch_dp_order_g(const GProb *gp, int first, int count, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_order_g, dim3(count), dim3(kPT), 0, s, gp, first, it);
}
void launch_dp_vplan_g(const GProb *gp, int first, int count, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_vplan_g, dim3(count), dim3(kPT), 0, s, gp, first, it);
}
void launch_dp_wplan_g(const GProb *gp, int first, int count, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_wplan_g, dim3(count), dim3(kPT), 0, s, gp, first, it);
}
void launch_dp_uplan_g(const GProb *gp, int first, int count, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_uplan_g, dim3(count), dim3(kPT), 0, s, gp, first, it);
}
void launch_residues_g(const GProb *gp, int first, int count, size_t P, int which,
                       hipStream_t s) {
  size_t bpp = (P / 4 + 255) / 256;
  if (bpp > 2048) bpp = 2048;
  hipLaunchKernelGGL(k_residues_g, dim3((unsigned)(count * bpp)), dim3(256), 0, s, gp, first,
                     (int)bpp, which);
}
void launch_flags_clear_g(const GProb *gp, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_flags_clear_g, dim3((count + 255) / 256), dim3(256), 0, s, gp, count);
}
void launch_count_running_g(const GProb *gp, int count, int *out, hipStream_t s) {
  hipLaunchKernelGGL(k_count_running_g, dim3(1), dim3(256), 0, s, gp, count, out);
}
void launch_gather_state_g(const GProb *gp, int count, char *out, size_t stride, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_state_g, dim3(count), dim3(256), 0, s, gp, out, stride);
}

void launch_dp_init(const PlanParams &p, const PlanBufs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_init, dim3(1), dim3(kPT), 0, s, p, b);
}
void launch_dp_order(const PlanParams &p, const PlanBufs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_order, dim3(1), dim3(kPT), 0, s, p, b);
}
void launch_dp_vplan(const PlanParams &p, const PlanBufs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_vplan, dim3(1), dim3(kPT), 0, s, p, b);
}
void launch_dp_wplan(const PlanParams &p, const PlanBufs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_wplan, dim3(1), dim3(kPT), 0, s, p, b);
}
void launch_dp_uplan(const PlanParams &p, const PlanBufs &b, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_uplan, dim3(1), dim3(kPT), 0, s, p, b);
}
void launch_residues_dev(const int8_t *planes, size_t pstride, size_t count, const ResWeights *w,
                         int8_t *res, const int *gate, hipStream_t s) {
  const size_t quads = count / 4;
  size_t blocks = (quads + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_residues_dev, dim3((unsigned)blocks), dim3(256), 0, s, planes, pstride,
                     count, w, res, gate);
}
void launch_fill_int(int *p, int n, int v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

}  // namespace refeig
