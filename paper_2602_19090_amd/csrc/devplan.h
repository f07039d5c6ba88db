// Planning of an iteration on the device: the working column order, beta and k_X, the
// modulus counts and reconstruction records of V by residues, the pair cutoffs and the block
// tables of the three products, the stop test and the report, computed by single-block
// kernels between the product kernels, so a solve enqueues its iterations without waiting
// for the host (and a fixed number of iterations can be captured in a HIP graph).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace refeig {

constexpr int kDevSortMax = 8192;   // columns the single-block planning kernels sort

// Per-iteration figures for the report (written by the planning kernels).
struct DevIter {
  int beta, kx, dv, dw, du, vres, lv, lw, lu;
  double pv, pw, pu, eps, gmin, lmax, delta;
};

// The planning state, kept in the workspace across iterations.
struct DevState {
  int done, stop_status, iters_done;
  int skip;   // grouped batches: the solve had stopped when this iteration began

  int eA_max;
  double hA;
  // the current iteration
  int kx, beta, eXmax, vres, vslice, ka_top;
  double gmin, lmax;       // of the iteration's entry estimates
  double gmin_w, lmax_w;   // of its Rayleigh quotients (the W and E~ products)
  double hX;
  int ka_l[kVLevels], N_l[kVLevels];
  int ares_ka[kVLevels], ares_n[kVLevels], ares_dirty[kVLevels];
  int gemm_v[4], gemm_w[4], gemm_u[4];   // slice GEMM: kl, kr, table entries
  double cx;
  int dmax_w;
  double eps_prev;
  ResWeights wX, wA[kVLevels];
  CrtRec recs[kVLevels];
  DevIter rep[32];
};

// Scalars every planning kernel reads (by value).
struct PlanParams {
  int n, npad, it, iters, fixed, kx_force, ka_max, d_extra, vmode, stop_rule, crt;
  double theta, delta_int, delta_k, xi, xi_stop, lgrowth_a, lsqn, target;
};

// Device pointers the planning kernels read and write (all in the workspace).
struct PlanBufs {
  DevState *st;
  const double *D;        // entry eigenvalue estimates (the caller's D, natural order)
  int *colmap;            // working position -> column
  double *gapsw;          // entry gaps in working order
  const int *eA;
  const double *mxA, *ssA;
  const int *eX, *cX;
  const double *mxX, *ssX;
  const double *lam;      // Rayleigh quotients (working order)
  const int *eR;
  const double *resmax;
  const int *eE;
  const double *emax;
  double *wtol;           // t_j, then g_j (2 npad)
  int *dcut[3];
  int *tab[3];
  int *vblk;
  const int *tcut;
  int *flags;
  int *mods;              // the moduli, all kCrtMax (for the residue store)
  double *skey;           // the W plan's sorted Rayleigh quotients (n), reused by the next
  int *sidx;              // iteration's order (their columns; D holds the same values then)
};

void launch_dp_init(const PlanParams &p, const PlanBufs &b, hipStream_t s);
void launch_dp_order(const PlanParams &p, const PlanBufs &b, hipStream_t s);
void launch_dp_vplan(const PlanParams &p, const PlanBufs &b, hipStream_t s);
void launch_dp_wplan(const PlanParams &p, const PlanBufs &b, hipStream_t s);
void launch_dp_uplan(const PlanParams &p, const PlanBufs &b, hipStream_t s);

// Residue planes with the weights (digit count, moduli) in device memory; gate (device, may be
// null): nothing is done unless *gate != 0.
void launch_residues_dev(const int8_t *planes, size_t pstride, size_t count, const ResWeights *w,
                         int8_t *res, const int *gate, hipStream_t s);
// Fill n ints with a value (graph-safe replacement of a memset).
void launch_fill_int(int *p, int n, int v, hipStream_t s);

}  // namespace refeig
