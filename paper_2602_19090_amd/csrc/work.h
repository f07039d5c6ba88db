// The workspace of one solve (device pointers carved from the caller's buffer), and the
// descriptor of one problem of a grouped batch as the grouped kernels read it.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "devplan.h"
#include "kernels.h"

namespace refeig {

constexpr int kMaxN = 8192;   // the column epilogues hold a whole column in registers
constexpr int kKxMax = 9;     // digit planes of X^(1) at most
constexpr int kKrMax = 12;    // ... of the residual
constexpr int kKeMax = 12;    // ... of E~
// Largest padded order run inside a grouped batch (larger problems of a batch run alone: they
// fill the device by themselves, and the grouped column epilogues hold 4 entries per thread).
constexpr int kGroupMaxNpad = 4096;

struct Work {
  int n = 0, npad = 0, ka = 0;
  size_t P = 0;
  int8_t *AP, *XP, *XPT, *RP, *EP;
  int8_t *ARES = nullptr, *XRES = nullptr;   // residue planes of the V product by residues
  int32_t *Cs;
  double *X1;
  int *eA, *cA, *eX, *cX, *eR, *eE, *flags;
  int *dcut[3];  // per-column last diagonal of V, W and X^(1) E~
  int *colmap;   // working column p holds column colmap[p] of the caller's X
  int *tcut;     // per-tile last diagonal of W (256 x 256 tiles)
  int *mods;     // moduli of the residue product of V
  CrtRec *recs;  // its reconstruction records, one per level (digit count of A)
  int *vblk;     // per 256-column block of V: slot count, level
  double *ssA, *ssX;   // column sums of squares of A and X (the residue product's bound)
  double *wtol;        // per column: W tile tightening t_j, then the column's own gap g_j
  int *tab[3];   // block tables of the V, W and X^(1) E~ products
  // grouped correction: coupling list, pair list, member table, Ritz data
  int *cpl, *g_pa, *g_pb, *g_col, *g_first, *g_k, *g_pos, *g_base;   // cpl: count, then pairs
  double *g_gh, *g_gl, *g_w, *g_Y, *g_mu, *g_mul;
  double *mxA, *mxX, *lam, *lam_lo, *r, *resmax, *emax;
  DevState *dst;   // device planning state
  double *gapsw;   // entry gaps in working order (device planning)
  double *skey;    // the last W plan's Rayleigh quotients in ascending order (device planning)
  int *sidx;       // ... and the column of each
};

// One problem of a grouped batch (device memory, one entry per problem). pp.it is not used:
// the grouped planning kernels take the iteration as an argument.
struct GProb {
  const double *A;
  double *X, *D;
  int lda, ldx, n, npad, ka;
  int gtile;   // rows of the product tile the grouped kernels use (128, or 256 when npad >= 1024)
  size_t P;
  Work w;
  PlanParams pp;
  PlanBufs pb;
};

// Launches over a grouped batch. gp: device array of the batch's problems; each step launch
// covers the size class gp[first .. first + count) (equal npad); the products run over the
// device-built work list of a tile group (consecutive problems with equal GEMM tile rows).
void launch_colstats_g(const GProb *gp, int first, int count, int npad, bool of_x, hipStream_t s);
void launch_split_g(const GProb *gp, int first, int count, int npad, bool of_x, hipStream_t s);
void launch_epi_v_g(const GProb *gp, int first, int count, int npad, bool crt, hipStream_t s);
void launch_tile_cutoffs_g(const GProb *gp, int first, int count, int npad, hipStream_t s);
void launch_epi_w_g(const GProb *gp, int first, int count, int npad, hipStream_t s);
void launch_epi_u_g(const GProb *gp, int first, int count, int npad, hipStream_t s);
void launch_scatter_g(const GProb *gp, int first, int count, int npad, hipStream_t s);
// which: 0 V by residues, 1 V by slices, 2 W, 3 X^(1) E~; items: room for every item the
// problems' plans can ask for; total and ctr: one int each.
void launch_worklist_g(const GProb *gp, int first, int count, int which, int tile, int2 *items,
                       int *total, int *ctr, hipStream_t s);
void launch_gemm_g(const GProb *gp, int tile, int blocks, const int2 *items, const int *total,
                   int *ctr, int which, hipStream_t s);
// Fill n bytes with digits in [-127, 127] from a hash of the index and seed (the tile tuner's
// synthetic planes).
void launch_fill_hash_i8(int8_t *p, size_t n, unsigned seed, hipStream_t s);
void launch_dp_init_g(const GProb *gp, int first, int count, hipStream_t s);
void launch_dp_order_g(const GProb *gp, int first, int count, int it, hipStream_t s);
void launch_dp_vplan_g(const GProb *gp, int first, int count, int it, hipStream_t s);
void launch_dp_wplan_g(const GProb *gp, int first, int count, int it, hipStream_t s);
void launch_dp_uplan_g(const GProb *gp, int first, int count, int it, hipStream_t s);
void launch_residues_g(const GProb *gp, int first, int count, size_t P, int which,
                       hipStream_t s);
void launch_flags_clear_g(const GProb *gp, int count, hipStream_t s);
void launch_count_running_g(const GProb *gp, int count, int *out, hipStream_t s);
void launch_gather_state_g(const GProb *gp, int count, char *out, size_t stride, hipStream_t s);

}  // namespace refeig
