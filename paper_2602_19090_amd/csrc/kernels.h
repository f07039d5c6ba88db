// Internal interface between the host orchestrator and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace refeig {

constexpr int kTile = 256;     // padding granule of every n x n operand
constexpr int kMaxDiag = 32;   // pair diagonals per product
constexpr int kEpiThreads = 1024;

// Flags raised by kernels (bitwise OR into a device int).
enum : int { FLAG_NONFINITE = 1, FLAG_TIE = 2, FLAG_RANGE = 4, FLAG_GAP = 8 };
// Any of these ends a solve with an error; kernels that write X and D skip their work once one
// is raised (the caller keeps the last completed iterate).
constexpr int kFlagsError = FLAG_NONFINITE | FLAG_TIE | FLAG_RANGE | FLAG_GAP;

struct DiagOrder {
  int q[kMaxDiag];  // launch position -> diagonal slot
};

// Column statistics of M (rows x cols, column-major, ld):
//   e[j] = floor(log2 max_i |M_ij|) + 1 (0 for a zero column),
//   c[j] = ceil(log2 max_i |M_ij|)      (0 for a zero column),
//   mx[j] = max_i |M_ij|.  Columns cols..cols_pad-1 get zeros.
// colmap (device, may be null): column j of the result is column colmap[j] of M.
// ss (optional): sum of squares of each column (plain FP64).
void launch_colstats(const double *M, int ld, int rows, int cols, int cols_pad, int *e, int *c,
                     double *mx, int *flags, hipStream_t s, const int *colmap = nullptr,
                     double *ss = nullptr);

// The largest number of nonzeros in a column of the symmetric A (= in a row): atomicMax
// into *kmax, which the caller zeroes.
void launch_row_nonzeros(const double *A, int lda, int n, int *kmax, hipStream_t s);

// 7-bit digit planes of M with column exponents e (see refeig_split_cols).
//  planes: k planes, plane stride pstride, element (i, j) at j*rpad + i.
//  trunc (optional, ld ldt): value of the k digits.
//  planesT (optional): kT planes of the transposed layout, element (i, j) at i*cpad + j.
// The grid covers the padded rpad x cpad area and writes zero digits outside.
// colmap (device, may be null): column j is read from column colmap[j] of M.
// kdev (device, may be null): the plane count k (and kT) read from device memory instead.
void launch_split_cols(const double *M, int ld, int rows, int cols, const int *e, int k,
                       int8_t *planes, size_t pstride, int rpad, int cpad, double *trunc, int ldt,
                       int8_t *planesT, size_t pstrideT, int kT, hipStream_t s,
                       const int *colmap = nullptr, const int *kdev = nullptr);

constexpr int kMaxRowBlocks = 64;
struct RowBlocks {
  int count;               // number of L row blocks (tile rows) in this launch
  int m[kMaxRowBlocks];    // their indices (units of gemm_tile_rows(npad) rows)
};

// Per-diagonal INT8 slice products (see refeig_slice_gemm) for diagonals
// d_min .. d_min + ndiag - 1, restricted to the L row blocks in rb (all row
// blocks when rb is null). The host issues one launch per group of row blocks
// that need the same diagonals, so every block of a diagonal does real work.
// ev_start / ev_stop (may be null) take the dispatch's own start / end times.
// kdim: reduction length (a multiple of 128; 0 means npad). The complex products use
// kdim = 2 npad: the imaginary parts are stacked after the real parts along K.
// same_plane: slot q holds the single product of plane q + 1 of L with plane q + 1 of R
// (the residue products, one modulus per slot) instead of diagonal d_min + q. mods (device,
// with same_plane): slot q is stored reduced mod mods[q] (symmetric, INT8, slot stride npad^2
// bytes) instead of as INT32.
void launch_slice_gemm(const int8_t *Lp, const int8_t *Rp, size_t pstride, int npad, int kl,
                       int kr, int d_min, int ndiag, int32_t *C, const RowBlocks *rb,
                       hipStream_t s, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr, int kdim = 0, bool same_plane = false,
                       const int *tcut = nullptr, const int *mods = nullptr, bool f8 = false,
                       const int *vblk = nullptr);
// vblk (device, with same_plane and npad >= 1024): per 256-row block of Lp (the output rows),
// {slot count N_J, level}: slots q >= N_J are skipped and the R operand of level l is the
// planes Rp + (l kCrtMax + q) pstride.
// f8 (npad >= 1024 only): the planes hold FP8 E4M3 codes of digits in [-15, 15].
// Digits (|d| <= 15) to FP8 E4M3 codes; a digit outside [-15, 15] sets *bad to 1.
void launch_digits_e4m3(const int8_t *in, uint8_t *out, size_t count, int *bad, hipStream_t s);
// The same products for npad >= 1024 in one launch of nblocks 256 x 256 blocks, block b
// computing the tile and diagonal slot of tab[b] (device memory; L row block | R row block
// << 8 | slot << 16, slot = d - d_min); the host orders the table. tcut as above.
// dp (device, may be null): {kl, kr, table entries} read from device memory; blocks at or
// beyond the entry count exit (the launch is sized for the largest table). npad < 1024: the
// 128 x 128 kernel, table entries in units of its tiles.
void launch_slice_gemm_table(const int8_t *Lp, const int8_t *Rp, size_t pstride, int npad,
                             int kl, int kr, int d_min, const int *tab, int nblocks, int32_t *C,
                             hipStream_t s, hipEvent_t ev_start = nullptr,
                             hipEvent_t ev_stop = nullptr, int kdim = 0,
                             const int *tcut = nullptr, const int *dp = nullptr);
// L rows per block tile of launch_slice_gemm for this npad.
int gemm_tile_rows(int npad);

// Epilogues sum, for output column j, the diagonals d_min .. min(d_min+ndiag-1, dcut[j]).
// Per-tile cutoffs of W (256 x 256 tiles, T a side): tcut[J T + I] = the last pair diagonal
// that keeps the W error of tile (column block J, row block I) within theta delta times the
// distance from each column's eigenvalue estimate to the nearest one of row block I;
// cx = 7 + log2(1.5 kx) + log2(sqrt n) - log2(theta delta). T <= kMaxTileSide.
constexpr int kMaxTileSide = 32;
// cxp, dmaxp (device, may be null): cx and dmax read from device memory instead.
void launch_tile_cutoffs(const double *lam, const int *eX, const int *eR, const double *resmax,
                         int n, int T, double cx, int dmax, int dextra, const double *tcol,
                         const double *gcol, int *tcut, hipStream_t s,
                         const double *cxp = nullptr, const int *dmaxp = nullptr);

// V epilogue fused with the column pass of Algorithm 1 (column j per block):
//   V_ij = sum_d 2^(eA_i + eX_j - 7d) C_d(i, j)  (double-word),
//   r_j = 1 - x_j^T x_j, lambda_j = x_j^T v_j / (1 - r_j) (double-word dots; lam gets
//   the FP64 value, lam_lo its low word), Res_ij = V_ij - x_ij lambda_j (pair arithmetic),
//   eR_j, resmax_j, and kr digit planes of Res (layout j*npad + i).
// ---- V by residues (an alternative to the slice products of V, see CrtRec): the integer
// product P = Ã X̃ of A's first ka digits and X^(1)'s kx digits is formed modulo N pairwise
// coprime odd moduli m_q <= 255 by N INT8 GEMMs of residue planes and reconstructed by the
// Chinese remainder theorem.
constexpr int kCrtMax = 28;   // moduli at most (over 200 bits of product)
constexpr int kVLevels = 4;   // digit counts of A (levels) in one residue product of V
constexpr int kCrtLimbs = 4, kCrtLimbBits = 34;   // limbs of the CRT fractions y_q / m_q
constexpr int kCrtPlanes = 18;
struct ResWeights {
  int N, k;
  int m[kCrtMax];
  float rmf[kCrtMax];           // fl32(1 / m_q): a rmf_q rounds to the nearest integer of
                                // a / m_q for |a| < 2^24 (a / m_q is never within 1 / (2 m_q)
                                // of a half-integer for odd m_q)
  int w[kCrtMax][kCrtPlanes];   // 128^(k-1-t) mod m_q in the symmetric range
  // the same weights as INT8, four planes to a dword: byte i of wp[q][g] is w[q][4g + i]
  // (zero beyond the planes), for the dot4 products of the residue kernel
  int wp[kCrtMax][(kCrtPlanes + 3) / 4];
};
// res plane q (stride pstride) = symmetric residue mod m_q of the integer sum_t d_t 128^(k-1-t)
// that the k digit planes encode at the same offset; count bytes per plane (a multiple of 4).
void launch_residues(const int8_t *planes, size_t pstride, size_t count, const ResWeights &w,
                     int8_t *res, hipStream_t s);
struct CrtRec {
  int N;
  int sh;                         // V = P 2^(eA_i + eX_j + sh)
  int m[kCrtMax];
  double rm[kCrtMax];             // fl(1 / m_q)
  double u[kCrtMax][3];           // y_q / m_q in triple-double, y_q = (M / m_q)^-1 mod m_q
  double M[3];                    // M = prod m_q in triple-double
  // The epilogue sums the N terms r_q u_q (r_q = the product mod m_q, symmetric) with u_q
  // truncated to kCrtLimbs limbs of kCrtLimbBits bits: u_q ~ sum_k L[q][k] 2^(-34 (k + 1)),
  // each L an integer below 2^34 held exactly in a double
  double L[kCrtMax][kCrtLimbs];
};
// V epilogue as launch_epi_v, with V rebuilt from the residues of the products (INT8 slot q
// of stride npad^2 bytes, reduced mod m_q by the GEMM) instead of summed from slice diagonals.
// recs (device): one record per level; vblk (device, may be null: level 0 for all): per
// 256-column block, its slot count and level.
// gate (device, may be null): the kernel does nothing while *gate == 0.
void launch_epi_v_crt(const int32_t *C, int npad, const CrtRec *recs, const int *vblk,
                      const int *eA, const int *eX, const double *X1, int n, double *lam,
                      double *lam_lo, double *r, int *eR, double *resmax, int8_t *Rpl, int kr,
                      int *flags, hipStream_t s, const int *gate = nullptr);

void launch_epi_v(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                  const int *eA, const int *eX, const double *X1, int n, double *lam,
                  double *lam_lo, double *r, int *eR, double *resmax, int8_t *Rplanes, int kr,
                  int *flags, hipStream_t s, const int *gate = nullptr);

// W epilogue (column j per block): W_ij = sum_d 2^(eX_i + eR_j - 7d) C_d(i, j),
//   e_ij = W_ij / (lambda_j - lambda_i) (difference of the double-word values),
//   e_jj = r_j / 2,  E'_ij = 2^eX_i e_ij,
//   eE_j (exponent of column j of E'), emax_j = max_i |e_ij|, ke digit planes of E'.
// cpl_count (may be null; the caller zeroes it): every pair (i, j), i != j, with
// |e_ij| > tau is counted, and the first cpl_cap are listed as (i, j) in cpl_pairs (in no
// particular order).
void launch_epi_w(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                  const int *eX, const int *eR, const double *lam, const double *lam_lo,
                  const double *r, int n, int *eE, double *emax, int8_t *Eplanes, int ke,
                  int *flags, hipStream_t s,
                  double tau = 0.0, int *cpl_count = nullptr, int *cpl_pairs = nullptr,
                  int cpl_cap = 0,
                  const int *tcut = nullptr);

// Grouped correction (Rayleigh-Ritz on strongly coupled columns). Groups hold at most
// kGroupMax members.
constexpr int kGroupMax = 128;
// For listed pairs q: gh/gl[q] = x_a^T x_b (double-word, columns of X1), wab[q] = w_ab
// (entry of W from the slots, as the W epilogue sums it), a = pa[q], b = pb[q].
void launch_group_gram(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                       const int *eX, const int *eR, const double *X1, int n, const int *pa,
                       const int *pb, int npairs, double *gh, double *gl, double *wab,
                       hipStream_t s, const int *tcut = nullptr);
// For each of nmem member slots m: column gcol[m], the group's slots start at gfirst[m],
// it has gk[m] members, this member is number gpos[m]; Ritz vectors row-major at
// Y + gbase[m], Ritz value mu[m] + mu_lo[m]. Rewrites that column's E' planes, eE and emax.
void launch_group_fix(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                      const int *eX, const int *eR, const double *lam, const double *lam_lo,
                      int n, const int *gcol, const int *gfirst, const int *gk, const int *gpos,
                      const int *gbase, const double *Y, const double *mu, const double *mu_lo,
                      int nmem, int *eE, double *emax, int8_t *Eplanes, int ke, int *flags,
                      hipStream_t s, const int *tcut = nullptr);

// Update: X_ij = hi(TwoSum(X1_ij, U_ij)), U_ij = sum_d 2^(eE_j - 7d) C_d(i, j); column j
// is written to column colmap[j] of X (colmap may be null).
// errflags (device, may be null): nothing is written once an error flag is raised.
void launch_epi_u(const int32_t *C, int npad, int d_min, int ndiag, const int *dcut,
                  const int *eE, const double *X1, int n, double *X, int ldx, hipStream_t s,
                  const int *colmap = nullptr, const int *errflags = nullptr);

// out[colmap[p]] = v[p] for p < n (colmap may be null); nothing once *errflags holds an error.
void launch_scatter(const double *v, const int *colmap, int n, double *out, hipStream_t s,
                    const int *errflags = nullptr);


// ---- complex Hermitian case. Complex matrices are interleaved (re, im), column-major,
// element (i, j) at 2 (i + j ld). Complex operand rows are realified: a digit plane holds
// K = 2 npad entries per row (real parts at k < npad, imaginary parts at npad + k) and has
// stride 2 npad^2; the products run as real slice GEMMs with kdim = 2 npad.

// Column statistics as launch_colstats over both parts (max_i max(|Re|, |Im|)).
void launch_colstats_c(const double *M, int ld, int rows, int cols, int cols_pad, int *e, int *c,
                       double *mx, int *flags, hipStream_t s, const int *colmap = nullptr);

// Realified digit planes with one exponent per column over both parts:
//   planes: row j = (Re M_.j ; Im M_.j);  planes2 (optional): row j = (-Im M_.j ; Re M_.j);
//   trunc (optional, complex, ld ldt): value of the k digits;
//   planesT (optional, kT planes): row i = (Re M_i. ; -Im M_i.).
void launch_split_c(const double *M, int ld, int rows, int cols, const int *e, int k,
                    int8_t *planes, int8_t *planes2, size_t pstride, int rpad, int cpad,
                    double *trunc, int ldt, int8_t *planesT, size_t pstrideT, int kT,
                    hipStream_t s, const int *colmap = nullptr);

// V epilogue + column pass (npad <= 4096): V = Vr + i Vi from the two products' slots,
// r_j = 1 - x_j^H x_j, lambda_j = Re(x_j^H v_j) / (1 - r_j), Res = V - x_j lambda_j, eR_j
// and resmax_j over both parts; planes of Res (Rpl) and of -i Res (Rpl2).
void launch_epi_v_c(const int32_t *Cr, const int32_t *Ci, int npad, int d_min, int ndiag,
                    const int *dcut, const int *eA, const int *eX, const double *X1, int n,
                    double *lam, double *lam_lo, double *r, int *eR, double *resmax,
                    int8_t *Rpl, int8_t *Rpl2, int kr, int *flags, hipStream_t s);

// W epilogue: e_ij = w_ij / (lambda_j - lambda_i), e_jj = r_j / 2, E' = 2^eX_i e, emax_j =
// max_i |e_ij| (modulus), eE_j; planes of E' (Epl) and of -i E' (Epl2).
void launch_epi_w_c(const int32_t *Cr, const int32_t *Ci, int npad, int d_min, int ndiag,
                    const int *dcut, const int *eX, const int *eR, const double *lam,
                    const double *lam_lo, const double *r, int n, int *eE, double *emax,
                    int8_t *Epl, int8_t *Epl2, int ke, int *flags, hipStream_t s);

// Update: X_.colmap[j] = X1_.j + U_.j (both parts).
void launch_epi_u_c(const int32_t *Cr, const int32_t *Ci, int npad, int d_min, int ndiag,
                    const int *dcut, const int *eE, const double *X1, int n, double *X, int ldx,
                    hipStream_t s, const int *colmap = nullptr);

}  // namespace refeig
