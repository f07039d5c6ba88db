/*
 * refeig.h - C ABI of the MI355X (gfx950) eigenvector-refinement library.
 *
 * The library refines approximate eigenvectors X^ and eigenvalues D^ of a real
 * symmetric matrix A (A X = X D, X^T X = I; Terao & Ozaki, arXiv 2602.19090,
 * Sec. 1) until the forward error ||X - X^|| reaches a prescribed delta > u
 * (Sec. 3.1). Each iteration is the Ogita-Aishima step of Algorithm 1
 * (Sec. 2.4) with the paper's cost cut (Sec. 3): X^ is replaced by its first
 * slice X^(1), whose grid is fixed by beta (the implementation rule of
 * Sec. 4.1), and every O(n^3) product runs through the Ozaki scheme
 * (Sec. 2.3) re-expressed for INT8 matrix cores: exponent-aligned 7-bit digit
 * planes, exact INT32 slice products, FP64 double-word slice sums.
 *
 * Conventions for every entry point:
 *  - Matrices are column-major (LAPACK): element (i, j) at i + j*ld, so
 *    eigenvector j is the contiguous column j. ld >= n.
 *  - "device" pointers are HIP device memory owned by the caller; the library
 *    never frees them. "host" pointers are ordinary host memory.
 *  - Work is enqueued on the given stream; entry points that return results
 *    in host memory synchronise that stream before returning.
 *  - Return values are refeig_status codes; no C++ exception crosses the ABI.
 *  - Calls that overlap on the same stream are serialised by the stream;
 *    calls on different streams must use different workspaces.
 */
#ifndef REFEIG_H
#define REFEIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *refeig_stream_t; /* a hipStream_t; NULL = default stream */

typedef enum {
    REFEIG_OK = 0,
    REFEIG_NOT_CONVERGED = 1, /* X, D hold the last iterate; the report says why        */
    REFEIG_E_ARG = -1,        /* bad size, pointer, leading dimension or option          */
    REFEIG_E_NONFINITE = -2,  /* NaN or Inf in A, X or D                                 */
    REFEIG_E_GAP = -3,        /* two eigenvalue estimates coincide (min gap 0): the
                                 paper assumes distinct, unclustered eigenvalues (Sec. 3.2) */
    REFEIG_E_RANGE = -4,      /* a row/column maximum outside [2^-400, 2^400]            */
    REFEIG_E_NOMEM = -5,      /* workspace too small or device allocation failed         */
    REFEIG_E_HIP = -6         /* a HIP runtime call failed                                */
} refeig_status;

typedef enum {
    REFEIG_OZAKI_INT8 = 0,  /* INT8 digit planes on MFMA (the hot path)                 */
    REFEIG_FP64_PLAIN = 2   /* the same iteration with FP64 slice products on DGEMM     */
} refeig_mode;

#define REFEIG_MAX_ITERS 32

typedef struct {
    int mode;            /* refeig_mode                                                  */
    int max_iter;        /* iteration limit (default 8)                                  */
    int fixed_iters;     /* > 0: run exactly this many iterations, no stop test          */
    int stop_rule;       /* stop after an iteration whose correction eps = max|E~|
                            satisfies eps^2 max|lambda| / (xi gap) <= target/delta_safety,
                            the post-update error that eq. (assume2) of Sec. 3.2
                            predicts, or eps <= target/delta_safety. An eps that
                            no longer halves is the products' noise floor: status
                            OK when eps <= target, else REFEIG_NOT_CONVERGED.
                            0: xi as below (default); 1: strict, xi = 1              */
    double delta_safety; /* internal delta = target / delta_safety (default 8)          */
    double xi;           /* xi of eq. (assume2); <= 0 means n, the Sec. 4.1 choice        */
    double theta;        /* share of the internal delta given to each product's
                            truncation (default 0.25)                                    */
    int ka_max;          /* maximum digit planes of A (default 18)                       */
    int d_extra;         /* extra pair diagonals added to every product (default 0)      */
    int verbose;         /* print per-iteration parameters to stderr                     */
    int kx_force;        /* > 0: digit planes of X^(1) fixed at this count (1..9) instead of
                            the beta rule of Sec. 4.1; 9 keeps X-hat at full FP64 precision,
                            the previous study's form without the X^(1) cut of Sec. 3.3
                            (an A/B for the paper's cost claim). 0: the beta rule.        */
    int schedule;        /* 1: adaptive accuracy, an extension beyond the paper (which aims
                            every iteration's products at the final delta): from the second
                            iteration on, with e the previous correction max|E~| (this
                            iteration's output error is then about e^4, the next one's
                            about e^8), the products aim at
                              max(delta, min(e^4 / 100,
                                  (0.1 / theta) sqrt(max(e^8, delta) gap / max|lambda|))):
                            the second bound keeps the error the loose products leave in
                            every entry of X, which the next iteration amplifies by about
                            max|lambda| / gap, at a tenth of that iteration's own output
                            error (gap: the smallest eigenvalue gap). 0: the paper's.      */
    int sparse_k;        /* > 0: the sparse-matrix rule of Sec. 4.3 with k = the largest
                            number of nonzeros in a row of A (refeig_row_nonzeros gives it):
                            xi = min(k^2, n) in beta (unless xi is set), and the error
                            growth of the products of A's planes is taken as min(k, sqrt n)
                            instead of sqrt n when the V product's diagonals are chosen.
                            0: the dense rule.                                          */
    int vmode;           /* how V = A X^(1) is formed. 1 (default): by residues, a product
                            algorithm other than the paper's slices: A cut to the digits
                            the V cutoff asks for and X^(1) are integers (the digit count
                            of A is chosen per 256-column block of V, in up to 4 levels
                            two digits apart), their product is formed exactly modulo N
                            pairwise coprime odd moduli <= 255 (one INT8 GEMM each; N is
                            sized per level from a Cauchy-Schwarz bound on the product,
                            22 for the top level at n = 8192, target 1e-14; at most 28) and
                            rebuilt by the Chinese remainder theorem; W and X^(1) E~ keep
                            the slice products. When a column's V tolerance lies below
                            what the reconstruction resolves, that iteration forms V by
                            slices instead. 0: the slice products of Sec. 2.3 for V too
                            (pair diagonals kept per column block). The Hermitian path
                            always uses slices.                                          */
    int plan;            /* where each iteration is planned (beta, k_X, cutoffs, modulus counts,
                            block tables): 0 (default) on the device, by small kernels between
                            the products, so the host enqueues the whole solve without waiting
                            (one wait per iteration for the stop test; none with fixed_iters);
                            1 on the host, which reads the device's column statistics three
                            times per iteration. group_tau > 0 and schedule = 1 always plan on
                            the host. Both give the same plan and bit-identical results.       */
    int enqueue_only;    /* 1: with fixed_iters > 0 and a caller workspace, device planning:
                            only enqueue the solve on the stream (no wait, no allocation, no
                            event; the stream may be under HIP graph capture). The return value
                            reports argument errors only; the status and report are read after
                            the stream has finished with refeig_read_report(work, ...).       */
    double group_tau;    /* > 0: grouped correction, an extension beyond the paper's
                            method (which assumes well-separated eigenvalues, Sec. 3.2):
                            every pair of columns whose first-order correction |e_ij|,
                            i != j, exceeds group_tau is linked; each linked group of
                            2..128 columns is corrected by the Rayleigh-Ritz problem on its
                            span (T y = mu G y, G = X_C^T X_C, T = X_C^T A X_C), which
                            resolves badly mixed or near-tied eigenvectors in one step.
                            0 (default): off, the paper's method.                       */
    double reserved_d[3];
} refeig_opts;

typedef struct {
    int status;                      /* final refeig_status                             */
    int iters;                       /* iterations performed                            */
    int beta[REFEIG_MAX_ITERS];      /* beta of Sec. 4.1 per iteration                  */
    int kx[REFEIG_MAX_ITERS];        /* digit planes of X^(1)                           */
    int dv[REFEIG_MAX_ITERS];        /* last pair diagonal kept in V = A X^(1)          */
    int dw[REFEIG_MAX_ITERS];        /* ... in W = X^(1)T (V - X^(1) D^)                */
    int du[REFEIG_MAX_ITERS];        /* ... in X^(1) E~                                 */
    int pairs[REFEIG_MAX_ITERS];     /* INT8 slice products (n x n x n) per iteration   */
    double eps[REFEIG_MAX_ITERS];    /* max |E~| per iteration                          */
    double ms_iter[REFEIG_MAX_ITERS];/* wall time per iteration (HIP events)            */
    double ms_gemm[REFEIG_MAX_ITERS];/* time in slice products per iteration            */
    int pairs_p[REFEIG_MAX_ITERS][3];   /* slice products of V, W, X^(1)E~ per iteration  */
    double pairs_f[REFEIG_MAX_ITERS][3];/* the same in units of one n x n x n product,
                                           counting per-column-block cutoffs exactly      */
    double ms_p[REFEIG_MAX_ITERS][3];   /* time of those three products, from the start of
                                           their first kernel dispatch to the end of their
                                           last (events taken by the dispatches)          */
    int launches_p[REFEIG_MAX_ITERS][3];/* slice-GEMM kernel dispatches of each product    */
    int groups[REFEIG_MAX_ITERS];    /* groups corrected by Rayleigh-Ritz (group_tau > 0) */
    double delta_it[REFEIG_MAX_ITERS];/* internal accuracy the iteration's products aimed at */
    double min_gap;                  /* min_{i != j} |lambda_i - lambda_j| (last)       */
    double max_abs_lambda;           /* max |lambda| (last)                             */
    double ms_total;
    int vres[REFEIG_MAX_ITERS];      /* 1: V formed by residues (vmode 1), 0: by slices  */
    double ms_phase[REFEIG_MAX_ITERS][5];/* device time of the iteration's phases (HIP
                                           events around each): column statistics of X,
                                           split of X^(1), V and the column pass, W and E~,
                                           the update; ms_iter minus their sum is the host
                                           planning and the copies it waits for           */
} refeig_report;

/* Defaults as documented in refeig_opts. Returns REFEIG_OK or REFEIG_E_ARG (o NULL). */
int refeig_default_opts(refeig_opts *o);

/* Device workspace needed by refine_eigvecs for order n (host out-pointer).
 * Returns REFEIG_E_ARG for n < 1 or n above the supported maximum (8192). */
int refeig_workspace_bytes(int n, const refeig_opts *o, size_t *bytes);

/* Refine X (n x n, device, column-major, ld ldx) and D (n, device) in place
 * for the symmetric A (device, ld lda; must be exactly symmetric, read only)
 * until max-abs forward error ~ target_fwd_err (Sec. 3.1; the paper's delta).
 * D on entry holds the eigenvalue estimates of X's columns (they set beta of
 * the first iteration); on return the Rayleigh quotients of the last X^(1).
 * work: device buffer of work_bytes >= refeig_workspace_bytes, or NULL to let
 * the library allocate (and free) it. report (host, may be NULL).
 * On REFEIG_OK / REFEIG_NOT_CONVERGED, X and D hold the last iterate. On a
 * negative status they hold the last completed iterate (unchanged if none). */
int refine_eigvecs(const double *A, int lda, double *X, int ldx, double *D, int n,
                   double target_fwd_err, const refeig_opts *o, void *work, size_t work_bytes,
                   refeig_stream_t stream, refeig_report *report);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): refine_eigvecs with the same arguments
 * minus the workspace, which lives in a static device array of the library (336 MiB, one
 * copy per GPU, held until the process ends; its device address is looked up once per
 * GPU). No hipMalloc, hipFree or allocating library call is made. Serves
 * 1 <= n <= REFEIG_NOALLOC_MAX_N with mode REFEIG_OZAKI_INT8 (REFEIG_E_NOMEM for larger n,
 * REFEIG_E_ARG for another mode); results are bit for bit those of refine_eigvecs. Every
 * call on one GPU uses that GPU's array, so calls that overlap on one GPU (different
 * streams or threads) race: serialise them. */
#define REFEIG_NOALLOC_MAX_N 1024
int refine_eigvecs_noalloc(const double *A, int lda, double *X, int ldx, double *D, int n,
                           double target_fwd_err, const refeig_opts *o, refeig_stream_t stream,
                           refeig_report *report);

/* The status and report of a solve enqueued with opts.enqueue_only, from its workspace
 * (device, as passed to refine_eigvecs; n and o as there). Synchronous: call it after the
 * stream has finished the solve (e.g. after a graph replay and a stream synchronisation). */
int refeig_read_report(const void *work, int n, const refeig_opts *o, int *status,
                       refeig_report *report);

/* Complex Hermitian extension (Sec. 5 names the Hermitian case as future
 * work): the same iteration for A = A^H with complex X. A and X are complex
 * matrices stored interleaved (real, imaginary) in column-major order, element
 * (i, j) at A[2 (i + j lda)] (real part) and A[2 (i + j lda) + 1] (imaginary
 * part), device pointers owned by the caller (e.g. torch complex128 tensors),
 * 16-byte aligned; lda, ldx count complex elements. D holds n real eigenvalue
 * estimates. r_i = 1 - x_i^H x_i, lambda_i = Re(x_i^H A x_i) / (1 - r_i),
 * W = X^H (A X - X D), e_ij = w_ij / (lambda_j - lambda_i), e_ii = r_i / 2;
 * X^(1) cuts both parts of a column on one grid, set by beta of Sec. 4.1 from
 * the column maximum over both parts. Each complex product is two real slice
 * products of reduction length 2n (real parts stacked above imaginary parts).
 * The forward error is measured in the modulus, up to a unit complex factor
 * per column. 1 <= n <= 4096. Options as refine_eigvecs, except that
 * group_tau, schedule and sparse_k must be 0 and mode REFEIG_OZAKI_INT8
 * (REFEIG_E_ARG otherwise); vmode is not used (slice products). Workspace:
 * refeig_herm_workspace_bytes, or NULL
 * (the library allocates and frees it). Statuses and report as
 * refine_eigvecs; pairs_f counts the slice products of both real GEMMs of a
 * complex product, in units of one real n x n x 2n product. */
int refeig_herm_workspace_bytes(int n, const refeig_opts *o, size_t *bytes);
int refine_eigvecs_herm(const double *A, int lda, double *X, int ldx, double *D, int n,
                        double target_fwd_err, const refeig_opts *o, void *work,
                        size_t work_bytes, refeig_stream_t stream, refeig_report *report);

/* Batched form of refine_eigvecs for `count` independent problems (the many-small-matrices
 * workload, one matrix per problem). Host arrays of length count hold each problem's order
 * n[i], device pointers A[i], X[i], D[i], leading dimensions and target_fwd_err[i]; o applies
 * to all. With device planning (o->plan == 0, group_tau == 0, schedule == 0: the defaults) the
 * solves advance together as a grouped batch: every step of an iteration is one launch per
 * group of problems with equal padded order, and the three products run as persistent kernels
 * over a device-built list of (problem, tile, slot) items. Problems run in chunks whose
 * workspaces total at most 16 GiB (the environment variable REFEIG_GROUP_CHUNK_MIB, read at each
 * call, overrides; the workspace query and the solve must see the same value); a problem whose
 * padded order exceeds 4096 runs alone after the chunks. With other options the problems run
 * concurrently on up to REFEIG_BATCH_LANES internal streams, each with its own slice of the
 * workspace. Either way every problem's result is bit for bit what refine_eigvecs returns for it
 * alone. work: device buffer of work_bytes >= refeig_batched_workspace_bytes(count, n, o), or
 * NULL (the library allocates and frees it). reports (host, count entries, may be NULL) receive
 * each problem's report and status (a grouped problem's ms_total is its chunk's wall time and
 * its per-iteration times are not taken). Returns REFEIG_OK when every problem did, else the
 * first negative per-problem status, else REFEIG_NOT_CONVERGED; REFEIG_E_ARG for count < 1 or a
 * NULL array (a problem with bad arguments of its own gets REFEIG_E_ARG in its report). */
#define REFEIG_BATCH_LANES 8
int refeig_batched_workspace_bytes(int count, const int *n, const refeig_opts *o, size_t *bytes);
int refine_eigvecs_batched(int count, const int *n, const double *const *A, const int *lda,
                           double *const *X, const int *ldx, double *const *D,
                           const double *target_fwd_err, const refeig_opts *o, void *work,
                           size_t work_bytes, refeig_stream_t stream, refeig_report *reports);

/* A grouped batch captured once in a HIP graph and replayed, for callers that refine batches of
 * the same shapes again and again (fixed_iters > 0 and device planning: grouped execution as
 * refine_eigvecs_batched, in one chunk; every padded order at most 4096). refeig_batch_create
 * (synchronous) carves the problems' workspaces from work (device, work_bytes >=
 * refeig_batch_workspace_bytes), uploads their descriptors and captures every launch of the solve
 * (all fixed_iters iterations) on an internal stream into a HIP graph; the arrays it takes are
 * those of refine_eigvecs_batched and the device buffers must stay allocated, at the same
 * addresses, until refeig_batch_destroy. refeig_batch_launch replays the graph on `stream` (NULL =
 * default): X and D are refined in place from whatever they hold when the replay runs, so the
 * caller rewrites them between replays (on that stream) to refine new data. refeig_batch_results
 * waits for the last replay and fills status[count] and reports (host, may be NULL); it returns
 * REFEIG_OK when every problem did, else the first negative status, else REFEIG_NOT_CONVERGED.
 * Each replay's results are bit for bit those of refine_eigvecs_batched (and of single calls).
 * REFEIG_E_ARG: options outside the above, bad arguments; REFEIG_E_NOMEM: work too small;
 * REFEIG_E_HIP: the capture or instantiation failed. Replays of one batch must not overlap. */
typedef struct refeig_batch refeig_batch;
int refeig_batch_workspace_bytes(int count, const int *n, const refeig_opts *o, size_t *bytes);
int refeig_batch_create(int count, const int *n, const double *const *A, const int *lda,
                        double *const *X, const int *ldx, double *const *D,
                        const double *target_fwd_err, const refeig_opts *o, void *work,
                        size_t work_bytes, refeig_batch **batch);
int refeig_batch_launch(refeig_batch *batch, refeig_stream_t stream);
int refeig_batch_results(refeig_batch *batch, int *status, refeig_report *reports);
int refeig_batch_destroy(refeig_batch *batch);

const char *refeig_strerror(int status);

/* Continuous-batching server for Algorithm 1 per request (the serving workload: requests
 * of uneven n that arrive while others run), with admission by HBM footprint.
 * refeig_server_create allocates one device arena of budget_bytes on the device current in
 * the calling thread and starts `lanes` host threads, each with its own stream (default
 * priority). A request's footprint is its workspace, refeig_server_request_bytes(n); it holds
 * that much of the arena from its start until it completes. A request starts when a lane is
 * free and its footprint fits in the arena's free space: the oldest pending one that fits
 * starts; one that does not fit yet may be passed by later ones at most 4 times, after which
 * nothing starts before it. Requests overlap on the device, and a short one does not wait
 * for a long one admitted before it. The machine's GPU runs 4 hardware queues per process by
 * default: with more than 4 lanes, lanes share queues.
 * refeig_server_submit queues one refine_eigvecs problem (device pointers as there; the caller
 * keeps A, X and D alive and untouched until the request is waited for) and returns at once
 * with a ticket. An event is recorded on `stream` (the caller's, NULL = default) at
 * submission; the lane waits for it before reading, so async writes of A, X or D that the
 * caller enqueued on that stream come first. REFEIG_E_NOMEM when the footprint exceeds the
 * budget (the request could never start), REFEIG_E_ARG for bad arguments.
 * refeig_server_wait blocks until the ticket's request is done and returns its status,
 * report (may be NULL) and completion time t_done (may be NULL; seconds on the monotonic
 * clock, CLOCK_MONOTONIC); a ticket is waited for once (REFEIG_E_ARG for an unknown or
 * already waited ticket). Each result is bit for bit what refine_eigvecs returns for that
 * problem alone. refeig_server_destroy waits for every submitted request, then frees
 * everything. */
typedef struct refeig_server refeig_server;
int refeig_server_create(int lanes, size_t budget_bytes, const refeig_opts *o,
                         refeig_server **server);
int refeig_server_submit(refeig_server *server, const double *A, int lda, double *X, int ldx,
                         double *D, int n, double target_fwd_err, refeig_stream_t stream,
                         int *ticket);
int refeig_server_wait(refeig_server *server, int ticket, int *status, refeig_report *report,
                       double *t_done);
int refeig_server_destroy(refeig_server *server);
/* Footprint of one request of order n in the server's arena (host out-pointer). */
int refeig_server_request_bytes(int n, const refeig_opts *o, size_t *bytes);

/* The largest number of nonzero entries in a row of A (device, n x n, ld lda),
 * the k of the sparse rule (Sec. 4.3). Synchronous; *k is a host int. */
int refeig_row_nonzeros(const double *A, int lda, int n, refeig_stream_t stream, int *k);

/* ---- host-only entry points: the planning the library does on the host, exposed
 * for checks on a machine without a GPU (no device memory is touched) ----------- */

/* beta of Sec. 4.1 (floor form, xi from o or n) and the digit-plane count of
 * X^(1), from the eigenvalue estimates lam (host, n) and the column statistics of
 * X (host arrays of n): e_j = floor(log2 max_i |x_ij|) + 1, c_j = ceil(log2 max_i
 * |x_ij|), mx_j = max_i |x_ij|. target_fwd_err as for refine_eigvecs (the rule
 * uses target / delta_safety). REFEIG_E_GAP if two estimates coincide. */
int refeig_host_beta(int n, const double *lam, const int *e, const int *c, const double *mx,
                     double target_fwd_err, const refeig_opts *o, int *beta, int *kx);

/* Host-only (no GPU needed): the plan of the residue product of V (vmode 1)
 * for ka1 digits of A, kx digits of X^(1) and reduction length npad, as the
 * solver builds it: *N moduli (odd, pairwise coprime, <= 255, largest first)
 * with prod m_q > 4 npad 128^(ka1 + kx); digit weights wA[q*18 + t] =
 * 128^(ka1-1-t) mod m_q and wX[q*18 + t] = 128^(kx-1-t) mod m_q in the
 * symmetric range; the reconstruction sums N terms, one per modulus:
 * U[3q..3q+2] = y_q / m_q as a triple-double, y_q = (M / m_q)^-1 mod m_q;
 * L[4q..4q+3] = the 34-bit limbs of y_q / m_q, floor(y_q / m_q 2^(34(k+1))) mod
 * 2^34 for k = 0..3 (integers in doubles; the V epilogue sums r_q L[q][k]);
 * M[0..2] = prod m_q (double-word, M[2] = 0). Arrays hold 28 moduli
 * (moduli: 28, wA, wX: 28*18, U: 28*3, L: 28*4 entries).
 * Returns REFEIG_E_ARG when more than 28 moduli would be needed. */
int refeig_host_crt_plan(int npad, int ka1, int kx, int *N, int *moduli, int *wA, int *wX,
                         double *U, double *L, double *M);
/* Host-only: the server's admission rule on a fake executor. count requests arrive at
 * t_arr[i] (seconds, ascending), each holding bytes[i] of an arena of budget bytes (both
 * rounded up to 256) for dur[i] seconds once started, served by `lanes` lanes; completions
 * are handled before arrivals at equal times. t_start[i] receives each request's start time
 * (-1 for a request larger than the budget, which never starts) and offset[i] (may be NULL)
 * its arena offset. */
int refeig_host_admission_sim(int count, const double *t_arr, const size_t *bytes,
                              const double *dur, int lanes, size_t budget, double *t_start,
                              size_t *offset);
/* Host-only: the product tile that grouped batches use for padded order npad on device
 * architecture arch (e.g. "gfx950"), as the tile cache holds it. Grouped batches run orders
 * from 1024 on the 256-row tile or, each entry of the 256-row plan split in four, on the
 * 128-row tile; both give the same results. The first batch that meets an order times both on
 * synthetic planes (in its own workspace) and records the faster in the cache, a JSON object
 * {"<arch>:<npad>": tile} in the file REFEIG_TUNE_CACHE names (else
 * $XDG_CACHE_HOME/refeig/tiles.json, else $HOME/.cache/refeig/tiles.json). REFEIG_TUNE=0 skips
 * the timing (cached choice, else 256); REFEIG_TILE=128 or 256 fixes the tile for every order.
 * *tile receives the cached tile (128 below npad 1024); returns REFEIG_OK when the cache holds
 * the order, REFEIG_NOT_CONVERGED when it does not (*tile = 256, the default), REFEIG_E_ARG
 * for bad arguments. */
int refeig_tile_cache_lookup(const char *arch, int npad, int *tile);

/* Working column order of an iteration: columns by the gap of their eigenvalue
 * estimate to its nearest neighbour, widest first, ties by eigenvalue.
 * order[p] = the column placed at working position p (host arrays of n). */
int refeig_host_column_order(int n, const double *lam, int *order);

/* The Rayleigh-Ritz problem of one group of k (2..128) columns, as the grouped
 * correction solves it: G (double-word Gram matrix, hi and lo parts, k x k
 * row-major), W (k x k row-major, w_ab), lam (double-word eigenvalue estimates).
 * T = W + G diag(lam), symmetrised; T y = mu G y. Y (k x k row-major) receives
 * the Ritz vector of member b in column b (the greedy largest-entry assignment,
 * signed so that its own entry is positive), mu_hi / mu_lo the Ritz values.
 * REFEIG_E_GAP if G is not positive definite, REFEIG_E_ARG for k out of range. */
int refeig_host_group_ritz(int k, const double *G_hi, const double *G_lo, const double *W,
                           const double *lam_hi, const double *lam_lo, double *Y,
                           double *mu_hi, double *mu_lo);

/* ---- entry points for bit-exact checks of the kernels -------------------- */

/* Column exponents and 7-bit digit planes of M (rows x cols, device, ld).
 * exps (device, cols ints): e_j with max_i |M_ij| < 2^e_j <= 2 max_i |M_ij|,
 * 0 for a zero column. planes (device, k * cols_pad * rows_pad bytes, where
 * rows_pad and cols_pad are rows and cols rounded up to 256): digit r (1..k)
 * of M_ij, sign(M_ij) * (floor(|M_ij| 2^(7r - e_j)) mod 128), at
 * planes[(r-1) * cols_pad * rows_pad + ((i / 64) * cols_pad + j) * 64 + i % 64]
 * (the K-blocked form: a plane is an operand with cols_pad rows j, each of
 * rows_pad entries i, cut into 64-entry blocks stored block by block); zero for
 * i >= rows or j >= cols. Errors: REFEIG_E_ARG (sizes, k outside 1..18),
 * REFEIG_E_NONFINITE (NaN/Inf in M), REFEIG_E_RANGE (e_j outside [-400, 400]).
 * trunc (device, may be NULL, ld rows): the value of the k digits.
 * This is the integer form of the error-free splitting of Sec. 2.3 (eq. a/x). */
int refeig_split_cols(const double *M, int ld, int rows, int cols, int k, int *exps,
                      int8_t *planes, double *trunc, refeig_stream_t stream);

/* refeig_split_cols with two more outputs of the splitter as the refinement runs it:
 * colmap (host, cols ints, may be NULL): column j of the result is column colmap[j] of M
 * (the working column order the solver folds into its reads of X; a permutation of 0..cols-1,
 * else REFEIG_E_ARG); exps and planes as refeig_split_cols for that column order.
 * planesT (device, kT * rows_pad * cols_pad bytes, may be NULL with kT = 0; 1 <= kT <= 9 when
 * given): the first kT digit planes in the transposed operand form, row i of the operand
 * holding the digits of row i of M (K index j): digit r of M_i,colmap[j] at
 * planesT[(r-1) * rows_pad * cols_pad + ((j / 64) * rows_pad + i) * 64 + j % 64] (the right
 * operand of the X^(1) E~ product, Algorithm 1 line 6 with the split of Sec. 2.3); zero
 * outside rows x cols. Errors as refeig_split_cols. */
int refeig_split_cols_ex(const double *M, int ld, int rows, int cols, int k, const int *colmap,
                         int *exps, int8_t *planes, double *trunc, int kT, int8_t *planesT,
                         refeig_stream_t stream);

/* Residue planes of the V product by residues (vmode 1; the Chinese-remainder form of the
 * error-free product of Sec. 2.3): the k digit planes at planes + t * plane_stride
 * (t = 0..k-1, digit t the most significant first, as refeig_split_cols writes them) encode
 * at each byte offset e < count the integer z = sum_t d_t 128^(k-1-t). For q = 0..nmod-1,
 * res[q * plane_stride + e] = z mod moduli[q] in the symmetric range
 * [-(m_q - 1) / 2, (m_q - 1) / 2] (int8). moduli (host): odd integers in [3, 255].
 * count a multiple of 4 (device pointers; every plane holds count bytes). Synchronous.
 * REFEIG_E_ARG: k outside 1..18, nmod outside 1..28, a bad modulus or count. */
int refeig_residue_planes(const int8_t *planes, size_t plane_stride, size_t count, int k,
                          int nmod, const int *moduli, int8_t *res, refeig_stream_t stream);

/* Residue products of the V product by residues: for q = 0..nmod-1,
 *   C[q][m][p] = (sum_k L_q[m][k] * R_{l q}[p][k]) mod moduli[q], symmetric range, int8,
 * at C + q*npad*npad + m*npad + p, with L_q and R_q residue planes in the K-blocked layout of
 * refeig_slice_gemm (plane stride plane_stride, npad a multiple of 256). vblk (host, may be
 * NULL; npad >= 1024 when given): per 256-row block b of L, {slot count c_b, level l_b}:
 * slots q >= c_b of that block's rows are not computed (C left as it was) and R_{l q} is
 * plane l_b * 28 + q of Rp (one residue set per digit count of A); NULL: c_b = nmod,
 * l_b = 0. Every slot sums npad terms below 127^2 exactly in INT32. Synchronous. */
int refeig_residue_gemm(const int8_t *Lp, const int8_t *Rp, size_t plane_stride, int npad,
                        int nmod, const int *moduli, const int *vblk, int8_t *C,
                        refeig_stream_t stream);

/* Exact per-diagonal slice products: for q = 0..ndiag-1 and d = d_min + q,
 *   C[q][m][p] = sum_{s + t = d, 1<=s<=kl, 1<=t<=kr} sum_k L_s[m][k] * R_t[p][k]
 * with L_s[m][k] at Lp + (s-1)*plane_stride + ((k / 64) * npad + m) * 64 + k % 64
 * (K-blocked, as refeig_split_cols writes), R_t likewise, and
 * C[q][m][p] at C + q*npad*npad + m*npad + p (int32, device). npad must be a
 * multiple of 256 and the planes zero-padded. The pairs of one diagonal must
 * satisfy pairs * npad * 127^2 < 2^31 (exact INT32 accumulation).  */
int refeig_slice_gemm(const int8_t *Lp, const int8_t *Rp, size_t plane_stride, int npad, int kl,
                      int kr, int d_min, int ndiag, int32_t *C, refeig_stream_t stream);

/* FP8 ablation of the slice products (the error-free products of Sec. 2.3, eq. mat_mul, with
 * 4-bit digits in FP8 E4M3 operands instead of 7-bit digits in INT8). refine_eigvecs does
 * not use it: at equal dense MFMA peaks (FP8 and INT8), a 4-bit digit carries 4 bits where
 * an INT8 digit carries 7, so the same accuracy needs about (7/4)^2 times the pairs.
 *
 * refeig_digits_to_e4m3: codes[i] = the E4M3 code (sign bit, 4 exponent bits with bias 7,
 * 3 mantissa bits) of the integer digits[i]; count entries, device pointers, the caller
 * owns both. Every integer in [-15, 15] is exact in E4M3. Returns REFEIG_E_ARG if a digit is
 * outside [-15, 15] (those codes are NaN) or a pointer is NULL with count > 0. Synchronous.
 *
 * refeig_slice_gemm_fp8: the products of refeig_slice_gemm, same plane layout, same C,
 * with Lp8 and Rp8 holding E4M3 codes of digits in [-15, 15]. The MFMA sums in FP32, which is
 * exact while pairs * npad * 15^2 < 2^24 for every diagonal (checked: REFEIG_E_ARG).
 * npad >= 1024, a multiple of 256. Synchronous. */
int refeig_digits_to_e4m3(const int8_t *digits, uint8_t *codes, size_t count,
                          refeig_stream_t stream);
int refeig_slice_gemm_fp8(const uint8_t *Lp8, const uint8_t *Rp8, size_t plane_stride, int npad,
                          int kl, int kr, int d_min, int ndiag, int32_t *C,
                          refeig_stream_t stream);

/* Measurement entry point, not part of the method: the matrix-core ceiling of the current GPU
 * for the slice product's instruction mix, the figure the product's achieved INT8 rate is
 * read against beside the published dense peak (the product is the cost that dominates,
 * Sec. 4). One block of 4 waves per CU issues the product's K-stage (32
 * v_mfma_i32_32x32x32_i8 per wave over a 128 x 128 wave tile) back to back for about
 * `seconds` (0 < seconds <= 10) on operands that change every stage:
 *   variant 0: operands in registers;
 *   variant 1: operands read from LDS as the product reads them;
 *   variant 2: variant 1 plus the LDS writes of the operand ring and a barrier per stage.
 * Outputs (host pointers): *ms the last run's time, *pops its INT8 rate in 10^15 operations
 * per second (2 per multiply-add), *ghz the shader clock over that run (s_memtime cycles over
 * the constant-rate s_memrealtime time, averaged over the blocks). Allocates and frees a few
 * KB of device memory; synchronous on `stream`. REFEIG_E_ARG for a bad variant, time or NULL
 * output; REFEIG_E_NOMEM / REFEIG_E_HIP on runtime failures. */
int refeig_mfma_ceiling(int variant, double seconds, refeig_stream_t stream, double *ms,
                        double *pops, double *ghz);

#ifdef __cplusplus
}
#endif

#endif
