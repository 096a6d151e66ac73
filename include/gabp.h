/*
 * gabp.h -- C ABI of a synchronous Gaussian belief propagation (GaBP) solver
 * for sparse symmetric linear systems A x = b on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Bickson, "Gaussian Belief Propagation: Theory and Application"
 * (arXiv:0811.2518).  The solution x* = A^-1 b is the vector of marginal means
 * of the Gaussian p(x) ~ exp(-x^T A x / 2 + b^T x) (Ch. 2 Sec. 2.1, Prop. 2.1).
 * Every directed edge i -> j of the graph of A carries a precision message
 * P_ij and a mean message; each sweep recomputes all of them from the previous
 * sweep's messages (synchronous scheduling, Ch. 2 Sec. 2.3) in the broadcast
 * form of Alg. 2 (Ch. 3 Sec. 3.3): node i forms P~_i = A_ii + sum_k P_ki and
 * the matching mean sum once, and each outgoing message subtracts the reverse
 * message j -> i.  Messages are held in information form (P_ij, h_ij = P_ij
 * mu_ij) as in the Weiss/Johnson form of the appendix.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Array arguments are DEVICE pointers owned by the caller and only borrowed
 *    for the duration of the call, unless stated "host".  All work is enqueued
 *    on the stream given at create time; calls that return a gabp_info wait for
 *    that stream before returning.
 *  * Matrices are full symmetric CSR with the diagonal stored: int32 row_ptr
 *    [n+1] (row_ptr[0] = 0), int32 col_idx [nnz] strictly increasing within a
 *    row, float64 vals [nnz].  The pattern and the values must be symmetric
 *    (|A_ij - A_ji| <= 1e-12 * max|A|) and every A_ii must be nonzero.
 *    gabp_create_augmented is the exception: it takes a rectangular B (no
 *    diagonal, no symmetry) and builds the symmetric matrix itself.
 *  * Nothing throws across the ABI.  A negative status is an error (outputs
 *    unspecified); GABP_NOT_CONVERGED still writes the last iterate.
 *    gabp_last_error() returns a description of the last failure.
 *  * A handle may be used by one host thread at a time.
 */
#ifndef GABP_H
#define GABP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gabp_ctx *gabp_handle;

typedef enum {
  GABP_OK = 0,
  GABP_NOT_CONVERGED = 1,     /* iteration cap reached; x holds the last iterate   */
  GABP_E_ARG = -1,            /* bad size, pointer, option or CSR structure        */
  GABP_E_NOT_SYMMETRIC = -2,  /* pattern or values of A not symmetric              */
  GABP_E_ZERO_DIAG = -3,      /* some A_ii missing or zero                         */
  GABP_E_NONFINITE = -4,      /* NaN/Inf in the input or in a message (P~_i = P_ji) */
  GABP_E_DIVERGED = -5,       /* residual grew past 1e8 * ||b|| or became NaN      */
  GABP_E_HIP = -6,            /* a HIP runtime call failed                         */
  GABP_E_OOM = -7             /* device allocation failed                          */
} gabp_status;

typedef enum {
  GABP_FP64 = 0,          /* messages, aggregates and residual in FP64              */
  GABP_FP32_REFINE = 1    /* FP32 messages inside an FP64 iterative-refinement loop  */
} gabp_precision;

/* Solver options.  Fill with gabp_default_opts() and change what is needed. */
typedef struct {
  int32_t precision;        /* gabp_precision                                       */
  int32_t check_every;      /* residual check period in sweeps (>= 1)               */
  int32_t edges_per_block;  /* message slots per 256-lane workgroup: 512, 1024 or   */
                            /* 2048; 0 = pick by timing at create (autotuner).  A   */
                            /* longer row gets a workgroup of its own (layouts 1,   */
                            /* 2) or is split over several (layouts 3, 4)           */
  int32_t inner_max_iter;   /* cap on inner sweeps per outer step                   */
  int32_t max_outer;        /* cap on outer steps (refinement / loading loop)       */
  int32_t flags;            /* GABP_FLAG_* bits                                     */
  int32_t layout;           /* message layout of the sweep kernels: 0 = pick by     */
                            /* timing at create, 1 = outgoing records + reverse-    */
                            /* slot index, 2 = node broadcast (edge pairs in place),*/
                            /* 3 = compact node broadcast (one incoming message per */
                            /* slot, the outgoing one recomputed by its sender),    */
                            /* 4 = colour-serial: SERIAL scheduling (Ch. 2 Sec.     */
                            /* 2.3) over the colour classes of a first-fit colouring*/
                            /* in row order -- a different iteration from 1-3, with */
                            /* fewer sweeps; never picked by the timing at create;  */
                            /* no precision reuse, no single loop, no gabp_messages */
  int32_t reserved;         /* must be 0                                            */
  double  gamma;            /* diagonal loading of Ch. 5: the inner solves use      */
                            /* A + gamma * diag(A); 0 = none; < 0 = chosen from an  */
                            /* estimate of rho(|R|) (walk-summability, Ch. 5.2)     */
  double  loading_delta;    /* margin for gamma < 0: gamma = (1+delta) rho - 1      */
  double  inner_tol;        /* inner relative residual target per outer step        */
  double  damping;          /* GABP_FLAG_SINGLE_LOOP: feedback step s in (0, 1]     */
} gabp_opts;

/* Reuse precision messages frozen by an earlier solve on the same handle: the
 * P messages depend on A only (the precision update of Alg. 2 has no b term), so later solves
 * and the adjoint solve run mean-only sweeps.  Without the flag every
 * gabp_solve runs the full synchronous iteration from zero messages.  Inside
 * one call, the outer loops freeze the precisions after the first inner solve
 * and run the later inner solves mean-only when diagonal loading is on (many
 * outer steps) or the flag is set; plain refinement without the flag runs
 * every inner solve from zero messages (two outer steps at the default
 * tolerances, where freezing would not pay). */
#define GABP_FLAG_REUSE_PRECISION 1

/* Profiling aid: time every main-mode sweep that carries the fused residual
 * check with HIP events attached to the dispatch (hipExtLaunchKernel), so the
 * interval is the kernel's own execution; totals land in gabp_info.sweep_ms /
 * timed_sweeps (at most 2048 sweeps per call are timed). */
#define GABP_FLAG_TIME_SWEEPS 2

/* With diagonal loading (gamma != 0): the single-loop form of the correction
 * method (Ch. 5 Sec. 5.3) instead of the double loop.  One FP64 sweep of
 * Alg. 2 on A + Gamma per outer step; the prior potentials of round t are
 * h^(t) = b + Gamma ((1 - s) x^(t-2) + s x^(t-1)) with s = opts.damping
 * (x^(-1) = 0, h^(0) = b), and the residual of A x = b itself is checked;
 * gabp_info.outer_iters = sweeps.  With GABP_FP32_REFINE the FP64 refinement
 * loop stays, and each inner correction solve A d = r runs this single loop
 * in FP32 (joint sweeps from zero messages, inner residual of A itself).
 * The handle uses the compact layout. */
#define GABP_FLAG_SINGLE_LOOP 4

/* Keep the caller's row order.  Without the flag, gabp_create of layouts 0-3
 * may renumber the rows internally (the caller never sees it) into 8 parts of
 * equal work.  The parts are grown breadth-first and refined by label
 * propagation, and part x is swept by the workgroups of XCD x, so that more
 * neighbour gathers hit that XCD's L2.  This is done only when the parts keep
 * clearly more edges inside than the caller's order does.  The iteration and
 * the results are unchanged up to the summation order of the residual norm. */
#define GABP_FLAG_NATURAL_ORDER 8

/* Aitken's extrapolation of the means (Ch. 3 Sec. 3.2, convergence
 * acceleration).  Plain FP64 only (precision FP64, gamma 0, no single loop);
 * the handle uses the compact layout (layout 0 or 3, else GABP_E_ARG).  The
 * sweeps are those of Alg. 2, unchanged; after sweep t >= 2 every node forms
 *   y_t = x_{t-2} - (x_{t-1} - x_{t-2})^2 / (x_t - 2 x_{t-1} + x_{t-2})
 * from its own last three means, or y_t = x_t where that second difference is
 * zero or the correction is not finite.  gabp_solve and gabp_backward return
 * y instead of x: the stop rule is applied to y_t on sweeps t >= 2 with
 * t % check_every == 0 or t == max_iter (tol <= 0: exactly max_iter >= 2
 * sweeps, y_{max_iter} returned), gabp_info.sweeps = t, and var (when asked
 * for) holds the variances of sweep t.  A large residual of y_t is not taken
 * for divergence (a node whose second difference nears zero can jump far for
 * one round); a NaN still is.  No precision messages are frozen for reuse.
 * With GABP_FLAG_TIME_SWEEPS every sweep is timed (the sweeps carry no fused
 * check; the Aitken step and the residual of y are not included). */
#define GABP_FLAG_AITKEN 16

/* Steffensen's iterations on the means (Ch. 3 Sec. 3.2, convergence
 * acceleration).  Plain FP64 only, compact layout, not together with
 * GABP_FLAG_AITKEN (else GABP_E_ARG).  The sweeps run in cycles of two.  A
 * cycle starts from an estimate s (the round-0 means b_i / A_ii for the
 * first), runs two sweeps of Alg. 2 to the means x_{t-1} and x_t, and forms
 *   y = s - (x_{t-1} - s)^2 / (x_t - 2 x_{t-1} + s)
 * (y = x_t where the second difference is zero or the correction is not
 * finite).  y then replaces the means of round t: node i's aggregate keeps
 * its precision P~_i and takes the mean y_i, so the messages of the next
 * sweep leave every node with y as its current mean, and y starts the next
 * cycle.  The stop rule is applied to y at the ends of cycles (rounds t with
 * t % check_every == 0, and the last cycle), through the fused check of the
 * following sweep; gabp_solve and gabp_backward return y and gabp_info.sweeps
 * is even.  At most 2 floor(max_iter / 2) sweeps run (max_iter >= 2; tol <= 0
 * runs all of them).  No precision messages are frozen for reuse.  Opt-in: on
 * the benchmark workloads and on the paper's own examples it needs more
 * sweeps than the plain iteration, and it can diverge where the plain
 * iteration converges (the reading of the re-entry of y is recorded with the
 * method's measurements in the design notes). */
#define GABP_FLAG_STEFFENSEN 64

/* Run one launch per sweep even where the whole solve fits one workgroup.
 * Without the flag, a plain FP64 solve (no reuse of frozen precisions, no
 * Aitken or Steffensen step, no sweep timing) on a compact-layout handle with
 * n <= 1024 rows, and either at most 4096 directed slots or at most 6 slots in
 * every row, runs every sweep, check and stop decision inside one launch of
 * 1024 lanes, with the messages in registers and the aggregates in LDS.  Both
 * paths perform the same operations; x, the variances and the messages agree
 * bit for bit, the reported residual up to its summation order. */
#define GABP_FLAG_MULTI_LAUNCH 32

/* Test aid for the compact layout (ignored by the other layouts; implies one
 * launch per sweep).  Before every sweep t the aggregate buffer that sweep t
 * writes (it holds round t-3, which no sweep reads again) and the half of the
 * slot-state buffer holding the other round parity (in^(t-1), which sweep t
 * must not touch) are filled with all-ones bit patterns (NaN in FP32 and
 * FP64); that half is saved before and restored after the sweep.  Once the
 * device status reports the end of the solve the fills are skipped, as are
 * the sweeps.  A solve that reads none of these stale words returns the same
 * bits as without the flag.  Costs two device copies and two fills per sweep,
 * and a save buffer of one slot-state half kept by the handle. */
#define GABP_FLAG_POISON_STALE 128

/* Test aid for the compact layout (implies one launch per sweep).  A solve to
 * a tolerance ends with the sweep that carries the check of the returned
 * round; when the residuals so far predict that round t-1 meets the
 * tolerance, launch t is instead the residual-only check of round t-1, and
 * sweep t (without that check) follows only if the check fails.  With this flag every checked launch from round 2
 * on is made that way, so both outcomes run constantly; the rounds, the
 * checks and the results are the same bits as without the flag, except in
 * the inner solves of the FP32 refinement: without the flag those check only
 * rounds 0-2, at least every fourth round, and the rounds from one before
 * the one their residuals predict to meet the inner tolerance, so they may
 * stop a few rounds later; with it they check every round.  Runs that a
 * freeze of the precisions follows (GABP_FLAG_REUSE_PRECISION, loading), and
 * Aitken's, Steffensen's and the single-loop runs, never take that form. */
#define GABP_FLAG_PREDICT_ALL 256

typedef struct {
  int32_t sweeps;        /* message sweeps run (inner sweeps summed over outer steps) */
  int32_t outer_iters;   /* outer steps (0 for the plain FP64 iteration)              */
  int32_t converged;     /* 1 if rel_residual <= tol                                  */
  int32_t status;        /* gabp_status of the call                                   */
  double  rel_residual;  /* ||b - A x||_2 / ||b||_2 of the returned x (||r|| if b = 0)*/
  double  gamma;         /* loading actually used (0 if none)                         */
  double  sweep_ms;      /* GABP_FLAG_TIME_SWEEPS: summed duration of the timed sweeps */
  int32_t timed_sweeps;  /* number of sweeps in sweep_ms                              */
  int32_t sweep_mode;    /* 0: joint (P, h) sweeps were timed, 1: h-only sweeps       */
} gabp_info;

/* Static properties of a handle (host struct). */
typedef struct {
  int64_t n;                /* unknowns                                   */
  int64_t num_offdiag;      /* directed message slots E = nnz - n         */
  int32_t edges_per_block;  /* slots per workgroup in the sweep kernel    */
  int32_t layout;           /* 1 = reverse-slot index, 2 = node broadcast,*/
                            /* 3 = compact node broadcast, 4 = colour-    */
                            /* serial                                     */
  int32_t xcd_parts;        /* 8 if the rows were renumbered into XCD     */
                            /* parts (GABP_FLAG_NATURAL_ORDER), else 0    */
  int32_t num_blocks;       /* workgroups per sweep launch                */
  int32_t max_degree;       /* largest off-diagonal row length            */
  int32_t precision;        /* gabp_precision                             */
  int64_t device_bytes;     /* device memory owned by the handle          */
  double  rho_lo, rho_hi;   /* bounds on rho(|R|) (walk-summability) when */
                            /* the loading was chosen automatically       */
  double  gamma;            /* loading applied to the inner solves        */
} gabp_props;

/* Default options: FP64, check every sweep, autotuned block size and layout,
 * no loading, inner_tol 1e-5, inner_max_iter 10000, max_outer 1000, reuse
 * flag on, damping 0.5. */
void gabp_default_opts(gabp_opts *opts);

/*
 * gabp_create -- ingest A and prepare the solver (Alg. 2: the
 * neighbourhoods N(i) and the priors P_ii = A_ii).
 *   n          number of unknowns (>= 0)
 *   row_ptr    device int32 [n+1]
 *   col_idx    device int32 [nnz]
 *   vals       device float64 [nnz]
 *   opts       host, nullable (defaults)
 *   stream     HIP stream for all of the handle's work (0 = default stream)
 *   out        host; receives the handle (NULL on failure)
 * Validates the CSR (GABP_E_ARG, GABP_E_NOT_SYMMETRIC, GABP_E_ZERO_DIAG,
 * GABP_E_NONFINITE), builds the off-diagonal CSR, the reverse-slot index and
 * the message buffers on the device.  The handle owns copies; the caller's
 * arrays may be freed after return.  Blocks until done.
 */
gabp_status gabp_create(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        const double *vals, const gabp_opts *opts, hipStream_t stream,
                        gabp_handle *out);

/*
 * gabp_solve -- solve A x = b.
 *   b          device float64 [n]
 *   x          device float64 [n] (output)
 *   var        device float64 [n] (output, nullable): 1 / P~_i, the GaBP
 *              marginal variances (exact on trees, Ch. 2.5; approximate on
 *              loopy graphs).  Plain FP64 mode only, else GABP_E_ARG.
 *   tol        stop when ||b - A x_t||_2 / ||b||_2 <= tol.  tol <= 0 runs
 *              exactly max_iter sweeps and returns x_{max_iter} (no checks).
 *   max_iter   cap on message sweeps (total, all outer steps)
 *   info       host, nullable
 * Plain FP64 (precision FP64, gamma 0): the synchronous iteration of Alg. 2,
 * x_t being the means formed from the messages of sweep t (x_0 = b_i / A_ii),
 * checked every check_every sweeps and at sweep max_iter.  Otherwise: the
 * correction loop x <- x + M^-1 (b - A x), M = A + Gamma (Ch. 5 eq. of the
 * iterative correction method; Gamma = 0 gives iterative refinement), the
 * residual in FP64 and M^-1 applied by GaBP sweeps (FP32 messages for
 * GABP_FP32_REFINE).  Returns GABP_OK, GABP_NOT_CONVERGED, GABP_E_DIVERGED or
 * GABP_E_NONFINITE.
 * Layout 4 replaces the synchronous sweep with a serial one.  A sweep
 * updates the colour classes in increasing colour order.  A node update
 * forms the node's aggregate from its current incoming messages (the mean
 * of that sweep) and overwrites its outgoing messages.  x_t collects the
 * means of sweep t.  Sweep 0, the prior, is checked only when max_iter = 0.
 */
gabp_status gabp_solve(gabp_handle h, const double *b, double *x, double *var,
                       double tol, int32_t max_iter, gabp_info *info);

/*
 * gabp_messages -- copy the messages left by the last gabp_solve that ran
 * with tol <= 0 (exactly max_iter sweeps), plain FP64 mode, layouts 1-3
 * (GABP_E_ARG for layout 4).
 *   P, hmsg    device float64 [num_offdiag] (outputs).  Slot s is the s-th
 *              stored off-diagonal entry (i, j) of A in CSR order (diagonal
 *              skipped) and holds the message i -> j: its precision P_ij and
 *              h_ij = P_ij mu_ij.
 */
gabp_status gabp_messages(gabp_handle h, double *P, double *hmsg);

/*
 * gabp_backward -- adjoint of x = A^-1 b for a scalar loss L(x).
 *   x          device float64 [n]: the solution returned by gabp_solve
 *   grad_x     device float64 [n]: dL/dx
 *   grad_b     device float64 [n] (output): lambda = A^-1 dL/dx (A symmetric)
 *   grad_vals  device float64 [nnz] (output, nullable), aligned with the CSR
 *              given to gabp_create: entry (i, j), i != j, receives
 *              -(lambda_i x_j + lambda_j x_i) (mirror entries move together);
 *              a diagonal entry receives -lambda_i x_i.
 *   tol, max_iter, info as in gabp_solve for the adjoint solve.
 * The adjoint solve is a second GaBP solve against A; with
 * GABP_FLAG_REUSE_PRECISION it reuses the precision messages of the forward
 * solve and runs mean-only sweeps.
 */
gabp_status gabp_backward(gabp_handle h, const double *x, const double *grad_x,
                          double *grad_b, double *grad_vals, double tol, int32_t max_iter,
                          gabp_info *info);

/*
 * gabp_create_augmented -- a general, possibly over-determined, system through
 * the symmetric augmented matrix of Ch. 5 Sec. 5.4 (extension to general
 * linear systems):
 *     K = [[D, B^T], [B, -gamma I]]   over the unknowns {x (n), z (m)},
 * so that B^T B is never formed.  Eliminating z = (B x - h) / gamma from
 * K {x, z} = {b, h} leaves (B^T B / gamma + D) x = b + B^T h / gamma; the
 * section's own matrix is D = I with right-hand side {0, h}, whose x-part is
 * the regularised least-squares solution (B^T B + gamma I)^-1 B^T h.
 *   m, n       B is m x n (m >= 1, n >= 1, m + n < 2^31)
 *   row_ptr, col_idx, vals   device CSR of B: int32 [m+1] (row_ptr[0] = 0),
 *              int32 [nnz] strictly increasing within a row and in [0, n),
 *              float64 [nnz], finite
 *   d          device float64 [n]: the diagonal D, finite and nonzero
 *   gamma      > 0, finite: the lower right block is -gamma I
 *   opts, stream, out   as gabp_create.  K is indefinite, so the plain
 *              iteration does not converge on it: the section runs the
 *              double loop of Ch. 5, i.e. opts->gamma != 0 (< 0: the loading
 *              picked from rho(|R|)).  With opts == NULL the defaults are
 *              used with opts->gamma = -1.
 * K (n + m unknowns, n + m + 2 nnz(B) stored entries, x first) is assembled
 * on the host at create and ingested as by gabp_create; the handle works with
 * every entry point that takes a single-system handle, on vectors of length
 * n + m.  Errors: GABP_E_ARG for a malformed B, d or gamma, otherwise those of
 * gabp_create.
 */
gabp_status gabp_create_augmented(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                  const double *vals, const double *d, double gamma,
                                  const gabp_opts *opts, hipStream_t stream, gabp_handle *out);

/*
 * gabp_plan_augmented -- the symmetric matrix K = [[D, B^T], [B, -gamma I]]
 * of Ch. 5 Sec. 5.4 that gabp_create_augmented would build, assembled on the
 * host, without a GPU.  All arrays are HOST arrays.
 *   m, n, row_ptr, col_idx, vals, d, gamma   as gabp_create_augmented
 *   K_row_ptr  int32 [n+m+1] (output, nullable)
 *   K_col      int32 [cap] (output, nullable), K_val float64 [cap] (output,
 *              nullable): K in full CSR, rows x first, columns increasing
 *   cap        room in K_col / K_val
 *   nnz_out    (output, nullable) stored entries of K, n + m + 2 nnz(B)
 * GABP_E_ARG for a malformed B, d or gamma (the checks of
 * gabp_create_augmented) or cap < *nnz_out when K_col or K_val is given.
 */
gabp_status gabp_plan_augmented(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                const double *vals, const double *d, double gamma, int32_t *K_row_ptr,
                                int32_t *K_col, double *K_val, int64_t cap, int64_t *nnz_out);

/*
 * gabp_solve_augmented -- solve K {x, z} = {b, h} on a handle made by
 * gabp_create_augmented and return the blocks (Ch. 5 Sec. 5.4).
 *   b          device float64 [n], nullable (zero)
 *   h          device float64 [m], nullable (zero)
 *   x          device float64 [n] (output)
 *   z          device float64 [m] (output, nullable)
 *   tol, max_iter, info   as gabp_solve; the residual is that of K.
 * GABP_E_ARG on a handle not made by gabp_create_augmented.
 */
gabp_status gabp_solve_augmented(gabp_handle hdl, const double *b, const double *h, double *x, double *z,
                                 double tol, int32_t max_iter, gabp_info *info);

/*
 * gabp_create_batched -- many independent systems in one handle.
 *   num_sys      number of systems (>= 1)
 *   sys_row_off  HOST int32 [num_sys+1]: system s owns global rows
 *                sys_row_off[s] .. sys_row_off[s+1]-1 (sys_row_off[0] = 0)
 *   row_ptr, col_idx, vals   device CSR of the block-diagonal matrix of all
 *                systems with GLOBAL column indices; an entry outside its
 *                system's block is GABP_E_ARG
 *   opts, stream, out        as gabp_create (precision must be FP32_REFINE;
 *                layout 0 = synchronous sweeps, 4 = colour-serial sweeps inside
 *                each system, colours by first fit in global row order as for
 *                gabp_get_colours; other layouts are GABP_E_ARG)
 */
gabp_status gabp_create_batched(int32_t num_sys, const int32_t *sys_row_off,
                                const int32_t *row_ptr, const int32_t *col_idx,
                                const double *vals, const gabp_opts *opts,
                                hipStream_t stream, gabp_handle *out);

/*
 * gabp_solve_batched -- solve every system for all of its right-hand sides.
 *   nrhs     HOST int32 [num_sys]: k_s >= 1 right-hand sides of system s
 *   rhs_off  HOST int64 [num_sys+1]: B and X offsets; system s uses the
 *            row-major block [n_s][k_s] at rhs_off[s] (rhs_off[s+1] -
 *            rhs_off[s] = n_s * k_s)
 *   B        device float64 [rhs_off[num_sys]]
 *   X        device float64 [rhs_off[num_sys]] (output)
 *   tol      per-RHS relative residual target (FP64 refinement)
 *   max_iter cap on the inner sweeps of each work item (all its outer steps)
 *   infos    HOST gabp_info [num_sys] (output, nullable)
 * One HIP graph runs two persistent kernels; it is captured when the call's
 * B, X, tol, max_iter, nrhs and rhs_off differ from the last call's and
 * replayed when they repeat.  The
 * first computes each system's precision messages once (FP32 P-only sweeps of
 * Alg. 2 until P~ settles, at most opts.inner_max_iter sweeps) and freezes the
 * h-update coefficients.  The second takes work items of 1, 2, 4 or 8
 * right-hand sides of one system, all reading that system's frozen
 * coefficients, and runs the FP64 refinement loop on each (FP64 residual,
 * FP32 h-only inner sweeps until the largest change of the correction is at
 * most opts.inner_tol times its largest magnitude, at most opts.max_outer
 * outer steps).  Returns the worst status over systems.  A tighter inner_tol
 * than gabp_default_opts' 1e-5 saves outer steps here: on the 4096-system
 * benchmark batch 2e-6 is the fastest of 1e-4 ... 1e-6.
 */
gabp_status gabp_solve_batched(gabp_handle h, const int32_t *nrhs, const int64_t *rhs_off,
                               const double *B, double *X, double tol, int32_t max_iter,
                               gabp_info *infos);

/* Load balance of the last gabp_solve_batched launch (host struct). */
typedef struct {
  int32_t num_items;        /* right-hand-side items: (system, group of 1, 2, 4  */
                            /* or 8 right-hand sides)                             */
  int32_t workgroups;       /* persistent workgroups of the right-hand sides     */
  double  makespan_ms;      /* first precision item start to last item end       */
                            /* (device clock)                                     */
  double  busy_ms;          /* sum of the item durations, both phases            */
  double  longest_item_ms;  /* duration of the longest right-hand-side item      */
  int64_t precision_sweeps; /* precision-phase sweeps summed over systems        */
  int64_t inner_sweeps;     /* right-hand-side sweeps summed over items          */
  int32_t longest_sys;      /* system of the longest item                        */
  int32_t longest_nrhs;     /* right-hand sides in that item                     */
  int32_t longest_sweeps;   /* its inner sweeps                                  */
  int32_t longest_psweeps;  /* precision-phase sweeps of its system              */
  double  longest_start_ms; /* its start after the first item's start            */
  int32_t precision_items;  /* systems of the precision phase (one item each)     */
  int32_t pad;
  double  precision_ms;     /* duration of the precision phase (device clock)    */
} gabp_batch_profile;

/* gabp_get_batch_profile -- load-balance figures of the last batched solve. */
gabp_status gabp_get_batch_profile(gabp_handle h, gabp_batch_profile *out);

/*
 * gabp_get_colours -- the colour classes of a layout-4 handle, the node
 * groups updated together by serial scheduling (Ch. 2 Sec. 2.3).
 *   colour       HOST int32 [n] (output, nullable): colour of each row of
 *                the matrix given to gabp_create.  First fit in row order:
 *                row i takes the smallest colour held by none of its stored
 *                neighbours j < i, so no two neighbours share a colour.
 *   num_colours  HOST (output, nullable): number of classes
 * Batched layout-4 handles: the colour of every global row (each system is
 * coloured on its own) and the largest number of classes of a system.
 * GABP_E_ARG for other handles.
 */
gabp_status gabp_get_colours(gabp_handle h, int32_t *colour, int32_t *num_colours);

/* Row plan of a handle (host struct), see gabp_plan_rows. */
typedef struct {
  int32_t num_colours;  /* colour classes (layout 4), else 0                 */
  int32_t xcd_parts;    /* 8 if the rows are renumbered into XCD parts, else 0 */
  int32_t num_blocks;   /* workgroups of a sweep over all rows                */
  int32_t num_chunks;   /* extra workgroups of a compact or colour-serial
                           sweep: a row with more than edges_per_block slots
                           is swept in chunks of edges_per_block slots       */
} gabp_plan;

/*
 * gabp_plan_rows -- the row plan gabp_create would make for this pattern
 * and these options, computed on the host, without a GPU.  That is the
 * colouring of layout 4 (serial scheduling, Ch. 2 Sec. 2.3), the XCD parts,
 * the internal row order and the workgroup partition.
 *   n, row_ptr, col_idx  HOST full CSR pattern (as gabp_create; values unused)
 *   opts       host, nullable: layout, flags and edges_per_block (0 = 512)
 *   perm       HOST int32 [n] (output, nullable): internal row of each row
 *   colour     HOST int32 [n] (output, nullable): colour of each row (layout 4)
 *   blk_row    HOST int32 [blk_cap] (output, nullable): the first internal
 *              row of every workgroup, then n (num_blocks + 1 entries; empty
 *              workgroups pad every XCD part of a group to the same count)
 *   class_blk  HOST int32 [num_colours + 1] (output, nullable, layout 4):
 *              the first workgroup of every colour class's launch, then
 *              num_blocks
 *   plan       HOST (output, nullable)
 * GABP_E_ARG for a malformed pattern (as gabp_create) or blk_cap too small.
 */
gabp_status gabp_plan_rows(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                           const gabp_opts *opts, int32_t *perm, int32_t *colour,
                           int32_t *blk_row, int32_t blk_cap, int32_t *class_blk, gabp_plan *plan);

/*
 * gabp_solve_noalloc -- for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the plain FP64 solve of gabp_create + gabp_solve (synchronous
 * Alg. 2, check every sweep) in one call that allocates nothing.
 *   n          unknowns, 0 <= n <= 1024 (larger: GABP_E_ARG)
 *   row_ptr, col_idx, vals   device full symmetric CSR as for gabp_create,
 *              at most 4096 off-diagonal entries (nnz - n; larger:
 *              GABP_E_ARG, detected on the device)
 *   b          device float64 [n]
 *   x          device float64 [n] (output)
 *   var        device float64 [n] (output, nullable): 1 / P~_i as gabp_solve
 *   tol, max_iter   as gabp_solve (tol <= 0: exactly max_iter sweeps)
 *   stream     the stream of the work; the current device must be its device
 *   info       host, nullable
 * Validation errors are those of gabp_create; solve statuses those of
 * gabp_solve.  The results equal those of gabp_create + gabp_solve bit for
 * bit.  Instead of allocating, the call uses a static device buffer of the
 * library (61.7 KB per device, held until the process ends) for the
 * validation flags, the split off-diagonal CSR and the status: calls that
 * overlap on one device share that buffer and race, so serialise them.  Blocks
 * until the stream has finished the solve.  gabp_last_error(NULL) describes a
 * failure.
 */
gabp_status gabp_solve_noalloc(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *vals,
                               const double *b, double *x, double *var, double tol, int32_t max_iter,
                               hipStream_t stream, gabp_info *info);

/* gabp_props -- static properties of a handle (host output). */
gabp_status gabp_get_props(gabp_handle h, gabp_props *props);

/* Release every resource of the handle (NULL is a no-op). */
void gabp_destroy(gabp_handle h);

/* Description of the last failure on h; NULL h gives the calling thread's
 * last gabp_create / gabp_create_batched failure.  Valid until the next call. */
const char *gabp_last_error(gabp_handle h);

#ifdef __cplusplus
}
#endif

#endif /* GABP_H */
