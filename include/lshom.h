/*
 * lshom - FFT-accelerated conjugate-gradient solver for the periodic
 * unit-cell (Lippmann-Schwinger) conduction problem on MI355X (gfx950).
 *
 * Method: Zeman, Vondrejc, Novak, Marek, "Accelerating a FFT-based solver for
 * numerical homogenization of periodic media by conjugate gradients",
 * J. Comput. Phys. 2010.  The library solves the collocation system
 * (I + B) e = e0 of Sec. 2.2, Eq. (15), with B = F^-1 Gamma0_hat F dL
 * (Eq. (16)), by the conjugate-gradient method of Sec. 2.3 (Saad's
 * Algorithm 6.18, named in Sec. 3).  Phases are isotropic, L = lambda I
 * (lshom_set_microstructure), or symmetric tensors per phase
 * (lshom_set_microstructure_tensor); the reference medium is L0 = l0 I
 * (lshom_set_reference) or any symmetric positive definite matrix
 * (lshom_set_reference_tensor, lshom_set_reference_mean); the cell may have
 * unequal side lengths (lshom_set_cell).
 *
 * Conventions shared by every entry point:
 *  - Grids are d = 2 or 3 dimensional, N[0..d) nodes per axis, C order (the
 *    last axis is contiguous).  Node j of an axis sits at coordinate j / N of
 *    the unit cell.  Every N[a] >= 3, and every prime factor of N[a] is one
 *    of 2, 3, 5, 7, 11, 13, 17 (lshom_check_problem states the size limits).
 *  - A real field with d components is stored component-major, FP64:
 *    field[a * |N| + flat_index], |N| = N[0] * ... * N[d-1].
 *  - Device pointers (suffix _dev) are HIP device memory owned by the caller;
 *    host pointers (suffix _host or plain arrays) are read during the call.
 *  - The library never allocates device memory: the caller provides one
 *    workspace (lshom_workspace_size / lshom_set_workspace).
 *  - Calls are blocking: work is queued on the context's stream after the
 *    caller's stream and the call returns when it has finished.
 *  - Errors are reported by status codes; no C++ exception crosses the ABI.
 *    lshom_last_error() returns a message owned by the context, valid until
 *    the next call on that context.
 */
#ifndef LSHOM_H
#define LSHOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lshom_status;

#define LSHOM_OK 0
#define LSHOM_ERR_INVALID_ARG (-1)   /* an argument is out of its domain */
#define LSHOM_ERR_STATE (-2)         /* call order: microstructure/workspace missing */
#define LSHOM_ERR_WORKSPACE (-3)     /* workspace absent or too small */
#define LSHOM_ERR_HIP (-4)           /* a HIP runtime call failed */
#define LSHOM_ERR_NOT_CONVERGED (-5) /* max_iter reached; last iterate returned */
#define LSHOM_ERR_BREAKDOWN (-6)     /* (p, A p) <= 0 or not finite; last iterate returned */
#define LSHOM_ERR_UNSUPPORTED (-7)   /* valid input outside what the library handles */

#define LSHOM_PRECISION_FP64 0  /* every step in FP64 */
#define LSHOM_PRECISION_MIXED 1 /* FP32 operator and vectors, FP64 dots and refresh */

#define LSHOM_METHOD_CG 0       /* conjugate gradients on Eq. (15) (Sec. 2.3, Sec. 3) */
#define LSHOM_METHOD_FFTH 1     /* the basic scheme: Neumann series of Sec. 2.3, Eq. (18) */
#define LSHOM_METHOD_BICG 2     /* biconjugate gradients on the nodal system (Sec. 2.3; Sec. 3) */
#define LSHOM_METHOD_PIPECG 3   /* CG with one reduction phase per iteration (pipelined, w = A r) */

#define LSHOM_NORM_RESIDUAL 0    /* stop when ||r|| <= tol ||e0|| (eta_r / l0, Eq. (22)) */
#define LSHOM_NORM_EQUILIBRIUM 1 /* stop when eta_e <= tol (Sec. 3, Eq. (21)) */

typedef struct lshom_ctx lshom_ctx;

/* Solver options; lshom_default_opts() fills the defaults shown. */
typedef struct lshom_solve_opts {
  int32_t max_iter;      /* 10000: CG iterations (operator applies in the loop) */
  int32_t precision;     /* LSHOM_PRECISION_FP64 */
  int32_t refresh_every; /* 50: mixed only, FP64 refresh at least this often */
  double refresh_drop;   /* 0.01: mixed only, refresh when ||r|| fell by this factor */
  int32_t graph_block;   /* 16: iterations per captured HIP graph launch (0: no graph) */
  int32_t true_residual; /* 1: recompute b - A x in FP64 after the loop (and eta_e, odd N) */
  int32_t method;        /* LSHOM_METHOD_CG; FFTH, BICG and PIPECG: FP64 only, no x0; BICG and
                            PIPECG: single solves, residual norm, no history, workspace from
                            lshom_workspace_size_for */
  int32_t norm;          /* LSHOM_NORM_RESIDUAL; EQUILIBRIUM: FP64 and odd N only */
  /*
   * NULL, or (single solves, FP64, odd N) a caller-owned device buffer of
   * 2 * history_len doubles receiving (eta_r, eta_e) of iterate m at
   * [2m], [2m + 1] for m < history_len.  CG: iterates x_0 .. x_iterations
   * (eta_r from the recursive residual); FFTH: e^0 .. e^(iterations - 1),
   * whose residual is the step to the next iterate.  Entries past the last
   * iterate are left untouched.
   */
  double* history_dev;
  int32_t history_len;   /* 0 */
} lshom_solve_opts;

/* Per-solve report. */
typedef struct lshom_solve_info {
  int32_t iterations;     /* CG iterations */
  int32_t applies_fp32;   /* FP32 operator applies in the loop (mixed) */
  int32_t applies_fp64;   /* FP64 operator applies, loop and refreshes */
  int32_t status;         /* status of this solve */
  int32_t warm_start_used;/* 1 if x0 was used (not rejected) */
  int32_t refreshes;      /* mixed: FP64 refreshes */
  double rel_res;         /* ||r|| / ||b|| of the recursive residual */
  double rel_res_true;    /* ||b - A x|| / ||b|| in FP64 (if computed, else -1) */
  double eta_r;           /* l0 ||r|| / ||b||, the residual norm of Sec. 3, Eq. (22) */
  double eta_e;           /* equilibrium norm of Sec. 3, Eq. (21) of the returned field
                             (computed with the FP64 true residual, odd N; else -1) */
} lshom_solve_info;

/* Fixed-size message for a status code (static storage). */
const char* lshom_status_string(lshom_status s);

/* Message of the last failed call on ctx ("" if none).  ctx may be NULL. */
const char* lshom_last_error(const lshom_ctx* ctx);

void lshom_default_opts(lshom_solve_opts* opts);

/*
 * Host-only validation of a problem statement (no device is touched):
 * d in {2, 3}; 3 <= N[a] <= 4096 with prime factors in {2, 3, 5, 7, 11, 13, 17};
 * fewer than 2^31 nodes; and the pass kernels' LDS footprint (one block holds
 * whole transform sequences and a twiddle table of N[a] entries, within
 * gfx950's 160 KiB of LDS per workgroup less 1 KiB for the kernels' static
 * use) fits for both precisions with scalar phases.  The last condition
 * bounds the axes far below 4096: the largest supported squares and cubes
 * are 1800^2 and 1224^3, and some smaller lengths whose radix plans need more
 * threads than a block holds (1458, 1620, 1728, 2048 in 2-D) are rejected
 * too.  A context further limits the LDS to what its device reports.  The same limits apply when a microstructure is set
 * (UNSUPPORTED there as well; tensor phases need somewhat more LDS);
 * 1 <= n_phases <= 256 with finite cond > 0; l0 finite > 0, or exactly 0 to
 * mean "the default (min + max) / 2" of Sec. 2.3, Eq. (19); E (d values, may
 * be NULL) finite; tol finite >= 0 (tol < 0 skips the check).
 * Returns LSHOM_OK or LSHOM_ERR_INVALID_ARG / LSHOM_ERR_UNSUPPORTED.
 */
lshom_status lshom_check_problem(int d, const int64_t* N, int n_phases, const double* cond,
                                 double l0, const double* E, double tol);

/*
 * Create a context on HIP device `device`.  hip_stream is the caller's
 * hipStream_t (NULL = the null stream); the context queues its work on a
 * private stream ordered after it.  *out is NULL on failure.
 */
lshom_status lshom_create(lshom_ctx** out, int device, void* hip_stream);
void lshom_destroy(lshom_ctx* ctx);

/*
 * The periodic microstructure: a digital image of phases sampled at the grid
 * nodes (Sec. 2.2, Eq. (17): dL is diagonal with entries dL(x^k)), with an
 * isotropic conductivity per phase (Sec. 3).  phase_dev holds prod(N) bytes,
 * C order, each < n_phases; it stays owned by the caller and must stay valid
 * until the next set_microstructure or destroy.  cond_host is copied.  Sets
 * l0 to the optimal (min + max) / 2 of Sec. 2.3, Eq. (19).  Invalidates the
 * workspace.
 */
lshom_status lshom_set_microstructure(lshom_ctx* ctx, int d, const int64_t* N,
                                      const uint8_t* phase_dev, int n_phases,
                                      const double* cond_host);

/*
 * As lshom_set_microstructure with a second-order conductivity tensor per
 * phase (Sec. 2.1, Eq. (1)): cond_tensor_host holds n_phases symmetric
 * positive-definite d x d matrices, row-major, copied.  n_phases is at most
 * 256 / (d (d + 1) / 2).  l0 defaults to (smallest + largest eigenvalue) / 2
 * over the phases (Sec. 2.3, Eq. (19)).  Single solves (lshom_solve,
 * lshom_homogenize, lshom_apply) with any method and precision.
 */
lshom_status lshom_set_microstructure_tensor(lshom_ctx* ctx, int d, const int64_t* N,
                                             const uint8_t* phase_dev, int n_phases,
                                             const double* cond_tensor_host);

/*
 * Side lengths of the periodic cell (Sec. 2.1, the cell prod (-Y_a, Y_a); d
 * finite values > 0, only their ratios matter).  The Green operator then
 * takes the wave vector xi_a = k_a / Y_a in place of the integer frequency
 * (and so does the equilibrium norm).  The default is a cubic cell.
 */
lshom_status lshom_set_cell(lshom_ctx* ctx, const double* lengths);

/* Reference medium L0 = l0 I (Sec. 2.1, Eq. (3); Sec. 3, Eq. (20)); finite, > 0. */
lshom_status lshom_set_reference(lshom_ctx* ctx, double l0);

/*
 * A general reference medium (Sec. 2.1, Eqs. (3) and (7): dL = L - L0 and the
 * Green operator xi (x) xi / (xi . L0 . xi)).  L0_host holds a symmetric
 * positive-definite d x d matrix, row-major, copied; INVALID_ARG otherwise.
 * A multiple of the identity acts as lshom_set_reference.  Otherwise:
 *  - scalar phases are turned into the tensors lambda I (the context then
 *    holds a tensor problem, as after lshom_set_microstructure_tensor; an
 *    attached workspace stays attached and is refilled);
 *  - CG and the basic scheme work in the energy product of L0,
 *    <u, v> = sum_x u . L0 . v, in which the system is self-adjoint: the
 *    residual test and rel_res, rel_res_true use ||r||_L0 / ||E||_L0, and
 *    eta_r uses tr(L0) / d in place of l0.  BiCG keeps Euclidean products.
 *  - eta_e (Eq. (21)) does not depend on L0.
 * Single solves only (lshom_solve, lshom_homogenize, lshom_apply); the
 * converged field does not depend on L0, the iteration count does.
 * lshom_set_reference returns to an isotropic reference.
 */
lshom_status lshom_set_reference_tensor(lshom_ctx* ctx, const double* L0_host);

/*
 * L0 = <L>, the cell average of the conductivity (phase counts of the
 * phase image times the phase tables), set as by lshom_set_reference_tensor
 * (a number for isotropic phases).  In the spectral coordinate of the
 * solver k_hat . <L> . k_hat is the diagonal of the operator, so this
 * reference is the Fourier-space Jacobi preconditioner of CG in the energy
 * product of L0 (Sec. 2.1, Eq. (7) with a general L0); CG does not depend on
 * the scale of L0, only on its shape.  Needs an attached workspace (it holds
 * the counts); WORKSPACE otherwise.
 */
lshom_status lshom_set_reference_mean(lshom_ctx* ctx);

/* Bytes of device workspace the current problem needs (both precisions). */
lshom_status lshom_workspace_size(const lshom_ctx* ctx, int precision, size_t* bytes);

/*
 * Bytes of device workspace a solve with these options needs (opts NULL =
 * defaults).  BiCG iterates on d-component nodal fields and needs seven of
 * them (x, r, r*, p, p*, A p, A^T p*) on top of the CG workspace; pipelined
 * CG uses the same extra area.
 */
lshom_status lshom_workspace_size_for(const lshom_ctx* ctx, const lshom_solve_opts* opts, size_t* bytes);

/* Attach caller-owned device workspace (256-byte aligned, >= the size above;
 * the largest of the layouts above that fits is used). */
lshom_status lshom_set_workspace(lshom_ctx* ctx, void* dev, size_t bytes);

/*
 * Solve (I + B) e = e0 with e0 = E at every node (Sec. 2.2, Eq. (15)) by CG,
 * or with opts->method = LSHOM_METHOD_FFTH by the basic scheme
 * e^(m+1) = e0 - B e^(m) (Eq. (18)).  Stops when ||r|| <= tol ||e0||
 * (recursive residual; for the basic scheme the step e^(m+1) - e^(m)), or
 * with LSHOM_METHOD_BICG by BiCG on the nodal fields (shadow residual
 * r0* = r0; info->applies_fp64 counts both products per iteration), or
 * with LSHOM_METHOD_PIPECG by pipelined CG (the iterates of CG in exact
 * arithmetic; both inner products of an iteration come from one reduction
 * in the update pass, so a distributed solve needs one all-reduce per
 * iteration, which can overlap the operator apply; the three extra
 * spectral vectors w = A r, s = A p, z = A s take the BiCG field area), or
 * with LSHOM_NORM_EQUILIBRIUM when eta_e <= tol, or after max_iter.  The
 * basic scheme tests iterate m in the apply that forms m + 1 and returns
 * e^(m+1).
 * x0_dev: NULL starts from e = E; otherwise a d x |N| FP64 field whose
 * admissible part E + P(x0) is used (P: projection on zero-mean curl-free
 * fields); it is rejected (start from E) if its residual is not finite or not
 * below the residual of E.
 * e_dev (d x |N| FP64, may be NULL) receives the field; leff_host (d values,
 * may be NULL) receives <lambda e> = L_eff E; info (may be NULL) the report.
 * NOT_CONVERGED and BREAKDOWN still write the last iterate and info; other
 * errors leave the outputs untouched.  E = 0 returns e = 0 at once.
 */
lshom_status lshom_solve(lshom_ctx* ctx, const double* E_host, double tol,
                         const lshom_solve_opts* opts, const double* x0_dev, double* e_dev,
                         double* leff_host, lshom_solve_info* info);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): lshom_solve for the
 * context's current microstructure with the library's own scratch as the
 * workspace, a file-scope device array of LSHOM_STATIC_WORKSPACE_BYTES per
 * GPU, held until the process ends.  No device memory is allocated or freed
 * and no graph is instantiated (iterations are launched one by one); the
 * caller still passes the outputs, and the context keeps the workspace it
 * had (lshom_set_workspace is not needed for this call).
 * Arguments, outputs and statuses as for lshom_solve, without a warm start.
 * Returns LSHOM_ERR_UNSUPPORTED when the problem and options need more than
 * LSHOM_STATIC_WORKSPACE_BYTES (lshom_workspace_size_for tells).  Every call
 * on one GPU uses the same array: calls from one process are serialised per
 * GPU (a call waits for the previous one), and each call initialises all it
 * reads.
 */
#define LSHOM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
lshom_status lshom_solve_static(lshom_ctx* ctx, const double* E_host, double tol,
                                const lshom_solve_opts* opts, double* e_dev, double* leff_host,
                                lshom_solve_info* info);

/*
 * Effective conductivity tensor from the d load cases E = e_b: column b of
 * leff_host (d x d, row-major) is <lambda e> for E = e_b.  infos: d reports
 * (may be NULL).  Returns the worst status.
 */
lshom_status lshom_homogenize(lshom_ctx* ctx, double tol, const lshom_solve_opts* opts,
                              double* leff_host, lshom_solve_info* infos);

/*
 * One FP64 operator apply on an arbitrary real field: q = (I + B) p of
 * Sec. 2.2, Eqs. (15)-(16).  p_dev and q_dev are d x |N| FP64 (may not alias).
 */
lshom_status lshom_apply(lshom_ctx* ctx, const double* p_dev, double* q_dev);

/*
 * Many independent problems (each an isotropic microstructure, reference
 * medium, load and tolerance as for lshom_solve) in one call.  Problems with
 * the same grid share every kernel launch (one block row per problem) and
 * advance together in captured graph blocks until each has met its own stop
 * test; grids are processed in turn.  d, N, phase_dev, n_phases and cond_host
 * as for lshom_set_microstructure; l0 <= 0 selects (min + max) / 2; E holds d
 * values; e_dev (d x |N| FP64) may be NULL.
 */
typedef struct lshom_problem {
  int32_t d;
  int64_t N[3];
  const uint8_t* phase_dev;
  int32_t n_phases;
  const double* cond_host;
  double l0;
  double E[3];
  double tol;
  double* e_dev;
  double cell[3];  /* side lengths of the cell (Sec. 2.1; Green operator at xi = k / Y); all 0: cubic */
  /* initial guess (d x |N| FP64, device, caller-owned, read during the call;
   * NULL: start from e = E), taken as for lshom_solve: projected to
   * E + P x0 and dropped in favour of e = E unless its residual is smaller */
  const double* x0_dev;
} lshom_problem;

/* Device workspace bytes lshom_solve_batched needs for these problems. */
lshom_status lshom_batch_workspace_size(lshom_ctx* ctx, int32_t n, const lshom_problem* probs,
                                        int precision, size_t* bytes);

/*
 * Solve n problems (each may carry its own warm start x0_dev, CG only;
 * opts->method and opts->norm apply to every problem, opts->history_dev must
 * be NULL).  A warm start that is dropped leaves its problem on e = E; the
 * report's warm_start_used says which happened.
 * ws_dev: caller-owned
 * device workspace of at least lshom_batch_workspace_size bytes, 256-byte
 * aligned (it is not kept after the call).  leff_host: n x 3 (row i is
 * <lambda e> of problem i, zero-padded); infos: n reports; both may be NULL.
 * Returns LSHOM_OK or the first non-OK per-problem status (each report holds
 * its own); argument or HIP errors abort the call.
 */
lshom_status lshom_solve_batched(lshom_ctx* ctx, int32_t n, const lshom_problem* probs,
                                 const lshom_solve_opts* opts, void* ws_dev, size_t ws_bytes,
                                 double* leff_host, lshom_solve_info* infos);

/*
 * Launch schedule of one grid at one precision: the radix order of each
 * axis's FFT (product = N[a]; radices 2..9) and the pass shapes (rows of the
 * last axis per row-pass block, an even number; whether a row-pass block
 * holds one component (row_split = 1) or all d; column tiles of the axis-0
 * and axis-1 passes; block sizes of the row and axis passes, 128 or 256
 * threads, 0 for the smallest that holds the batch).  Results do not depend on the schedule beyond
 * floating-point rounding.
 */
typedef struct lshom_schedule {
  int32_t d;
  int64_t N[3];
  int32_t precision;
  int32_t rows_per_block;
  int32_t tile0;
  int32_t tile1;
  int32_t row_split;
  int32_t threads_row;
  int32_t threads_col;
  int32_t nstages[3];
  int32_t radix[3][16];
  double ms_per_iter;  /* autotuned device time of one CG iteration's passes (0: not measured) */
  int32_t tail_rows;   /* 0: the schedule of the grid; > 0: used instead by batched launches that
                          cover at most this many unfinished problems (the tail of a batch) */
} lshom_schedule;

/* Schedule the current problem uses at `precision`. */
lshom_status lshom_get_schedule(lshom_ctx* ctx, int precision, lshom_schedule* out);

/*
 * Register a schedule for its grid and precision (used by later solves of
 * that grid, single or batched; applied at once to the current problem when
 * the grid matches).  INVALID_ARG if it does not factor N or does not fit the
 * FFT batch or LDS limits.
 */
lshom_status lshom_set_schedule(lshom_ctx* ctx, const lshom_schedule* s);

/*
 * Autotuner: time every pass kind of one CG iteration under candidate radix
 * orders and launch shapes (HIP events over `reps` launches each) on the
 * current problem, keep the fastest per pass kind, register and apply it;
 * best (may be NULL) receives it.  Overwrites the internal vectors (call it
 * between solves).
 */
lshom_status lshom_autotune(lshom_ctx* ctx, int precision, int reps, lshom_schedule* best);

/*
 * Autotuner for batched solves: for every distinct grid among the problems,
 * tune on that grid's whole batch (same launches as lshom_solve_batched) and
 * register the result.  ws_dev / ws_bytes as for lshom_solve_batched.
 * best (may be NULL) receives up to *n_best schedules; *n_best (may be NULL)
 * the number of grids.
 */
lshom_status lshom_autotune_batched(lshom_ctx* ctx, int32_t n, const lshom_problem* probs, int precision,
                                    int reps, void* ws_dev, size_t ws_bytes, lshom_schedule* best,
                                    int32_t* n_best);

/* Write the registered schedules as JSON lines keyed by GPU architecture,
 * d, N and precision (one object per line); read them back (entries of other
 * architectures are skipped).  Returns INVALID_ARG on I/O or parse errors. */
lshom_status lshom_save_schedules(lshom_ctx* ctx, const char* path);
lshom_status lshom_load_schedules(lshom_ctx* ctx, const char* path);

/* Kernel classes reported by lshom_time_passes. */
#define LSHOM_PASS_AXIS0_INVERSE 0  /* p = r + beta p, i khat p, inverse FFT along axis 0 */
#define LSHOM_PASS_AXIS1_INVERSE 1  /* 3-D: inverse FFT along axis 1 */
#define LSHOM_PASS_ROW 2            /* last axis: inverse FFT, dL (E + u), forward FFT */
#define LSHOM_PASS_AXIS1_FORWARD 3  /* 3-D: forward FFT along axis 1 */
#define LSHOM_PASS_AXIS0_FORWARD 4  /* forward FFT along axis 0, Gamma0 projection, q, (p, q) */
#define LSHOM_PASS_UPDATE 5         /* x += alpha p, r -= alpha q, (r, r) */
#define LSHOM_PASS_COUNT 6

/*
 * Device time of each pass kernel of one CG iteration (Sec. 2.3: the apply of
 * Eq. (16) plus the CG vector updates) for the current problem at `precision`:
 * every kernel is launched `reps` times back to back on the context stream,
 * with the same launch shape and buffers as in lshom_solve, between two HIP
 * events.  ms_out[LSHOM_PASS_COUNT] receives the average milliseconds per
 * launch (0 for passes a 2-D problem does not have); bytes_out (may be NULL)
 * the minimum HBM bytes each launch must move (its algorithmic traffic).
 * Overwrites the solver's internal vectors: call it between solves.
 */
lshom_status lshom_time_passes(lshom_ctx* ctx, int precision, int reps, double* ms_out,
                               double* bytes_out);

/*
 * Pass timing inside real solves.  While enabled, lshom_solve and
 * lshom_solve_batched on this context queue their CG iterations without HIP
 * graph capture and bracket every pass-kernel launch of the CG loop with a
 * pair of HIP events on the context stream.  lshom_get_pass_timing returns,
 * per pass class, the summed device milliseconds, the number of launches and
 * the algorithmic HBM bytes of the work those launches did (the per-problem
 * bytes of lshom_time_passes times the CG iterations the problems actually
 * advanced; launches for problems that had already stopped count zero
 * bytes).  Enabling (or disabling) resets the sums.  Arrays hold
 * LSHOM_PASS_COUNT entries; any may be NULL.
 */
lshom_status lshom_set_pass_timing(lshom_ctx* ctx, int enable);
lshom_status lshom_get_pass_timing(lshom_ctx* ctx, double* ms_out, double* bytes_out, int64_t* launches_out);

#ifdef __cplusplus
}
#endif

#endif /* LSHOM_H */
