/*
 * halp.h -- C ABI of an MI355X (gfx950) solver for linear programs based on
 * restarted Halpern PDHG (rHPDHG) and its reflected variant (r2HPDHG).
 *
 * Method: H. Lu and J. Yang, "Restarted Halpern PDHG for Linear Programming",
 * arXiv 2407.16144 (2024).  The PDHG operator T is Section 2, eq. (pdhg); the
 * Halpern step eq. (hpdhg); the restarted loop Algorithm 1; the adaptive
 * restart rule eq. (adaptive-restart) in Section 3; infeasibility
 * certificates from the infimal displacement vector, Section 5; the reflected
 * step eq. (hrpdhg) and Algorithm 2 in Section 6; the relative-KKT
 * termination criterion, preprocessing and primal weight "as cuPDLP" in
 * Section 7.
 *
 * Problem, for every entry point:
 *
 *     minimise  c^T x   subject to   A x = b,   G x >= h,   lb <= x <= ub
 *
 * given as one CSR matrix K = [A; G] with the m_eq equality rows first and
 * the m_ineq inequality rows after them, right-hand side rhs = [b; h], and
 * bounds that may be -INFINITY / +INFINITY.  Duals use the sign in which
 * y_i >= 0 on inequality rows (Lagrangian c^T x - y^T (K x - rhs)).
 *
 * Conventions
 *  - Every function returns an lp_err code (LP_OK = 0 or a negative error)
 *    and never aborts; lp_last_error() returns this thread's last message.
 *  - lp_create / lp_batch_create / lp_server_submit COPY all inputs; the
 *    caller keeps ownership of its arrays.  With inputs_on_device = 1 every
 *    array pointer is HIP device memory (e.g. a torch tensor's data_ptr());
 *    otherwise host memory.
 *  - Host CSR input may have unsorted or duplicate column indices within a
 *    row (duplicates are summed).  Device CSR input must have strictly
 *    increasing column indices within each row.
 *  - Rejected with LP_ERR_INVALID: n < 1, negative row counts, row_ptr not
 *    starting at 0 or decreasing, a column index out of range, NaN/Inf in
 *    val, c or rhs, NaN bounds, lb > ub, lb = +inf or ub = -inf, more than
 *    2^31 - 1 stored entries.
 *  - Solutions and certificates are returned in the ORIGINAL (unscaled)
 *    space, as float64.
 *  - A handle is not thread-safe.  Different handles may run concurrently
 *    on different streams.  `stream` is a hipStream_t; NULL makes the
 *    handle create (and own) a stream of its own.
 *  - Each handle owns its device memory until it is destroyed.
 */
#ifndef HALP_H
#define HALP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LP_OK = 0,
  LP_ERR_INVALID = -1, /* bad argument or malformed LP */
  LP_ERR_OOM = -2,     /* device memory (or reserved capacity) exhausted */
  LP_ERR_DEVICE = -3,  /* HIP runtime error */
  LP_ERR_STATE = -4    /* call not valid in the handle's current state */
} lp_err;

typedef enum {
  LP_UNSOLVED = 0,
  LP_OPTIMAL = 1,            /* relative KKT error <= tol at the returned point */
  LP_PRIMAL_INFEASIBLE = 2,  /* Farkas ray in y-space, see lp_get_certificate */
  LP_DUAL_INFEASIBLE = 3,    /* unbounded ray in x-space, see lp_get_certificate */
  LP_ITER_LIMIT = 4,
  LP_TIME_LIMIT = 5,
  LP_NUMERICAL = 6           /* NaN or Inf in a reduction */
} lp_status_code;

/* LP_METHOD_RAPDHG: restarted average PDHG, the base method of PDLP / cuPDLP
 * that the paper compares with (Sections 2 and 7): plain PDHG steps within
 * an epoch, candidates and restart points at the epoch's running average
 * (the average of Proposition 1), restarts on cuPDLP's KKT-based rule. */
typedef enum { LP_METHOD_RHPDHG = 0, LP_METHOD_R2HPDHG = 1, LP_METHOD_RAPDHG = 2 } lp_method;
typedef enum { LP_PREC_FP64 = 0, LP_PREC_FP32 = 1 } lp_precision;

typedef enum {
  LP_RESTART_ADAPTIVE = 0,
  LP_RESTART_FIXED = 1,
  LP_RESTART_NONE = 2
} lp_restart_mode;

typedef struct {
  int method;               /* lp_method; default r2HPDHG (Algorithm 2) */
  int precision;            /* lp_precision; FP32 stores K, K^T and the iterate
                               streams in float with float accumulation; norms,
                               KKT, restart and step-size scalars stay float64 */
  int ruiz_iters;           /* Ruiz infinity-norm passes (default 10) */
  double pc_alpha;          /* Pock-Chambolle exponent (default 1; <= 0 disables) */
  int check_every;          /* C: restart / termination checks at k % C == 0 (64) */
  double restart_beta;      /* adaptive restart factor, 1/e (eq. (adaptive-restart)) */
  double artificial_restart;/* also restart when k >= this * total (0.36; 0 = off) */
  double step_safety;       /* eta = step_safety / sigma_hat (0.9) */
  int power_max_iters;      /* power iteration cap (1000) */
  int power_min_iters;      /* minimum power iterations (20) */
  double power_rtol;        /* power iteration stop: relative change (1e-4) */
  double eps_infeas;        /* relative tolerance of the Farkas tests (1e-8) */
  int primal_weight;        /* 1: PDLP primal-weight updates; 0: tau = sigma = eta */
  uint64_t seed;            /* SplitMix64 seed of the power-iteration start */
  double eta;               /* > 0: fixed step size, power iteration skipped */
  double omega0;            /* > 0: fixed initial primal weight */
  int chunk;                /* iterations per launched chunk / graph (64) */
  int use_graph;            /* 1: replay chunks as a captured hipGraph */
  int profile;              /* k > 0: time every k-th chunk's two kernels with HIP
                               events on the solver's stream (see lp_kernel_times) */
  int64_t slice_min_bytes;  /* column-slice K (K^T) when the vector its product
                               gathers exceeds this many bytes (default 2 MiB, half
                               the 4 MB L2 of one XCD; < 0 never): in sorted groups
                               (slice_sort = 1) into the fewest of 2, 4 or 8 slices
                               that keep each slice within it, or more where that
                               allows larger groups; in row-major slice tiles
                               (slice_sort = 0) into 8, one per XCD */
  double polish_tol;        /* FP32 precision: when the requested tolerance is
                               below this (default 1e-3), solve in FP32 to this
                               tolerance (or to the stall rule, or for at most a
                               tenth of max_iter), then continue in FP64 from the
                               FP32 candidate (same scaling and step) to the request
                               with the rest of max_iter: lp_solve, lp_batch_solve
                               and FP32 servers */
  int verbose;              /* k > 0: progress line on stderr every k seconds of a solve */
  int64_t cache_budget_bytes; /* bytes of vectors and matrix tiles meant to stay in the
                               last-level cache between steps (default 208 MiB of the
                               256 MB Infinity Cache); the remaining tiles are read with
                               non-temporal loads; < 0: every tile read normally */
  int64_t stall_checks;     /* FP32 phase of a polished solve: an LP moves on to the FP64
                               phase after this many checks without a 10% drop of its
                               best relative KKT error (default 200; 0: only at polish_tol) */
  int restart_mode;         /* lp_restart_mode: LP_RESTART_ADAPTIVE (default; eq.
                               (adaptive-restart) plus the artificial rule),
                               LP_RESTART_FIXED (eq. (fixed-restart): at the first check
                               with k >= fixed_restart_len), LP_RESTART_NONE */
  int64_t fixed_restart_len; /* k* of LP_RESTART_FIXED (>= 1) */
  int xcd_pin;              /* 1 (default): in schedules of 16 or more LPs, each LP's
                               workgroups run on one XCD (its gathered vectors stay in
                               that XCD's L2); 0: every LP spread over all XCDs */
  int tile_rows;            /* SpMV tile shapes (chosen by paper_2407_16144_amd.autotune):
                               rows per plain workgroup tile, 1..256 (default 256; a
                               tile holds at most 1024 entries, longer rows are split
                               off into their own strided tiles) */
  int slice_entries;        /* entries per column-slice tile: 256, 512 (default) or 1024 */
  int slice_rows;           /* rows per sliced row group, 1..256 (default 128) */
  int slice_sort;           /* 1 (default): products whose gathered vector exceeds
                               slice_min_bytes, and products large enough for sorted
                               groups of more rows than a plain block, are stored in
                               sorted groups (row groups x column slices, entries in
                               column order) whose products are added into the row sums
                               with LDS atomics (faster; the order of the additions
                               within a row, and so the last bits of the iterates, may
                               differ from run to run); 0: sliced products in row-major
                               slice tiles with fixed-order sums (slice_entries,
                               slice_rows) */
  int sort_rows;            /* most rows per sorted group or column-sorted block,
                               1..16384 (default 16384).  Sorted groups: the largest
                               group that leaves at least group_blocks workgroups per
                               product and fits the packed column index (fewer rows when
                               a slice is wider than 2^(32 - log2 rows)).  Column-sorted
                               plain blocks: at most 2048 rows, sized for the LPs that
                               share the launches: max(256, rows / 64) with 12 or more
                               live LPs, else about 768 workgroups per product over the
                               live LPs (down to 64 rows); engines re-block their
                               running LPs as others finish */
  int plain_sort;           /* products neither sliced nor in sorted groups (those of
                               small and mid-size LPs): 1 (default) stores the rows of at
                               most 1024 entries in column-sorted blocks (see sort_rows)
                               with LDS-atomic row sums (same caveat as slice_sort);
                               0: plain tiles (tile_rows) with fixed-order sums */
  int group_threads;        /* threads per workgroup of the sorted-group slice kernels:
                               256, 512 or 1024; 0 (default): enough for about eight
                               waves per CU over the product's workgroups */
  int group_batched;        /* 1 (default): each thread issues the gathers of a batch of
                               entries together, then adds them into the LDS row sums;
                               0: one gather per add */
  int group_blocks;         /* fewest workgroups a product stored in sorted groups is cut
                               into (default 240, about one per CU): groups get as many
                               rows as that allows */
  int polish_weight;        /* FP32 precision: primal weight of the FP64 phase, which
                               starts from the FP32 candidate: 1 (default) the FP32
                               phase's last weight; 0 the LP's initial weight
                               ||c~|| / ||q~||, as the method starts (fewer
                               iterations on many LPs, an objective further from the
                               optimum at the same tolerance); 2 the initial weight
                               when the FP32 phase reached polish_tol, else the last */
} lp_options;

typedef struct {
  int status;               /* lp_status_code */
  int ray;                  /* which candidate certified infeasibility: 1 = T(z)-z, 2 = z-z0 */
  int64_t iters;            /* evaluations of T (one K and one K^T product each) */
  int64_t restarts;
  int64_t checks;
  double pobj, dobj;        /* c^T x and the bound-aware dual objective */
  double rel_kkt;           /* max of the three relative errors below */
  double rel_primal, rel_dual, rel_gap;
  double omega, eta, sigma_hat;
  int power_iters;
  int64_t polish_iters;     /* FP64 iterations after an FP32 phase (0 if none) */
  double seconds;           /* wall time of the last lp_solve / batch solve */
  int64_t active_changes;   /* two-stage diagnostics (Section 4): variables whose T(z) sits
                               at a different bound (or leaves / reaches one) and
                               inequality rows whose dual leaves / reaches zero, between
                               the last two checks of the final phase */
  int64_t ident_iters;      /* iterations at the last check where any activity changed:
                               the observed end of the identification stage */
} lp_result;

/* Fills *opt with the defaults listed above. */
void lp_default_options(lp_options* opt);

/* ---------------------------------------------------------------- one LP */

typedef struct lp_solver lp_solver;

/* Copies the LP, builds the explicit transpose K^T, rescales (Ruiz passes and
 * Pock-Chambolle), estimates ||K~||_2 by power iteration and prepares the
 * iterates z^{0,0} = (clamp(0, lb, ub), 0).  row_ptr has m_eq + m_ineq + 1
 * entries, col_idx and val have row_ptr[m] entries, c/lb/ub have n, rhs has
 * m_eq + m_ineq.  opt may be NULL (defaults).  On success *out owns the
 * handle. */
int lp_create(lp_solver** out, int64_t n, int64_t m_eq, int64_t m_ineq, const int32_t* row_ptr,
              const int32_t* col_idx, const double* val, const double* c, const double* rhs,
              const double* lb, const double* ub, int inputs_on_device, void* stream,
              const lp_options* opt);

/* lp_create for CSR input whose row pointers are 64-bit (int64_t, m + 1
 * entries, host or device memory like the other arrays); every entry must
 * lie in [0, 2^31 - 1] (the solver stores at most 2^31 - 1 entries per LP),
 * else LP_ERR_INVALID.  Device row pointers are narrowed on `stream` into a
 * temporary int32 array that the call frees before it returns. */
int lp_create64(lp_solver** out, int64_t n, int64_t m_eq, int64_t m_ineq, const int64_t* row_ptr,
                const int32_t* col_idx, const double* val, const double* c, const double* rhs,
                const double* lb, const double* ub, int inputs_on_device, void* stream,
                const lp_options* opt);

/* Runs restarted (reflected) Halpern PDHG until the relative KKT error at the
 * check candidate T(z) is <= rel_kkt_tol (LP_OPTIMAL), an infeasibility
 * certificate passes its Farkas test, the first check at or after max_iter
 * evaluations of T (LP_ITER_LIMIT), or time_limit_s seconds (LP_TIME_LIMIT;
 * < 0 means none).  Checks happen every `check_every` inner iterations, so
 * the iteration limit is honoured at that granularity.  A handle solves once. */
int lp_solve(lp_solver* s, double rel_kkt_tol, int64_t max_iter, double time_limit_s);

/* Status and statistics of the last solve. */
int lp_status(const lp_solver* s, lp_result* out);

/* The candidate of the last check, unscaled: x (n entries), y (m entries).
 * Either pointer may be NULL.  to_device = 1 writes device memory. */
int lp_get_solution(const lp_solver* s, double* x, double* y, int to_device);

/* After LP_PRIMAL_INFEASIBLE: a ray y (m entries, y_ineq >= 0) with
 * rhs^T y > max_{lb<=x<=ub} (K^T y)^T x up to eps_infeas.  After
 * LP_DUAL_INFEASIBLE: a ray d (n entries) in the recession cone of the box
 * with c^T d < 0, A d = 0, G d >= 0 up to eps_infeas.  LP_ERR_STATE
 * otherwise. */
int lp_get_certificate(const lp_solver* s, double* ray, int to_device);

/* Durations (ms) of the four kernels of a step, summed over the steps timed
 * with HIP events on the solver's stream (options.profile > 0: every
 * profile-th chunk of steps is launched without a graph and timed).  The
 * slice kernels compute the per-XCD column-slice partial products of a
 * column-sliced K^T (primal) or K (dual); where no row group is sliced they
 * launch nothing and their sums stay at (event overhead) ~0. */
typedef struct {
  double primal_slice_ms;
  double primal_ms;          /* primal_step: K^T y and the x half of eq. (pdhg) + Halpern blend */
  double dual_slice_ms;
  double dual_ms;            /* dual_step: K(2x+ - x), the y half of eq. (pdhg), controller */
  double event_pair_ms;      /* two events recorded back to back (no kernel between):
                                the timing overhead contained in each figure above */
  double nnz, n, m;          /* matrix entries, variables and rows of the LPs the timed
                                steps processed, summed over those steps */
  int64_t steps;             /* number of timed steps */
} lp_kernel_timing;

/* Fills *out.  LP_ERR_INVALID for a NULL argument. */
int lp_kernel_times(const lp_solver* s, lp_kernel_timing* out);

/* The constraint matrix as the solver holds it after the preprocessing of
 * Section 7 (Ruiz and Pock-Chambolle scaling), K~ = D1 K D2 (transpose = 0,
 * m rows) or the explicit transpose K~^T the solver builds for the K^T y
 * product (transpose = 1, n rows), as CSR in host arrays supplied by the
 * caller: row_ptr (rows + 1 entries, from 0), col_idx and val (nnz entries
 * each, at least 1; column indices from 0, values in FP64).  Entries of a
 * row are in the order the solver stores them: ascending columns for a
 * product stored in row order.  Only a product stored in row order can be
 * read: one kept in column slices or column-sorted blocks or groups (the
 * default layouts for most LPs; options slice_sort = 0, plain_sort = 0 and
 * slice_min_bytes = -1 keep row order) gives LP_ERR_STATE.  LP_ERR_INVALID
 * for a NULL pointer or a transpose other than 0 or 1. */
int lp_get_scaled_matrix(const lp_solver* s, int transpose, int32_t* row_ptr, int32_t* col_idx, double* val);

void lp_destroy(lp_solver* s);

/* Message of this thread's last error ("" if none). */
const char* lp_last_error(void);

/* ---------------------------------------------------------------- batches */

/* One LP of a batch or a serving request; same array conventions as
 * lp_create. */
typedef struct {
  int64_t n, m_eq, m_ineq;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
  const double* c;
  const double* rhs;
  const double* lb;
  const double* ub;
} lp_problem;

typedef struct lp_batch lp_batch;

/* Many independent LPs stored as one block-diagonal CSR (per-LP offsets),
 * advanced together: every step is one launch over all LPs' rows of K^T and
 * one over all rows of K.  Each LP keeps its own step size, primal weight,
 * Halpern counter, restart state and status, so an LP's result does not
 * depend on what else is in the batch. */
int lp_batch_create(lp_batch** out, int count, const lp_problem* problems, int inputs_on_device,
                    void* stream, const lp_options* opt);
/* Solves every LP of the batch (same tolerance and iteration limit). */
int lp_batch_solve(lp_batch* b, double rel_kkt_tol, int64_t max_iter, double time_limit_s);
int lp_batch_status(const lp_batch* b, int index, lp_result* out);
int lp_batch_get_solution(const lp_batch* b, int index, double* x, double* y, int to_device);
int lp_batch_get_certificate(const lp_batch* b, int index, double* ray, int to_device);
int lp_batch_kernel_times(const lp_batch* b, lp_kernel_timing* out);
void lp_batch_destroy(lp_batch* b);

/* ---------------------------------------------------------------- serving */

typedef struct lp_server lp_server;

/* A continuous-batching solver: submitted LPs wait in a FIFO queue, are
 * admitted when a slot and enough of the reserved device memory are free,
 * advance together with every other live LP, and retire as soon as they
 * finish (results are copied to host memory and their memory is reused).
 * hbm_budget_bytes bounds the device memory the server allocates: FP32
 * servers give half of it to the FP32 engine and half to the FP64 polish
 * engine (with its staging buffer); of each half, three quarters hold the
 * live LPs and one quarter the transient buffers of an admission (about 48
 * bytes per stored entry of the LPs admitted in one step, which caps how
 * much one step admits).  Served LPs are never column-sliced
 * (opt->slice_min_bytes is ignored), so no buffer is allocated while
 * serving beyond the small workgroup schedules. */
int lp_server_create(lp_server** out, int64_t hbm_budget_bytes, int max_slots, void* stream,
                     const lp_options* opt);
/* Copies the LP (host arrays) into the queue; *ticket identifies it.
 * t_arrival is the caller's timestamp (seconds, any origin) used for the
 * latency figures; LP_ERR_INVALID if the LP alone can never fit. */
int lp_server_submit(lp_server* s, const lp_problem* p, double rel_kkt_tol, int64_t max_iter,
                     double t_arrival, int64_t* ticket);
/* Admits what fits, advances all live LPs by `chunks` chunks, retires the
 * finished ones.  *n_done receives how many finished during this call. */
int lp_server_step(lp_server* s, int chunks, int* n_done);
/* 1 in *done if the ticket has finished (then *out holds its result and
 * *t_done the server's clock, in the same units as t_arrival). */
int lp_server_poll(lp_server* s, int64_t ticket, int* done, lp_result* out, double* t_done);
/* The finished ticket's unscaled solution (host memory). */
int lp_server_get_solution(lp_server* s, int64_t ticket, double* x, double* y);
/* The finished ticket's certificate, as lp_get_certificate (host memory:
 * m entries after LP_PRIMAL_INFEASIBLE, n after LP_DUAL_INFEASIBLE);
 * LP_ERR_STATE for a ticket that is not finished or was not found
 * infeasible. */
int lp_server_get_certificate(lp_server* s, int64_t ticket, double* ray);
/* Forget a finished ticket. */
int lp_server_release(lp_server* s, int64_t ticket);
/* The server's clock: seconds since lp_server_create (use it for t_arrival). */
int lp_server_clock(const lp_server* s, double* now);
/* Queue length, live LPs and reserved bytes in use. */
int lp_server_info(const lp_server* s, int* queued, int* live, int64_t* bytes_in_use);
void lp_server_destroy(lp_server* s);

/* ---------------------------------------------------------------- no allocation */

/* Bytes of the static device workspace that lp_solve_static draws on: one
 * array per GPU, part of the library's device code, held by every GPU the
 * library runs on until the process ends. */
#define LP_STATIC_WORKSPACE_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc, code that prepares a graph capture):
 * lp_create + lp_solve + lp_get_solution + lp_destroy of one LP in a single
 * call that allocates no device memory and no pinned host memory.  Every
 * device buffer of the solve (the copied LP, K^T, scaled data, iterates,
 * schedules, partial sums, sort buffers) is carved out of the static
 * workspace of the current GPU and cleared before use; results equal those
 * of lp_create + lp_solve with the same options and use_graph = 0.
 *  - row_ptr .. ub: device pointers, same layout as lp_create (inputs are
 *    copied; the caller keeps ownership).  x (n) and y (m_eq + m_ineq)
 *    receive the unscaled candidate of the last check in DEVICE memory;
 *    either may be NULL.  *out receives the status and statistics.
 *  - stream: a hipStream_t, or NULL for the null stream; the call returns
 *    after its work on the stream has finished.
 *  - FP64 only: opt->precision must be LP_PREC_FP64 (LP_ERR_INVALID
 *    otherwise); opt->use_graph and opt->profile are ignored (no graphs,
 *    no events).
 *  - LP_ERR_OOM, with the bytes needed in lp_last_error(), when the LP does
 *    not fit LP_STATIC_WORKSPACE_BYTES (roughly up to 1M stored entries);
 *    the check happens before any buffer beyond the workspace would be used.
 *  - All calls on one GPU share that GPU's workspace, which keeps the last
 *    call's contents: two calls overlapping on one GPU would race, so the
 *    library serialises the calls of a process with a lock. */
int lp_solve_static(int64_t n, int64_t m_eq, int64_t m_ineq, const int32_t* row_ptr, const int32_t* col_idx,
                    const double* val, const double* c, const double* rhs, const double* lb, const double* ub,
                    void* stream, const lp_options* opt, double rel_kkt_tol, int64_t max_iter,
                    double time_limit_s, double* x, double* y, lp_result* out);

#ifdef __cplusplus
}
#endif

#endif /* HALP_H */
