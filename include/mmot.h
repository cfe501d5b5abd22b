/*
 * mmot.h -- C ABI of the MI355X graph-structured multi-marginal Sinkhorn solver
 * for dynamic multi-commodity min-cost network flow.
 *
 * Method: Haasler, Ringh, Chen, Karlsson, "Scalable computation of dynamic flow
 * problems via multi-marginal graph-structured optimal transport".  The solver
 * runs Algorithm 2 (Section 4.3): entropy-regularised problem
 * "multicommodity_reg", whose optimum is M = K (.) U (Theorem 3/4) with
 * K = exp(-C/eps) and scalings U^(0,1), u_t, U^(0,TT) (eq. U_multicommodity),
 * computed by the Sinkhorn updates of eq. sinkhorn_multicommodity using the
 * message recursions of Theorem 5 and the marginals of Corollary 1.
 *
 * Conventions used throughout this header
 *   n   number of states (graph nodes); L commodities; T transitions, so the
 *       marginals sit at times 0..T (the paper's TT = T + 1 time marginals).
 *   Source distribution R^(0,1) at time 0, sink distribution R^(0,TT) at
 *   time T, capacity d on the summed occupancy at the interior times 1..T-1.
 *   All array arguments are DEVICE pointers owned by the caller unless the
 *   parameter name ends in _host.  Matrices in the paper's L x n orientation
 *   are row-major with the commodity index slowest ("l * n + i").
 *   A solver never allocates device memory: every buffer it keeps lives in
 *   the caller-provided workspace (size from mmot_query_workspace).  All work
 *   is enqueued on the stream given to mmot_create (a hipStream_t passed as
 *   void*, NULL = default stream); calls that return host data synchronise it.
 *   Calls on one solver are not thread-safe; distinct solvers are independent.
 * Errors: every call returns mmot_status; MMOT_OK on success.  On error no
 *   output is written and the solver (if any) stays usable unless stated.
 */
#ifndef MMOT_H
#define MMOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mmot_status {
  MMOT_OK = 0,
  MMOT_EINVAL = 1,        /* bad sizes, eps, NaN/negative data, unsorted CSR, unequal or zero masses */
  MMOT_ENOMEM = 2,        /* workspace smaller than mmot_query_workspace reported */
  MMOT_EINFEASIBLE = 3,   /* a positive source/sink entry faces a zero message (Theorem 4 support) */
  MMOT_ENUMERIC = 4,      /* non-finite values appeared, or a scaled-domain solver that passed its
                             AUTO probe met a zero message later (range exceeded in the scaled domain) */
  MMOT_EHIP = 5,          /* a HIP runtime call failed */
  MMOT_EAGAIN = 6,        /* pool: request does not fit the HBM budget right now */
  MMOT_EUNSUPPORTED = 7   /* option combination not implemented */
} mmot_status;

enum { MMOT_CSR = 0, MMOT_DENSE = 1 };
/* arithmetic of the K-products (messages); FP64 reductions are used for stats either way */
enum { MMOT_FP32 = 0, MMOT_FP64 = 1, MMOT_BF16 = 2 /* dense only: BF16 MFMA + FP32 polish */ };
/* range control: SCALED keeps per-commodity FP64 log offsets on linear panels,
   LOG keeps log2-values (log-sum-exp products); AUTO picks from a range estimate */
enum { MMOT_DOMAIN_AUTO = 0, MMOT_DOMAIN_SCALED = 1, MMOT_DOMAIN_LOG = 2 };

/* Problem data (eq. multicommodity / multicommodity_reg).  kind == MMOT_CSR:
 * the allowed moves i -> j (time tau to tau+1) are the CSR entries of C
 * (rowptr[n+1], colidx[nnz] sorted ascending within each row, cost[nnz]);
 * waiting is a diagonal entry.  kind == MMOT_DENSE: cost_dense[n*n],
 * row-major, +INF marks a forbidden move.  Negative finite costs are allowed.
 * state_cost: per-commodity state cost C_L (L x n) charged at interior times,
 * or NULL (K_L = 1).  cap: n values (cap_per_step = 0, same at every interior
 * time) or (T-1) x n (cap_per_step = 1); +INF = uncapacitated; must be > 0.
 * src = R^(0,1), dst = R^(0,TT): L x n, >= 0, each commodity's row sums equal
 * (relative 1e-9) and positive (a commodity without mass is rejected: drop it
 * from the problem instead). */
typedef struct mmot_problem {
  int32_t n, L, T;
  double eps;
  int32_t kind;
  int32_t cap_per_step;
  int64_t nnz;
  const int32_t* rowptr;
  const int32_t* colidx;
  const double* cost;
  const double* cost_dense;
  const double* state_cost;
  const double* cap;
  const double* src;
  const double* dst;
  /* 1: a time-varying network (Section 3.3, one cost matrix C_tau per move
   * tau -> tau+1).  CSR: cost holds T x nnz values, row tau for the moves from
   * time tau to tau+1, all with the pattern of rowptr/colidx; an entry may be
   * +INF to close that move at that step.  Dense: cost_dense holds T x n x n
   * values (matrix tau for the move tau -> tau+1; the workspace then holds T
   * copies of K and K^T).  0: cost holds nnz values used at every step
   * (finite), cost_dense one n x n matrix. */
  int32_t cost_per_step;
  /* Commodity-dependent capacities (the extension at the end of Section 3):
   * P_{0,t}[l, i] <= D_t[l, i] at the interior times, D >= 0, +INF = no bound,
   * 0 closes state i to commodity l.  L x n values used at every interior
   * time (cap_comm_per_step = 0) or (T-1) x L x n (index ((t-1)*L + l)*n + i,
   * cap_comm_per_step = 1).  NULL = none.  Sparse and dense networks (dense:
   * w_t is applied in the epilogue of the forward and backward products).
   * Each adds one dual scaling w_t (L x n, in [0, 1]) per interior time; see
   * mmot_get_comm_duals. */
  const double* cap_comm;
  int32_t cap_comm_per_step;
} mmot_problem;

typedef struct mmot_options {
  int32_t precision;     /* MMOT_FP32 (default), MMOT_FP64, MMOT_BF16 */
  int32_t domain;        /* MMOT_DOMAIN_AUTO (default) / SCALED / LOG */
  int32_t check_every;   /* mmot_solve: iterations between convergence checks (default 10) */
  int32_t calib_every;   /* re-centre the range offsets every this many iterations (default 10; the first 3 always) */
  int32_t polish_iters;  /* BF16: FP32 iterations appended by mmot_solve (default 20) */
  int32_t use_graph;     /* capture one iteration in a HIP graph (default 1) */
  double tol;            /* mmot_solve: stop when src_resid <= tol and cap_viol <= tol (default 1e-6) */
  /* 1 (default): room for the forward messages of every time (T - 1 more n x L
   * panels without state costs or commodity capacities, on a fixed network when
   * sparse; the
   * last Sinkhorn sweep of each mmot_iterate / mmot_solve chunk fills them), so
   * that the convergence check after it takes its statistics from the fresh
   * backward sweep it needs anyway (Corollary 1: P_t = u_t sum_l hatPsi_t Psi_t
   * K_L), without an extra update-free forward sweep.  0: two rolling forward
   * panels.  The serving pool runs 0 (mmot_pool_submit rejects 1 with
   * MMOT_EUNSUPPORTED).  The two give the same statistics up to rounding order
   * and the same iterates. */
  int32_t keep_forward;
} mmot_options;

/* Convergence / dual statistics of the current iterate (FP64 reductions).
 * dual_obj: dual objective of Theorem 3 at the current scalings,
 *   eps*(<log U01,R01> + <log U0T,R0T> + sum_t <log u_t,d_t> + sum_t <log w_t,D_t>)
 *   - eps*<K,U> (the w_t term only with commodity capacities).
 * src_resid: sum|P_{0,1} - R01| / sum R01; cap_viol: max_t,i (P_t - d)_+ / d,
 *   and max_t,l,i (P_{0,t} - D_t)_+ / D_t with commodity capacities;
 * mass_drift: max over times of |mass(t) - mass(T)| / mass(T) (Corollary 1
 * makes it zero in exact arithmetic); dual_gap: eps*(<log U,P - R> terms). */
typedef struct mmot_stats {
  int32_t iters;
  int32_t converged;
  int32_t domain;        /* domain actually used */
  int32_t precision;     /* precision actually used */
  double dual_obj;
  double src_resid;
  double cap_viol;
  double mass_drift;
  double dual_gap;
  double mass;
} mmot_stats;

typedef struct mmot_solver mmot_solver;

/* Fill *opt with the defaults listed above. */
void mmot_default_options(mmot_options* opt);

/* Bytes of device workspace mmot_create needs for this problem and options.
 * Only sizes, kinds and precision are read; the optional arrays (state_cost,
 * cap_comm) are only tested for NULL (no device data is touched).
 * EINVAL on bad sizes; EUNSUPPORTED on an unsupported combination. */
mmot_status mmot_query_workspace(const mmot_problem* prob, const mmot_options* opt, size_t* bytes_host);

/* Build a solver: validates the problem on the device, forms K (CSR of K and
 * of K^T, or dense K/K^T), converts R01/R0T/C_L/d to the internal state-major
 * layout and sets the initial scalings (u = 1, U0T = 1 on supp R0T).
 * ws: device buffer of ws_bytes >= the queried size, 256-byte aligned, owned by
 * the caller and kept alive until mmot_destroy.  The problem arrays may be
 * freed after this call returns.  Synchronises the stream.
 * *out receives a host-side handle.  EINVAL / ENOMEM / EHIP on failure. */
mmot_status mmot_create(const mmot_problem* prob, const mmot_options* opt, void* ws, size_t ws_bytes,
                        void* stream, mmot_solver** out);

/* Enqueue n_iter Sinkhorn iterations (Algorithm 2 loop body: backward sweep,
 * source update, forward sweep with capacity updates, sink update).
 * Asynchronous unless stats_host != NULL: then a check pass computes the
 * statistics of the resulting iterate and the call synchronises.
 * Returns EINFEASIBLE / ENUMERIC if the device flagged such a condition
 * (checked only when stats_host != NULL). */
mmot_status mmot_iterate(mmot_solver* s, int32_t n_iter, mmot_stats* stats_host);

/* Iterate with a convergence check every opt.check_every iterations until
 * converged or max_iter iterations; BF16 solvers then run polish_iters FP32
 * iterations.  Synchronous; fills *stats_host (nullable). */
mmot_status mmot_solve(mmot_solver* s, int32_t max_iter, mmot_stats* stats_host);

/* Statistics of the current iterate (one update-free pass).  Synchronous. */
mmot_status mmot_stats_now(mmot_solver* s, mmot_stats* stats_host);

/* Projections of the current plan M = K (.) U (Theorem 5, Corollary 1):
 * occ[(T+1) * n] = occupancy P_t (row t = time t), always written;
 * per_comm[(T+1) * L * n] = P_{0,t} (index (t*L + l)*n + i), optional (NULL).
 * Asynchronous (device outputs). */
mmot_status mmot_occupancy(mmot_solver* s, double* occ, double* per_comm);

/* The same for a window of commodities (a full P_{0,t} of a large problem is
 * (T+1) x L x n doubles; the window pages through it): occ as above;
 * per_comm[(T+1) * comm_count * n] = P_{0,t} of commodities comm_first ..
 * comm_first + comm_count - 1 (index (t*comm_count + k)*n + i for commodity
 * comm_first + k), optional (NULL: comm_first and comm_count are ignored).
 * MMOT_EINVAL unless 0 <= comm_first and 1 <= comm_count <= L - comm_first.
 * Asynchronous (device outputs). */
mmot_status mmot_occupancy_window(mmot_solver* s, double* occ, double* per_comm, int32_t comm_first,
                                  int32_t comm_count);

/* Aggregate edge flows (bi-marginal projections P_{t,t+1} summed over
 * commodities, eq. proj_discrete_bi), t = 0..T-1.  CSR problems:
 * flow[t * nnz + e] = mass moving along CSR entry e between times t and t+1.
 * Dense problems: flow[(t * n + i) * n + j] = mass moving from state i to
 * state j (T * n * n doubles, zero where C_ij = +INF), the commodity sum of
 * each time one MFMA product.  cost_host (nullable): transport cost <C, M> =
 * move costs + interior state costs (eq. cost_multicommodity); synchronises. */
mmot_status mmot_edge_flows(mmot_solver* s, double* flow, double* cost_host);

/* Natural-log dual scalings of the current iterate: log_src, log_dst (L x n,
 * -INF off the support), log_cap ((T-1) x n, <= 0).  Asynchronous. */
mmot_status mmot_get_log_duals(mmot_solver* s, double* log_src, double* log_dst, double* log_cap);

/* Warm start / resume: replace the scalings (same layout as above). Only
 * log_dst and log_cap matter for the next iteration (log_src is recomputed by
 * its first source update).  Asynchronous. */
mmot_status mmot_set_log_duals(mmot_solver* s, const double* log_src, const double* log_dst,
                               const double* log_cap);

/* Commodity-capacity duals (problems with cap_comm): natural logs of the
 * scalings w_t, (T-1) x L x n (index ((t-1)*L + l)*n + i), <= 0, -INF where
 * D_t = 0.  In the forward sweep, at each interior time, w_t is projected
 * first (w_t = min(D_t ./ P_{0,t} without w_t, 1) with the current u_t), then
 * u_t.  EINVAL for a solver without commodity capacities.  get: asynchronous
 * device output.  set (warm start / resume, same layout, values clamped at 0):
 * asynchronous; the next iteration recomputes the messages. */
mmot_status mmot_get_comm_duals(mmot_solver* s, double* log_w);
mmot_status mmot_set_comm_duals(mmot_solver* s, const double* log_w);

/* Release host-side resources (the workspace stays the caller's). */
void mmot_destroy(mmot_solver* s);

const char* mmot_status_str(mmot_status st);

/* Dense solvers created with MMOT_BF16: switch the K-products between BF16
 * MFMA (MMOT_BF16) and FP32 MFMA (MMOT_FP32, the polish precision) for the
 * following iterations.  Other solvers accept only their own precision.
 * EUNSUPPORTED otherwise. */
mmot_status mmot_set_precision(mmot_solver* s, int32_t precision);

/* Iterations completed so far. */
int64_t mmot_iterations(const mmot_solver* s);

/* Profiling helper: average device time (ms, HIP events on the solver's
 * stream) of `reps` back-to-back launches of one sweep step, cycling through
 * the interior times as a sweep does; forward != 0: the forward product with
 * its capacity-update epilogue (the u it computes goes to scratch), else the
 * backward product.  Message panels are left needing a fresh backward sweep
 * (done automatically by the next call that needs them).  Synchronous.
 * EUNSUPPORTED for a forward step of a CSR problem with T = 1 (its only
 * forward product is the sink update). */
mmot_status mmot_time_step(mmot_solver* s, int32_t forward, int32_t reps, double* avg_ms_host);

/* One whole solve that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): mmot_create, mmot_solve(max_iter), mmot_occupancy and
 * mmot_destroy in one call, with the solver workspace taken from a static
 * device array of MMOT_STATIC_WORKSPACE_BYTES that the library holds on each
 * GPU it runs on until the process ends, and the solver's host state on the
 * call's stack.  The caller passes the problem (device inputs, as for
 * mmot_create), occ ((T+1) * n doubles on the device, NULL for none), stats
 * (host, nullable) and the stream, which must belong to the current device.
 * Same results as that sequence of calls (same kernels; iterations are
 * launched directly, never through captured graphs).  ENOMEM when the problem's
 * workspace (mmot_query_workspace, with the options given: keep_forward = 0
 * needs T - 1 panels fewer) exceeds MMOT_STATIC_WORKSPACE_BYTES; the
 * other errors as mmot_create and mmot_solve.  The array is shared by every
 * call on a GPU and keeps the last call's contents (the set-up initialises
 * everything a solve reads): calls that overlap on one GPU -- from several host
 * threads or on streams that are not ordered -- race.  Returns after the solve
 * has finished on the stream; the occupancy is written asynchronously after it. */
#define MMOT_STATIC_WORKSPACE_BYTES ((size_t)256 << 20)
mmot_status mmot_solve_static(const mmot_problem* prob, const mmot_options* opt, int32_t max_iter, double* occ,
                              mmot_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * Serving pool: continuous batching of many solves on one GPU.
 *
 * Each admitted request is a solver (FP32, CSR) whose scalings and messages
 * stay resident in its own caller-provided workspace.  Requests run in one of
 * two kinds of lane, chosen at admission from the size of one sweep step:
 *  - batched lane (steps too small to fill the GPU): the request's schedule is
 *    recorded as a list of kernel work items and kept on the device; one
 *    launch ("tick", on the pool's stream) runs the next item of every batched
 *    request at once, so many small solves share the GPU;
 *  - dedicated lane (steps that fill the GPU alone): such requests run one at
 *    a time, in admission order, with their own captured iteration graphs on
 *    a pool-owned stream, next to the batched lane (two of them together would
 *    only stretch both);
 *  - express lanes (two): a small request admitted while fewer than two
 *    requests run in the batched lane replays its own graphs on a pool-owned
 *    stream instead (alone, that finishes sooner than one kernel per tick).
 * Either way a request's schedule is exactly the one mmot_solve would run
 * (check_every iterations, then a convergence check, until converged or
 * max_iter), so its result is bitwise the same alone, in any mix, and as a
 * plain solver.  Admission is by HBM footprint: the sum of admitted workspace
 * sizes never exceeds the budget.  Set-up work (validation, operators, the
 * domain probe) runs on a pool-owned stream and does not wait for queued
 * ticks.  The pool allocates no device memory: a request's workspace (sized by
 * mmot_pool_query_workspace) holds its solver and, after it, the program area
 * of its recorded work items (368 bytes per kernel of a check_every-iteration
 * chunk plus its check pass), so the budget counts every byte a request uses.
 * A tick runs at most 64 requests' items; the others wait for later ticks
 * (round-robin), each request's items always running in their recorded order.
 * ------------------------------------------------------------------------- */
typedef struct mmot_pool mmot_pool;

/* hbm_budget: bytes of workspace (mmot_pool_query_workspace sizes) the pool
 * may have admitted at once. */
mmot_status mmot_pool_create(size_t hbm_budget, void* stream, mmot_pool** out);

/* Workspace bytes of one pool request: the solver's (mmot_query_workspace),
 * 256 bytes of alignment, and its program area of (check_every + 1) * (2 T + 8)
 * + 8 work items of 368 bytes.  Same errors as mmot_query_workspace, and
 * EUNSUPPORTED for keep_forward = 1 (as mmot_pool_submit). */
mmot_status mmot_pool_query_workspace(const mmot_problem* prob, const mmot_options* opt, size_t* bytes);

/* Admit one request: validates and sets up a solver in ws (>= the size from
 * mmot_pool_query_workspace, ENOMEM otherwise; the caller keeps it alive until
 * mmot_pool_release) and schedules it.  EAGAIN when admitting it would exceed
 * the budget (nothing is done; retry after a release); EUNSUPPORTED unless CSR
 * and MMOT_FP32 with keep_forward = 0, or if a recorded chunk would not fit its
 * program area.
 * *ticket identifies the request.  Synchronous with respect to its own set-up
 * only. */
mmot_status mmot_pool_submit(mmot_pool* pool, const mmot_problem* prob, const mmot_options* opt, void* ws,
                             size_t ws_bytes, int32_t max_iter, uint64_t* ticket);

/* Collect finished chunks, schedule the next ones, and launch up to max_ticks
 * ticks of the batched lane (returns early when no batched request has work
 * ready; the dedicated lane runs on its own).  The host runs at most 16 ticks
 * ahead of the device.  *n_running (nullable) receives the number of
 * unfinished requests. */
mmot_status mmot_pool_run(mmot_pool* pool, int32_t max_ticks, int32_t* n_running);

/* State of a request: *state = 0 running, 1 converged or max_iter reached,
 * 2 failed (the call then returns the failure status).  *stats (nullable):
 * statistics of its latest check. */
mmot_status mmot_pool_poll(mmot_pool* pool, uint64_t ticket, int32_t* state, mmot_stats* stats);

/* The solver of a request (for mmot_occupancy / mmot_edge_flows /
 * mmot_get_log_duals on finished requests, which then run on the pool's
 * stream); NULL for an unknown ticket. */
mmot_solver* mmot_pool_solver(mmot_pool* pool, uint64_t ticket);

/* Free a finished request's slot and budget (EAGAIN while it is running). */
mmot_status mmot_pool_release(mmot_pool* pool, uint64_t ticket);

void mmot_pool_destroy(mmot_pool* pool);

#ifdef __cplusplus
}
#endif
#endif /* MMOT_H */
