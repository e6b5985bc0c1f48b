/* libl0l2 — MI355X (gfx950) library for the node relaxations of the l0-l2
 * branch-and-bound method of arXiv 2602.04551 ("A GPU-accelerated Nonlinear
 * Branch-and-Bound Framework for Sparse Linear Models").
 *
 * Problem (eq. original, Sec. 1):   min_beta 1/2 ||y - X beta||^2 + lambda0 ||beta||_0
 *                                              + lambda2 ||beta||_2^2
 * in its perspective big-M form (eq. perspective, Sec. 2.1) with box |beta_i| <= M.
 * A BnB node is a pair (F0, F1) of coordinates fixed to z = 0 / z = 1 (Sec. 2.2);
 * its interval relaxation (eq. relaxnode / relaxnode2, Sec. 3.1) is solved by
 * ADMM (eq. admm-update), bounded from below by the dual of Prop. 1 (Sec. 3.1.2),
 * and rounded into an incumbent refined by the fast proximal gradient method of
 * Sec. 3.3-3.4.
 *
 * Conventions for every entry point:
 *  - Return value: 0 (L0L2_OK) on success, a negative L0L2_E_* code on failure.
 *    No entry point throws, aborts or exits; l0l2_last_error() gives a message.
 *  - Matrices are dense.  X is column-major n x p (element (i, j) at X[i + j*n]).
 *    Per-node arrays are node-major: row k of a K x p array holds node k.
 *  - Fixing codes are one byte per coordinate: L0L2_FREE, L0L2_FIX0 (z = 0,
 *    coordinate in F0) or L0L2_FIX1 (z = 1, coordinate in F1).
 *  - "Device" buffers are caller-owned GPU memory on the context's device; the
 *    library reads and writes them on the context's stream and never frees them.
 *  - A context is used by one host thread at a time (l0l2_cancel excepted).
 *  - Synchronisation: work runs on the context's stream, ordered after what the
 *    caller's stream (given to l0l2_create) holds at the call and before what it
 *    receives afterwards.  l0l2_admm_sweeps, l0l2_dual_bound, l0l2_round_branch
 *    and the refinement entry points return without waiting for the device.
 *    l0l2_solve_node_batch waits at the end of every block of check_every sweeps
 *    (the host reads two counters there to switch precision and to stop) but not
 *    for its final copies; l0l2_set_data, l0l2_bnb_solve, l0l2_matching_pursuit,
 *    l0l2_exact_objective and the server calls return host results and wait.
 */
#ifndef L0L2_H
#define L0L2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    L0L2_OK = 0,
    L0L2_E_INVALID = -1,     /* bad argument (shape, NaN/Inf input, out-of-range option) */
    L0L2_E_NODATA = -2,      /* l0l2_set_data has not been called on this context */
    L0L2_E_OOM = -3,         /* device memory allocation failed */
    L0L2_E_DEVICE = -4,      /* a HIP runtime call failed */
    L0L2_E_NUMERIC = -5,     /* factorisation failed (matrix not positive definite) */
    L0L2_E_TIMEOUT = -6,     /* time limit reached before certification */
    L0L2_E_CANCELLED = -7,   /* stopped by l0l2_cancel / l0l2_server_cancel */
    L0L2_E_UNSUPPORTED = -8  /* option not available in this build */
};

/* Precision of the X products inside the ADMM sweep.  FP64: everything in FP64.
 * FP32 (mixed): sweeps in FP32 while a batch converges, then anchored sweeps
 * until each node meets its tolerance: the node state and update are FP64, an
 * FP64 product anchors every block and the FP32 products act on the movement
 * since that anchor only (FP32 sweeps alone stall near a relative gap of
 * 1e-6 .. 1e-5); node state returned in FP32.  BF16: the transformed design
 * matrix is stored as two BF16 terms (hi + lo), the node operand is split into
 * two BF16 halves, accumulation is FP32; the BF16 phase ends in anchored sweeps
 * as in FP32 mode.  FP8: the transformed design matrix is stored as
 * FP8 e4m3 codes with one FP32 scale per column (s_j = max_i |Xh_ij| / 448,
 * one byte per element), the codes are widened to BF16 in the products and
 * every sweep is anchored (an FP64 product every block, the reduced products
 * act on the movement since the anchor only), so the iterates converge to the
 * FP64 fixed point; node state returned in FP32.  In every mode the dual bound
 * and the incumbent objective are computed in FP64 with the original X. */
enum { L0L2_FP64 = 0, L0L2_FP32 = 1, L0L2_BF16 = 2, L0L2_FP8 = 3 };

enum { L0L2_FREE = 0, L0L2_FIX0 = 1, L0L2_FIX1 = 2 };

typedef struct l0l2_ctx l0l2_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t (NULL
 * = the device's null stream) on which all work of this context is issued. */
int l0l2_create(int device, void *hip_stream, l0l2_ctx **out);
void l0l2_destroy(l0l2_ctx *ctx);
/* Message of the last failed call on ctx (empty string if none); valid until the
 * next call on ctx.  ctx may be NULL (then: message of the last failed create). */
const char *l0l2_last_error(const l0l2_ctx *ctx);
/* Size of the state element for the current precision: 8 (FP64) or 4. */
int l0l2_state_bytes(const l0l2_ctx *ctx);

/* Load one instance and precompute what the whole tree shares (Sec. 3.1.1:
 * c = X^T y and the factor behind D = (X^T X + rho I)^{-1}, computed once for
 * the entire tree).  X (n x p column-major FP64) and y (n FP64) are host
 * pointers when ptrs_on_device == 0, device pointers otherwise; the library
 * copies them and the caller keeps ownership.  Requires n, p >= 1, finite
 * X and y, lambda0 >= 0, lambda2 > 0, M > 0 (INFINITY allowed), rho > 0.
 * x_precision is one of L0L2_FP64, L0L2_FP32, L0L2_BF16, L0L2_FP8.  Replaces
 * any previous instance on ctx. */
int l0l2_set_data(l0l2_ctx *ctx, const double *X, const double *y, int64_t n, int64_t p,
                  double lambda0, double lambda2, double M, double rho,
                  int x_precision, int ptrs_on_device);

typedef struct {
    double tol_node;   /* stop a node when (P(beta) - LB) / |P(beta)| <= tol_node */
    int max_iter;      /* ADMM sweeps per node (>= 1) */
    int check_every;   /* the gap is evaluated every check_every sweeps and at max_iter */
} l0l2_admm_opts;

/* Run exactly `sweeps` ADMM sweeps (eq. admm-update) on K nodes, without gap
 * checks.  codes: device, K x p uint8.  beta, v: device, K x p state elements
 * (double for FP64, float otherwise), read as the start and overwritten with
 * the result; b_out: device, K x p state elements, receives the last b.  The
 * F0 fixings are imposed on beta before the first sweep (Sec. 3.1.3).  FP8 mode
 * gives L0L2_E_UNSUPPORTED (its sweeps only run anchored inside a solve). */
int l0l2_admm_sweeps(l0l2_ctx *ctx, int K, const uint8_t *codes, void *beta, void *v,
                     void *b_out, int sweeps);

/* Rigorous dual lower bound (Prop. 1, eq. dual) of K nodes at r = y - X b:
 * evaluated in FP64 with the original X and lowered by an a-priori bound on
 * its rounding error, so that lb[k] <= the exact dual value at that r, which
 * is <= the node's relaxation value.  codes: device K x p; b: device K x p
 * state elements; lb: device K doubles. */
int l0l2_dual_bound(l0l2_ctx *ctx, int K, const uint8_t *codes, const void *b, double *lb);

/* Solve K node relaxations by ADMM from the warm starts (beta, v) (device, K x p
 * state elements, overwritten with the final iterates).  Outputs (device, K each):
 * lb = rigorous bound of the last gap check, primal = P(beta) of eq. relaxnode2
 * in FP64, iters = sweeps done, status = 0 converged / 1 reached max_iter. */
int l0l2_solve_node_batch(l0l2_ctx *ctx, int K, const uint8_t *codes, void *beta, void *v,
                          const l0l2_admm_opts *opts, double *lb, double *primal,
                          int32_t *iters, int32_t *status);

/* Continuous batching of node relaxations (the batching pattern's slot refill,
 * Sec. 3.2's batch of K nodes kept full): N queued nodes run through K slots;
 * at every block boundary (check_every sweeps) the slots whose nodes retired
 * (gap <= tol_node, or max_iter sweeps of their own done) hand over their
 * results and take the next queued nodes, in queue order, until the queue is
 * empty.  Each node counts its own sweeps.  FP64 mode runs the plain FP64
 * sweeps; FP32, BF16 and FP8 modes run anchored from the first sweep (FP64
 * state, an FP64 anchor product per block, the reduced products on the
 * movement since it), so a node joining a running batch needs no phase of its
 * own.  codes: device N x p uint8; beta, v: device N x p state elements (FP64,
 * or FP32 in the reduced modes), the warm starts, overwritten with each node's
 * final iterates; outputs (device, N each) as in l0l2_solve_node_batch.
 * Waits at every block boundary. */
int l0l2_solve_node_queue(l0l2_ctx *ctx, int N, const uint8_t *codes, void *beta, void *v, int K,
                          const l0l2_admm_opts *opts, double *lb, double *primal, int32_t *iters,
                          int32_t *status);

/* Block statistics of the last l0l2_solve_node_batch or l0l2_solve_node_queue
 * on ctx: *blocks = blocks of sweeps issued, *sparse_blocks = those with fewer
 * than 1/8 of the padded batch still live, *node_blocks = the live nodes summed
 * over the blocks (node_blocks / (blocks x padded K) is the batch's occupancy).
 * Any pointer may be NULL. */
int l0l2_batch_stats(l0l2_ctx *ctx, int64_t *blocks, int64_t *sparse_blocks, int64_t *node_blocks);

/* Rounding and branching for K nodes (Sec. 3.3; branching rule: most fractional
 * z_j, score floored to a 2^-20 grid, ties to the smallest index; when all free
 * scores are 0, the free index of largest |beta_j|).  z_j follows App. A.1.
 * Outputs (device): support (K x p uint8, S = F1 u {free j : z_j >= 1/2}),
 * support_size (K), branch_j (K, -1 when no coordinate is free), z_up (K,
 * 1 when z at branch_j >= 1/2). */
int l0l2_round_branch(l0l2_ctx *ctx, int K, const uint8_t *codes, const void *beta,
                      uint8_t *support, int32_t *support_size, int32_t *branch_j,
                      int32_t *z_up);

typedef struct {
    double tol;        /* stop when |U(beta+) - U(beta)| <= tol * max(1, U(beta+)) */
    int max_iter;      /* outer iterations */
} l0l2_fista_opts;

/* Incumbent refinement (eqs. fpg_extrapolate .. fpg_armijo, batched as in
 * Sec. 3.4) of K supports in FP64.  support: device K x p uint8 (0/1).
 * beta_start: device K x p state elements (the node iterates; only entries on
 * the support are read).  beta_out: device K x p doubles, receives the refined
 * coefficients, zero off the support (may alias beta_start in FP64 mode).
 * obj: device K doubles, F(S, beta) = 1/2||y - X_S beta_S||^2 + lambda2
 * ||beta_S||^2 + lambda0 |S|.  iters: device K int32 (may be NULL).
 * Supports of up to 1024 coordinates are refined with their per-coordinate
 * state in LDS; wider ones (p > 1024 only) by a second kernel whose state
 * lives in a workspace of at most 64 slots of 44 p bytes (at most 256 MiB),
 * the widest supports taking turns in the slots. */
int l0l2_refine_incumbent(l0l2_ctx *ctx, int K, const uint8_t *support, const void *beta_start,
                          double *beta_out, const l0l2_fista_opts *opts, double *obj, int32_t *iters);

/* Allocation-free form of l0l2_refine_incumbent, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts and results as
 * l0l2_refine_incumbent (the same kernels, bit-identical outputs), except:
 *  - the FP64 residual rows of supports wider than 64 coordinates live in a
 *    fixed device scratch of 32 MiB (each device the library runs on holds
 *    its own copy until the process ends); K x (n rounded up to a multiple of
 *    128) x 8 bytes must fit in it, else L0L2_E_INVALID (n = 1000: K <= 4096;
 *    n = 5000: K <= 819);
 *  - supports wider than 1024 coordinates are not refined: their obj is NaN
 *    and their iters -1 (their beta_out row keeps the converted start);
 *  - no device memory is allocated or freed and no library routine that
 *    allocates is called; the call is not timed by l0l2_profile_*;
 *  - it returns without waiting: the outputs are ready in stream order on the
 *    context's stream (and on the caller's stream given to l0l2_create).
 * Every call on one device shares that device's scratch: calls that overlap
 * on one device (contexts on different streams, or threads) race and must be
 * serialised by the caller.  Nothing in the scratch needs to start at zero
 * (each residual row is written before it is read). */
int l0l2_refine_incumbent_noalloc(l0l2_ctx *ctx, int K, const uint8_t *support, const void *beta_start,
                                  double *beta_out, const l0l2_fista_opts *opts, double *obj, int32_t *iters);

/* Objective of one support solved to full FP64 accuracy (box-constrained ridge
 * on S; used for the certified value of the final incumbent).  support and
 * beta_out (p doubles) are host pointers. */
int l0l2_exact_objective(l0l2_ctx *ctx, const uint8_t *support, double *beta_out, double *obj);

/* Matching-pursuit root heuristic (Sec. 3.5; forward and backward scores of
 * App. A.2), FP64 with the original X.  From the empty support, a forward
 * step adds the j outside S of smallest Delta_j = -b c_j + D_j b^2 / 2 + lambda0
 * (c_j = X_j^T r, D_j = ||X_j||^2 + 2 lambda2, b = clip(c_j / D_j, -M, M), r the
 * residual y - X beta; the other coefficients frozen), a backward step removes
 * the j in S of smallest Delta_j = beta_j c_j + (||X_j||^2 / 2 - lambda2) beta_j^2
 * - lambda0; a step is taken only when its Delta_j < 0, ties go to the smallest
 * index, steps alternate forward / backward, and the run ends when a forward
 * step and the backward step after it both take nothing, or after max_moves
 * moves (>= 1).  Host outputs: support (p bytes, 0/1), beta (p doubles, the
 * heuristic's coefficients, zero off S), *obj = F(S, beta) including
 * lambda0 |S|, moves (room for max_moves int32, may be NULL: j + 1 for an
 * addition of j, -(j + 1) for a removal, in order), *n_moves.  Waits for the
 * device. */
int l0l2_matching_pursuit(l0l2_ctx *ctx, int max_moves, uint8_t *support, double *beta, double *obj,
                          int32_t *moves, int32_t *n_moves);

enum { L0L2_BEST_FIRST = 0, L0L2_DFS = 1 };

typedef struct {
    int64_t id, parent;
    int32_t depth, branch_j, decision, iters;   /* decision: 0 branched, 1 pruned after its
                                                   solve, 2 leaf, 3 pruned at selection */
    int32_t support_size, admm_status;
    double lb, primal, ub_node, ub_global;
} l0l2_trace_rec;

typedef struct {
    int K;                 /* nodes per batch (Alg. 1); 0: chosen by l0l2_tune_batch_size
                              (k_max 1024, frac 0.9) once per instance */
    int policy;            /* L0L2_BEST_FIRST or L0L2_DFS */
    double eps_prune;      /* prune when LB >= UB (1 - eps_prune) */
    double gap_tol;        /* stop when (UB - LB) / UB <= gap_tol; 0 runs to exhaustion */
    double time_limit_s;   /* <= 0: none */
    int64_t max_nodes;     /* node solves budget */
    int max_iter_root;     /* ADMM sweeps at the root */
    l0l2_admm_opts admm;
    l0l2_fista_opts fista;
    l0l2_trace_rec *trace; /* optional host buffer of trace_cap records (NULL: none) */
    int64_t trace_cap;
    int root_heuristic;    /* 1: before the root, the support of l0l2_matching_pursuit
                              (max_moves 4 min(n, p)) solved exactly seeds the incumbent
                              (Sec. 3.5); 0: none */
    const uint8_t *init_support; /* optional host array of p bytes (0/1): a support whose
                              exact objective at the current penalties seeds the incumbent
                              (the better of it and the heuristic's); NULL: none */
    int warm_root;         /* 1: the root relaxation starts from the root iterates of the
                              previous l0l2_bnb_solve on this context (same instance and
                              precision, any penalties; Sec. 3.1.3's warm start across
                              solves), else from zero */
} l0l2_bnb_opts;

typedef struct {
    double ub;             /* incumbent objective from the node refinements */
    double certified;      /* F of the incumbent support solved exactly */
    double lb;             /* global lower bound at exit: the smallest bound over the closed
                              (pruned or leaf) and the open nodes, at most ub; when the tree
                              is exhausted it is at least ub (1 - eps_prune) */
    int64_t nodes_solved, nodes_pruned, trace_len, batches;
    double seconds;
    int status;            /* 0 exhausted (certified), 1 node budget, 2 gap_tol, 3 time limit */
    int64_t support_len;
    int32_t *support;      /* library-owned until l0l2_result_free */
    double *beta;          /* p entries, library-owned until l0l2_result_free */
} l0l2_bnb_result;

/* Branch and bound of Alg. 1 on the instance of ctx, to certification when
 * gap_tol = 0.  Node relaxations, rounding, branching and refinement run on the
 * GPU in batches of K; the host keeps the frontier (best-first by (LB, id), or
 * LIFO), the incumbent and the pruning decisions.  Fills *out. */
int l0l2_bnb_solve(l0l2_ctx *ctx, const l0l2_bnb_opts *opts, l0l2_bnb_result *out);
void l0l2_result_free(l0l2_bnb_result *res);

/* New penalties (lambda0 >= 0, lambda2 > 0, M > 0 or INFINITY) for the instance
 * of ctx, keeping everything l0l2_set_data precomputed (c, the factor, the
 * transformed operands and the Gram matrix depend on X, y and rho only), so a
 * sequence of solves over a lambda0 grid (Sec. 4.1, selection of lambda0)
 * pays the precompute once. */
int l0l2_set_penalties(l0l2_ctx *ctx, double lambda0, double lambda2, double M);

/* The smallest lambda0 at which the empty support is not improved by adding any
 * single coordinate (the forward scores of App. A.2 at S = {} with lambda0 = 0:
 * max_j (b_j c_j - D_j b_j^2 / 2), b_j = clip(c_j / D_j, -M, M),
 * D_j = ||X_j||^2 + 2 lambda2, c = X^T y): the top of a decreasing lambda0 grid. */
int l0l2_lambda0_max(l0l2_ctx *ctx, double *out);

/* Branch and bound along a decreasing lambda0 grid (Sec. 4.1's regularization
 * path): for i = 0 .. m-1, the penalties become (lambda0s[i], lambda2, M) of the
 * current instance and l0l2_bnb_solve(opts) runs with the previous grid point's
 * certified support as init_support and, for i > 0, warm_root = 1 (the previous
 * root iterates).  results[i] receives each solve's result (release each with
 * l0l2_result_free).  On return the instance keeps the last grid point's
 * penalties.  A failed solve stops the path with its error code; the results
 * filled before it are valid. */
int l0l2_bnb_path(l0l2_ctx *ctx, const l0l2_bnb_opts *opts, int m, const double *lambda0s,
                  l0l2_bnb_result *results);

/* Node-batch size by measurement (the batch axis of the autotuner; the batch
 * size K of Alg. 1 is the paper's parameter for how many nodes are solved at
 * once).  Each candidate K = 32, 64, ..., up to k_max (powers of two) solves a
 * batch of K nodes of the instance with every coordinate free from a cold start
 * for 20 sweeps (two gap checks, zero tolerance so that no node retires) in the
 * context's precision, once to settle tiles and graphs and once timed; the
 * chosen K is the smallest whose node-sweeps per second reach frac (0 < frac
 * <= 1) of the best candidate's.  *k_out receives it; rates (host, may be NULL,
 * room for 12 entries) receives each candidate's node-sweeps per second and
 * *n_rates (may be NULL) their count.  The choice is kept with the instance for
 * l0l2_bnb_solve with K = 0.  Requires 32 <= k_max <= 65536; uses the context's
 * batch workspace (grown to k_max nodes). */
int l0l2_tune_batch_size(l0l2_ctx *ctx, int k_max, double frac, int *k_out, double *rates, int *n_rates);

/* ---- Serving: branch and bound for many instances on one device ---------- */

/* Estimated device bytes one instance of n x p needs at batch size K in the
 * given precision (instance copies, precompute peak, batch workspace, a
 * warm-start reserve of 16 K slots, and where the default b-update form is the
 * Gram form, G's copies and the second W buffer), plus a tenth and 16 MiB for
 * the small buffers and captured graphs.  Used for admission; the pool of parent
 * states can outgrow its reserve on large trees. */
size_t l0l2_footprint_bytes(int64_t n, int64_t p, int precision, int K);

typedef struct l0l2_server l0l2_server;

typedef struct {
    double submit_s, admit_s, done_s;   /* seconds since the server was created */
    size_t footprint_bytes;             /* reserved from the HBM budget while running */
    size_t peak_bytes;                  /* device bytes its context held at most (l0l2_memory_stats) */
} l0l2_request_stats;

/* Create a server on `device`.  hbm_budget_bytes bounds the summed footprints
 * of the instances running at once (0 = 80% of the free device memory now);
 * at most max_concurrent instances run at once, each with its own context and
 * HIP stream for its branch and bound, their blocks of ADMM sweeps batched
 * into shared launches by the server's executor (l0l2_server_set_batching).
 * opts (copied; its trace buffer is ignored) applies to every request.
 * Requests are admitted in arrival order as workers and budget free up
 * (arrivals join while others are on the GPU). */
int l0l2_server_create(int device, size_t hbm_budget_bytes, int max_concurrent, const l0l2_bnb_opts *opts,
                       l0l2_server **out);
/* Queue one instance (host X column-major n x p, host y; copied before return).
 * Returns L0L2_E_OOM when its footprint alone exceeds the budget. */
int l0l2_server_submit(l0l2_server *srv, const double *X, const double *y, int64_t n, int64_t p,
                       double lambda0, double lambda2, double M, double rho, int precision,
                       int64_t *req_id);
/* Wait up to timeout_s seconds (< 0: no limit) for request req_id.  On success
 * *out holds its certified result (arrays owned by the caller from then on:
 * release with l0l2_result_free) and *stats (may be NULL) its timing.  A request
 * can be collected once.  L0L2_E_TIMEOUT if it is not finished in time; the
 * request's own error code if its solve failed. */
int l0l2_server_wait(l0l2_server *srv, int64_t req_id, double timeout_s, l0l2_bnb_result *out,
                     l0l2_request_stats *stats);
const char *l0l2_server_last_error(const l0l2_server *srv);
/* Cancel request req_id: a queued request ends at once with L0L2_E_CANCELLED
 * (its wait returns that code); a running one stops at its next batch and ends
 * the same way; a finished one is left as it is.  L0L2_E_INVALID for an unknown
 * or already collected id. */
int l0l2_server_cancel(l0l2_server *srv, int64_t req_id);
/* Stop admitting, end queued requests as cancelled, ask running ones to stop
 * (they end cancelled at their next batch), wait for the workers and for the
 * threads already inside l0l2_server_wait, free all.  No call on srv may start
 * once destroy has begun.  Server contexts choose tile shapes by a size rule
 * (no timing under contention), so an instance runs the same kernels alone and
 * beside others. */
int l0l2_server_destroy(l0l2_server *srv);

/* Batching across instances (the batched node solves of Sec. 3.2 pooled over
 * the admitted instances).  on = 1 (the default): instances admitted
 * after the call hand every block of ADMM sweeps to the server's executor,
 * which runs all blocks waiting when it becomes free together on one stream:
 * the sweep contractions of FP32-, FP64- and BF16-mode instances whose batches
 * use the 32 x 32 register tile (node batches below 128, or grids too small
 * for the 128 x 128 tile; BF16 then takes the split form) go out as one
 * grouped launch per contraction kind covering up to 8 instances, the other
 * sweeps launch by launch; FP8-mode instances keep their own streams.  on = 0: each instance replays
 * its own captured blocks on its own stream.  Results
 * are identical either way (a grouped tile computes what the instance's own
 * launch would).  Errors: L0L2_E_INVALID for a null server or on outside {0, 1}. */
int l0l2_server_set_batching(l0l2_server *srv, int on);

/* Executor counters since the server was created (any pointer may be NULL):
 * rounds run, blocks run in them, grouped contraction launches, and the
 * instance contractions those launches carried (members / launches = mean
 * instances per shared launch). */
int l0l2_server_batching_stats(l0l2_server *srv, int64_t *rounds, int64_t *blocks, int64_t *launches,
                               int64_t *members);

/* Tile shapes of the two sweep contractions (output rows x nodes / waves):
 * register tiles whose waves split the contraction range, 0 = 32x32/4,
 * 1 = 32x32/8, 2 = 32x32/16 (8 in FP64), 3 = 16x32/8, 4 = 32x16/8, 5 = 16x16/4,
 * 6 = 64x32/8, 7 = 32x64/8, 8 = 64x64/4; LDS-staged tiles (4 waves), 9 = 64x64,
 * 10 = 128x64, 11 = 128x128; for the contraction over p only (xw_shape), the
 * range cut into slices whose partial products are then added in slice order
 * (more workgroups when n x nodes is small and p long): 12, 13, 17 = 128x128
 * LDS-staged in 2 / 4 / 8 slices, 14, 15 = 16x16/4 in 4 / 8 slices, 16 = 32x32/4
 * in 4 slices.  By default (both -1) each live bucket (the live node count
 * rounded up to a power of two, at most the padded batch) is timed once with
 * every shape whose node tile divides it, on the live batch, and the fastest
 * kept per instance (in the reduced modes also for the anchor's FP64
 * product); fixed shapes serve tests and tuning studies (they cover the whole
 * padded batch, and one whose node tile does not divide it makes the solve
 * calls fail with L0L2_E_INVALID).  Results do not depend on the
 * shape beyond rounding of the summation order.  BF16 mode maps shapes 0-11 to
 * its own three (0 = 32x32 register tile, 1 = 64x64 and 2 = 128x128 LDS-staged,
 * larger values taken as 2) and the sliced shapes of the contraction over p
 * to its 32x32 register tile in 4 slices (14, 16) or 8 (15) and to its 128x128
 * LDS-staged tile in 4 slices (12, 13) or 8 (17); FP8 mode maps the contraction
 * over n the same way and its contraction over p to the 32x32 register tile,
 * unsliced for 0-11, in 4 slices for 14 and 16, 8 for 15, and to its 128x128
 * LDS-staged tile in 4 slices for 12 and 13, 8 for 17.  A sliced shape never
 * uses more slices than the range has 32-wide chunks. */
int l0l2_set_tiles(l0l2_ctx *ctx, int xw_shape, int xtu_shape);

/* Form of the b-update of the ADMM sweep (Sec. 3.1.1: b = D w with
 * D = (X^T X + rho I)^{-1}).  1: through the folded operand Xh = L^{-1} X
 * (S = X X^T + rho I = L L^T), b = (w - Xh^T (Xh w)) / rho, two contractions of
 * 2 n p flops per node per sweep.  2: through the p x p Gram matrix G = Xh^T Xh,
 * b = (w - G w) / rho, one contraction of 2 p^2 flops (the paper's p x p D,
 * here in the form I - rho D).  0 (default): the Gram form in FP32 and BF16
 * modes where it can win (p < 2 n, its 2 p^2 flops against the folded form's
 * 4 n p, and padded p at most 8192), chosen by measurement: on the instance's
 * first solve one sweep of each form is timed on the batch (every node masked,
 * best of three) and the faster is kept for the instance; elsewhere the folded
 * operand.  The Gram form exists in FP32 and BF16 modes only (FP64 and FP8
 * always use the folded operand; l0l2_admm_sweeps always does).  G is built in
 * FP64 (the anchors), then FP32 (FP32 mode) or a BF16 hi/lo pair of its FP32
 * value (BF16 mode), on the first solve that uses it (and freed if the folded
 * form wins the measurement). */
int l0l2_set_bupdate_form(l0l2_ctx *ctx, int form);
/* The b-update form in use: *form = 1 folded, 2 Gram; *ms_folded / *ms_gram
 * (may be NULL) the measured time of one sweep of each (0 when the choice was
 * not measured: forced, not a candidate, or before the first solve). */
int l0l2_bupdate_form(l0l2_ctx *ctx, int *form, double *ms_folded, double *ms_gram);

/* Device memory the library holds (device allocations of its calls; caller-owned
 * buffers are not counted): for ctx, the buffers that calls on ctx allocated
 * (instance copies, factors, workspace, and the transient buffers of each
 * call while they live); for ctx == NULL, the whole process.  *in_use: bytes
 * held now; *peak: the largest in_use since the counter was created or last
 * reset; reset_peak != 0 then sets peak to in_use.  Either pointer may be
 * NULL.  Safe to call from any thread. */
int l0l2_memory_stats(l0l2_ctx *ctx, size_t *in_use, size_t *peak, int reset_peak);

/* Ask the call running on ctx (or, if none is running, the next one) to stop:
 * l0l2_solve_node_batch, l0l2_bnb_solve and l0l2_matching_pursuit test the
 * request at each block of sweeps, batch or group of steps and then return
 * L0L2_E_CANCELLED (outputs unspecified, the context stays usable); the
 * request is consumed by that return.  The one entry point that may be called
 * from another thread than the one using ctx. */
int l0l2_cancel(l0l2_ctx *ctx);

/* Products of the BF16 Gram-form sweeps.  3: every sweep multiplies with the
 * split form (G as a BF16 hi/lo pair times the node operand split into two
 * BF16 halves: three MFMA products, FP32 accumulation).  1 (default): blocks
 * of single-term sweeps wherever the LDS-staged tiles are chosen: each block is
 * anchored (FP32 phase: its first sweep is a split-form sweep whose product
 * z = G w_a and operand w_a become the anchor; FP64 phase: the FP64 anchor
 * product), and its other sweeps multiply only d = W - w_a, rounded to one BF16
 * term, by G rounded to one BF16 term (one MFMA product), taking
 * G W = z + G d; the product's error then scales with the movement since the
 * anchor.  FP32, FP64 and FP8 modes ignore the setting.  Returns
 * L0L2_E_INVALID for other values. */
int l0l2_set_bf16_terms(l0l2_ctx *ctx, int terms);

/* Rows of the single-term sweep's largest LDS-staged tile (the Gram form's
 * 128-node tile): 128 (default) keeps the 128 x 128 tile; 256, where the padded
 * p is a multiple of 256, takes a 256 x 128 tile (one workgroup per compute
 * unit, each wave a 128 x 64 block: fewer operand bytes staged per MFMA, but
 * one wave per SIMD; slower at n = p = 5000).  The results are
 * those of the same contraction in another tile order: bounds agree to the
 * node tolerance, not bit for bit.  Returns L0L2_E_INVALID for other values. */
int l0l2_set_bf16_tile_rows(l0l2_ctx *ctx, int rows);

/* Opt-in timing of the library's kernels with HIP events recorded on the
 * context stream around each launch (adds one event pair per launch).
 * l0l2_profile_enable clears the counters and switches timing on (1) or off (0).
 * l0l2_profile_query returns the number of timed launches and their summed
 * duration in milliseconds for one kernel family: "gemm_xw.f32" / "gemm_xw.f64"
 * (contraction over p of a sweep in FP32 / FP64), "admm_xtu.f32" /
 * "admm_xtu.f64" (contraction over n with the prox/V epilogue), "gap_check"
 * (the FP64 gap evaluation, all of its kernels), "round_branch", "fista",
 * "anchor.f64" (the two FP64 products that start each block of anchored
 * sweeps; in FP32 mode those sweeps count as the FP32 families, in BF16 mode as
 * the BF16 ones), "gemm_xw.fp8" / "admm_xtu.fp8" (the two products of an
 * anchored sweep in FP8 mode).
 * units (may be NULL) receives the work the timed launches did: for the sweep
 * families the number of node-iterations of nodes that were still active
 * (columns of converged nodes are not counted).  Unknown names give
 * L0L2_E_INVALID. */
int l0l2_profile_enable(l0l2_ctx *ctx, int enable);
int l0l2_profile_query(l0l2_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms,
                       int64_t *units);

#ifdef __cplusplus
}
#endif
#endif
