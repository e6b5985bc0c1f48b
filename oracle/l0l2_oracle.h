/* Plain FP64 single-threaded CPU oracle for the l0-l2 branch-and-bound method of
 * "A GPU-accelerated Nonlinear Branch-and-Bound Framework for Sparse Linear
 * Models" (arXiv 2602.04551).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP library: every formula below is written out again from the paper.
 *
 * Parity status of each function (what pins it; the pins live in tests/):
 *   orc_T, orc_psi, orc_prox   pinned: brute-force 1-D minimisation
 *   orc_h, orc_nu              pinned: brute-force convex conjugate
 *   orc_b_update               pinned: (X^T X + rho I) b = w to 1e-12
 *   orc_create_factored        pinned: same b-update and node solves as orc_create
 *   orc_dual_value/bound       pinned: weak duality for random r, strong duality
 *   orc_node_admm              pinned: gap -> 0, fully-fixed special cases
 *   orc_fista / exact          pinned: Cholesky ridge and scipy bounded LSQ
 *   orc_bnb                    pinned: enumeration of all supports, p <= 14
 *   orc_mp_deltas              pinned: brute-force 1-D minimisation / direct
 *                              objective differences
 *   orc_matching_pursuit       pinned: each move lowers F by its Delta; no
 *                              improving single move at exit; global optimum
 *                              on orthonormal designs (enumeration)
 *   trajectory details (iteration counts, node counts) are parity unpinned
 *   beyond this oracle: the paper prints no worked example.
 *
 * Conventions: X is column-major n x p (column i is X + i*n); codes are one
 * byte per coordinate: 0 free, 1 fixed to zero (F0), 2 fixed to one (F1).
 */
#ifndef L0L2_ORACLE_H
#define L0L2_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FREE = 0, ORC_FIX0 = 1, ORC_FIX1 = 2 };

/* --- scalar pieces --------------------------------------------------------- */
double orc_T(double t, double a, double m);                                   /* eq. Tdef */
double orc_psi(double beta, int code, double l0, double l2, double M);       /* eq. psi */
double orc_prox(double bt, int code, double l0, double l2, double M, double rho); /* eq. minbetalower */
double orc_h(double x, double l0, double l2, double M);                      /* eq. hdef */
double orc_nu(double x, int code, double l0, double l2, double M);           /* eq. nudef */
double orc_z(double beta, int code, double l0, double l2, double M);         /* App. A.1 z* */

/* --- instance -------------------------------------------------------------- */
typedef struct orc_inst orc_inst;
orc_inst *orc_create(const double *X, const double *y, int64_t n, int64_t p,
                     double lambda0, double lambda2, double M, double rho);
/* The same with the once-per-tree factor supplied: D = (X^T X + rho I)^{-1}
   (p x p) when n >= p, else the lower Cholesky factor of X X^T + rho I (n x n),
   column-major; copied. */
orc_inst *orc_create_factored(const double *X, const double *y, int64_t n, int64_t p,
                              double lambda0, double lambda2, double M, double rho,
                              const double *factor);
void orc_free(orc_inst *);
const double *orc_c(const orc_inst *);                /* X^T y */

/* b = (X^T X + rho I)^{-1} w (eq. b_update; Woodbury form when p > n) */
void orc_b_update(const orc_inst *, const double *w, double *b);
/* one ADMM sweep in place: w = c + rho beta - v; b = D w; beta = prox(b + v/rho);
   v += rho (b - beta)  (eq. admm-update); b receives the new b. */
void orc_admm_sweep(const orc_inst *, const uint8_t *codes, double *beta, double *v, double *b);

double orc_primal(const orc_inst *, const uint8_t *codes, const double *beta);   /* eq. relaxnode2 */
double orc_dual_value(const orc_inst *, const uint8_t *codes, const double *r);  /* eq. dual, plain */
double orc_dual_bound(const orc_inst *, const uint8_t *codes, const double *r);  /* with rounding margin */

/* Node relaxation by ADMM from the warm start (beta, v).  Stops when the
   relative primal-dual gap (P(beta) - LB)/|P(beta)| <= tol at a check iteration
   (every check_every sweeps, and at max_iter).  Returns 0 converged, 1 hit
   max_iter.  lb is the rigorous bound at r = y - X b of the last check. */
int orc_node_admm(const orc_inst *, const uint8_t *codes, double *beta, double *v, double *b,
                  double tol, int max_iter, int check_every,
                  double *lb, double *primal, int *iters);

/* rounding and branching (Sec. 3.3 and the branching rule) */
int orc_support(const orc_inst *, const uint8_t *codes, const double *beta, uint8_t *mask);
int orc_branch(const orc_inst *, const uint8_t *codes, const double *beta);

/* fast proximal gradient on the support (eq. fpg_extrapolate..fpg_armijo).
   beta: p entries, in = start (only the support is read), out = refined
   (zero off the support).  Returns F(S, beta) = U_S(beta) + lambda0 |S|. */
double orc_fista(const orc_inst *, const uint8_t *mask, double *beta,
                 double tol, int max_iter, int *iters);
/* F(S) solved to full FP64 accuracy (Cholesky ridge; coordinate descent on the
   box-constrained QP when the box binds).  beta (p) receives the minimiser. */
double orc_exact_objective(const orc_inst *, const uint8_t *mask, double *beta);
/* F(S, beta) evaluated as written (eq. upperboundbeta plus lambda0 |S|) */
double orc_objective(const orc_inst *, const uint8_t *mask, const double *beta);

/* --- matching-pursuit root heuristic (Sec. 3.5, App. A.2) ----------------- */
/* Objective change of each single-coordinate move at (mask, beta), residual r =
   y - X beta given, other coordinates frozen: an addition for j outside the
   support (bnew[j] = its coefficient), a removal for j in it (bnew[j] = 0). */
void orc_mp_deltas(const orc_inst *, const uint8_t *mask, const double *beta, const double *r,
                   double *delta, double *bnew);
/* Alternating forward / backward steps from the empty support until neither
   moves or max_moves moves; moves[t] = j + 1 (addition) or -(j + 1) (removal).
   Returns the number of moves; mask and beta (p) receive the result. */
int orc_matching_pursuit(const orc_inst *, int max_moves, uint8_t *mask, double *beta, int32_t *moves);

/* --- depth-first branch and bound (Alg. 1 with K = 1 and a LIFO frontier) --- */
typedef struct {
    double tol_node;      /* node gap tolerance */
    int max_iter;         /* ADMM sweeps per non-root node */
    int max_iter_root;    /* ADMM sweeps at the root */
    int check_every;      /* gap checked every this many sweeps */
    double eps_prune;     /* prune when LB >= UB (1 - eps_prune) */
    double gap_tol;       /* stop when (UB - LB_global)/UB <= gap_tol; 0 = run to exhaustion */
    int64_t max_nodes;    /* node solves budget */
    double fista_tol;
    int fista_max_iter;
} orc_bnb_opts;

typedef struct {
    int64_t id, parent;
    int32_t depth, branch_j, decision, iters;   /* decision: 0 branched, 1 pruned after solve,
                                                   2 leaf, 3 pruned at selection */
    int32_t support_size, admm_status;
    double lb, primal, ub_node, ub_global;
} orc_trace_rec;

typedef struct {
    double ub;            /* incumbent F from the node refinements */
    double certified;     /* exact F of the incumbent support */
    double lb_global;     /* min LB over open nodes at exit (= ub when exhausted) */
    int64_t nodes_solved, nodes_pruned, trace_len;
    int status;           /* 0 exhausted (certified), 1 node budget, 2 gap_tol reached */
} orc_bnb_result;

/* mask_out, beta_out: p entries.  trace: capacity trace_cap records (may be NULL). */
int orc_bnb(const orc_inst *, const orc_bnb_opts *, orc_bnb_result *,
            uint8_t *mask_out, double *beta_out, orc_trace_rec *trace, int64_t trace_cap);

#ifdef __cplusplus
}
#endif
#endif
