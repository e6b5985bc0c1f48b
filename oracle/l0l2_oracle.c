/* Plain FP64 CPU oracle: see l0l2_oracle.h.  TEST INFRASTRUCTURE ONLY.
 *
 * Every routine is a direct transcription of a definition in the paper
 * (arXiv 2602.04551), written for a reader to check by eye: no blocking, no
 * fusion, no reordering beyond what the definitions state.  Readings taken
 * where the paper is silent or inconsistent are marked "Reading:".
 */
#include "l0l2_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Scalar pieces                                                              */
/* ------------------------------------------------------------------------- */

/* Box-constrained soft threshold T(t; a, m), eq. (Tdef). */
double orc_T(double t, double a, double m) {
    double at = fabs(t);
    double s = (t > 0) - (t < 0);
    if (at <= a) return 0.0;
    if (at <= a + m) return (at - a) * s;
    return m * s;
}

static double clip(double x, double m) { return x > m ? m : (x < -m ? -m : x); }

/* psi_i(beta; lambda0, lambda2, M), eq. (psi), for |beta| <= M (infinite outside
 * the box and, on F0, off zero). */
double orc_psi(double beta, int code, double l0, double l2, double M) {
    double ab = fabs(beta);
    if (ab > M) return INFINITY;
    if (code == ORC_FIX0) return beta == 0.0 ? 0.0 : INFINITY;
    if (code == ORC_FIX1) return l0 + l2 * beta * beta;
    double s = sqrt(l0 / l2);
    if (s <= M) {
        if (ab >= s) return l0 + l2 * beta * beta;
        return 2.0 * sqrt(l0 * l2) * ab;
    }
    return (l0 / M + l2 * M) * ab;
}

/* argmin_b rho/2 (b - bt)^2 + psi(b) over |b| <= M, eq. (minbetalower).
 * Reading: the free case with sqrt(l0/l2) > M uses the single soft threshold for
 * every bt (App. A.1, case 4 of the beta-update derivation); the ridge branch
 * |bt| >= a + s applies only when sqrt(l0/l2) <= M (case 3(b)). */
double orc_prox(double bt, int code, double l0, double l2, double M, double rho) {
    if (code == ORC_FIX0) return 0.0;
    if (code == ORC_FIX1) return clip(rho / (rho + 2.0 * l2) * bt, M);
    double s = sqrt(l0 / l2);
    if (s <= M) {
        double a = 2.0 * sqrt(l0 * l2) / rho;
        if (fabs(bt) >= a + s) return clip(rho / (rho + 2.0 * l2) * bt, M);
        return orc_T(bt, a, M);
    }
    return orc_T(bt, l0 / (M * rho) + l2 * M / rho, M);
}

/* h(x), eq. (hdef), x >= 0. */
double orc_h(double x, double l0, double l2, double M) {
    if (x <= 2.0 * M * l2) return x * x / (4.0 * l2) - l0;
    return M * x - l0 - l2 * M * M;
}

/* nu_i(x), eq. (nudef), x >= 0. */
double orc_nu(double x, int code, double l0, double l2, double M) {
    if (code == ORC_FIX0) return 0.0;
    if (code == ORC_FIX1) return orc_h(x, l0, l2, M);
    if (sqrt(l0 / l2) <= M) {
        double h = orc_h(x, l0, l2, M);
        return h > 0.0 ? h : 0.0;
    }
    double t = M * x - l0 - l2 * M * M;
    return t > 0.0 ? t : 0.0;
}

/* z_i at the relaxation optimum for a given beta_i (App. A.1, derivation of
 * eq. relaxnode2, cases 1-3). */
double orc_z(double beta, int code, double l0, double l2, double M) {
    if (code == ORC_FIX0) return 0.0;
    if (code == ORC_FIX1) return 1.0;
    double s = sqrt(l0 / l2);
    double ab = fabs(beta);
    if (s <= M) return ab >= s ? 1.0 : ab / s;
    return ab / M;
}

/* ------------------------------------------------------------------------- */
/* Instance and the b-update                                                  */
/* ------------------------------------------------------------------------- */

struct orc_inst {
    int64_t n, p;
    double *X, *y;
    double l0, l2, M, rho;
    double *c;      /* X^T y */
    double *colnrm; /* ||X_i||_2 */
    int dform;      /* 1: D = (X^T X + rho I)^{-1} stored (n >= p); 0: Woodbury */
    double *D;      /* p x p, column-major */
    double *L;      /* n x n lower Cholesky factor of X X^T + rho I (column-major) */
};

#define XC(in, i, j) ((in)->X[(size_t)(j) * (size_t)(in)->n + (size_t)(i)])

/* In-place lower Cholesky of the m x m column-major SPD matrix A. */
static int cholesky(double *A, int64_t m) {
    for (int64_t j = 0; j < m; ++j) {
        double d = A[j * m + j];
        for (int64_t k = 0; k < j; ++k) d -= A[k * m + j] * A[k * m + j];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        A[j * m + j] = d;
        for (int64_t i = j + 1; i < m; ++i) {
            double s = A[j * m + i];
            for (int64_t k = 0; k < j; ++k) s -= A[k * m + i] * A[k * m + j];
            A[j * m + i] = s / d;
        }
        for (int64_t i = 0; i < j; ++i) A[j * m + i] = 0.0;
    }
    return 0;
}

/* Solve L L^T x = rhs in place (L lower, column-major m x m). */
static void chol_solve(const double *L, int64_t m, double *x) {
    for (int64_t i = 0; i < m; ++i) {
        double s = x[i];
        for (int64_t k = 0; k < i; ++k) s -= L[k * m + i] * x[k];
        x[i] = s / L[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double s = x[i];
        for (int64_t k = i + 1; k < m; ++k) s -= L[i * m + k] * x[k];
        x[i] = s / L[i * m + i];
    }
}

/* Instance data every constructor fills: copies of X and y, c = X^T y, ||X_j||. */
static orc_inst *inst_common(const double *X, const double *y, int64_t n, int64_t p,
                             double lambda0, double lambda2, double M, double rho) {
    if (n < 1 || p < 1 || !(lambda0 >= 0) || !(lambda2 > 0) || !(M > 0) || !(rho > 0)) return NULL;
    orc_inst *in = (orc_inst *)calloc(1, sizeof(orc_inst));
    in->n = n; in->p = p; in->l0 = lambda0; in->l2 = lambda2; in->M = M; in->rho = rho;
    in->X = (double *)malloc(sizeof(double) * (size_t)n * (size_t)p);
    in->y = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(in->X, X, sizeof(double) * (size_t)n * (size_t)p);
    memcpy(in->y, y, sizeof(double) * (size_t)n);
    in->c = (double *)malloc(sizeof(double) * (size_t)p);
    in->colnrm = (double *)malloc(sizeof(double) * (size_t)p);
    for (int64_t j = 0; j < p; ++j) {
        double s = 0.0, q = 0.0;
        for (int64_t i = 0; i < n; ++i) { s += XC(in, i, j) * in->y[i]; q += XC(in, i, j) * XC(in, i, j); }
        in->c[j] = s;
        in->colnrm[j] = sqrt(q);
    }
    in->dform = (n >= p);
    return in;
}

orc_inst *orc_create(const double *X, const double *y, int64_t n, int64_t p,
                     double lambda0, double lambda2, double M, double rho) {
    orc_inst *in = inst_common(X, y, n, p, lambda0, lambda2, M, rho);
    if (!in) return NULL;
    /* Precompute D once for the whole tree (Sec. 3.1.1, update for b).  Reading:
     * the printed Woodbury form carries 1/rho^2 where (1/rho)(I - X^T (X X^T +
     * rho I)^{-1} X) is the identity; the latter is used. */
    if (in->dform) {
        double *A = (double *)malloc(sizeof(double) * (size_t)p * (size_t)p);
        for (int64_t j = 0; j < p; ++j)
            for (int64_t i = 0; i < p; ++i) {
                double s = 0.0;
                for (int64_t k = 0; k < n; ++k) s += XC(in, k, i) * XC(in, k, j);
                A[j * p + i] = s + (i == j ? rho : 0.0);
            }
        if (cholesky(A, p) != 0) { free(A); orc_free(in); return NULL; }
        in->D = (double *)malloc(sizeof(double) * (size_t)p * (size_t)p);
        double *e = (double *)malloc(sizeof(double) * (size_t)p);
        for (int64_t j = 0; j < p; ++j) {
            for (int64_t i = 0; i < p; ++i) e[i] = (i == j);
            chol_solve(A, p, e);
            memcpy(in->D + j * p, e, sizeof(double) * (size_t)p);
        }
        free(e);
        free(A);
    } else {
        in->L = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int64_t k = 0; k < p; ++k) s += XC(in, i, k) * XC(in, j, k);
                in->L[j * n + i] = s + (i == j ? rho : 0.0);
            }
        if (cholesky(in->L, n) != 0) { orc_free(in); return NULL; }
    }
    return in;
}

/* The same instance with the once-per-tree factor supplied by the caller (for
 * large instances, where it comes from a library factorisation): D =
 * (X^T X + rho I)^{-1} (p x p) when n >= p, else the lower Cholesky factor L of
 * X X^T + rho I (n x n), column-major either way.  Everything else is computed
 * here exactly as in orc_create. */
orc_inst *orc_create_factored(const double *X, const double *y, int64_t n, int64_t p,
                              double lambda0, double lambda2, double M, double rho, const double *factor) {
    if (!factor) return NULL;
    orc_inst *in = inst_common(X, y, n, p, lambda0, lambda2, M, rho);
    if (!in) return NULL;
    int64_t m = in->dform ? p : n;
    double *F = (double *)malloc(sizeof(double) * (size_t)m * (size_t)m);
    memcpy(F, factor, sizeof(double) * (size_t)m * (size_t)m);
    if (in->dform) in->D = F;
    else in->L = F;
    return in;
}

void orc_free(orc_inst *in) {
    if (!in) return;
    free(in->X); free(in->y); free(in->c); free(in->colnrm); free(in->D); free(in->L);
    free(in);
}

const double *orc_c(const orc_inst *in) { return in->c; }

/* b = D w with D = (X^T X + rho I)^{-1}, eq. (b_update). */
void orc_b_update(const orc_inst *in, const double *w, double *b) {
    int64_t n = in->n, p = in->p;
    if (in->dform) {
        for (int64_t i = 0; i < p; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < p; ++j) s += in->D[j * p + i] * w[j];
            b[i] = s;
        }
        return;
    }
    /* Woodbury: b = (1/rho) (w - X^T (X X^T + rho I)^{-1} X w) */
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < p; ++j) s += XC(in, i, j) * w[j];
        u[i] = s;
    }
    chol_solve(in->L, n, u);
    for (int64_t j = 0; j < p; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += XC(in, i, j) * u[i];
        b[j] = (w[j] - s) / in->rho;
    }
    free(u);
}

/* One ADMM sweep, eq. (admm-update) with the closed forms of Sec. 3.1.1. */
void orc_admm_sweep(const orc_inst *in, const uint8_t *codes, double *beta, double *v, double *b) {
    int64_t p = in->p;
    double rho = in->rho;
    double *w = (double *)malloc(sizeof(double) * (size_t)p);
    for (int64_t i = 0; i < p; ++i) w[i] = in->c[i] + rho * beta[i] - v[i];
    orc_b_update(in, w, b);
    for (int64_t i = 0; i < p; ++i) {
        double bt = b[i] + v[i] / rho;
        beta[i] = orc_prox(bt, codes[i], in->l0, in->l2, in->M, rho);
        v[i] = v[i] + rho * (b[i] - beta[i]);
    }
    free(w);
}

/* ------------------------------------------------------------------------- */
/* Primal value and dual bound                                                */
/* ------------------------------------------------------------------------- */

/* Objective of eq. (relaxnode2) at beta. */
double orc_primal(const orc_inst *in, const uint8_t *codes, const double *beta) {
    int64_t n = in->n, p = in->p;
    double rr = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < p; ++j) s += XC(in, i, j) * beta[j];
        double r = in->y[i] - s;
        rr += r * r;
    }
    double ps = 0.0;
    for (int64_t j = 0; j < p; ++j) ps += orc_psi(beta[j], codes[j], in->l0, in->l2, in->M);
    return 0.5 * rr + ps;
}

/* Dual objective of eq. (dual) at r, evaluated as written. */
double orc_dual_value(const orc_inst *in, const uint8_t *codes, const double *r) {
    int64_t n = in->n, p = in->p;
    double rr = 0.0, yr = 0.0;
    for (int64_t i = 0; i < n; ++i) { rr += r[i] * r[i]; yr += in->y[i] * r[i]; }
    double sn = 0.0;
    for (int64_t j = 0; j < p; ++j) {
        double g = 0.0;
        for (int64_t i = 0; i < n; ++i) g += XC(in, i, j) * r[i];
        sn += orc_nu(fabs(g), codes[j], in->l0, in->l2, in->M);
    }
    return -0.5 * rr + yr - sn;
}

static double gamma_k(double k) {
    const double u = DBL_EPSILON / 2.0;
    return k * u / (1.0 - k * u);
}

/* Rigorous lower bound: Prop. 1(1) says D(r) <= p* for every r; this returns a
 * floating-point number that is <= the exact D(r) of the stored vector r.
 * Reading (the paper evaluates D(r) without rounding analysis): with u = 2^-53
 * and gamma_k = k u / (1 - k u), every dot product of length k carries an
 * error <= gamma_k |a|^T |b| in any summation order; nu_i is nondecreasing on
 * [0, inf) so it is evaluated at an upper bound x+ of |X_i^T r|; each nu value
 * is raised by its own evaluation error; the sums are bounded the same way. */
double orc_dual_bound(const orc_inst *in, const uint8_t *codes, const double *r) {
    const double u = DBL_EPSILON / 2.0;
    int64_t n = in->n, p = in->p;
    double l0 = in->l0, l2 = in->l2, M = in->M;
    double rr = 0.0, yr = 0.0, ayr = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        rr += r[i] * r[i];
        yr += in->y[i] * r[i];
        ayr += fabs(in->y[i]) * fabs(r[i]);
    }
    double q = -0.5 * rr + yr;
    double nr = sqrt(rr);
    double gn = gamma_k((double)n);
    double sum_nu = 0.0, sum_anu = 0.0;
    int free_quad = sqrt(l0 / l2) <= M;
    for (int64_t j = 0; j < p; ++j) {
        if (codes[j] == ORC_FIX0) continue;
        double g = 0.0;
        for (int64_t i = 0; i < n; ++i) g += XC(in, i, j) * r[i];
        double e = 2.0 * gn * in->colnrm[j] * nr;
        double x = (fabs(g) + e) * (1.0 + 4.0 * u);
        double val, mag;
        if (codes[j] == ORC_FIX1 || free_quad) {
            if (x <= 2.0 * M * l2) { val = x * x / (4.0 * l2) - l0; mag = x * x / (4.0 * l2) + l0; }
            else { val = M * x - l0 - l2 * M * M; mag = M * x + l0 + l2 * M * M; }
        } else {
            val = M * x - l0 - l2 * M * M; mag = M * x + l0 + l2 * M * M;
        }
        val += gamma_k(4.0) * mag;             /* upper bound of the exact value */
        if (codes[j] == ORC_FREE && val < 0.0) val = 0.0;   /* [.]_+ */
        sum_nu += val;
        sum_anu += fabs(val);
    }
    double margin = 2.0 * gamma_k((double)n + 2.0) * (0.5 * rr + ayr)
                  + 2.0 * gamma_k((double)p) * sum_anu
                  + 4.0 * u * (fabs(q) + fabs(sum_nu));
    return (q - sum_nu) - margin;
}

/* ------------------------------------------------------------------------- */
/* Node relaxation by ADMM                                                    */
/* ------------------------------------------------------------------------- */

int orc_node_admm(const orc_inst *in, const uint8_t *codes, double *beta, double *v, double *b,
                  double tol, int max_iter, int check_every,
                  double *lb, double *primal, int *iters) {
    int64_t n = in->n, p = in->p;
    if (max_iter < 1) max_iter = 1;
    if (check_every < 1) check_every = 1;
    /* Warm start: the fixings of the node are imposed on beta (Sec. 3.1.3). */
    for (int64_t j = 0; j < p; ++j)
        if (codes[j] == ORC_FIX0) beta[j] = 0.0;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    int status = 1, t = 0;
    double LB = -INFINITY, P = INFINITY;
    while (t < max_iter) {
        orc_admm_sweep(in, codes, beta, v, b);
        ++t;
        if (t % check_every == 0 || t == max_iter) {
            /* r_hat = y - X b_hat (Sec. 3.1.2) */
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int64_t j = 0; j < p; ++j) s += XC(in, i, j) * b[j];
                r[i] = in->y[i] - s;
            }
            LB = orc_dual_bound(in, codes, r);
            P = orc_primal(in, codes, beta);
            double den = fabs(P) > 1e-300 ? fabs(P) : 1e-300;
            if ((P - LB) / den <= tol) { status = 0; break; }
        }
    }
    free(r);
    *lb = LB;
    *primal = P;
    *iters = t;
    return status;
}

/* ------------------------------------------------------------------------- */
/* Rounding, branching, incumbent                                             */
/* ------------------------------------------------------------------------- */

/* S = F1 u {free i : z_i >= 1/2} (Sec. 3.3, rounding of z). */
int orc_support(const orc_inst *in, const uint8_t *codes, const double *beta, uint8_t *mask) {
    int cnt = 0;
    for (int64_t j = 0; j < in->p; ++j) {
        double z = orc_z(beta[j], codes[j], in->l0, in->l2, in->M);
        mask[j] = (codes[j] == ORC_FIX1) || (codes[j] == ORC_FREE && z >= 0.5);
        cnt += mask[j];
    }
    return cnt;
}

/* Reading (the paper says only "select j"): most fractional free z, score
 * min(z, 1-z) floored to a 2^-20 grid, ties to the smallest index; when every
 * free score is 0, the free index of largest |beta| (ties smallest index).
 * Returns -1 when no coordinate is free. */
int orc_branch(const orc_inst *in, const uint8_t *codes, const double *beta) {
    int64_t best = -1, bestabs = -1;
    double bscore = -1.0, babs = -1.0;
    for (int64_t j = 0; j < in->p; ++j) {
        if (codes[j] != ORC_FREE) continue;
        double z = orc_z(beta[j], codes[j], in->l0, in->l2, in->M);
        double f = z < 1.0 - z ? z : 1.0 - z;
        double sc = floor(f * 1048576.0);
        if (sc > bscore) { bscore = sc; best = j; }
        if (fabs(beta[j]) > babs) { babs = fabs(beta[j]); bestabs = j; }
    }
    if (best < 0) return -1;
    if (bscore <= 0.0) return (int)bestabs;
    return (int)best;
}

/* U_S(beta) of eq. (upperboundbeta), beta indexed by the compact support list. */
static double U_S(const orc_inst *in, const int64_t *S, int64_t k, const double *bs, double *res) {
    int64_t n = in->n;
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t a = 0; a < k; ++a) s += XC(in, i, S[a]) * bs[a];
        double r = s - in->y[i];
        if (res) res[i] = r;
        rr += r * r;
    }
    for (int64_t a = 0; a < k; ++a) bb += bs[a] * bs[a];
    return 0.5 * rr + in->l2 * bb;
}

static int64_t support_list(const orc_inst *in, const uint8_t *mask, int64_t *S) {
    int64_t k = 0;
    for (int64_t j = 0; j < in->p; ++j)
        if (mask[j]) S[k++] = j;
    return k;
}

double orc_objective(const orc_inst *in, const uint8_t *mask, const double *beta) {
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)in->p);
    int64_t k = support_list(in, mask, S);
    double *bs = (double *)malloc(sizeof(double) * (size_t)(k ? k : 1));
    for (int64_t a = 0; a < k; ++a) bs[a] = beta[S[a]];
    double f = U_S(in, S, k, bs, NULL) + in->l0 * (double)k;
    free(bs); free(S);
    return f;
}

/* Fast proximal gradient with Nesterov extrapolation t/(t+3) and backtracking
 * (eqs. fpg_extrapolate, fpg_grad, fpg_step, fpg_armijo).  Reading of the
 * unstated constants: start at the node iterate on S; step alpha_0 =
 * 4 / (||X_S||_F^2 + 2 lambda2), halved on each Armijo failure (at most 60
 * times per iteration) and carried to the next iteration; stop when
 * |U(beta+) - U(beta)| <= tol max(1, U(beta+)) or max|beta+ - beta| <= 1e-10,
 * or after max_iter iterations. */
double orc_fista(const orc_inst *in, const uint8_t *mask, double *beta,
                 double tol, int max_iter, int *iters) {
    int64_t n = in->n, p = in->p;
    double l2 = in->l2, M = in->M;
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)p);
    int64_t k = support_list(in, mask, S);
    int it = 0;
    if (k == 0) {
        for (int64_t j = 0; j < p; ++j) beta[j] = 0.0;
        free(S);
        if (iters) *iters = 0;
        double yy = 0.0;
        for (int64_t i = 0; i < n; ++i) yy += in->y[i] * in->y[i];
        return 0.5 * yy;
    }
    double *cur = (double *)malloc(sizeof(double) * (size_t)k);
    double *prev = (double *)malloc(sizeof(double) * (size_t)k);
    double *ext = (double *)malloc(sizeof(double) * (size_t)k);
    double *nxt = (double *)malloc(sizeof(double) * (size_t)k);
    double *grad = (double *)malloc(sizeof(double) * (size_t)k);
    double *res = (double *)malloc(sizeof(double) * (size_t)n);
    double fro = 0.0;
    for (int64_t a = 0; a < k; ++a) {
        cur[a] = clip(beta[S[a]], M);
        prev[a] = cur[a];
        fro += in->colnrm[S[a]] * in->colnrm[S[a]];
    }
    double alpha = 4.0 / (fro + 2.0 * l2);
    double Ucur = U_S(in, S, k, cur, NULL);
    for (it = 0; it < max_iter;) {
        double mom = (double)it / ((double)it + 3.0);
        for (int64_t a = 0; a < k; ++a) ext[a] = cur[a] + mom * (cur[a] - prev[a]);
        double Uext = U_S(in, S, k, ext, res);   /* res = X_S ext - y */
        for (int64_t a = 0; a < k; ++a) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += XC(in, i, S[a]) * res[i];
            grad[a] = s + 2.0 * l2 * ext[a];
        }
        double Unxt = 0.0;
        for (int bt = 0; bt <= 60; ++bt) {
            double gd = 0.0, dd = 0.0;
            for (int64_t a = 0; a < k; ++a) {
                nxt[a] = clip(ext[a] - alpha * grad[a], M);
                double d = nxt[a] - ext[a];
                gd += grad[a] * d;
                dd += d * d;
            }
            Unxt = U_S(in, S, k, nxt, NULL);
            if (Unxt <= Uext + gd + dd / (2.0 * alpha) || bt == 60) break;
            alpha *= 0.5;
        }
        ++it;
        double dmax = 0.0;
        for (int64_t a = 0; a < k; ++a) {
            double d = fabs(nxt[a] - cur[a]);
            if (d > dmax) dmax = d;
        }
        double dU = fabs(Unxt - Ucur);
        for (int64_t a = 0; a < k; ++a) { prev[a] = cur[a]; cur[a] = nxt[a]; }
        Ucur = Unxt;
        if (dU <= tol * (Ucur > 1.0 ? Ucur : 1.0) || dmax <= 1e-10) break;
    }
    for (int64_t j = 0; j < p; ++j) beta[j] = 0.0;
    for (int64_t a = 0; a < k; ++a) beta[S[a]] = cur[a];
    double f = U_S(in, S, k, cur, NULL) + in->l0 * (double)k;
    free(cur); free(prev); free(ext); free(nxt); free(grad); free(res); free(S);
    if (iters) *iters = it;
    return f;
}

/* min over |beta| <= M of U_S(beta), solved to full precision (used only to
 * report the certified objective of the final support). */
double orc_exact_objective(const orc_inst *in, const uint8_t *mask, double *beta) {
    int64_t n = in->n, p = in->p;
    double l2 = in->l2, M = in->M;
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)p);
    int64_t k = support_list(in, mask, S);
    for (int64_t j = 0; j < p; ++j) beta[j] = 0.0;
    if (k == 0) {
        free(S);
        double yy = 0.0;
        for (int64_t i = 0; i < n; ++i) yy += in->y[i] * in->y[i];
        return 0.5 * yy;
    }
    double *H = (double *)malloc(sizeof(double) * (size_t)(k * k));
    double *L = (double *)malloc(sizeof(double) * (size_t)(k * k));
    double *g = (double *)malloc(sizeof(double) * (size_t)k);
    double *bs = (double *)malloc(sizeof(double) * (size_t)k);
    for (int64_t a = 0; a < k; ++a) {
        g[a] = in->c[S[a]];
        for (int64_t b2 = 0; b2 < k; ++b2) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += XC(in, i, S[a]) * XC(in, i, S[b2]);
            H[b2 * k + a] = s + (a == b2 ? 2.0 * l2 : 0.0);
        }
    }
    memcpy(L, H, sizeof(double) * (size_t)(k * k));
    memcpy(bs, g, sizeof(double) * (size_t)k);
    int boxed = 0;
    if (cholesky(L, k) == 0) {
        chol_solve(L, k, bs);
        for (int64_t a = 0; a < k; ++a) if (fabs(bs[a]) > M) boxed = 1;
    } else {
        boxed = 1;
        for (int64_t a = 0; a < k; ++a) bs[a] = 0.0;
    }
    if (boxed) {
        /* coordinate descent on 1/2 b^T H b - g^T b over the box */
        for (int64_t a = 0; a < k; ++a) bs[a] = clip(bs[a], M);
        for (int sweep = 0; sweep < 200000; ++sweep) {
            double dmax = 0.0, bmax = 0.0;
            for (int64_t a = 0; a < k; ++a) {
                double s = g[a];
                for (int64_t b2 = 0; b2 < k; ++b2) if (b2 != a) s -= H[b2 * k + a] * bs[b2];
                double nv = clip(s / H[a * k + a], M);
                double d = fabs(nv - bs[a]);
                if (d > dmax) dmax = d;
                bs[a] = nv;
                if (fabs(nv) > bmax) bmax = fabs(nv);
            }
            if (dmax <= 1e-16 * (bmax > 1.0 ? bmax : 1.0)) break;
        }
    }
    for (int64_t a = 0; a < k; ++a) beta[S[a]] = bs[a];
    double f = U_S(in, S, k, bs, NULL) + in->l0 * (double)k;
    free(H); free(L); free(g); free(bs); free(S);
    return f;
}

/* ------------------------------------------------------------------------- */
/* Matching-pursuit root heuristic (Sec. 3.5, App. A.2)                       */
/* ------------------------------------------------------------------------- */

/* Objective change of each single-coordinate move at (mask, beta) with the
 * residual r = y - X beta given, the other coordinates frozen (App. A.2):
 *   j outside the support: adding j with b = clip(c_j / D_j, -M, M),
 *     c_j = X_j^T r, D_j = ||X_j||^2 + 2 lambda2,
 *     Delta_j = -b c_j + D_j b^2 / 2 + lambda0            (bnew[j] = b);
 *   j in the support: removing it (beta_j -> 0),
 *     Delta_j = beta_j c_j + (||X_j||^2 / 2 - lambda2) beta_j^2 - lambda0
 *                                                         (bnew[j] = 0). */
void orc_mp_deltas(const orc_inst *in, const uint8_t *mask, const double *beta, const double *r,
                   double *delta, double *bnew) {
    const int64_t n = in->n, p = in->p;
    for (int64_t j = 0; j < p; ++j) {
        double c = 0.0, q = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            c += XC(in, i, j) * r[i];
            q += XC(in, i, j) * XC(in, i, j);
        }
        if (mask[j]) {
            const double b = beta[j];
            delta[j] = b * c + (0.5 * q - in->l2) * b * b - in->l0;
            bnew[j] = 0.0;
        } else {
            const double D = q + 2.0 * in->l2;
            const double b = clip(c / D, in->M);
            delta[j] = -b * c + 0.5 * D * b * b + in->l0;
            bnew[j] = b;
        }
    }
}

/* From S = {} and beta = 0 (r = y), alternate a forward step (the addition of
 * smallest Delta_j among j outside S, taken when Delta_j < 0) and a backward
 * step (the removal of smallest Delta_j among j in S, taken when Delta_j < 0),
 * each recomputing c = X^T r at the current residual, which is updated
 * exactly (r -= X_j b on an addition, r += X_j beta_j on a removal); stop when
 * a forward and the following backward step both take no move, or after
 * max_moves moves.  Ties go to the smallest index.  Fills mask and beta (p
 * entries) and moves (room for max_moves: j + 1 for an addition of j, -(j + 1)
 * for a removal), returns the number of moves. */
int orc_matching_pursuit(const orc_inst *in, int max_moves, uint8_t *mask, double *beta, int32_t *moves) {
    const int64_t n = in->n, p = in->p;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *delta = (double *)malloc(sizeof(double) * (size_t)p);
    double *bnew = (double *)malloc(sizeof(double) * (size_t)p);
    memcpy(r, in->y, sizeof(double) * (size_t)n);
    memset(mask, 0, (size_t)p);
    for (int64_t j = 0; j < p; ++j) beta[j] = 0.0;
    int nm = 0;
    while (nm < max_moves) {
        int moved = 0;
        for (int phase = 0; phase < 2 && nm < max_moves; ++phase) {
            const int want = phase == 0 ? 0 : 1;    /* forward: j outside S; backward: j in S */
            orc_mp_deltas(in, mask, beta, r, delta, bnew);
            int64_t best = -1;
            for (int64_t j = 0; j < p; ++j)
                if ((mask[j] != 0) == want && delta[j] < 0.0 && (best < 0 || delta[j] < delta[best])) best = j;
            if (best < 0) continue;
            if (phase == 0) {
                const double b = bnew[best];
                for (int64_t i = 0; i < n; ++i) r[i] = r[i] - XC(in, i, best) * b;
                beta[best] = b;
                mask[best] = 1;
                moves[nm++] = (int32_t)(best + 1);
            } else {
                const double b = beta[best];
                for (int64_t i = 0; i < n; ++i) r[i] = r[i] + XC(in, i, best) * b;
                beta[best] = 0.0;
                mask[best] = 0;
                moves[nm++] = (int32_t)(-(best + 1));
            }
            moved = 1;
        }
        if (!moved) break;
    }
    free(r); free(delta); free(bnew);
    return nm;
}

/* ------------------------------------------------------------------------- */
/* Depth-first branch and bound                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint8_t *codes;
    double *beta, *v;
    double lb_parent;
    int64_t id, parent;
    int32_t depth;
} orc_node;

static void node_free(orc_node *u) { free(u->codes); free(u->beta); free(u->v); }

/* Alg. 1 with batch size K = 1 and a LIFO frontier.  Readings: a node is pruned
 * when its bound reaches UB (1 - eps_prune) (eps_prune absorbs the inexactness
 * of the ADMM bound at tolerance tol_node); a child inherits max(LB_u,
 * inherited bound) and is discarded at selection when that already prunes it;
 * a node with no free coordinate is closed after its incumbent is taken; the
 * child that agrees with the rounded z_j is explored first. */
int orc_bnb(const orc_inst *in, const orc_bnb_opts *o, orc_bnb_result *res,
            uint8_t *mask_out, double *beta_out, orc_trace_rec *trace, int64_t trace_cap) {
    int64_t n = in->n, p = in->p;
    int64_t cap = 2 * p + 8, top = 0;
    orc_node *stack = (orc_node *)calloc((size_t)cap, sizeof(orc_node));
    double *b = (double *)calloc((size_t)p, sizeof(double));
    uint8_t *mask = (uint8_t *)malloc((size_t)p);
    double *bf = (double *)malloc(sizeof(double) * (size_t)p);
    uint8_t *inc_mask = (uint8_t *)calloc((size_t)p, 1);
    double *inc_beta = (double *)calloc((size_t)p, sizeof(double));
    double UB = INFINITY;
    int have_inc = 0;
    int64_t next_id = 1, solved = 0, pruned = 0, tl = 0;
    int status = 0;
    (void)n;

    orc_node root = {0};
    root.codes = (uint8_t *)calloc((size_t)p, 1);
    root.beta = (double *)calloc((size_t)p, sizeof(double));
    root.v = (double *)calloc((size_t)p, sizeof(double));
    root.lb_parent = -INFINITY;
    root.id = 0; root.parent = -1; root.depth = 0;
    stack[top++] = root;

    while (top > 0) {
        if (o->gap_tol > 0.0 && have_inc) {
            double lbg = INFINITY;
            for (int64_t s = 0; s < top; ++s) if (stack[s].lb_parent < lbg) lbg = stack[s].lb_parent;
            if (UB - lbg <= o->gap_tol * fabs(UB)) { status = 2; break; }
        }
        orc_node u = stack[--top];
        orc_trace_rec rec;
        memset(&rec, 0, sizeof rec);
        rec.id = u.id; rec.parent = u.parent; rec.depth = u.depth; rec.branch_j = -1;
        if (have_inc && u.lb_parent >= UB * (1.0 - o->eps_prune)) {
            ++pruned;
            rec.decision = 3; rec.lb = u.lb_parent; rec.ub_global = UB;
            if (trace && tl < trace_cap) trace[tl] = rec;
            ++tl;
            node_free(&u);
            continue;
        }
        if (solved >= o->max_nodes) { stack[top++] = u; status = 1; break; }
        double lb, primal;
        int iters;
        int st = orc_node_admm(in, u.codes, u.beta, u.v, b, o->tol_node,
                               u.id == 0 ? o->max_iter_root : o->max_iter, o->check_every,
                               &lb, &primal, &iters);
        ++solved;
        double lb_eff = lb > u.lb_parent ? lb : u.lb_parent;
        rec.lb = lb_eff; rec.primal = primal; rec.iters = iters; rec.admm_status = st;
        if (have_inc && lb_eff >= UB * (1.0 - o->eps_prune)) {
            ++pruned;
            rec.decision = 1; rec.ub_global = UB;
            if (trace && tl < trace_cap) trace[tl] = rec;
            ++tl;
            node_free(&u);
            continue;
        }
        int k = orc_support(in, u.codes, u.beta, mask);
        memcpy(bf, u.beta, sizeof(double) * (size_t)p);
        int fit;
        double ub_u = orc_fista(in, mask, bf, o->fista_tol, o->fista_max_iter, &fit);
        rec.ub_node = ub_u; rec.support_size = k;
        if (ub_u < UB) {
            UB = ub_u;
            have_inc = 1;
            memcpy(inc_mask, mask, (size_t)p);
            memcpy(inc_beta, bf, sizeof(double) * (size_t)p);
        }
        rec.ub_global = UB;
        int j = orc_branch(in, u.codes, u.beta);
        if (j < 0) {
            rec.decision = 2;
            if (trace && tl < trace_cap) trace[tl] = rec;
            ++tl;
            node_free(&u);
            continue;
        }
        rec.decision = 0; rec.branch_j = j;
        if (trace && tl < trace_cap) trace[tl] = rec;
        ++tl;
        orc_node c0, c1;
        c0.codes = (uint8_t *)malloc((size_t)p); memcpy(c0.codes, u.codes, (size_t)p); c0.codes[j] = ORC_FIX0;
        c1.codes = u.codes; c1.codes[j] = ORC_FIX1;
        c0.beta = (double *)malloc(sizeof(double) * (size_t)p); memcpy(c0.beta, u.beta, sizeof(double) * (size_t)p);
        c0.v = (double *)malloc(sizeof(double) * (size_t)p); memcpy(c0.v, u.v, sizeof(double) * (size_t)p);
        c1.beta = u.beta; c1.v = u.v;
        c0.lb_parent = c1.lb_parent = lb_eff;
        c0.parent = c1.parent = u.id;
        c0.depth = c1.depth = u.depth + 1;
        c0.id = next_id++;
        c1.id = next_id++;
        double zj = orc_z(u.beta[j], ORC_FREE, in->l0, in->l2, in->M);
        if (top + 2 > cap) { cap *= 2; stack = (orc_node *)realloc(stack, sizeof(orc_node) * (size_t)cap); }
        if (zj >= 0.5) { stack[top++] = c0; stack[top++] = c1; }
        else { stack[top++] = c1; stack[top++] = c0; }
    }
    double lbg = UB;
    for (int64_t s = 0; s < top; ++s) if (stack[s].lb_parent < lbg) lbg = stack[s].lb_parent;
    for (int64_t s = 0; s < top; ++s) node_free(&stack[s]);
    free(stack);
    res->ub = UB;
    res->lb_global = status == 0 ? UB : lbg;
    res->nodes_solved = solved;
    res->nodes_pruned = pruned;
    res->trace_len = tl;
    res->status = status;
    res->certified = have_inc ? orc_exact_objective(in, inc_mask, beta_out) : INFINITY;
    memcpy(mask_out, inc_mask, (size_t)p);
    free(b); free(mask); free(bf); free(inc_mask); free(inc_beta);
    return 0;
}
