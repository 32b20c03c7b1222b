/*
 * FP64 CPU oracle for the superiorized simultaneous band+box projection method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant with the HIP
 * library: it is written independently from the paper, plainly and slowly, in
 * double precision throughout.
 *
 * What it computes (paper, Section 2.1):
 *   - projection onto one linear constraint set (Section 2.1.1, the half-space
 *     formula), generalised to a two-sided band l_i <= <a_i,x> <= u_i: the point
 *     moves along a_i by (clip(r_i) - r_i)/||a_i||^2 with r_i = <a_i,x>;
 *   - the relaxed projection x + lambda (P(x) - x) (eq. RelaxedProjection),
 *     applied to the weighted simultaneous combination sum_i w_i P_i(x) with
 *     w_i > 0, sum w_i = 1 (the weights of eq. WeightedProximity), and the
 *     other simultaneous basic algorithms of the appendix's table of methods
 *     (DROP, extrapolated Landweber, Landweber with error-minimising
 *     relaxation) and the CQ iteration of Section 2.1.1;
 *   - the weighted proximity 1/2 sum_i w_i ||P_i(x) - x||^2 (eq. WeightedProximity);
 *   - a projection onto the box lo <= x <= hi after every step (Section 2.3.3,
 *     the BoxProjection applied after each iteration);
 *   - the superiorized iteration of Algorithm 1 with power-law step sizes
 *     beta = gamma * alpha^ell (Section 2.1.2) and restarts of ell;
 *   - dose-volume constraints (Section 2.3.3) as sets in the output space of
 *     the split problem (eq. Split): for a structure S of N_S rows, "at most
 *     V N_S rows above d" or "at least V N_S rows at or above d", with the
 *     nearest-point projection of the structure's values A_S x onto that set;
 *   - the objectives: squared norm (the L2 perturbation of Section 2.3.1), the
 *     L1 norm (the L1 perturbation of the same section, subgradient sign(x)),
 *     total variation of a 2-D image (Section 2.3.1, TV equation), and a linear
 *     dose objective c^T x (Section 2.3.3, mean-dose objective up to scale).
 *
 * Readings taken where the paper is silent or ambiguous are listed in the
 * design notes of the repository; the ones this file depends on are restated
 * at the point of use.
 *
 * Parallelism: only loops whose iterations are independent (one output per
 * row or per column) run under OpenMP, so every result is independent of the
 * thread count.  All reductions are plain sequential loops.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OBJ_NONE 0
#define ORC_OBJ_SQNORM 1
#define ORC_OBJ_TV2D 2
#define ORC_OBJ_LINEAR 3
#define ORC_OBJ_L1 4     /* ||x||_1 (Section 2.3.1), subgradient sign(x) with sign(0) = 0 */

/* basic (feasibility-seeking) algorithms of the appendix's table of methods */
#define ORC_BASIC_SIMULT 0 /* weighted simultaneous projection */
#define ORC_BASIC_DROP 1   /* diagonally relaxed orthogonal projections */
#define ORC_BASIC_CQ 2     /* CQ iteration with the Frobenius bound */
#define ORC_BASIC_EL 3     /* extrapolated Landweber */
#define ORC_BASIC_EMR 4    /* Landweber with error-minimising relaxation */
#define ORC_BASIC_ART 5    /* sequential projections (Kaczmarz / ART), one sweep per iteration; oracle only */

/* step-size rules of the perturbation phase (Section 2.1.2) */
#define ORC_STEP_POWER 0    /* beta = gamma * alpha^ell, ell one per trial */
#define ORC_STEP_ADAPTIVE 1 /* beta = (f(x^k) - f_ref) / ||g(x^k)|| when f(x^k) > f_ref, else no step */

/* dose-volume constraint senses (Section 2.3.3) */
#define ORC_DVC_MAX 0 /* D_V <= d: at most floor(V N_S) rows of the structure above d */
#define ORC_DVC_MIN 1 /* D_V >= d: at least ceil(V N_S) rows of the structure at or above d */

typedef struct {
    int64_t row_begin, row_end; /* the structure's rows [row_begin, row_end) */
    int32_t sense;              /* ORC_DVC_* */
    int32_t pad_;
    double fraction;            /* V in [0, 1] */
    double dose;                /* d */
} orc_dvc;

typedef struct {
    int64_t m, n;
    const int64_t *row_ptr; /* m+1 */
    const int32_t *col;     /* nnz */
    const double *val;      /* nnz */
    const double *lower;    /* m, may hold -inf */
    const double *upper;    /* m, may hold +inf */
    const double *w;        /* m, weights, w_i > 0, sum 1 */
    const double *box_lo;   /* n */
    const double *box_hi;   /* n */
    double lambda;
    int32_t obj;
    int32_t tv_rows, tv_cols;
    int32_t max_trials;
    double tv_eps;
    const double *lin_c; /* n */
    double gamma, alpha;
    int32_t n_red, restart_every;
    int32_t basic;          /* ORC_BASIC_*: the feasibility-seeking step */
    const double *col_nnz;  /* n, nonzeros per column for DROP, or NULL to count them from val */
    /* stopping rules (Section 2.2.1 and the superiorized variant of Section
     * 2.2.3; the variance rule of Section 2.3.2); stop_on = 0 disables all */
    int32_t stop_on;
    int32_t stop_n;      /* N: consecutive iterations with a small proximity change */
    int32_t stop_max;    /* N_max (0: none) */
    double stop_prox;    /* P* */
    double stop_dprox;   /* Delta P* */
    double stop_dobj;    /* Delta f* */
    double stop_var;     /* variance threshold (0: rule off) */
    /* dose-volume constraints: each owns a block of rows whose lower/upper are
     * replaced, at every point, by the bands its projection sets */
    int32_t n_dvc;
    int32_t pad_;
    const orc_dvc *dvc;
    /* optional column copy of A (orc_build_csc), used by the transposed
     * product when present: col_ptr[n+1], each column's rows ascending */
    const int64_t *csc_ptr;
    const int32_t *csc_row;
    const double *csc_val;
    int32_t step_rule; /* ORC_STEP_* */
    int32_t pad2_;
} orc_problem;

typedef struct {
    int64_t k;        /* outer iterations completed */
    int64_t ell;      /* exponent of the power-law step, one per trial */
    int64_t restarts; /* restarts performed so far */
    int64_t trials;   /* trial points evaluated, total */
    int64_t accepts;  /* trial points accepted, total */
    int64_t cap_hits; /* reduction steps that hit the trial cap */
    /* stopping-rule bookkeeping */
    int32_t stop_reason; /* ORC_STOP_*: 0 while running */
    int32_t dp_run;      /* consecutive iterations with Delta P < Delta P* */
    int32_t feas_ok;     /* the proximity rules held at the last iteration */
    int32_t pad_;
    double p_last;       /* proximity recorded at the last iteration (NaN before the first) */
    double f_last;       /* f(x^k) of the last iteration's phase */
    double var_n, var_mean, var_m2; /* running count, mean and squared deviations of omega */
    double f_ref; /* f where the last perturbation phase ended (NaN before the first): the adaptive step's reference */
} orc_state;

#define ORC_STOP_PROX 1    /* P <= P* */
#define ORC_STOP_DPROX 2   /* Delta P < Delta P* for N consecutive iterations */
#define ORC_STOP_MAXIT 3   /* N_max iterations */
#define ORC_STOP_VAR 4     /* variance of the relative iterate changes below its threshold */
#define ORC_STOP_SM 5      /* a proximity rule and Delta f < Delta f* (superiorized runs) */

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* r = A x, one inner product <a_i, x> per row. */
void orc_matvec(const orc_problem *P, const double *x, double *r)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P->m; ++i) {
        double s = 0.0;
        for (int64_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) s += P->val[p] * x[P->col[p]];
        r[i] = s;
    }
}

/* y = A^T c: y_j = sum_i a_ij c_i, the terms added in ascending row order.
 * With the column copy each column is one independent sum (the same terms in
 * the same order as the row-after-row accumulation, so the result is the
 * same bit for bit); without it the rows are accumulated one after another. */
void orc_matvec_t(const orc_problem *P, const double *c, double *y)
{
    if (P->csc_ptr) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t j = 0; j < P->n; ++j) {
            double s = 0.0;
            for (int64_t p = P->csc_ptr[j]; p < P->csc_ptr[j + 1]; ++p) s += P->csc_val[p] * c[P->csc_row[p]];
            y[j] = s;
        }
        return;
    }
    for (int64_t j = 0; j < P->n; ++j) y[j] = 0.0;
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) y[P->col[p]] += P->val[p] * c[i];
}

/* The column copy of A: a stable counting sort of the entries by column, so
 * the rows of each column stay in ascending order.  col_ptr has n+1 entries,
 * rows and vals nnz each (caller-owned). */
void orc_build_csc(const orc_problem *P, int64_t *col_ptr, int32_t *rows, double *vals)
{
    const int64_t nnz = P->row_ptr[P->m];
    for (int64_t j = 0; j <= P->n; ++j) col_ptr[j] = 0;
    for (int64_t p = 0; p < nnz; ++p) col_ptr[P->col[p] + 1] += 1;
    for (int64_t j = 0; j < P->n; ++j) col_ptr[j + 1] += col_ptr[j];
    int64_t *next = malloc(sizeof(int64_t) * (P->n > 0 ? P->n : 1));
    for (int64_t j = 0; j < P->n; ++j) next[j] = col_ptr[j];
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) {
            const int64_t q = next[P->col[p]]++;
            rows[q] = (int32_t)i;
            vals[q] = P->val[p];
        }
    free(next);
}

/* OpenMP threads used by the parallel loops (n > 0), and the current count. */
void orc_set_threads(int32_t n)
{
    if (n > 0) omp_set_num_threads(n);
}

int32_t orc_max_threads(void) { return (int32_t)omp_get_max_threads(); }

/* q_i = ||a_i||^2 */
void orc_row_sqnorms(const orc_problem *P, double *q)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P->m; ++i) {
        double s = 0.0;
        for (int64_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) s += P->val[p] * P->val[p];
        q[i] = s;
    }
}

/*
 * Dose-volume constraints.  The structure's values d_i = r_i (i in S) are
 * ranked from the highest down by their exact (double) values; equal values
 * are ranked by row index.  The nearest point of the set
 *   MAX: at most k = floor(V N_S) values above d  keeps the k highest values
 *        and lowers every other value above d to d;
 *   MIN: at least k = ceil(V N_S) values at or above d  raises the k highest
 *        values to d where they are below it and keeps the others;
 * (changing the k highest is the cheapest choice in both cases, the squared
 * distance being a sum over the changed values; where the k-th and (k+1)-th
 * values are equal the nearest point is not unique and the lower row index
 * is kept among the k).  As bands on the rows: MAX gives (-inf, +inf) to the
 * k highest and (-inf, d] to the rest, MIN gives [d, +inf) to the k highest
 * and (-inf, +inf) to the rest.
 */
typedef struct {
    double key;
    int64_t row;
} ranked;

static int by_value_then_row(const void *a, const void *b)
{
    const ranked *p = a, *q = b;
    if (p->key != q->key) return p->key > q->key ? -1 : 1; /* higher value first */
    return p->row < q->row ? -1 : (p->row > q->row ? 1 : 0);
}

int64_t orc_dvc_count(const orc_dvc *g)
{
    const int64_t N = g->row_end - g->row_begin;
    double kv = g->sense == ORC_DVC_MAX ? floor(g->fraction * (double)N) : ceil(g->fraction * (double)N);
    if (kv < 0.0) kv = 0.0;
    if (kv > (double)N) kv = (double)N;
    return (int64_t)kv;
}

/* lo/up: the bands every row has at the point with row values r. */
static void effective_bands(const orc_problem *P, const double *r, double *lo, double *up)
{
    for (int64_t i = 0; i < P->m; ++i) {
        lo[i] = P->lower[i];
        up[i] = P->upper[i];
    }
    for (int32_t g = 0; g < P->n_dvc; ++g) {
        const orc_dvc *G = &P->dvc[g];
        const int64_t N = G->row_end - G->row_begin, k = orc_dvc_count(G);
        ranked *order = malloc(sizeof(ranked) * (N > 0 ? N : 1));
        for (int64_t p = 0; p < N; ++p) {
            order[p].key = r[G->row_begin + p];
            order[p].row = G->row_begin + p;
        }
        qsort(order, (size_t)N, sizeof(ranked), by_value_then_row);
        for (int64_t p = 0; p < N; ++p) {
            const int64_t i = order[p].row;
            const int top = p < k;
            if (G->sense == ORC_DVC_MAX) {
                lo[i] = -INFINITY;
                up[i] = top ? INFINITY : G->dose;
            } else {
                lo[i] = top ? G->dose : -INFINITY;
                up[i] = INFINITY;
            }
        }
        free(order);
    }
}

/* For each dose-volume constraint g at the point x: the k-th and (k+1)-th
 * highest values of its structure (k as in orc_dvc_count; +inf when k = 0,
 * -inf when k = N_S).  Where the two are close the nearest point of the set
 * is nearly a tie, and a computation whose values carry rounding errors may
 * keep the other row. */
void orc_dvc_boundary(const orc_problem *P, const double *x, double *kth, double *next)
{
    double *r = malloc(sizeof(double) * P->m);
    orc_matvec(P, x, r);
    for (int32_t g = 0; g < P->n_dvc; ++g) {
        const orc_dvc *G = &P->dvc[g];
        const int64_t N = G->row_end - G->row_begin, k = orc_dvc_count(G);
        ranked *order = malloc(sizeof(ranked) * (N > 0 ? N : 1));
        for (int64_t p = 0; p < N; ++p) {
            order[p].key = r[G->row_begin + p];
            order[p].row = G->row_begin + p;
        }
        qsort(order, (size_t)N, sizeof(ranked), by_value_then_row);
        kth[g] = k > 0 ? order[k - 1].key : INFINITY;
        next[g] = k < N ? order[k].key : -INFINITY;
        free(order);
    }
    free(r);
}

/*
 * Weighted proximity (eq. WeightedProximity): 1/2 sum_i w_i ||P_i(x) - x||^2.
 * For a band, P_i(x) - x = ((clip(r_i) - r_i)/||a_i||^2) a_i, whose norm is
 * |clip(r_i) - r_i| / ||a_i||.  A row with a_i = 0 is the whole space when its
 * band holds 0 and is skipped here (it cannot be projected onto otherwise).
 * lo/up are the bands at this point (effective_bands).
 */
static double proximity_q(const orc_problem *P, const double *q, const double *r, const double *lo,
                          const double *up)
{
    double s = 0.0;
    for (int64_t i = 0; i < P->m; ++i) {
        if (!(q[i] > 0.0)) continue;
        double t = clampd(r[i], lo[i], up[i]) - r[i];
        double dist = fabs(t) / sqrt(q[i]);
        s += P->w[i] * dist * dist;
    }
    return 0.5 * s;
}

double orc_proximity(const orc_problem *P, const double *x)
{
    double *q = malloc(sizeof(double) * P->m), *r = malloc(sizeof(double) * P->m),
           *lo = malloc(sizeof(double) * P->m), *up = malloc(sizeof(double) * P->m);
    orc_row_sqnorms(P, q);
    orc_matvec(P, x, r);
    effective_bands(P, r, lo, up);
    double v = proximity_q(P, q, r, lo, up);
    free(q);
    free(r);
    free(lo);
    free(up);
    return v;
}

/* The bands at x (for tests): lo/up of length m. */
void orc_bands_at(const orc_problem *P, const double *x, double *lo, double *up)
{
    double *r = malloc(sizeof(double) * P->m);
    orc_matvec(P, x, r);
    effective_bands(P, r, lo, up);
    free(r);
}

/*
 * One feasibility-seeking step T of the chosen basic algorithm (in place),
 * then the box projection.  t_i = clip(r_i) - r_i is the band residual at the
 * input point (for an equality band l_i = u_i = b_i it is b_i - <a_i,x>, the
 * negative of the residual A x - b the table of methods writes).  With
 * D = diag(w_i/||a_i||^2) and W = diag(w_i):
 *   SIMULT  x + lambda A^T D t: the relaxed weighted sum of the single-band
 *           projections, since P_i(x) - x = (t_i/||a_i||^2) a_i;
 *   DROP    x + lambda Z A^T D t, Z_j = 1/(nonzeros in column j), 0 for an
 *           empty column;
 *   CQ      x + lambda A^T t / ||A||_F^2: the CQ iteration with Q the bands
 *           and gamma = lambda / L*, L* the squared Frobenius norm bound
 *           (Section 2.1.1); the box plays C;
 *   EL      x + lambda sigma A^T D t, sigma = t^T D t / ||A^T D t||^2;
 *   EMR     x + lambda sigma y, y = A^T W t, sigma = ||y||^2 / sum_i w_i (A y)_i^2;
 *   ART     one sweep over the rows in order, each projecting the current
 *           point onto its band: x <- x + lambda (clip(<a_i,x>) - <a_i,x>) /
 *           ||a_i||^2 a_i (the sequential row of the table of methods; rows
 *           with a_i = 0 are skipped; dose-volume rows keep the bands set at
 *           the sweep's start);
 * sigma = 0 when its denominator is 0 (then y = 0 too).  The bands of
 * dose-volume rows are those their projection sets at the input point (the
 * split problem's P_Q).  Returns the
 * proximity at the input point.  Scratch: r[m], c[m], y[n]; zc[n] holds the
 * DROP column factors (unused otherwise).
 */
static double feas_step(const orc_problem *P, const double *q, const double *zc, double *x, double *r, double *c,
                        double *y)
{
    orc_matvec(P, x, r);
    double *lo = malloc(sizeof(double) * P->m), *up = malloc(sizeof(double) * P->m);
    effective_bands(P, r, lo, up);
    double prox = proximity_q(P, q, r, lo, up);
    if (P->basic == ORC_BASIC_ART) {
        for (int64_t i = 0; i < P->m; ++i) {
            if (!(q[i] > 0.0)) continue;
            double ri = 0.0;
            for (int64_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) ri += P->val[p] * x[P->col[p]];
            const double step = P->lambda * (clampd(ri, lo[i], up[i]) - ri) / q[i];
            for (int64_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) x[P->col[p]] += step * P->val[p];
        }
        for (int64_t j = 0; j < P->n; ++j) x[j] = clampd(x[j], P->box_lo[j], P->box_hi[j]);
        free(lo);
        free(up);
        return prox;
    }
    double fro2 = 0.0;
    if (P->basic == ORC_BASIC_CQ)
        for (int64_t i = 0; i < P->m; ++i) fro2 += q[i];
    for (int64_t i = 0; i < P->m; ++i) {
        double t = clampd(r[i], lo[i], up[i]) - r[i];
        r[i] = t; /* r now holds t */
        switch (P->basic) {
        case ORC_BASIC_CQ:
            c[i] = fro2 > 0.0 ? t / fro2 : 0.0;
            break;
        case ORC_BASIC_EMR:
            c[i] = P->w[i] * t;
            break;
        default: /* w_i (P_i(x) - x) = w_i * t / ||a_i||^2 * a_i */
            c[i] = (q[i] > 0.0) ? P->w[i] * t / q[i] : 0.0;
        }
    }
    free(lo);
    free(up);
    orc_matvec_t(P, c, y);
    double sigma = 1.0;
    if (P->basic == ORC_BASIC_EL) {
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < P->m; ++i) num += c[i] * r[i]; /* t^T D t */
        for (int64_t j = 0; j < P->n; ++j) den += y[j] * y[j];
        sigma = den > 0.0 ? num / den : 0.0;
    } else if (P->basic == ORC_BASIC_EMR) {
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < P->n; ++j) num += y[j] * y[j];
        orc_matvec(P, y, r); /* r = A y */
        for (int64_t i = 0; i < P->m; ++i) den += P->w[i] * r[i] * r[i];
        sigma = den > 0.0 ? num / den : 0.0;
    }
    for (int64_t j = 0; j < P->n; ++j) {
        const double yj = (P->basic == ORC_BASIC_DROP) ? zc[j] * y[j] : y[j];
        x[j] = clampd(x[j] + P->lambda * sigma * yj, P->box_lo[j], P->box_hi[j]);
    }
    return prox;
}

/* DROP column factors Z_j = 1/(nonzeros in column j), 0 for an empty column. */
static void drop_factors(const orc_problem *P, double *zc)
{
    for (int64_t j = 0; j < P->n; ++j) zc[j] = 0.0;
    if (P->col_nnz) {
        for (int64_t j = 0; j < P->n; ++j) zc[j] = P->col_nnz[j];
    } else {
        for (int64_t p = 0; p < P->row_ptr[P->m]; ++p)
            if (P->val[p] != 0.0) zc[P->col[p]] += 1.0;
    }
    for (int64_t j = 0; j < P->n; ++j) zc[j] = zc[j] > 0.0 ? 1.0 / zc[j] : 0.0;
}

double orc_step(const orc_problem *P, double *x)
{
    double *q = malloc(sizeof(double) * P->m), *r = malloc(sizeof(double) * P->m),
           *c = malloc(sizeof(double) * P->m), *y = malloc(sizeof(double) * P->n),
           *zc = malloc(sizeof(double) * P->n);
    orc_row_sqnorms(P, q);
    drop_factors(P, zc);
    double v = feas_step(P, q, zc, x, r, c, y);
    free(q);
    free(r);
    free(c);
    free(y);
    free(zc);
    return v;
}

/*
 * Total variation of an R x C image stored row-major (pixel (i,j) at i*C + j),
 * summed over forward differences with i <= R-2 and j <= C-2 (the TV equation
 * of Section 2.3.1), smoothed by eps: each term is sqrt(dx^2 + dy^2 + eps^2)
 * with dx = X[i+1,j] - X[i,j] and dy = X[i,j+1] - X[i,j].
 */
static double tv_value(const orc_problem *P, const double *x)
{
    const int64_t R = P->tv_rows, C = P->tv_cols;
    const double e2 = P->tv_eps * P->tv_eps;
    double s = 0.0;
    for (int64_t i = 0; i + 1 < R; ++i)
        for (int64_t j = 0; j + 1 < C; ++j) {
            double x0 = x[i * C + j];
            double dx = x[(i + 1) * C + j] - x0;
            double dy = x[i * C + j + 1] - x0;
            s += sqrt(dx * dx + dy * dy + e2);
        }
    return s;
}

/* Gradient of the smoothed TV: each term's derivative scattered onto its three
 * pixels.  With eps = 0 a term with a zero root contributes nothing (the zero
 * subgradient). */
static void tv_grad(const orc_problem *P, const double *x, double *g)
{
    const int64_t R = P->tv_rows, C = P->tv_cols;
    const double e2 = P->tv_eps * P->tv_eps;
    for (int64_t p = 0; p < R * C; ++p) g[p] = 0.0;
    for (int64_t i = 0; i + 1 < R; ++i)
        for (int64_t j = 0; j + 1 < C; ++j) {
            double x0 = x[i * C + j];
            double dx = x[(i + 1) * C + j] - x0;
            double dy = x[i * C + j + 1] - x0;
            double tau = sqrt(dx * dx + dy * dy + e2);
            if (!(tau > 0.0)) continue;
            g[i * C + j] -= (dx + dy) / tau;
            g[(i + 1) * C + j] += dx / tau;
            g[i * C + j + 1] += dy / tau;
        }
}

double orc_objective(const orc_problem *P, const double *x)
{
    double s = 0.0;
    switch (P->obj) {
    case ORC_OBJ_SQNORM:
        for (int64_t j = 0; j < P->n; ++j) s += x[j] * x[j];
        return s;
    case ORC_OBJ_LINEAR:
        for (int64_t j = 0; j < P->n; ++j) s += P->lin_c[j] * x[j];
        return s;
    case ORC_OBJ_L1:
        for (int64_t j = 0; j < P->n; ++j) s += fabs(x[j]);
        return s;
    case ORC_OBJ_TV2D:
        return tv_value(P, x);
    default:
        return 0.0;
    }
}

void orc_gradient(const orc_problem *P, const double *x, double *g)
{
    switch (P->obj) {
    case ORC_OBJ_SQNORM:
        for (int64_t j = 0; j < P->n; ++j) g[j] = 2.0 * x[j];
        return;
    case ORC_OBJ_LINEAR:
        for (int64_t j = 0; j < P->n; ++j) g[j] = P->lin_c[j];
        return;
    case ORC_OBJ_L1:
        for (int64_t j = 0; j < P->n; ++j) g[j] = x[j] > 0.0 ? 1.0 : (x[j] < 0.0 ? -1.0 : 0.0);
        return;
    case ORC_OBJ_TV2D:
        tv_grad(P, x, g);
        return;
    default:
        for (int64_t j = 0; j < P->n; ++j) g[j] = 0.0;
    }
}

/*
 * Algorithm 1 (superiorized version of a feasibility-seeking algorithm), run
 * for K outer iterations from the state in *st (so a run can be split and
 * resumed).  With perturb == 0 only the feasibility step runs.
 *
 * Perturbation phase of outer iteration k, from x^{k,0} = x^k:
 *   - restarts: when restart_every > 0 and k is a positive multiple of it, the
 *     restart count r grows by one and ell is set to r (Section 2.1.2);
 *   - the direction is the normalised negative gradient v = -g/||g|| taken at
 *     x^k and kept for the whole phase; if ||g|| = 0 the phase is skipped;
 *   - each of the n_red reduction steps tries z = x^{k,n} + beta v with
 *     beta = gamma * alpha^ell, ell growing by one per trial, and accepts the
 *     first z with f(z) <= f(x^{k,n}); the number of trials per reduction step
 *     is capped at max_trials, and a step that reaches the cap ends the phase.
 * Then x^{k+1} = T(x^{k,n}).
 *
 * Per-iteration records (each may be NULL): proximity at the point T acts on,
 * objective at x^k, objective after the phase, trials and accepted trials.
 */
/*
 * Stopping rules, checked when P->stop_on (Section 2.2.1: P <= P*, or the
 * relative proximity change |P^{k+1} - P^k| / max{1, P^k} below Delta P* for
 * N consecutive iterations, or N_max iterations; Section 2.2.3: a superiorized
 * run stops when one of the two proximity rules holds and the relative change
 * of the objective |f^{k+1} - f^k| / max{1, f^k}, f^k = f(x^k), is below
 * Delta f*; Section 2.3.2: the variance of omega_i = ||x^i - x^{i-1}|| /
 * ||x^i||, i = 1..k, below a threshold).  P^k is the proximity recorded for
 * iteration k.  A superiorized run learns f(x^{k+1}) when its next phase
 * opens, so its rule is checked there, before that iteration perturbs.
 * omega_i = 0 when x^i = 0.  A stopped run does nothing more.
 */
static int stop_after_step(const orc_problem *P, orc_state *st, int sm, double prox, double f_start,
                           const double *x_prev, const double *x)
{
    if (st->stop_reason) return 1;
    if (!isnan(st->p_last)) {
        const double dp = fabs(prox - st->p_last) / fmax(1.0, st->p_last);
        st->dp_run = dp < P->stop_dprox ? st->dp_run + 1 : 0;
    }
    st->p_last = prox;
    const int by_prox = prox <= P->stop_prox, by_dprox = st->dp_run >= P->stop_n;
    if (sm) {
        st->feas_ok = by_prox || by_dprox;
        st->f_last = f_start;
    } else if (by_prox) {
        st->stop_reason = ORC_STOP_PROX;
    } else if (by_dprox) {
        st->stop_reason = ORC_STOP_DPROX;
    }
    if (!st->stop_reason && P->stop_max > 0 && st->k >= P->stop_max) st->stop_reason = ORC_STOP_MAXIT;
    if (P->stop_var > 0.0) {
        double dd = 0.0, xx = 0.0;
        for (int64_t j = 0; j < P->n; ++j) {
            dd += (x[j] - x_prev[j]) * (x[j] - x_prev[j]);
            xx += x[j] * x[j];
        }
        const double om = xx > 0.0 ? sqrt(dd) / sqrt(xx) : 0.0;
        /* running mean and sum of squared deviations (Welford) */
        st->var_n += 1.0;
        const double delta = om - st->var_mean;
        st->var_mean += delta / st->var_n;
        st->var_m2 += delta * (om - st->var_mean);
        if (!st->stop_reason && st->var_n >= 2.0 && st->var_m2 / (st->var_n - 1.0) < P->stop_var)
            st->stop_reason = ORC_STOP_VAR;
    }
    return st->stop_reason != 0;
}

/* A fresh stopping-rule state. */
void orc_stop_reset(orc_state *st)
{
    st->stop_reason = 0;
    st->dp_run = 0;
    st->feas_ok = 0;
    st->p_last = NAN;
    st->f_last = NAN;
    st->var_n = st->var_mean = st->var_m2 = 0.0;
}

/*
 * The perturbation phase of outer iteration st->k at x (in place), from
 * f(x^k) = f_start:
 *   - restarts: when restart_every > 0 and k is a positive multiple of it, the
 *     restart count r grows by one and ell is set to r (Section 2.1.2);
 *   - the direction is the normalised negative gradient v = -g/||g|| taken at
 *     x^k and kept for the whole phase; if ||g|| = 0 the phase is skipped;
 *   - each of the n_red reduction steps tries z = x^{k,n} + beta v with
 *     beta = gamma * alpha^ell, ell growing by one per trial, and accepts the
 *     first z with f(z) <= f(x^{k,n}); the number of trials per reduction step
 *     is capped at max_trials, and a step that reaches the cap ends the phase.
 * With the adaptive rule (ORC_STEP_ADAPTIVE; the step size of Nikazad et al.
 * in Section 2.1.2, whose reference value the paper does not define) the
 * phase instead tries the one step beta = (f(x^k) - f_ref) / ||g|| along v
 * when f(x^k) > f_ref, accepted under the same test f(z) <= f(x^k) (a
 * rejected step leaves x^k), and then sets f_ref to f after the phase: the
 * value the point the feasibility step acts on has.  Before the first phase
 * f_ref is f(x^0), so the first iteration does not perturb.  ell counts the
 * trial; n_red, max_trials and the power law do not apply.
 * Returns f after the phase (f_start when nothing was accepted); counts the
 * trials and accepted trials.  Scratch: g, v, z of length n.
 */
static double phase_steps(const orc_problem *P, double *x, orc_state *st, double f_start, double *g, double *v,
                          double *z, int32_t *trials, int32_t *accepts);

static double perturbation_phase(const orc_problem *P, double *x, orc_state *st, double f_start, double *g, double *v,
                                 double *z, int32_t *trials, int32_t *accepts)
{
    const double f = phase_steps(P, x, st, f_start, g, v, z, trials, accepts);
    st->f_ref = f; /* where this phase ended (the adaptive step's next reference) */
    return f;
}

static double phase_steps(const orc_problem *P, double *x, orc_state *st, double f_start, double *g, double *v,
                          double *z, int32_t *trials, int32_t *accepts)
{
    const int64_t n = P->n, k = st->k;
    if (P->restart_every > 0 && k > 0 && k % P->restart_every == 0) {
        st->restarts += 1;
        st->ell = st->restarts;
    }
    orc_gradient(P, x, g);
    double gg = 0.0;
    for (int64_t j = 0; j < n; ++j) gg += g[j] * g[j];
    const double gn = sqrt(gg);
    if (P->step_rule == ORC_STEP_ADAPTIVE) {
        double f_cur = f_start;
        if (!isnan(st->f_ref) && gn > 0.0 && f_start > st->f_ref) {
            const double beta = (f_start - st->f_ref) / gn;
            for (int64_t j = 0; j < n; ++j) z[j] = x[j] - beta * g[j] / gn;
            const double fz = orc_objective(P, z);
            st->ell += 1;
            *trials += 1;
            if (fz <= f_start) {
                memcpy(x, z, sizeof(double) * n);
                f_cur = fz;
                *accepts += 1;
            }
        }
        return f_cur;
    }
    if (!(gn > 0.0)) return f_start;
    for (int64_t j = 0; j < n; ++j) v[j] = -g[j] / gn;
    double f_cur = f_start;
    int32_t nr = 0;
    while (nr < P->n_red) {
        int accepted = 0;
        for (int32_t t = 0; t < P->max_trials; ++t) {
            const double beta = P->gamma * pow(P->alpha, (double)st->ell);
            st->ell += 1;
            for (int64_t j = 0; j < n; ++j) z[j] = x[j] + beta * v[j];
            const double fz = orc_objective(P, z);
            *trials += 1;
            if (fz <= f_cur) {
                memcpy(x, z, sizeof(double) * n);
                f_cur = fz;
                accepted = 1;
                *accepts += 1;
                break;
            }
        }
        if (!accepted) {
            st->cap_hits += 1;
            break;
        }
        nr += 1;
    }
    return f_cur;
}

/* The perturbation phase alone, as outer iteration st->k would run it, on x
 * (in place): the point z^k the feasibility step then acts on.  The state's
 * ell, restarts and cap hits advance as in orc_run; k and the trial totals
 * do not.  Without an objective nothing changes.  Returns -2 when out of
 * memory. */
int orc_perturb(const orc_problem *P, double *x, orc_state *st)
{
    if (P->obj == ORC_OBJ_NONE) return 0;
    double *g = malloc(sizeof(double) * P->n), *v = malloc(sizeof(double) * P->n), *z = malloc(sizeof(double) * P->n);
    if (!g || !v || !z) {
        free(g); free(v); free(z);
        return -2;
    }
    int32_t trials = 0, accepts = 0;
    perturbation_phase(P, x, st, orc_objective(P, x), g, v, z, &trials, &accepts);
    free(g); free(v); free(z);
    return 0;
}

/* What every iteration reuses: the row norms q[m] and the DROP column
 * factors zc[n]. */
void orc_prepare(const orc_problem *P, double *q, double *zc)
{
    orc_row_sqnorms(P, q);
    drop_factors(P, zc);
}

/* orc_run with q and zc from orc_prepare. */
int orc_run_prepared(const orc_problem *P, const double *q, const double *zc, double *x, int64_t K, int32_t perturb,
                     orc_state *st, double *hist_prox, double *hist_f_start, double *hist_f_end, int32_t *hist_trials,
                     int32_t *hist_accepts)
{
    const int64_t m = P->m, n = P->n;
    double *r = malloc(sizeof(double) * m), *c = malloc(sizeof(double) * m), *y = malloc(sizeof(double) * n),
           *g = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n),
           *xp = malloc(sizeof(double) * n);
    if (!r || !c || !y || !g || !v || !z || !xp) {
        free(r); free(c); free(y); free(g); free(v); free(z); free(xp);
        return -2;
    }
    const int sm = perturb && P->obj != ORC_OBJ_NONE;
    for (int64_t it = 0; it < K; ++it) {
        if (hist_prox) hist_prox[it] = NAN;
        if (hist_f_start) hist_f_start[it] = NAN;
        if (hist_f_end) hist_f_end[it] = NAN;
        if (hist_trials) hist_trials[it] = 0;
        if (hist_accepts) hist_accepts[it] = 0;
        if (P->stop_on && st->stop_reason) continue;
        int32_t trials = 0, accepts = 0;
        double f_start = NAN, f_end = NAN;
        memcpy(xp, x, sizeof(double) * n);
        if (sm) {
            f_start = f_end = orc_objective(P, x);
            if (P->stop_on && st->feas_ok && !isnan(st->f_last) &&
                fabs(f_start - st->f_last) / fmax(1.0, st->f_last) < P->stop_dobj) {
                st->stop_reason = ORC_STOP_SM; /* this iteration does not run */
                if (hist_f_start) hist_f_start[it] = NAN;
                continue;
            }
            f_end = perturbation_phase(P, x, st, f_start, g, v, z, &trials, &accepts);
        }
        double prox = feas_step(P, q, zc, x, r, c, y);
        if (hist_prox) hist_prox[it] = prox;
        if (hist_f_start) hist_f_start[it] = f_start;
        if (hist_f_end) hist_f_end[it] = f_end;
        if (hist_trials) hist_trials[it] = trials;
        if (hist_accepts) hist_accepts[it] = accepts;
        st->trials += trials;
        st->accepts += accepts;
        st->k += 1;
        if (P->stop_on) stop_after_step(P, st, sm, prox, f_start, xp, x);
    }
    free(r); free(c); free(y); free(g); free(v); free(z); free(xp);
    return 0;
}

int orc_run(const orc_problem *P, double *x, int64_t K, int32_t perturb, orc_state *st, double *hist_prox,
            double *hist_f_start, double *hist_f_end, int32_t *hist_trials, int32_t *hist_accepts)
{
    double *q = malloc(sizeof(double) * P->m), *zc = malloc(sizeof(double) * P->n);
    if (!q || !zc) {
        free(q); free(zc);
        return -2;
    }
    orc_prepare(P, q, zc);
    const int rc = orc_run_prepared(P, q, zc, x, K, perturb, st, hist_prox, hist_f_start, hist_f_end, hist_trials,
                                    hist_accepts);
    free(q); free(zc);
    return rc;
}

/*
 * Rounding of float32 values to bfloat16, round-to-nearest-even on the
 * float32 bit pattern (the upper 16 bits are kept).  Inputs are float32 values
 * held in doubles.
 */
void orc_round_bf16(const double *in, double *out, int64_t count)
{
    for (int64_t p = 0; p < count; ++p) {
        float f = (float)in[p];
        uint32_t u;
        memcpy(&u, &f, sizeof u);
        if ((u & 0x7f800000u) != 0x7f800000u) {
            uint32_t keep_lsb = (u >> 16) & 1u;
            u += 0x7fffu + keep_lsb;
        }
        u &= 0xffff0000u;
        memcpy(&f, &u, sizeof f);
        out[p] = (double)f;
    }
}

/*
 * Storage in IEEE binary16 after one global power-of-two scale s = 2^(14 - e),
 * e = ceil(log2(max |a|)), so the largest magnitude lands in (2^13, 2^14].
 * Each value a*s (exact, s a power of two) is rounded to the nearest binary16
 * value, ties to even, including the subnormal range (quantum 2^-24), and the
 * stored operator is that value divided by s.  Returns s (1 if all zero).
 */
double orc_round_f16_scaled(const double *in, double *out, int64_t count)
{
    double amax = 0.0;
    for (int64_t p = 0; p < count; ++p) amax = fmax(amax, fabs(in[p]));
    if (!(amax > 0.0)) {
        for (int64_t p = 0; p < count; ++p) out[p] = in[p];
        return 1.0;
    }
    int e;
    double mant = frexp(amax, &e); /* amax = mant * 2^e, mant in [0.5, 1) */
    int ce = (mant == 0.5) ? e - 1 : e; /* ceil(log2(amax)) */
    double s = ldexp(1.0, 14 - ce);
    for (int64_t p = 0; p < count; ++p) {
        double v = in[p] * s;
        double a = fabs(v);
        double quantum;
        if (a < ldexp(1.0, -14)) {
            quantum = ldexp(1.0, -24);
        } else {
            int ev;
            frexp(a, &ev); /* a in [2^(ev-1), 2^ev) */
            quantum = ldexp(1.0, (ev - 1) - 10);
        }
        double rq = nearbyint(v / quantum) * quantum; /* default mode: ties to even */
        out[p] = rq / s;
    }
    return s;
}
