/*
 * smx: superiorized simultaneous band+box projection on AMD MI355X (gfx950).
 *
 * C ABI of the HIP library libsmx.so.  Plain pointers and sizes only.
 *
 * Problem (paper, Section 2.1.1 and Section 2.3.3): find x in R^n with
 *     lower_i <= <a_i, x> <= upper_i   (i = 1..m, the rows of a sparse A)
 *     box_lo_j <= x_j <= box_hi_j
 * while reducing a secondary objective f (superiorization, Section 2.1.2).
 *
 * One feasibility step (the basic algorithm T) is the relaxed simultaneous
 * projection (eq. RelaxedProjection applied to the weighted combination of
 * the single-band projections of Section 2.1.1, with the weights of eq.
 * WeightedProximity), followed by the box projection (Section 2.3.3):
 *     r = A z,  t_i = clip(r_i, lower_i, upper_i) - r_i,
 *     x = clip( z + lambda * A^T (D t), box_lo, box_hi ),  D_i = w_i / ||a_i||^2.
 * One outer iteration of Algorithm 1 first perturbs x^k to z^k along
 * v = -grad f / ||grad f|| with power-law steps beta = gamma * alpha^ell, accepting
 * a trial only if it does not increase f, then applies T.
 *
 * Several right-hand sides ("slices", B of them) may share one A.  Every
 * per-slice vector is stored slice-interleaved: element j of slice s sits at
 * index j*B + s.
 *
 * Conventions:
 *   - Every call returns an int status (SMX_OK or a negative SMX_E* code) and
 *     never throws, aborts or exits; smx_last_error() describes the last failure
 *     on the calling thread.
 *   - "stream" arguments are hipStream_t values passed as void* (NULL means the
 *     null stream).  Work is enqueued asynchronously on the problem's stream.
 *   - Device pointers refer to memory on the device that is current when the
 *     object is created; an object must be used with that device current.
 *   - Distinct handles may be used from distinct threads concurrently; one
 *     handle must not be used by two threads at once.
 */
#ifndef SMX_H
#define SMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMX_VERSION_MAJOR 0
#define SMX_VERSION_MINOR 1

/* status codes */
#define SMX_OK 0
#define SMX_EINVAL (-1)   /* an argument is invalid; nothing was changed */
#define SMX_ENOMEM (-2)   /* device or host allocation failed, or a budget is exceeded */
#define SMX_EDEVICE (-3)  /* a HIP runtime call failed */
#define SMX_ESTATE (-4)   /* the call is not valid in the object's current state */
#define SMX_ENUMERIC (-5) /* a non-finite value was produced on the device */

/* storage of A's values (the indices are always exact) */
#define SMX_STORE_F32 0  /* float32 values */
#define SMX_STORE_BF16 1 /* bfloat16, round-to-nearest-even from float32 */
#define SMX_STORE_F16 2  /* binary16 after one global power-of-two scale */

/* secondary objectives f */
#define SMX_OBJ_NONE 0   /* feasibility only */
#define SMX_OBJ_SQNORM 1 /* f = ||x||^2, the L2 perturbation (Section 2.3.1) */
#define SMX_OBJ_TV2D 2   /* smoothed total variation of an R x C image (Section 2.3.1) */
#define SMX_OBJ_LINEAR 3 /* f = c^T x, e.g. summed dose (Section 2.3.3) */
#define SMX_OBJ_L1 4     /* f = ||x||_1, the L1 perturbation (Section 2.3.1); subgradient sign(x), 0 at 0 */

/* basic (feasibility-seeking) algorithms: the step T applied after the
 * perturbation (the appendix's table of methods; CQ from Section 2.1.1).  With
 * t_i = clip(<a_i,z>, l_i, u_i) - <a_i,z>, D = diag(w_i/||a_i||^2), W = diag(w_i):
 *   SIMULT  x = P_box(z + lambda A^T D t)              weighted simultaneous projection
 *   DROP    x = P_box(z + lambda Z A^T D t)            Z_j = 1/(nonzeros in column j)
 *   CQ      x = P_box(z + lambda A^T t / ||A||_F^2)    CQ with the Frobenius bound, C = the box
 *   EL      x = P_box(z + lambda sigma A^T D t)        sigma = t^T D t / ||A^T D t||^2
 *   EMR     x = P_box(z + lambda sigma y), y = A^T W t, sigma = ||y||^2 / sum_i w_i (A y)_i^2
 * (sigma = 0 when its denominator is 0).  The proximity is the same for all. */
#define SMX_BASIC_SIMULT 0
#define SMX_BASIC_DROP 1
#define SMX_BASIC_CQ 2
#define SMX_BASIC_EL 3
#define SMX_BASIC_EMR 4

/* perturbation step sizes (smx_problem_desc.step_rule) */
#define SMX_STEP_POWER 0
#define SMX_STEP_ADAPTIVE 1

/* launch form of the perturbation phase (smx_set_phase_form) */
#define SMX_PHASE_AUTO 0       /* one launch for short flat problems, else one launch per trial batch */
#define SMX_PHASE_ONE_LAUNCH 1 /* one launch per phase (squared norm, L1, linear; n <= 20,000) */
#define SMX_PHASE_BATCHES 2    /* a direction launch, trial launches, a closing launch */
#define SMX_PHASE_CLOSED_FORM 3 /* linear objective: a direction launch, then the trials in closed form */

/* smx_run flags */
#define SMX_RUN_PERTURB 1u /* run the perturbation phase of Algorithm 1 */
#define SMX_RUN_GRAPH 2u   /* replay captured HIP graphs of several iterations */

typedef struct smx_operator smx_operator;
typedef struct smx_problem smx_problem;

/* A sparse matrix in CSR form.  row_ptr[0] = 0, row_ptr non-decreasing,
 * row_ptr[m] = nnz, 0 <= col_idx < n, values finite.  Column indices within a
 * row need not be sorted; repeated (row, col) pairs are summed. */
typedef struct {
    int64_t m, n, nnz;
    const int32_t *row_ptr; /* m+1 */
    const int32_t *col_idx; /* nnz */
    const float *val;       /* nnz */
    int32_t on_device;      /* 0: host pointers, 1: device pointers */
} smx_csr;

/*
 * Dose-volume constraint (Section 2.3.3) on a structure whose voxels are the
 * rows [row_begin, row_end) of A, N = row_end - row_begin of them.
 * SMX_DVC_MAX (D_V <= dose): at most k = floor(fraction * N) rows may lie above
 * dose.  SMX_DVC_MIN (D_V >= dose): at least k = ceil(fraction * N) rows must
 * reach dose.  Such a constraint is a set in the output space of the split
 * problem (eq. Split); at every point its rows are ranked by <a_i, x> rounded
 * to float32, highest first, equal values by row index, and the nearest point
 * of the set gives the k highest rows the band (-inf, +inf) (MAX) or
 * [dose, +inf) (MIN) and the others (-inf, dose] (MAX) or (-inf, +inf) (MIN).
 * These bands take the place of the rows' lower/upper entries, which are
 * ignored; the rows otherwise take part in the step and the proximity like any
 * other row (weights, D, the basic algorithm).
 */
typedef struct {
    int64_t row_begin, row_end; /* 0 <= row_begin < row_end <= m */
    int32_t sense;              /* SMX_DVC_MAX or SMX_DVC_MIN */
    int32_t reserved;           /* 0 */
    double fraction;            /* V, in [0, 1] */
    double dose;                /* d, finite */
} smx_dvc;

#define SMX_DVC_MAX 0
#define SMX_DVC_MIN 1
#define SMX_MAX_DVC 16 /* constraints per problem */

/* Everything about one problem except A.  All arrays are copied at creation. */
typedef struct {
    int32_t B;               /* slices sharing A: a power of two, 1..32 */
    const float *lower;      /* m*B, slice-interleaved; -INFINITY allowed */
    const float *upper;      /* m*B; +INFINITY allowed; lower <= upper */
    const double *weights;   /* m, > 0 (normalised to sum 1 here), or NULL for 1/m */
    const float *box_lo;     /* n, or NULL for -INFINITY */
    const float *box_hi;     /* n, or NULL for +INFINITY; box_lo <= box_hi */
    double lambda;           /* relaxation parameter, 0 < lambda <= 2 (DROP:
                                0 < lambda <= 2 / max_i w_i with the weights
                                normalised to sum 1) */
    int32_t obj_kind;        /* SMX_OBJ_* */
    int32_t tv_rows, tv_cols; /* SMX_OBJ_TV2D: image shape, rows*cols = n,
                                pixel (i,j) is unknown i*tv_cols + j */
    double tv_eps;           /* SMX_OBJ_TV2D smoothing, >= 0 */
    const float *linear_c;   /* SMX_OBJ_LINEAR: c, n entries, nonzero */
    double gamma;            /* step kernel, > 0 */
    double alpha;            /* step ratio, 0 < alpha < 1 */
    int32_t n_red;           /* reduction steps per perturbation phase, >= 1 */
    int32_t restart_every;   /* restart ell every this many iterations; 0: never */
    int32_t max_trials;      /* trial cap per reduction step, 1..1024 */
    int32_t refine_iters;    /* low-precision operators only: the last iterations
                                of every smx_run use the float32 operator;
                                -1 means ceil(K/20) */
    int32_t history_cap;     /* per-iteration records kept (0: none) */
    int32_t on_device;       /* 0: the arrays above are host pointers, 1: device */
    int32_t basic;           /* SMX_BASIC_*; SMX_BASIC_SIMULT (0) is the default */
    /* Stopping rules, checked on the device after every iteration (a stopped
     * slice stays idle; smx_run still returns after its K iterations).
     * Section 2.2.1: the proximity P of the iteration <= stop_prox, or the
     * relative change |P^{k+1} - P^k| / max{1, P^k} < stop_dprox for stop_n
     * consecutive iterations, or stop_max_iters iterations (0: none).  A
     * perturbed run with an objective (Section 2.2.3) stops instead when one
     * of the two proximity rules held at the last iteration and the objective
     * change |f(x^{k+1}) - f(x^k)| / max{1, f(x^k)} < stop_dobj; it is checked
     * when the next perturbation phase opens.  stop_var > 0 adds the rule of
     * Section 2.3.2: the sample variance of omega_i = ||x^i - x^{i-1}|| /
     * ||x^i|| over the run falls below stop_var. */
    int32_t stop_on;         /* 0: no stopping rule */
    int32_t stop_n;          /* N >= 1 */
    int64_t stop_max_iters;  /* >= 0 */
    double stop_prox;        /* P* */
    double stop_dprox;       /* Delta P* */
    double stop_dobj;        /* Delta f* */
    double stop_var;         /* >= 0; 0 disables the variance rule */
    /* Dose-volume constraints (host array of n_dvc entries, 0..SMX_MAX_DVC):
     * their row blocks follow one another (dvc[g+1].row_begin ==
     * dvc[g].row_end).  A problem with any runs the two passes (never the
     * fused pass). */
    int32_t n_dvc;
    int32_t reserved_dvc;    /* 0 */
    const smx_dvc *dvc;
    /* Step size of the perturbation phase (Section 2.1.2): SMX_STEP_POWER, the
     * power law gamma alpha^ell of Algorithm 1; or SMX_STEP_ADAPTIVE, the
     * subgradient-projection step beta_k = (f(x^k) - f_ref) / ||g(x^k)|| when
     * f(x^k) > f_ref and no step otherwise, where f_ref is the objective value
     * at which the previous perturbation phase ended (f(x^0) before the first
     * phase, so the first iteration does not perturb).  The adaptive phase
     * tries that one step along v = -g/||g|| and keeps it when f does not
     * increase (n_red, max_trials, gamma and alpha do not apply; ell counts
     * the trial). */
    int32_t step_rule;
    int32_t reserved_step;   /* 0 */
} smx_problem_desc;

/* Per-slice iteration state, as checkpointed by smx_get_state. */
typedef struct {
    int64_t k;        /* outer iterations completed */
    int64_t ell;      /* exponent of the next power-law trial step */
    int64_t restarts; /* restarts so far */
    int64_t trials;   /* trial points evaluated, total */
    int64_t accepts;  /* trial points accepted, total */
    int64_t cap_hits; /* reduction steps that reached max_trials */
    /* stopping-rule bookkeeping (restored by smx_set_state, so a resumed run
     * stops where an uninterrupted one would) */
    int32_t stop_reason; /* SMX_STOP_*; 0 while the slice runs */
    int32_t dp_run;      /* consecutive iterations with a small proximity change */
    int32_t feas_ok;     /* a proximity rule held at the last iteration */
    int32_t reserved;
    double p_last;       /* proximity recorded at the last iteration (NaN before the first) */
    double f_last;       /* f(x^k) of the last perturbation phase (NaN if none) */
    double var_n, var_mean, var_m2; /* running count, mean and squared deviations of
                                       the relative iterate changes */
    double f_ref;        /* f where the last perturbation phase ended (NaN before the
                            first): the adaptive step's reference value */
} smx_slice_state;

/* why a slice stopped (smx_stop_status) */
#define SMX_STOP_NONE 0
#define SMX_STOP_PROX 1  /* proximity <= stop_prox */
#define SMX_STOP_DPROX 2 /* relative proximity change < stop_dprox for stop_n iterations */
#define SMX_STOP_MAXIT 3 /* stop_max_iters iterations */
#define SMX_STOP_VAR 4   /* variance of the relative iterate changes < stop_var */
#define SMX_STOP_SM 5    /* superiorized: a proximity rule and objective change < stop_dobj */

/* Library version.  Both pointers must be non-NULL. */
int smx_version(int *major, int *minor);

/* Measurement aid, not a step of the method: one read-only pass over bytes
 * of device memory at buf (16-byte aligned, a positive multiple of 16 bytes)
 * by grid workgroups of 256 threads, each thread reading 16-byte words four
 * at a time and each workgroup storing the float sum of what it read into
 * partials[grid] (device memory, caller-owned).  Enqueued on stream (NULL:
 * the default stream), no synchronisation: timing it with events around the
 * call gives the rate at which a kernel that only reads HBM moves bytes on
 * this device, the ceiling the passes' achieved bandwidth is compared with.
 * Errors: SMX_EINVAL for NULL pointers, a misaligned or empty buffer, or grid
 * outside 1..65535; SMX_EDEVICE for a launch failure. */
int smx_read_rate_probe(const void *buf, size_t bytes, float *partials, int32_t grid, void *stream);

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next smx_* call on this thread. */
const char *smx_last_error(void);

/*
 * Create an operator from A: deep-copies the CSR (host or device input) into
 * library-owned device buffers laid out for the kernels (row-aligned CSR and a
 * column-major copy for A^T), computes the float64 row norms ||a_i||^2 from the
 * stored values, and, for SMX_STORE_BF16/F16, a reduced-precision copy.  With
 * keep_f32 != 0 a reduced-precision operator also keeps the float32 copy used
 * by refinement iterations.  A reduced-precision layout whose index range fits
 * in 16 bits (the CSR when n <= 65536, the column copy when m <= 65536) is
 * also held packed: each entry one 32-bit word, value in the low half and
 * index in the high half; the passes read that copy, 4 bytes per entry.
 * The caller may free its buffers on return.
 * Errors: SMX_EINVAL for m or n < 1, no nonzeros at all (nnz = 0: every band
 * would be the constant 0), nnz != row_ptr[m], a decreasing row_ptr,
 * a column index outside [0,n), a non-finite value, or sizes beyond 2^31-1
 * entries; SMX_ENOMEM when device memory runs out (nothing is leaked).
 */
int smx_operator_create(const smx_csr *A, int32_t value_storage, int32_t keep_f32, void *stream,
                        smx_operator **out);

/*
 * smx_operator_create for an operator whose unknowns are the pixels of an
 * image_rows x image_cols image (pixel (i, j) is unknown i * image_cols + j;
 * image_rows * image_cols must equal n).  Beside the layouts above, the
 * library groups A's columns by 8 x 8 pixel tiles with each tile's rows listed
 * once: a ray crosses several pixels of a tile, so the transposed product
 * stages the tile's rows of the residual in LDS and gathers from there.  One-
 * slice problems on such an operator use that layout for A^T when it is the
 * faster one (smx_autotune times both).  Errors as smx_operator_create, and
 * SMX_EINVAL when the image does not match n.  A tile touching more than 16384
 * rows leaves the operator without the tile layout (not an error).
 */
int smx_operator_create_image(const smx_csr *A, int32_t value_storage, int32_t keep_f32, int32_t image_rows,
                              int32_t image_cols, void *stream, smx_operator **out);

/* Release an operator once every problem created from it is destroyed
 * (operators are reference counted).  NULL is accepted. */
int smx_operator_destroy(smx_operator *op);

/* Free an operator's row-panel layout of the column copy (operators with
 * more than 40,448 rows build it for the one-slice row-panel pass 2: offsets
 * of every column in every panel, and for rows past 16 bits a copy of the
 * rows as 16-bit offsets within their panel, packed beside reduced-precision
 * values) for callers whose problems will not use that pass: multi-slice
 * problems never do, one-slice problems choose the fused pass or the column
 * pass without it.  On the radiotherapy operator with bf16 values that is
 * about 2.4 GB.  Problems created afterwards simply lack the panel pass.
 * Errors: SMX_EINVAL for NULL, SMX_ESTATE while any problem created from the
 * operator exists (it may be using the layout).  SMX_OK when there is no
 * layout to free. */
int smx_operator_release_panels(smx_operator *op);

/* Device bytes the operator would take for A of this shape and storage,
 * without allocating anything (an upper bound: row and column padding is
 * counted at its maximum). */
int smx_operator_footprint(int64_t m, int64_t n, int64_t nnz, int32_t value_storage, int32_t keep_f32,
                           size_t *bytes);

/*
 * Device bytes, without allocating anything, of an operator of this shape and
 * storage (*operator_bytes, an upper bound as smx_operator_footprint's; with
 * image_rows x image_cols = n, of the image operator smx_operator_create_image
 * makes, tile layout included; 0 x 0 for a plain operator) and of
 * a problem with this descriptor on it (*problem_bytes: exactly what
 * smx_problem_create allocates on the current device -- bands, box, weights,
 * iterate, gradient, residual, states, D, step weights, the extrapolated
 * steps' y, the dose-volume buffers, the fused pass's partial vectors, the
 * panel pass's per-panel sums, every kernel's per-workgroup partials and the
 * history -- summed from the plan the creation allocates by).  desc may be
 * NULL (*problem_bytes = 0); its arrays are not read.  Not counted:
 * smx_autotune's temporary copies of the iterate, residual and states, and
 * captured graphs.  Used for admission by HBM footprint (the serving pattern).
 * Errors: SMX_EINVAL for a NULL output, an invalid shape or storage, or an
 * invalid descriptor field the sizes depend on (B, basic algorithm,
 * objective, TV image, max_trials, history_cap, dose-volume table), or an
 * image that does not match n.
 */
int smx_footprint(int64_t m, int64_t n, int64_t nnz, int32_t value_storage, int32_t keep_f32, int32_t image_rows,
                  int32_t image_cols, const smx_problem_desc *desc, size_t *operator_bytes, size_t *problem_bytes);

/*
 * Create a problem on an operator.  Validates and copies the descriptor's
 * arrays; sets x to 0 for every slice and the iteration state to k = ell =
 * restarts = 0.  Errors (SMX_EINVAL): B not a power of two in 1..32, any
 * lower > upper or NaN bound, a weight <= 0 or non-finite, box_lo > box_hi,
 * lambda outside its range, an unknown basic algorithm, gamma <= 0, alpha
 * outside (0,1), n_red < 1, max_trials outside 1..1024, TV with rows*cols !=
 * n, LINEAR with a NULL c, dose-volume constraints whose row blocks are empty,
 * outside [0, m) or not consecutive, whose fraction is outside [0, 1], whose
 * dose is not finite or whose sense is unknown.  EL and EMR keep y (n*B
 * doubles) and apply the step after it is complete (with the fused pass, its
 * apply kernel keeps y instead of moving x); EMR adds a pass over A per
 * iteration for sum_i w_i (A y)_i^2.
 */
int smx_problem_create(smx_operator *op, const smx_problem_desc *desc, void *stream, smx_problem **out);

/* Destroy a problem (waits for its stream).  NULL is accepted. */
int smx_problem_destroy(smx_problem *p);

/* Convenience: operator plus problem in one call; the problem owns the
 * operator's only reference. */
int smx_create(const smx_csr *A, int32_t value_storage, const smx_problem_desc *desc, void *stream,
               smx_problem **out);

/* Change the stream later work of this problem is enqueued on. */
int smx_set_stream(smx_problem *p, void *stream);

/* Copy the iterate in (n*B floats, slice-interleaved; host or device).  Also
 * resets no state: use smx_set_state for that. */
int smx_set_x(smx_problem *p, const float *x, int32_t on_device);

/* Copy the iterate out (n*B floats).  Synchronises for host output. */
int smx_get_x(smx_problem *p, float *out, int32_t on_device);

/*
 * Enqueue K outer iterations (Algorithm 1 with SMX_RUN_PERTURB and an
 * objective, else K feasibility steps).  With a reduced-precision operator the
 * last refine_iters of the K iterations use the float32 operator.
 * SMX_RUN_GRAPH replays captured graphs of several iterations.
 * Asynchronous; returns SMX_EINVAL for K < 0.
 */
int smx_run(smx_problem *p, int32_t K, uint32_t flags);

/* Wait for the problem's stream.  Returns SMX_ENUMERIC if a non-finite
 * proximity or objective was produced since the last check. */
int smx_sync(smx_problem *p);

/* Proximity 1/2 sum_i w_i ||P_i(x) - x||^2 (eq. WeightedProximity) and the
 * objective f at the current x, one double per slice each (either may be
 * NULL).  Synchronises. */
int smx_query(smx_problem *p, double *proximity, double *objective);

/* Per-iteration records of the first min(k, history_cap) iterations, each
 * [iteration][slice] (row-major, B per iteration): proximity at the point the
 * feasibility step acted on, objective at x^k and after the perturbation phase
 * (NaN when no phase ran), trials and accepted trials.  Any pointer may be
 * NULL.  *n_out receives the number of iterations written (<= cap). */
int smx_get_history(smx_problem *p, double *prox, double *f_start, double *f_end, int32_t *trials,
                    int32_t *accepts, int32_t cap, int32_t *n_out);

/* Checkpoint: the per-slice states (B entries) and the iterate (n*B floats,
 * host).  smx_set_state restores both exactly. */
int smx_get_state(smx_problem *p, smx_slice_state *states, float *x);
int smx_set_state(smx_problem *p, const smx_slice_state *states, const float *x);

/* Shape of the problem. */
int smx_problem_dims(const smx_problem *p, int64_t *m, int64_t *n, int64_t *nnz, int32_t *B);

/*
 * Slots (serving): the B slices of a problem are independent slots sharing
 * the operator.  smx_slot_load copies one slot's bands (m floats each) and
 * starting point (n floats; host or device) into slot `slot`, resets its
 * state (k = ell = restarts = 0, counters 0) and lets it run `budget` more
 * iterations: later smx_run calls advance it until its k reaches budget, then
 * leave it untouched.  budget = 0 loads the data and keeps the slot idle.
 * Errors: slot outside [0,B), lower > upper, NaN bounds -> SMX_EINVAL.
 * The copies are ordered on the problem's stream; smx_slot_load returns after
 * they complete.  A slot's results do not depend on the other slots.
 */
int smx_slot_load(smx_problem *p, int32_t slot, const float *lower, const float *upper, const float *x0,
                  int32_t on_device, int64_t budget);

/*
 * smx_slot_load without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the staging of the slot's bands and starting point
 * (2m + n floats, which smx_slot_load allocates per call) and the flags of
 * their validation live in a fixed 32 MiB scratch array inside the library,
 * one per device, resident from the first smx_problem_create on that device
 * until the process ends.  Arguments,
 * results and errors as smx_slot_load (host or device input, copied in order
 * on the problem's stream; returns after the copies complete), and
 * SMX_EINVAL, with nothing changed, when 256 + 4(2m + n) bytes (each part
 * rounded up to 256) exceed the scratch: 2m + n up to about 8.39M floats.
 * Bounds are checked on the device after staging; an invalid slot is
 * reported before anything in the problem changes.  Every call on a device
 * shares that device's scratch and leaves its contents there: calls that
 * overlap on one device (from several threads) race.
 */
int smx_slot_load_noalloc(smx_problem *p, int32_t slot, const float *lower, const float *upper, const float *x0,
                          int32_t on_device, int64_t budget);

/* Stop advancing a slot (its iterate and state stay as they are). */
int smx_slot_disable(smx_problem *p, int32_t slot);

/* Per-slot iterations completed (k[B]) and whether the slot still runs
 * (live[B]); either may be NULL.  Synchronises. */
int smx_slot_status(smx_problem *p, int64_t *k, int32_t *live);

/* One slot's iterate (n floats) to host or device memory. */
int smx_slot_get_x(smx_problem *p, int32_t slot, float *out, int32_t on_device);

/* Autotuner (batching pattern): times candidate launch shapes of both passes
 * (row blocks streamed through LDS, or 8..64 lanes per row with 4 or 8
 * entries per load, at several grid sizes) on this problem's operator, `reps`
 * launches each, and keeps the fastest for later runs.  Runs on scratch
 * copies, so the iterate, state and history are unchanged.  Synchronises.
 * Results do not depend on the shape beyond float64 summation order.  With
 * the environment variable SMX_TUNE_LOG=1 each candidate's mean time is
 * printed to stderr.
 *
 * Other environment variables, read when an operator or problem is created
 * (they pick starting shapes; smx_autotune may replace them):
 *   SMX_PASS_MODE=rows|interleaved  lanes-per-row passes / interleaved-lane
 *                                   pass 1 (one slice)
 *   SMX_PASS_MODE=lds               both passes with the gathered vector's
 *                                   first 40,448 entries in LDS (one slice)
 *   SMX_PASS_MODE=panels            pass 2 in row panels of 40,448 rows, each
 *                                   panel's residual in LDS (one slice,
 *                                   m > 40,448)
 *   SMX_TILES=0|1                   image operators: never use the tile pass 2,
 *                                   or start every problem whose tiles fit on it
 *   SMX_TILE=4|8|16                 image operators: tile edge (default 8) */
int smx_autotune(smx_problem *p, int32_t reps);

/* Fused single pass for one-slice problems (B = 1).  The two passes of a
 * feasibility step read the same entries, so when an LDS copy of y = A^T c
 * fits on a CU (n up to about 20k unknowns in float64, 40k in float32) one
 * pass over the CSR forms c and adds c_i a_i into per-workgroup copies of y,
 * reading A once per iteration instead of twice; a small kernel sums the
 * copies and applies the box.
 *   mode 1 (the default): use the fused pass where it is available (the
 *          autotuner may still keep the two passes when they time faster);
 *   mode 0: always the two passes.
 * The two passes add in a fixed order, so repeated runs, graph replays and
 * checkpoint/resume are bitwise reproducible.  The fused pass adds into LDS
 * with atomics, so its results are reproducible up to float64 summation
 * order only.  Errors: SMX_EINVAL for another mode.  SMX_OK also where no
 * fused pass is available (mode 1 then changes nothing). */
int smx_set_fused(smx_problem *p, int32_t mode);

/* Launch form of the perturbation phase of Algorithm 1 (Section 2.1.2: the
 * normalised negative (sub)gradient, the trial steps with the nonascent test,
 * n_red reduction steps).  The phase is a chain of reductions over x: the
 * direction's norm and f(x^k), then f at each batch of trial points.
 *   SMX_PHASE_BATCHES: a direction launch, trial launches over the whole
 *     device (one for a short first batch of each reduction step, one for the
 *     rest up to the trial cap), a closing launch;
 *   SMX_PHASE_ONE_LAUNCH: the whole phase in one workgroup per slice, x and
 *     the direction in its LDS, trials in batches of 8 (squared norm, L1 and
 *     linear objectives, n <= 20,000);
 *   SMX_PHASE_CLOSED_FORM (linear objective f = c^T x): the direction
 *     launch (f(x^k), ||c||), then one launch in which every workgroup takes
 *     each trial's value from f(x + t v) = f(x) - t ||c|| (v = -c/||c||), so
 *     no trial needs a pass over x, and adds the accepted step.  On the
 *     fused pass (not EL or EMR) the previous iteration's apply kernel
 *     leaves the direction's partial sums, so the direction launch goes;
 *     with z in LDS the pass itself opens the phase and stages
 *     z = x + s v, and the phase takes no launch of its own;
 *   SMX_PHASE_AUTO (the default): ONE_LAUNCH for those objectives up to
 *     n = 8,192 (there the chain of launches, not the arithmetic, sets the
 *     phase's time; one workgroup reads x at one compute unit's rate, so on
 *     longer vectors it is no faster than the chain), else CLOSED_FORM for
 *     the linear objective, else BATCHES.
 * Every form accepts the same trial (the first acceptable one in order) and
 * keeps the same state; they differ in the order of the float64 sums of f
 * (and CLOSED_FORM in taking a trial's value from the identity), so a
 * decision taken within rounding of the acceptance threshold can differ
 * between them.  Errors: SMX_EINVAL for another form, SMX_ESTATE for
 * ONE_LAUNCH on an objective or size it does not take or CLOSED_FORM on
 * another objective. */
int smx_set_phase_form(smx_problem *p, int32_t form);

/* Pin the launch shape of the fused pass instead of the default or the
 * autotuner's choice: lanes per row (8, 16, 32), entries per load (4, 8) and
 * cap: 0 to read a row's entries again for the scatter, or 256/(lpr*vec) (16
 * or 32 lanes only) to keep 256 entries of each row in registers.  With
 * z_in_lds != 0 (problems whose n is at most about 20k): every workgroup
 * first copies the whole point z into LDS beside a float32 copy of y and
 * gathers from there instead of from memory; cap is then 0 or 16/vec (each
 * lane keeps 16 entries of its row in registers for the scatter).
 * Results do not depend on the shape beyond floating-point summation order.
 * Errors: SMX_ESTATE when the problem has no fused pass, SMX_EINVAL for
 * another shape. */
int smx_set_fused_shape(smx_problem *p, int32_t lpr, int32_t vec, int32_t cap, int32_t z_in_lds);

/* Why each slice stopped (reason[B], SMX_STOP_*; 0 while it runs).
 * Synchronises. */
int smx_stop_status(smx_problem *p, int32_t *reason);

/* JSON description of the launch shapes in use, of the device bytes the
 * problem ("device_bytes") and its operator ("operator_bytes") hold and of
 * the launches one perturbation phase takes ("phase_launches")
 * (NUL-terminated, truncated to cap bytes); *need (if non-NULL) receives the
 * full size. */
int smx_describe(const smx_problem *p, char *buf, size_t cap, size_t *need);

/* Mean device time (milliseconds) per launch of the two passes (with the
 * fused pass: of the fused pass and of its apply kernel) recorded by the last
 * smx_run made with SMX_RUN_GRAPH clear and timing enabled through
 * smx_set_timing; zero launches give 0. */
int smx_set_timing(smx_problem *p, int32_t enable);
int smx_get_timing(smx_problem *p, double *pass1_ms, double *pass2_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* SMX_H */
