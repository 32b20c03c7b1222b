// Internal declarations shared by the kernels and the host runtime of libsmx.
// Not part of the public ABI (include/smx.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace smx {

constexpr int kBlock = 256;    // threads per workgroup for every kernel (4 waves of 64)
constexpr int kRowAlign = 8;   // entries of every row/column start at a multiple of this
constexpr int kTrialChunk = 32; // trial steps evaluated (and their totals read) per register batch
constexpr int kFirstWidth = 8;  // least width of the first trial batch of a reduction step
constexpr int kTrialBlock = 1024; // threads of a TV trial workgroup (one 16 x 16 tile)
constexpr int kTile = 16;      // TV tile edge (kTile*kTile = kBlock)
constexpr int kFusedBlock = 1024; // threads of a fused-pass workgroup (one per CU: its LDS holds y)
constexpr int kFusedRcBlock = 512; // the same for the register-cached fused pass
constexpr int kSmallPhaseBlock = 1024; // threads of the one-launch perturbation phase (one workgroup per slice)
constexpr int kSmallPhaseMaxN = 20000; // longest x it takes (x and the direction in LDS, 8 bytes an entry)
constexpr int kSmallPhaseAutoN = 8192; // longest x it is the default for
constexpr int kSmallTrials = 8;        // trials per batch there
constexpr int kApplyBlock = 1024;  // threads of the fused pass's apply kernel (16 waves share a column's partials)

// Stored formats of A's entries.  The packed kinds hold one 32-bit word per
// entry: the 16-bit value in the low half, a 16-bit index in the high half
// (used when the layout's index range fits in 16 bits).
// VK_F32U16: float32 values beside a uint16 index array (a layout whose
// index range fits in 16 bits, one-slice passes).
enum ValKind : int { VK_F32 = 0, VK_BF16 = 1, VK_F16 = 2, VK_BF16P = 3, VK_F16P = 4, VK_F32U16 = 5 };
enum ObjKind : int { OBJ_NONE = 0, OBJ_SQNORM = 1, OBJ_TV2D = 2, OBJ_LINEAR = 3, OBJ_L1 = 4 };

// Device view of one row-aligned sparse layout: the CSR of A (pass 1) or the
// CSR of A^T (pass 2).  Row r owns entries [ptr[r], ptr[r+1]); both ends are
// multiples of kRowAlign, padding entries hold value 0 and a valid index.
struct SpView {
    const int32_t *ptr;
    const int32_t *idx;
    const void *val; // float, bf16 bits (uint16), binary16, or packed words, by ValKind
    int64_t rows;
    float vscale_inv; // operator value = stored value * vscale_inv
};

// Per-slice iteration state, resident on the device.  Only the one-workgroup
// kernels (phase opening, trial decision, end of iteration) write it.
struct SliceState {
    double f_cur;   // objective at the current point of the perturbation phase
    double f_start; // objective at x^k (NaN when no phase ran this iteration)
    double gn;      // norm of the gradient of this phase
    double s_acc;   // accepted step length along v in this phase (z = x + s_acc v)
    double prox;    // proximity at the last feasibility step's input point
    long long k;      // outer iterations completed
    long long k_end;  // iterations stop advancing here (budget)
    long long ell;    // exponent of the next trial step
    long long restarts;
    long long trials;   // totals
    long long accepts;
    long long cap_hits;
    int n_done;     // reduction steps completed in this phase
    int phase;      // 1 while the phase is still trying
    int step_tried; // trials spent in the current reduction step
    int trials_it;  // this iteration
    int accepts_it;
    int live;       // the current iteration runs (enabled and k < k_end)
    int applied;    // the accepted step of this phase has been added to x
    int enabled;    // slice participates at all
    int nonfinite;  // a non-finite proximity or objective was seen
    int need_last;  // trials the last completed reduction step used (sizes the next first batch)
    // stopping rules (stop_on = 0: run the iterations asked for)
    int stop_on, stop_n, stop_reason; // reason: STOP_* once stopped (the slice then stays idle)
    int dp_run;                       // consecutive iterations with a small proximity change
    int feas_ok;                      // a proximity rule held at the last iteration (superiorized runs)
    int ran;                          // the slice ran the iteration that just ended
    long long stop_max;               // iteration cap (0: none)
    double stop_prox, stop_dprox, stop_dobj, stop_var;
    double p_last, f_last;            // last recorded proximity; f(x^k) of the last phase
    double var_n, var_mean, var_m2;   // running statistics of the relative iterate changes
    double f_ref;   // f where the last perturbation phase ended (NaN before the first): the adaptive step's reference
    double beta_ad; // the adaptive step of the current phase
};

enum StopReason : int { STOP_NONE = 0, STOP_PROX = 1, STOP_DPROX = 2, STOP_MAXIT = 3, STOP_VAR = 4, STOP_SM = 5 };

// Stopping-rule parameters given at problem creation.
struct StopParams {
    int on, n;
    long long max_iters;
    double prox, dprox, dobj, var;
};

struct PertParams {
    int obj;
    int B;
    long long n;
    int tv_rows, tv_cols;
    double tv_eps2;
    double gamma, alpha;
    int n_red, restart_every, max_trials;
    int first_width; // trials evaluated by a trial launch that starts a reduction step
    int adaptive;    // 1: the adaptive step (one trial per phase, beta from the state); 0: the power law
};

// The linear objective's perturbation phase taken inside the fused pass with
// z in LDS (one slice): the direction partials the last apply kernel left
// (sum c_j^2 and sum c_j x_j per workgroup), and the state buffer the phase's
// state goes to.  c == nullptr: no phase in the pass.
struct LinPhase {
    const float *c;
    const double *part;
    int nparts;
    SliceState *st_out;
    PertParams pp;
};

struct Hist {
    double *prox;
    double *f_start;
    double *f_end;
    int *trials;
    int *accepts;
    long long cap;
};

constexpr int kStreamEntries = 2048; // entries per row block of the streaming pass kernels

struct PassCfg {
    int mode; // 0: a group of lpr lanes per row; 1: row blocks streamed through LDS;
              // 2: (pass 2 of an image operator) image tiles, lpr lanes per column;
              // 3: (one slice) lpr lanes per row, the gathered vector's first xlds
              //    entries staged in LDS by every workgroup (one per CU);
              // 5: (pass 2, one slice) the column copy in row panels, each
              //    panel's rows of c staged in LDS
    int lpr;  // lanes per row (mode 0): 2, 4, 8, 16, 32 or 64
    int vec;  // entries per lane per load: 4 or 8
    int grid; // workgroups
    int xlds = 0; // mode 3: entries of the gathered vector held in LDS (<= kLdsPassFloats)
};

constexpr int kLdsPassBlock = 1024;   // threads of an LDS-staged pass workgroup
constexpr int kLdsPassFloats = 40448; // its LDS copy of the gathered vector (158 KB)

// Row weights of pass 1: c_i = S_i t_i and the proximity term D_i t_i^2 (S = D
// for the weighted simultaneous step; 1/||A||_F^2 for CQ; w for the
// error-minimising step).  In quadratic-form mode the gathered vector is y
// and the only output is the partial of sum_i S_i (A y)_i^2.
struct RowW {
    const float *D;
    const float *S;
    int qform;
    // rows [dose_lo, dose_hi), the dose-volume rows, only store r = <a_i, z>
    // (float64) into dose[(i - dose_lo) * B + s]: their bands are set after
    // the pass (NULL: no such rows)
    double *dose;
    long long dose_lo, dose_hi;
};

// ---- dose-volume constraints ----
// A constraint's rows are ranked by a 64-bit key: the order-preserving bits of
// the float32-rounded value in the high half, the complement of the row's
// position in its block in the low half (equal values rank by row), so keys are
// unique.  The k-th highest key is found by a radix select over 11-bit digits
// (at most six rounds: shifts 53, 42, 31, 20, 9 and a last 9-bit digit), one
// launch per round; a round's last workgroup of a constraint picks the digit.
constexpr int kMaxDvc = 16;
constexpr int kDvcChunk = 2048; // rows per workgroup of the selection and band kernels
constexpr int kDvcBins = 2048;  // 11-bit digits
constexpr int kDvcRounds = 6;

struct DvcTable {
    int n;                       // constraints
    int nblk;                    // workgroups per slice over all constraints
    long long lo, span;          // rows [lo, lo + span) hold every constraint
    long long begin[kMaxDvc], end[kMaxDvc];
    long long k[kMaxDvc];        // rows ranked "high": floor(V N) (MAX) or ceil(V N) (MIN)
    double dose[kMaxDvc];
    int sense[kMaxDvc];          // 0: at most k above dose, 1: at least k at or above dose
    int blk_begin[kMaxDvc + 1];  // workgroups [blk_begin[g], blk_begin[g+1]) cover constraint g
};

// Selection state of one constraint and slice.
struct DvcSel {
    unsigned long long prefix; // digits fixed so far
    unsigned long long thr;    // mode 2: rows with key >= thr rank high
    long long krem;            // rank still to find below the prefix
    int mode;                  // 0: searching, 1: no row ranks high, 2: threshold, 3: every row ranks high
    int pad;
};

// Column step of pass 2 (and of the fused pass's apply kernel):
// x = clip(z + lambda * zcol_j * y_j, lo, hi) (zcol NULL: factor 1), or, when
// defer != 0, y itself into ybuf (float64; also rounded into ybuf32 when that
// is not NULL, the vector EMR's second product gathers) with per-workgroup
// partials of ||y||^2 in ypart (the extrapolated steps apply x in
// k_step_apply).
struct ColStep {
    const float *lo, *hi;
    float lambda;
    const float *zcol;
    double *ybuf;
    float *ybuf32;
    double *ypart;
    int defer;
};

// Launch shape of the fused single pass (one slice).
struct FusedCfg {
    int lpr;   // lanes per row: 8, 16 or 32
    int vec;   // entries per lane per load: 4 or 8
    int cap;   // 0: entries re-read for the scatter; else chunks per lane kept in
               // registers (cap * lpr * vec = 256 entries; with zl, 16 a lane)
    int grid;  // workgroups, each with an LDS copy of y
    int acc64; // 1: float64 LDS accumulators, 0: float32
    int zl = 0; // 1: z staged in LDS beside a float32 y (k_fused_zl, k_fused_zlr; acc64 = 0)
};

// Column layout grouped by image tiles (A^T for an operator whose unknowns
// are the pixels of an image): tile t owns the columns tcol[pptr[t] ..
// pptr[t+1]) (its pixels, in row order inside the tile) and the rows
// rlist[rptr[t] .. rptr[t+1]) that touch them (ascending).  A is the CSR of
// the tile columns in that order, whose indices are 16-bit positions in the
// tile's row list: a float32 copy (values beside a uint16 index array) and/or
// packed 16-bit words.  Rays crossing a tile touch many of its pixels, so the
// pass stages the tile's rows of c in LDS once and gathers from there.
struct TileView {
    SpView A;
    const int32_t *tcol;
    const int32_t *pptr;
    const int32_t *rptr;
    const int32_t *rlist;
    int ntiles;
    int max_rows; // most rows of one tile (LDS floats the pass needs)
};

// Row blocks of a row-aligned layout for the streaming kernels: block b holds
// rows [rb[b], rb[b+1]), at most kBlock rows and at most kStreamEntries
// entries, or a single longer row.
struct RowBlocks {
    const int32_t *rb;
    int nblk;
};

// ---- launchers (kernels.hip) ----
hipError_t launch_rownorm(const SpView &A, int vk, double *q, hipStream_t s);
hipError_t launch_make_D(const double *q, const double *w, float *D, int64_t m, hipStream_t s);
hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t count, hipStream_t s);
hipError_t launch_to_f16(const float *src, uint16_t *dst, int64_t count, float scale, hipStream_t s);
hipError_t launch_pack16u(const uint16_t *val16, const uint16_t *idx16, uint32_t *packed, int64_t count, hipStream_t s);
hipError_t launch_pack16(const uint16_t *val16, const int32_t *idx, uint32_t *packed, int64_t count, hipStream_t s);
hipError_t launch_init_state(SliceState *st, int B, StopParams sp, hipStream_t s);
// the variance rule: xprev = x at the start of an iteration; after it,
// per-workgroup partials of ||x - xprev||^2 and ||x||^2 (norms) and, in one
// workgroup, the running variance of their ratio and the stop decision
hipError_t launch_copy(float *dst, const float *src, int64_t count, hipStream_t s);
hipError_t launch_iter_norms(const float *x, const float *xprev, int64_t n, int B, double *partials, int *nparts,
                             hipStream_t s);
hipError_t launch_stop_var(SliceState *st, int B, const double *partials, int nparts, hipStream_t s);
hipError_t launch_fill(float *p, float v, int64_t count, hipStream_t s);
// slots of a multi-slice problem (serving)
hipError_t launch_put_column(float *dst, const float *src, int64_t rows, int B, int slot, hipStream_t s);
hipError_t launch_get_column(float *dst, const float *src, int64_t rows, int B, int slot, hipStream_t s);
// flag[0..1] = {bit 0: a NaN bound, bit 1: lower > upper; the lowest such row}
// for m staged bands (flag is cleared first, in the same stream)
hipError_t launch_check_bands(const float *lo, const float *up, int64_t m, unsigned *flag, hipStream_t s);
hipError_t launch_reset_slot(SliceState *st, int slot, int64_t budget, hipStream_t s);
hipError_t launch_disable_slot(SliceState *st, int slot, hipStream_t s);

constexpr int kMaxPassGrid = 4096; // workgroups of a pass kernel (one proximity partial each)

// pass 1: r = A x, t = clip(r) - r, c = D t, one proximity partial per
// workgroup (query != 0: every slice runs, whatever its state)
hipError_t launch_pass1(const PassCfg &cfg, const SpView &A, const RowBlocks &RB, int vk, const float *x,
                        const float *lower, const float *upper, RowW w, float *c, const SliceState *st, int B,
                        int query, double *partials, hipStream_t s);
// The column copy split into row panels of P rows (the last one shorter):
// pp[p*n + j] is the first entry of column j whose row is >= p*P, for p = 0
// .. np (pp[np*n + j] ends the column's entries); ypanel holds np*n partial
// sums.
struct PanelView {
    const int32_t *pp = nullptr;
    int np = 0, P = 0;
    long long m = 0;
    double *ypanel = nullptr;
    int local = 0; // 1: the entries' indices are rows within their panel (16-bit copy), 0: global rows
};

// pass 2 in row panels (one slice): each panel's rows of c staged in LDS,
// per-panel column sums, then the sums in panel order and the column step
hipError_t launch_pass2_panels(const PassCfg &cfg, const SpView &At, const PanelView &PV, int vk, const float *c,
                               float *x, ColStep cs, const SliceState *st_in, SliceState *st_out, const double *part1,
                               int nparts1, Hist h, hipStream_t s);

// raises the dynamic-LDS limit of every LDS-staged pass kernel (once per
// process; outside any stream capture, before the first such launch)
hipError_t prepare_lds_passes();
// pass 2: x = clip(x + lambda A^T c, lo, hi); workgroup 0 also ends the
// iteration (proximity from pass 1's partials, history, k + 1) into st_out
hipError_t launch_pass2(const PassCfg &cfg, const SpView &At, const RowBlocks &RB, int vk, const float *c, float *x,
                        ColStep cs, const SliceState *st_in, SliceState *st_out, int B, const double *part1,
                        int nparts1, Hist h, hipStream_t s);
// pass 2 over the image-tile column layout: per tile, the rows of c it needs
// (B values each) staged in LDS, then y_j and the column step for its pixels
hipError_t launch_pass2_tiles(const PassCfg &cfg, const TileView &T, int vk, const float *c, float *x, ColStep cs,
                              const SliceState *st_in, SliceState *st_out, int B, const double *part1, int nparts1,
                              Hist h, hipStream_t s);
// whether a tile's staged rows of c (B floats each) fit the 64 KB of LDS the
// tile passes use
inline bool tiles_fit(int max_rows, int B) { return int64_t(max_rows) * B * 4 <= 65536; }
// x = clip(z + lambda * sigma_s * y, lo, hi) for the extrapolated steps, sigma_s
// per slice from the partials: EL (emr = 0) t^T D t / ||y||^2 from pass 1's
// and pass 2's partials, EMR (emr = 1) ||y||^2 / sum w (A y)^2 from pass 2's and
// the quadratic-form pass's; closes the iteration.
hipError_t launch_step_apply(int64_t n, int B, const double *y, float *x, const float *lo, const float *hi,
                             float lambda, int emr, const double *part1, int nparts1, const double *party, int npartsy,
                             const double *partq, int npartsq, const SliceState *st_in, SliceState *st_out, Hist h,
                             hipStream_t s);
// fused pass over the CSR: r = A z, t, c = D t, the proximity partial per
// workgroup, and one partial vector of y = A^T c per workgroup in ypart
// (grid x n, float64 or float32 by cfg.acc64).  lds_bytes: dynamic LDS it needs.
size_t fused_lds_bytes(int64_t n, int acc64);
// dynamic LDS of the fused pass with z in LDS (z and a float32 y)
size_t fused_zl_lds_bytes(int64_t n);
// chunks of a row the fused pass with z in LDS keeps in registers for the
// scatter (cap != 0): 16 entries a lane (more, beside the LDS reads in
// flight, would not fit the 128 registers of a 1024-thread workgroup's lane)
constexpr int fused_zl_cap(int lpr, int vec) { return lpr > 0 ? 16 / vec : 0; }
// lp (shapes with z in LDS, one slice): the linear objective's phase opened
// from its partials and z = x + s v staged instead of x; the phase's state
// goes to lp->st_out.
hipError_t launch_fused(const FusedCfg &cfg, const SpView &A, int vk, int64_t n, const float *x, const float *lower,
                        const float *upper, RowW w, const SliceState *st, double *partials, void *ypart,
                        hipStream_t s, const LinPhase *lp = nullptr);
// workgroups of the fused pass's apply kernel (its ||y||^2 partials in deferred mode)
int fused_apply_grid(int64_t n);
// x = clip(z + lambda * sum of the partial vectors, lo, hi), closing the
// iteration; in deferred mode (cs.defer) y itself into cs.ybuf (and ybuf32)
// with fused_apply_grid(n) partials of ||y||^2 in cs.ypart (the extrapolated
// steps then apply x in k_step_apply)
// lin_part (with lin_c): also the linear objective's direction partials of
// the x written, for the next phase (fused_apply_grid(n) slots, not in the
// deferred mode)
// lin_z != 0 (with lin_c): x holds x^k and the pass took the linear phase, so
// z_j = x_j + s v_j is formed here from the phase's state in st_in.
hipError_t launch_fused_apply(const FusedCfg &cfg, int64_t n, const void *ypart, int nvec, float *x, ColStep cs,
                              const SliceState *st_in, SliceState *st_out, const double *part1, Hist h,
                              hipStream_t s, const float *lin_c = nullptr, double *lin_part = nullptr,
                              int lin_z = 0);
// the same direction partials of x alone (one slice)
hipError_t launch_lin_partials(const float *x, const float *c, int64_t n, double *part, hipStream_t s);
// y partials of rows [r_lo, r_hi) whose c is set (the dose-volume rows of a
// fused-pass problem, after their ranking): grid float32 vectors of n at ypart
hipError_t prepare_scatter_rows(int vk, int64_t n);
hipError_t launch_scatter_rows(const SpView &A, int vk, int64_t n, long long r_lo, long long r_hi, const float *c,
                               const SliceState *st, float *ypart, int grid, hipStream_t s);
// largest dynamic LDS one fused workgroup may take on the current device, after
// the kernel's attributes are raised to it (0 if that fails)
size_t fused_lds_limit();
// raise the dynamic-LDS attribute of the fused kernel of this shape (call
// before its first launch, outside stream capture)
hipError_t prepare_fused(const FusedCfg &cfg, int vk, int64_t n);
// query: proximity from pass 1's partials into out[B]
// dose-volume constraints after pass 1 (which stored the rows' values in
// dose): the radix-select rounds (keys, per-constraint histograms in hist,
// which must start zeroed and are left zeroed, selection state in sel), then
// the bands of the rows, their c = S t, and their proximity terms (partials in
// epart, nblk * B), added in a fixed order to pass 1's partial 0 of each slice
// (part1 with nparts1 partials per slice).
hipError_t launch_dvc(const DvcTable &T, const double *dose, unsigned long long *key, unsigned *hist, DvcSel *sel,
                      const float *D, const float *S, float *c, double *epart, double *part1, int nparts1,
                      const SliceState *st, int B, int query, hipStream_t s);

hipError_t launch_query_prox(SliceState *st, int B, const double *partials, int nparts, double *out, hipStream_t s);

int phase_grid(const PertParams &pp);
// gradient and per-tile partials [2][B*tiles] of ||g||^2 and f(x) (eval_only: no gradient)
hipError_t launch_phase(const PertParams &pp, const float *x, float *g, const float *lin_c, const SliceState *st,
                        int eval_only, double *partials, hipStream_t s);
// f(x) per slice from eval_only phase partials into out[B]
hipError_t launch_eval_objective(SliceState *st, const PertParams &pp, const double *partials, double *out,
                                 hipStream_t s);
// One trial launch: derives the state (first: the phase opening from the
// gradient partials; otherwise the previous launch's decision from its trial
// partials), then with `evaluate` the next batch of trial steps (partials
// [max_trials][B*tiles] into part_out), or adds the accepted step to x once
// the phase is over.  The derived state goes to st_out.
// the closing launch of a phase (one workgroup per slice)
// Whether the perturbation phase runs as one launch (flat objectives, short
// vectors), and that launch: state st_in in, st_out out.
bool phase_in_one_launch(const PertParams &pp);
// raises the one-launch phase's dynamic LDS limit on the current device to
// what the longest x takes (outside any capture)
hipError_t prepare_phase_small();
hipError_t launch_phase_small(const PertParams &pp, float *x, const float *lin_c, const SliceState *st_in,
                              SliceState *st_out, hipStream_t s);
// The linear objective's phase after launch_phase (its partials in
// part_phase): trials in closed form, the accepted step added to x.
hipError_t launch_trial_linear(const PertParams &pp, float *x, const float *c, const SliceState *st_in,
                               SliceState *st_out, const double *part_phase, hipStream_t s, int nt = 0);
hipError_t launch_trial_close(const PertParams &pp, float *x, const float *g, const SliceState *st_in,
                              SliceState *st_out, const double *part_prev, hipStream_t s);
hipError_t launch_trial(const PertParams &pp, float *x, const float *g, const SliceState *st_in, SliceState *st_out,
                        int first, int evaluate, const double *part_prev, double *part_out, hipStream_t s);

} // namespace smx
