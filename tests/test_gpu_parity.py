"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: the float32 path must match the oracle to a relative 1e-5 on the
iterate (norm-wise), on every per-iteration proximity and on the final
proximity and objective; the sequence of trial counts (the decisions of
Algorithm 1) must match exactly.  The reduced-precision storage paths are
compared with the oracle run on the same rounded operator (1e-5) and with the
oracle on the float32 operator (2e-2 on proximity and objective).
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-5


@pytest.fixture(scope="module")
def smx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd as smx

    smx.lib()
    return smx


def say(msg):
    print(f"[case] {msg}", flush=True)


def rel(a, b, floor=0.0):
    return float(np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) / max(np.linalg.norm(b), floor, 1e-300))


ELEM_FLOOR = 1e-2


def sup(a, b):
    """Largest entry error of a against b on the scale of b's largest entry."""
    a, b = np.asarray(a, float).reshape(-1), np.asarray(b, float).reshape(-1)
    return float(np.max(np.abs(a - b)) / max(float(np.abs(b).max()), 1e-300)) if b.size else 0.0



def elem(a, b):
    """Worst element-wise relative difference of a against the reference b:
    max_j |a_j - b_j| / max(|b_j|, ELEM_FLOOR max|b|).  Entries below 1 % of
    the largest are compared on that scale: their float32 rounding inherits
    the magnitude of the terms that cancel in them (a step's y_j sums
    contributions on the scale of the whole iterate), so 1e-5 of it is about
    two float32 units of the largest entry, while a wrong entry (a missed
    column, a boundary pixel) is off by far more."""
    a, b = np.asarray(a, float).reshape(-1), np.asarray(b, float).reshape(-1)
    if b.size == 0:
        return 0.0
    scale = np.maximum(np.abs(b), ELEM_FLOOR * max(float(np.abs(b).max()), 1e-300))
    return float(np.max(np.abs(a - b) / scale))


# Dose-volume constraints: the device ranks a structure's rows by their values
# rounded to float32, the oracle by exact values.  Where the k-th and (k+1)-th
# highest values of a structure lie closer than this (relative), and the choice
# between them changes a band (the (k+1)-th lies above the dose of an "at
# most" constraint, or the k-th below the dose of an "at least" one), both
# choices are nearest points of the set to within float32 resolution.
TIE_REL = 1e-5


def dvc_margin(P, dvc, z):
    """Smallest relative gap between the k-th and (k+1)-th value over the
    constraints whose choice between them changes a band at the point z
    (inf when none does)."""
    if not dvc:
        return np.inf
    kth, nxt = P.dvc_boundary(z)
    out = np.inf
    for g, d in enumerate(dvc):
        a, b = kth[g], nxt[g]
        if not (np.isfinite(a) and np.isfinite(b)):
            continue
        if d["sense"] == W.DVC_MAX and not b > d["dose"]:
            continue
        if d["sense"] == W.DVC_MIN and not a < d["dose"]:
            continue
        out = min(out, abs(a - b) / max(abs(a), abs(b), 1e-30))
    return out


def dvc_trajectory_margin(w, K, perturb=True, s=0, value_round=None, refine=0):
    """The smallest dvc_margin over the points the feasibility steps of the
    oracle's run act on (its iterate rounded to float32 after every
    iteration, as the device stores it)."""
    P32 = oracle.from_workload(w, s)
    Pr = P32 if value_round is None else oracle.from_workload(w, s, value_round=value_round)
    x = w.x0[:, s].astype(np.float32).astype(np.float64)
    st, worst = None, np.inf
    for k in range(K):
        P = Pr if k < K - refine else P32
        z = P.perturb(x, st)[0] if perturb else x
        worst = min(worst, dvc_margin(P, w.dvc, z))
        x, st, _ = P.run(x, 1, perturb=perturb, state=st)
        x = x.astype(np.float32).astype(np.float64)
    return worst


def gpu_run(smx, w, K, perturb=True, storage="f32", graph=False, refine_iters=-1, fused=True, phase_form=None,
            fused_shape=None):
    p = smx.problem_from_workload(w, storage=storage, history_cap=K, refine_iters=refine_iters, fused=fused)
    if phase_form is not None:
        p.set_phase_form(phase_form)
    if fused_shape is not None:
        p.set_fused_shape(*fused_shape)
    p.run(K, perturb=perturb, graph=graph)
    p.sync()
    x = p.get_x().cpu().numpy().astype(np.float64)
    prox, obj = p.query()
    h = p.history()
    st, _ = p.get_state()
    p.close()
    return x, prox, obj, h, st


def oracle_run(w, K, perturb=True, s=0, value_round=None, refine=0):
    """Oracle run for slice s; with value_round, the first K-refine iterations
    use the rounded operator and the last `refine` the float32 one."""
    P32 = oracle.from_workload(w, s)
    if value_round is None or refine >= K:
        x, st, h = P32.run(w.x0[:, s], K, perturb=perturb)
        return x, st, h, P32
    Pr = oracle.from_workload(w, s, value_round=value_round)
    x, st, h1 = Pr.run(w.x0[:, s], K - refine, perturb=perturb)
    if refine == 0:
        return x, st, h1, P32
    x, st, h2 = P32.run(x, refine, perturb=perturb, state=st)
    h = oracle.History(*(np.concatenate([a, b]) for a, b in zip(
        (h1.prox, h1.f_start, h1.f_end, h1.trials, h1.accepts),
        (h2.prox, h2.f_start, h2.f_end, h2.trials, h2.accepts))))
    return x, st, h, P32


def storage_deviation(w, K, perturb=True, s=0, value_round=None, refine=0):
    """Deviation forced by float32 storage of the iterate alone: the oracle's
    trajectory with x rounded to float32 after every iteration, against its
    pure float64 trajectory (relative, for x, the proximity and the objective).
    Every float32 path carries at least this much; TV amplifies it."""
    P32 = oracle.from_workload(w, s)
    Pr = P32 if value_round is None else oracle.from_workload(w, s, value_round=value_round)
    x64, _, _, _ = oracle_run(w, K, perturb, s, value_round=value_round, refine=refine)
    x = w.x0[:, s].astype(np.float32).astype(np.float64)
    st = None
    for k in range(K):
        P = Pr if k < K - refine else P32
        x, st, _ = P.run(x, 1, perturb=perturb, state=st)
        x = x.astype(np.float32).astype(np.float64)
    dx = rel(x, x64)
    dp = abs(P32.proximity(x) - P32.proximity(x64)) / max(abs(P32.proximity(x64)), 1e-300)
    df = abs(P32.objective(x) - P32.objective(x64)) / max(abs(P32.objective(x64)), 1e-300)
    storage_deviation.elem = elem(x, x64)
    storage_deviation.sup = sup(x, x64)
    return dx, dp, df


def check_parity(smx, w, K, perturb=True, tol=RTOL, storage="f32", value_round=None, refine_iters=-1,
                 sensitive=False, fused=True, phase_form=None, fused_shape=None):
    """End-to-end parity.  With sensitive=True (TV problems, whose gradient
    amplifies rounding of the iterate), the iterate and proximity tolerances
    are max(tol, 10 x the deviation float32 storage of the iterate alone
    forces: the kernels store four float32 quantities per iteration, the
    perturbed point, the gradient, the weighted residual and the iterate, where
    the emulation rounds one), and the objective must agree to first order
    with the iterate's difference: |df| <= 2 ||grad f|| ||dx|| + tol |f|, and
    so must the final proximity (grad P = -A^T D t).  The strict
    per-iteration check is the lockstep test.  The iterate is compared
    norm-wise, by its largest entry error against its largest entry (sup)
    and element by element (elem); the last two within max(tol, 30 x the
    same deviation float32 storage of the iterate alone forces: the kernels'
    element-wise deviations run up to ~16 x that emulation's over the parity
    cases, as their norm-wise ones run up to ~12 x, and on TV, EL and EMR
    problems, whose steps amplify rounding where the iterate is nearly flat
    or the system inconsistent, both concentrate on a few entries).  With dose-volume constraints
    the case must keep every ranking decision of the oracle's run clear of
    float32 near-ties (dvc_trajectory_margin above TIE_REL), so that the
    device and the oracle pick the same nearest point."""
    say(f"{w.name} m={w.m} n={w.n} nnz={w.nnz} K={K} perturb={perturb} obj={w.obj} storage={storage} "
        f"fused={fused} phase_form={phase_form} fused_shape={fused_shape}")
    x, prox, obj, h, st = gpu_run(smx, w, K, perturb, storage=storage, refine_iters=refine_iters, fused=fused,
                                  phase_form=phase_form, fused_shape=fused_shape)
    refine = 0
    if storage != "f32":
        refine = refine_iters if refine_iters >= 0 else (K + 19) // 20
    for s in range(w.B):
        if getattr(w, "dvc", None):
            mg = dvc_trajectory_margin(w, K, perturb, s, value_round=value_round, refine=refine)
            print(f"  slice {s}: smallest dose-volume ranking margin {mg:.2e}", flush=True)
            assert mg > TIE_REL, f"the case passes a float32 near-tie of a ranking ({mg:.2e}); choose another seed"
        xo, sto, ho, P = oracle_run(w, K, perturb, s, value_round=value_round, refine=refine)
        tx = tp = tol
        r, re = rel(x[:, s], xo), elem(x[:, s], xo)
        f_slack = 0.0
        dx, dp, df = storage_deviation(w, K, perturb, s, value_round=value_round, refine=refine)
        te, ts = max(tol, 30 * storage_deviation.elem), max(tol, 30 * storage_deviation.sup)
        if sensitive:
            tx, tp = max(tol, 10 * dx), max(tol, 10 * dp)
            f_slack = 2.0 * np.linalg.norm(P.gradient(xo)) * np.linalg.norm(x[:, s] - xo)
        print(f"  storage-only deviation x {dx:.2e} (element-wise {storage_deviation.elem:.2e}) "
              f"prox {dp:.2e} f {df:.2e}", flush=True)
        print(f"  slice {s}: iterate rel err {r:.3e} (tol {tx:.1e}), element-wise {re:.3e} (tol {te:.1e}), "
              f"largest entry error {sup(x[:, s], xo):.3e} (tol {ts:.1e})", flush=True)
        assert np.array_equal(h["trials"][:, s], ho.trials), "trial sequence differs"
        assert np.array_equal(h["accepts"][:, s], ho.accepts), "accept sequence differs"
        assert r <= tx, f"slice {s}: iterate rel err {r:.3e}"
        assert sup(x[:, s], xo) <= ts, f"slice {s}: largest entry error {sup(x[:, s], xo):.3e} of the largest entry"
        assert re <= te, f"slice {s}: element-wise iterate err {re:.3e}"
        assert st[s]["ell"] == sto.ell and st[s]["restarts"] == sto.restarts and st[s]["k"] == K
        assert st[s]["cap_hits"] == sto.cap_hits
        pfloor = 1e-6 * max(abs(ho.prox[0]), 1e-300)
        np.testing.assert_allclose(h["prox"][:, s], ho.prox, rtol=tp, atol=pfloor)
        po, fo = P.proximity(xo), P.objective(xo)
        p_slack = 0.0
        if sensitive:  # first order in the iterate's difference: grad P = -A^T D t
            ro = P.matvec(xo)
            q = P.row_sqnorms()
            dt = np.where(q > 0, P.w / np.where(q > 0, q, 1.0), 0.0) * (np.clip(ro, P.lower, P.upper) - ro)
            p_slack = 2.0 * np.linalg.norm(P.matvec_t(dt)) * np.linalg.norm(x[:, s] - xo)
        assert abs(prox[s] - po) <= p_slack + tp * max(abs(po), pfloor), (prox[s], po, p_slack)
        assert abs(obj[s] - fo) <= f_slack + tol * max(abs(fo), 1e-12), (obj[s], fo, f_slack)
    return x, h


# ---------------------------------------------------------------------------
# float32 path
# ---------------------------------------------------------------------------

def test_dense_consistent(smx):
    w = W.dense_small()
    check_parity(smx, w, w.K)


def test_dense_unperturbed_consistent_proximity_decreases(smx):
    w = W.dense_small()
    _, h = check_parity(smx, w, 60, perturb=False)
    d = np.diff(h["prox"][:, 0])
    assert np.all(d <= 1e-6 * h["prox"][0, 0])


@pytest.mark.parametrize("obj", [W.OBJ_NONE, W.OBJ_SQNORM, W.OBJ_LINEAR, W.OBJ_TV2D, W.OBJ_L1])
def test_random_sparse_edge_rows(smx, obj):
    """Skewed row lengths, empty rows, two full-length rows, one-sided and
    equality bands, restarts and two reduction steps."""
    w = W.random_sparse(3000, 2000, 12, seed=40 + obj, empty_frac=0.08, long_rows=2, obj=obj,
                        tv_shape=(40, 50), K=25)
    check_parity(smx, w, w.K, perturb=obj != W.OBJ_NONE, sensitive=obj == W.OBJ_TV2D)


def test_ct_small_tv(smx):
    w = W.ct(N=48, n_angles=36, seed=7, K=60)
    check_parity(smx, w, w.K, sensitive=True)


def test_ct_small_tv_paper_parameters(smx):
    w = W.ct(N=48, n_angles=36, seed=8, K=60, variant="paper")
    check_parity(smx, w, w.K, sensitive=True)


STATE_FIELDS = ("k", "ell", "restarts", "trials", "accepts", "cap_hits", "stop_reason", "dp_run", "feas_ok",
                "p_last", "f_last", "var_n", "var_mean", "var_m2", "f_ref")


def device_state(so):
    """An oracle state as the device's per-slice state record."""
    out = {}
    for f in STATE_FIELDS:
        v = getattr(so, f)
        out[f] = (None if v != v else float(v)) if isinstance(v, float) else int(v)
    return out


def step_from_oracle(p, P, x, so, graph=False, perturb=True):
    """One iteration from an oracle-made point: x (float32 values) and state so
    are loaded into the device, which runs one iteration; the oracle runs the
    same iteration from the same point.  Returns (device x, device state,
    oracle x, oracle state, the oracle's proximity at the point its step acted
    on).  The device records its own in its history at index so.k when its
    history holds that many iterations."""
    p.set_state([device_state(so)], x.astype(np.float32).reshape(-1, 1))
    xo, so1, ho = P.run(x.astype(np.float64), 1, perturb=perturb, state=so)
    p.run(1, perturb=perturb, graph=graph)
    states1, xg = p.get_state()
    return xg[:, 0].astype(np.float64), states1[0], xo, so1, float(ho.prox[0])


def near_tie_step(P, w, x, so, perturb=True):
    """Whether the feasibility step from the oracle point (x, so) meets a
    dose-volume ranking near-tie (dvc_margin below TIE_REL)."""
    if not getattr(w, "dvc", None):
        return False
    z = P.perturb(x, so)[0] if perturb else x
    return dvc_margin(P, w.dvc, z) < TIE_REL


def check_step(xg, sg, xo, so1, tie, tol, k):
    """One oracle-driven iteration: decisions exactly and, unless the step met
    a dose-volume near-tie (where either of the near-equal rows may keep its
    value and the two nearest points differ in that row's band), the iterate
    norm-wise and element-wise to tol.  The step's proximity (unique: the
    distance to a nearest point) is compared from the histories afterwards
    (check_step_proximities).  Returns the norm-wise difference (0 at a
    near-tie)."""
    assert sg["trials"] == so1.trials and sg["accepts"] == so1.accepts, k
    assert sg["ell"] == so1.ell and sg["restarts"] == so1.restarts and sg["k"] == so1.k, k
    if tie:
        print(f"  iteration {k}: dose-volume near-tie, iterate not compared", flush=True)
        return 0.0
    r, re = rel(xg, xo), elem(xg, xo)
    assert r <= tol, f"iteration {k}: rel err {r:.3e}"
    assert re <= tol, f"iteration {k}: element-wise err {re:.3e}"
    return r


def check_step_proximities(p, ks, prox_oracle, tol):
    """The proximity each oracle-driven step recorded on the device (history
    index k) against the oracle's, to tol (relative)."""
    hp = p.history()["prox"][:, 0]
    for k, po in zip(ks, prox_oracle):
        assert abs(hp[k] - po) <= tol * max(abs(po), 1e-300), (k, hp[k], po)


def lockstep(smx, w, K, tol=RTOL):
    """Per-iteration check driven by the oracle: the oracle runs its own
    trajectory with the iterate rounded to float32 after every iteration; each
    of its iterates and states is loaded into the device, which runs that one
    iteration.  The iterates must agree to tol (norm-wise and element by
    element), every step's proximity to tol and the decisions (trials,
    accepts, ell, restarts) exactly (check_step)."""
    p = smx.problem_from_workload(w, history_cap=K)
    P = oracle.from_workload(w)
    x = w.x0[:, 0].astype(np.float32).astype(np.float64)
    so = oracle.State()
    worst, po = 0.0, []
    for k in range(K):
        tie = near_tie_step(P, w, x, so)
        xg, sg, xo, so1, pk = step_from_oracle(p, P, x, so)
        worst = max(worst, check_step(xg, sg, xo, so1, tie, tol, k))
        po.append(pk)
        x, so = xo.astype(np.float32).astype(np.float64), so1
    check_step_proximities(p, range(K), po, tol)
    p.close()
    return worst


def test_ct_small_tv_lockstep(smx):
    w = W.ct(N=48, n_angles=36, seed=7, K=40, variant="paper")
    say("ct48 lockstep (paper parameters)")
    worst = lockstep(smx, w, w.K)
    print(f"  worst per-iteration rel err {worst:.3e}", flush=True)


def test_seismic_small_tv(smx):
    w = W.seismic(rows=30, cols=60, n_src=15, n_rec=30, seed=9, K=80, variant="paper")
    check_parity(smx, w, w.K, sensitive=True)


def test_seismic_small_tv_lockstep(smx):
    w = W.seismic(rows=30, cols=60, n_src=15, n_rec=30, seed=9, K=40, variant="paper")
    say("seismic lockstep (paper parameters)")
    worst = lockstep(smx, w, w.K)
    print(f"  worst per-iteration rel err {worst:.3e}", flush=True)


@pytest.mark.parametrize("obj,noise", [(W.OBJ_L1, 0.0), (W.OBJ_L1, 0.05), (W.OBJ_SQNORM, 0.0),
                                       (W.OBJ_TV2D, 0.05)])
def test_seismic_fresnel_drop(smx, obj, noise):
    """Band rows of the first-Fresnel-zone model, DROP steps, equality bands
    (noise-free and with 5 % noise, Section 2.3.1) and the L1, squared-norm and
    TV perturbations."""
    w = W.seismic_fresnel(N=48, n_src=12, n_rec=24, seed=11, noise=noise, obj=obj, K=40)
    check_parity(smx, w, w.K, sensitive=obj == W.OBJ_TV2D)


def test_seismic_fresnel_l1_lockstep(smx):
    w = W.seismic_fresnel(N=48, n_src=12, n_rec=24, seed=11, noise=0.05, obj=W.OBJ_L1, K=30)
    say("seismic fresnel lockstep (DROP, L1)")
    worst = lockstep(smx, w, w.K)
    print(f"  worst per-iteration rel err {worst:.3e}", flush=True)


def test_rt_small_linear_infeasible(smx):
    w = W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=10, K=40)
    assert w.meta["n_overlap"] > 0
    check_parity(smx, w, w.K)


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (5, 3)])
def test_tiny_shapes(smx, shape):
    m, n = shape
    rng = np.random.default_rng(m * 100 + n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    rp = np.arange(0, m * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), m)
    r = A.astype(np.float64) @ rng.uniform(0, 1, n)
    w = W.Workload(name=f"tiny{m}x{n}", m=m, n=n, row_ptr=rp, col_idx=ci, val=A.reshape(-1),
                   lower=(r - 0.1).astype(np.float32)[:, None], upper=(r + 0.1).astype(np.float32)[:, None],
                   box_lo=np.zeros(n, np.float32), box_hi=np.ones(n, np.float32),
                   x0=rng.uniform(0, 1, (n, 1)).astype(np.float32), obj=W.OBJ_SQNORM, gamma=0.3, alpha=0.9,
                   n_red=2, K=15)
    check_parity(smx, w, w.K)


# ---------------------------------------------------------------------------
# reduced-precision storage
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_lowp_matches_oracle_on_rounded_operator(smx, storage):
    w = W.ct(N=48, n_angles=36, seed=11, K=40)
    check_parity(smx, w, w.K, storage=storage, value_round=storage, sensitive=True)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_lowp_wide_operator_32bit_indices(smx, storage):
    """Reduced-precision values beside 32-bit column indices (n above the
    16-bit index range, so neither the packed words nor the 16-bit index
    arrays serve; the rows' chunks are loaded as raw words and decoded after
    all of them are requested): against the oracle on the rounded
    operator."""
    w = W.random_sparse(4000, 70000, 40, seed=71, long_rows=4, long_len=900, obj=W.OBJ_L1, K=12)
    check_parity(smx, w, w.K, storage=storage, value_round=storage)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_lowp_against_float_operator(smx, storage):
    """Against the oracle on the float32 operator: proximity and objective
    within 2e-2 after K iterations (with the float32 refinement tail)."""
    w = W.ct(N=64, n_angles=48, seed=12, K=60)
    say(f"{storage} vs float operator")
    x, prox, obj, h, st = gpu_run(smx, w, w.K, storage=storage)
    xo, sto, ho, P = oracle_run(w, w.K)
    po, fo = P.proximity(xo), P.objective(xo)
    assert abs(prox[0] - po) <= 2e-2 * abs(po)
    assert abs(obj[0] - fo) <= 2e-2 * abs(fo)


# ---------------------------------------------------------------------------
# execution modes
# ---------------------------------------------------------------------------

def test_graph_replay_is_bitwise_eager(smx):
    w = W.ct(N=48, n_angles=36, seed=13, K=37)
    say("graph vs eager (two passes)")
    xe, pe, fe, he, _ = gpu_run(smx, w, w.K, graph=False, fused=False)
    xg, pg, fg, hg, _ = gpu_run(smx, w, w.K, graph=True, fused=False)
    assert np.array_equal(xe, xg)
    assert np.array_equal(he["trials"], hg["trials"])
    assert np.array_equal(he["prox"], hg["prox"])


@pytest.mark.parametrize("form", ["one_launch", "closed_form"])
def test_phase_forms_graph_and_resume_bitwise(smx, form):
    """The one-launch and closed-form phases (two passes, so every sum has a
    fixed order): graph replay equals eager launches, and a run stopped,
    checkpointed and resumed equals the run straight through, bit for bit."""
    w = W.random_sparse(3000, 2000, 12, seed=43, empty_frac=0.08, long_rows=2, obj=W.OBJ_LINEAR, K=23)
    f = smx.PHASE_ONE_LAUNCH if form == "one_launch" else smx.PHASE_CLOSED_FORM
    say(f"graph, eager and resume with the {form} phase")
    xe, pe, fe, he, se = gpu_run(smx, w, w.K, graph=False, fused=False, phase_form=f)
    xg, pg, fg, hg, sg = gpu_run(smx, w, w.K, graph=True, fused=False, phase_form=f)
    assert np.array_equal(xe, xg) and np.array_equal(he["prox"], hg["prox"]) and se == sg
    p = smx.problem_from_workload(w, history_cap=0, fused=False)
    p.set_phase_form(f)
    p.run(9, graph=True)
    p.sync()
    states, x1 = p.get_state()
    p.close()
    q = smx.problem_from_workload(w, history_cap=0, fused=False)
    q.set_phase_form(f)
    q.set_state(states, x1)
    q.run(w.K - 9, graph=True)
    q.sync()
    xb = q.get_x().cpu().numpy().astype(np.float64)
    sb, _ = q.get_state()
    q.close()
    assert np.array_equal(xe, xb) and sb == se


def test_repeat_is_bitwise(smx):
    w = W.random_sparse(2000, 1500, 20, seed=14, obj=W.OBJ_TV2D, tv_shape=(30, 50), K=20)
    say("repeat (two passes)")
    a = gpu_run(smx, w, w.K, fused=False)
    b = gpu_run(smx, w, w.K, fused=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_checkpoint_resume_bitwise(smx):
    w = W.ct(N=40, n_angles=30, seed=15, K=30, variant="paper")
    say("checkpoint/resume (two passes)")
    xa, _, _, _, sa = gpu_run(smx, w, w.K, fused=False)
    p = smx.problem_from_workload(w, history_cap=0, fused=False)
    p.run(11)
    p.sync()
    states, x1 = p.get_state()
    p.close()
    q = smx.problem_from_workload(w, history_cap=0, fused=False)
    q.set_state(states, x1)
    q.run(w.K - 11)
    q.sync()
    xb = q.get_x().cpu().numpy()
    sb, _ = q.get_state()
    q.close()
    assert np.array_equal(xa, xb.astype(np.float64))
    assert sa == sb


def test_query_at_given_point(smx):
    """Proximity and objective evaluated by the kernels at a seeded point
    loaded into the device agree with the oracle evaluated at that point."""
    w = W.seismic(rows=30, cols=60, n_src=15, n_rec=30, seed=16, K=30)
    say("query at a loaded point")
    x = W.synthetic_iterate(w, seed=17)
    p = smx.problem_from_workload(w, history_cap=0)
    p.set_x(x)
    prox, obj = p.query()
    p.close()
    P = oracle.from_workload(w)
    assert prox[0] == pytest.approx(P.proximity(x[:, 0].astype(np.float64)), rel=2e-6)
    assert obj[0] == pytest.approx(P.objective(x[:, 0].astype(np.float64)), rel=2e-6)


def test_timing_counts_launches(smx):
    w = W.ct(N=32, n_angles=24, seed=17, K=12)
    p = smx.problem_from_workload(w)
    p.set_timing(True)
    p.run(12)
    p.sync()
    t1, t2, n = p.timing()
    p.close()
    assert n == 12 and t1 > 0 and t2 > 0


def test_invalid_problem_args(smx):
    w = W.ct(N=16, n_angles=8, seed=18, K=5)
    op = smx.Operator(w.m, w.n, w.row_ptr, w.col_idx, w.val)
    bad = [
        dict(lam=0.0), dict(lam=2.5), dict(alpha=1.0), dict(gamma=0.0), dict(n_red=0), dict(max_trials=0),
        dict(tv_rows=5),
    ]
    for kw in bad:
        args = dict(lower=w.lower, upper=w.upper, obj=W.OBJ_TV2D, tv_rows=16, tv_cols=16, tv_eps=1e-3)
        args.update(kw)
        with pytest.raises(smx.SmxError) as e:
            smx.Problem(op, **args)
        assert e.value.code == smx.EINVAL, kw
    lo = w.lower.copy()
    lo[3, 0] = w.upper[3, 0] + 1
    with pytest.raises(smx.SmxError):
        smx.Problem(op, lower=lo, upper=w.upper)
    with pytest.raises(smx.SmxError):
        smx.Problem(op, lower=w.lower, upper=w.upper, obj=W.OBJ_LINEAR)
    op.close()


# ---------------------------------------------------------------------------
# full size CT (the benchmarked configuration)
# ---------------------------------------------------------------------------

def test_ct256_full_bench_configuration(smx):
    w = W.ct(N=256, seed=2, K=200)
    check_parity(smx, w, w.K, sensitive=True)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_interleaved_lane_pass1(smx, storage, monkeypatch):
    """Pass 1 with interleaved lanes (lane l of a row takes entries l, l + 16,
    ...) against the oracle, on skewed rows and on CT."""
    monkeypatch.setenv("SMX_PASS_MODE", "interleaved")
    w = W.random_sparse(3000, 2000, 12, seed=44, empty_frac=0.08, long_rows=2, obj=W.OBJ_SQNORM, K=20)
    p = smx.problem_from_workload(w, storage=storage)
    assert p.describe()[storage]["pass1"]["vec"] == 1
    p.close()
    vr = None if storage == "f32" else storage
    check_parity(smx, w, w.K, storage=storage, value_round=vr)
    wc = W.ct(N=48, n_angles=36, seed=45, K=30)
    check_parity(smx, wc, wc.K, storage=storage, value_round=vr, sensitive=True)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_lds_staged_passes(smx, storage, monkeypatch):
    """Both passes with the gathered vector's first 40,448 entries staged in
    LDS (x for pass 1, c for pass 2): vectors longer than that (gathers from
    LDS and from memory), ones that fit whole with a length not a multiple of
    four, CT with TV, and EMR with dose-volume constraints (its kept y and
    quadratic-form pass)."""
    monkeypatch.setenv("SMX_PASS_MODE", "lds")
    vr = None if storage == "f32" else storage
    wl = W.random_sparse(2500, 50001, 30, seed=46, empty_frac=0.05, long_rows=3, long_len=45000,
                         obj=W.OBJ_SQNORM, K=15)
    p = smx.problem_from_workload(wl, storage=storage, fused=False)
    d = p.describe()[storage]
    p.close()
    assert d["pass1"]["mode"] == "lds" and d["pass2"]["mode"] == "lds", d
    assert d["pass1"]["xlds"] == 40448 and d["pass2"]["xlds"] == 2500, d
    assert not (d["fused"] or {}).get("in_use"), d
    check_parity(smx, wl, wl.K, storage=storage, value_round=vr, fused=False)
    wt = W.random_sparse(45001, 3000, 8, seed=49, empty_frac=0.05, long_rows=2, obj=W.OBJ_LINEAR, K=12)
    check_parity(smx, wt, wt.K, storage=storage, value_round=vr, fused=False)
    ws = W.random_sparse(3000, 2001, 12, seed=47, empty_frac=0.08, long_rows=2, obj=W.OBJ_L1, K=20)
    check_parity(smx, ws, ws.K, storage=storage, value_round=vr, fused=False)
    wc = W.ct(N=48, n_angles=36, seed=48, K=30)
    check_parity(smx, wc, wc.K, storage=storage, value_round=vr, sensitive=True, fused=False)
    wd = _dvc_rt(W.BASIC_EMR, K=15)
    check_parity(smx, wd, wd.K, storage=storage, value_round=vr, refine_iters=0)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_row_panel_pass2(smx, storage, monkeypatch):
    """Pass 2 over the column copy in row panels of 40,448 rows (c's rows of
    a panel staged in LDS, per-panel sums added in panel order): 100,001 rows
    make three panels, the last one short, read through the copy with 16-bit
    offsets within the panel; the plain step, EMR's kept y and DROP's column
    factors, against the oracle; then 50,001 rows (two panels)."""
    monkeypatch.setenv("SMX_PASS_MODE", "panels")
    vr = None if storage == "f32" else storage
    w = W.random_sparse(100001, 700, 6, seed=50, empty_frac=0.05, long_rows=3, long_len=650, obj=W.OBJ_SQNORM,
                        K=10)
    p = smx.problem_from_workload(w, storage=storage, fused=False)
    d = p.describe()[storage]
    p.close()
    assert d["pass2"]["mode"] == "panels" and not (d["fused"] or {}).get("in_use"), d
    check_parity(smx, w, w.K, storage=storage, value_round=vr, fused=False)
    for method in ("emr", "drop"):
        wb = _with_basic(w, method)
        check_parity(smx, wb, wb.K, storage=storage, value_round=vr, fused=False)
    # 50,001 rows fit 16 bits: the column copy's own rows (packed with the
    # values for bf16), offset by the panel's first row
    w2 = W.random_sparse(50001, 600, 6, seed=51, empty_frac=0.05, long_rows=2, long_len=550, obj=W.OBJ_LINEAR,
                         K=10)
    p = smx.problem_from_workload(w2, storage=storage, fused=False)
    assert p.describe()[storage]["pass2"]["mode"] == "panels"
    p.close()
    check_parity(smx, w2, w2.K, storage=storage, value_round=vr, fused=False)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_lanes_per_row_kernels(smx, storage, monkeypatch):
    """The lanes-per-row pass kernels (the alternative launch shape) give the
    same results as the oracle too."""
    monkeypatch.setenv("SMX_PASS_MODE", "rows")
    w = W.random_sparse(2500, 1800, 30, seed=19, empty_frac=0.05, long_rows=3, obj=W.OBJ_SQNORM, K=15)
    if storage == "f32":
        check_parity(smx, w, w.K)
    else:
        check_parity(smx, w, w.K, storage="bf16", value_round="bf16")


def test_long_rows_stream_kernel(smx):
    """Rows and columns longer than one streamed row block (2048 entries)."""
    w = W.random_sparse(600, 5000, 40, seed=20, empty_frac=0.05, long_rows=4, long_len=4500,
                        obj=W.OBJ_LINEAR, K=12)
    check_parity(smx, w, w.K)


def test_autotuned_shapes_keep_parity(smx):
    """After autotuning (launch shapes picked by timing), results still match
    the oracle, and tuning leaves the iterate and state untouched."""
    w = W.ct(N=64, n_angles=48, seed=21, K=30)
    say("autotune")
    p = smx.problem_from_workload(w, history_cap=w.K)
    x_before = p.get_x().cpu().numpy().copy()
    shapes = p.autotune(reps=3)
    print(f"  shapes {shapes}", flush=True)
    assert shapes["tuned"]
    assert np.array_equal(p.get_x().cpu().numpy(), x_before)
    p.run(w.K)
    p.sync()
    x = p.get_x().cpu().numpy()[:, 0].astype(np.float64)
    h = p.history()
    p.close()
    xo, sto, ho, P = oracle_run(w, w.K)
    assert np.array_equal(h["trials"][:, 0], ho.trials)
    dx, _, _ = storage_deviation(w, w.K)
    assert rel(x, xo) <= max(RTOL, 10 * dx)


# ---------------------------------------------------------------------------
# fused single pass (one slice, y = A^T c accumulated in LDS)
# ---------------------------------------------------------------------------

def _fused_info(smx, w, storage="f32"):
    p = smx.problem_from_workload(w, storage=storage)
    d = p.describe()
    p.close()
    kind = storage if storage != "f32" else "f32"
    return d[kind]["fused"]


@pytest.mark.parametrize("case", ["rt", "ct_tv", "edge_rows", "sqnorm_paper"])
def test_fused_pass_parity(smx, case):
    """The fused pass against the oracle on each objective, with empty rows,
    rows longer than a lane group's reach and an infeasible band set."""
    if case == "rt":
        w = W.rt(grid=(24, 24, 12), beamlets=(7, 7), seed=50, K=25)
    elif case == "ct_tv":
        w = W.ct(N=40, n_angles=30, seed=51, K=30)
    elif case == "edge_rows":
        w = W.random_sparse(3000, 2500, 25, seed=52, empty_frac=0.05, long_rows=4, long_len=2200,
                            obj=W.OBJ_LINEAR, K=15)
    else:
        w = W.random_sparse(2000, 1200, 30, seed=53, obj=W.OBJ_SQNORM, K=20).with_params(
            gamma=5.0, n_red=4, restart_every=7)
    info = _fused_info(smx, w)
    assert info is not None and info["in_use"] and info["acc"] == "f64", info
    check_parity(smx, w, w.K, sensitive=(w.obj == W.OBJ_TV2D))


def test_fused_float32_accumulators(smx):
    """n too large for a float64 LDS copy of y but within a float32 one."""
    w = W.random_sparse(4000, 30000, 40, seed=54, obj=W.OBJ_SQNORM, K=12)
    info = _fused_info(smx, w)
    assert info is not None and info["in_use"] and info["acc"] == "f32", info
    check_parity(smx, w, w.K)


def test_fused_absent_when_y_does_not_fit(smx):
    w = W.random_sparse(500, 70000, 20, seed=55, obj=W.OBJ_NONE, K=3)
    assert _fused_info(smx, w) is None


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_fused_reduced_precision(smx, storage):
    w = W.rt(grid=(24, 24, 12), beamlets=(7, 7), seed=56, K=20)
    info = _fused_info(smx, w, storage)
    assert info is not None and info["in_use"], info
    check_parity(smx, w, w.K, storage=storage, value_round=storage, refine_iters=0)


def test_fused_agrees_with_two_passes(smx):
    w = W.ct(N=48, n_angles=36, seed=57, K=25)
    say("fused vs two passes")
    xf, pf, ff, hf, _ = gpu_run(smx, w, w.K, fused=True)
    xt, pt, ft, ht, _ = gpu_run(smx, w, w.K, fused=False)
    assert np.array_equal(hf["trials"], ht["trials"])
    dx, _, _ = storage_deviation(w, w.K)
    assert rel(xf, xt) <= max(RTOL, 10 * dx)
    np.testing.assert_allclose(hf["prox"], ht["prox"], rtol=max(RTOL, 10 * dx))


def test_fused_graph_replay_and_tiny_grids(smx):
    """Graph replay of the fused pass, and an operator with fewer rows than
    fused workgroups (most workgroups get no rows)."""
    w = W.random_sparse(40, 30, 6, seed=58, obj=W.OBJ_SQNORM, K=23)
    info = _fused_info(smx, w)
    assert info is not None and info["in_use"] and info["grid"] > w.m
    say("fused graph replay, tiny grid")
    xe, _, _, he, _ = gpu_run(smx, w, w.K, graph=False)
    xg, _, _, hg, _ = gpu_run(smx, w, w.K, graph=True)
    assert np.array_equal(he["trials"], hg["trials"])
    assert rel(xg, xe) <= RTOL
    check_parity(smx, w, w.K)


def test_set_fused_switches_kernels(smx):
    w = W.ct(N=24, n_angles=16, seed=59, K=5)
    p = smx.problem_from_workload(w)
    assert p.fused_in_use()
    p.set_fused(False)
    assert not p.fused_in_use()
    p.set_fused(True)
    assert p.fused_in_use()
    with pytest.raises(smx.SmxError):
        smx.check(smx.lib().smx_set_fused(p.handle, 2))
    p.close()


PHASE_CASES = {
    "rt_linear": lambda: W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=10, K=40),
    "sqnorm_two_steps": lambda: W.random_sparse(3000, 2000, 12, seed=41, empty_frac=0.08, long_rows=2,
                                                obj=W.OBJ_SQNORM, K=25),
    "l1": lambda: W.random_sparse(3000, 2000, 12, seed=44, empty_frac=0.08, long_rows=2, obj=W.OBJ_L1, K=25),
    "dense_sqnorm": lambda: W.dense_small(),
    "batched_l1": lambda: W.random_sparse(2000, 1500, 10, seed=48, B=4, obj=W.OBJ_L1, K=20),
    "sqnorm_longest_x": lambda: W.random_sparse(4000, 20000, 40, seed=45, obj=W.OBJ_SQNORM, K=12),
}


PHASE_FORM_RUNS = [(c, f) for c in PHASE_CASES for f in ("one_launch", "batches")] + \
    [("rt_linear", "closed_form"), ("linear_two_steps", "closed_form"), ("linear_two_steps", "batches")]
PHASE_CASES["linear_two_steps"] = lambda: W.random_sparse(3000, 2000, 12, seed=42, empty_frac=0.08, long_rows=2,
                                                         obj=W.OBJ_LINEAR, K=25)


@pytest.mark.parametrize("case,form", PHASE_FORM_RUNS)
def test_phase_forms_parity(smx, case, form):
    """The perturbation phase in one launch per slice, as the chain of
    trial-batch launches and, for the linear objective, with its trials in
    closed form: each against the oracle, with the same trial and acceptance
    sequence (n = 20,000 is the longest x the one-launch form takes; the
    linear cases have restarts and two reduction steps)."""
    w = PHASE_CASES[case]()
    f = {"one_launch": smx.PHASE_ONE_LAUNCH, "batches": smx.PHASE_BATCHES,
         "closed_form": smx.PHASE_CLOSED_FORM}[form]
    check_parity(smx, w, w.K, phase_form=f)


def linear_phase_launches(p):
    """Launches of the closed-form linear phase the library reports for p: none
    when the fused pass with z in LDS takes it, one when the fused pass's apply
    kernel only leaves it the direction partials, two otherwise."""
    for v in p.describe().values():
        if isinstance(v, dict) and isinstance(v.get("fused"), dict) and v["fused"]["in_use"]:
            return 0 if v["fused"]["zl"] else 1
    return 2


@pytest.mark.parametrize("shape", [(8, 8, 2, 1), (8, 4, 0, 1), (8, 4, 0, 0)])
def test_closed_form_partials_from_apply(smx, shape):
    """The closed-form linear phase on the fused pass takes its direction
    partials from the previous iteration's apply kernel (and from a
    partials launch where a run, or a run of iterations of one value kind,
    starts); with z in LDS the pass itself opens the phase and stages
    z = x + s v, and the apply kernel forms z_j again (no launch of its
    own), with z gathered one closed-form launch adds the step: against the
    oracle with the bf16 operator and a float32 refinement tail (a change of
    value kind mid-run), and across a checkpoint and resume."""
    w = W.random_sparse(6000, 9000, 20, seed=51, empty_frac=0.05, obj=W.OBJ_LINEAR, K=24)
    p = smx.problem_from_workload(w)
    p.set_fused_shape(*shape)
    assert p.fused_in_use() and p.describe()["phase_launches"] == (0 if shape[3] else 1)
    p.close()
    check_parity(smx, w, w.K, storage="bf16", value_round="bf16", refine_iters=5, fused_shape=shape)
    say(f"closed-form phase on the fused pass {shape}, checkpoint and resume")
    p = smx.problem_from_workload(w, history_cap=0)
    p.set_fused_shape(*shape)
    p.run(10, graph=True)
    p.sync()
    states, x1 = p.get_state()
    p.close()
    q = smx.problem_from_workload(w, history_cap=0)
    q.set_fused_shape(*shape)
    q.set_state(states, x1)
    q.run(w.K - 10, graph=True)
    q.sync()
    x = q.get_x().cpu().numpy()[:, 0].astype(np.float64)
    sq, _ = q.get_state()
    q.close()
    xo, sto, ho, _ = oracle_run(w, w.K)
    assert rel(x, xo) <= RTOL and sq[0]["ell"] == sto.ell and sq[0]["trials"] == sto.trials


def test_phase_form_choice_and_args(smx):
    """Auto picks one launch for flat objectives up to n = 8,192, the closed
    form for the linear objective beyond, and the batches otherwise; one
    launch can be asked for up to n = 20,000, the closed form for the linear
    objective, and each is refused where it does not apply."""
    for w, launches, eligible in ((W.random_sparse(300, 200, 8, seed=46, obj=W.OBJ_SQNORM, K=3), 1, True),
                                  (W.random_sparse(300, 8193, 8, seed=49, obj=W.OBJ_LINEAR, K=3), None, True),
                                  (W.random_sparse(300, 20001, 8, seed=47, obj=W.OBJ_L1, K=3), None, False),
                                  (W.ct(N=24, n_angles=16, seed=59, K=5), None, False)):
        p = smx.problem_from_workload(w)
        d = p.describe()
        if launches is not None:
            assert d["phase_launches"] == launches
        elif w.obj == W.OBJ_LINEAR:  # closed form: in the fused pass, or after its apply kernel's partials
            assert d["phase_launches"] == linear_phase_launches(p)
        else:
            assert d["phase_launches"] > 1
        if eligible:
            p.set_phase_form(smx.PHASE_ONE_LAUNCH)
            assert p.describe()["phase_launches"] == 1
        else:
            with pytest.raises(smx.SmxError, match="ESTATE"):
                p.set_phase_form(smx.PHASE_ONE_LAUNCH)
        if w.obj == W.OBJ_LINEAR:
            p.set_phase_form(smx.PHASE_CLOSED_FORM)
            assert p.describe()["phase_launches"] == linear_phase_launches(p)
        else:
            with pytest.raises(smx.SmxError, match="ESTATE"):
                p.set_phase_form(smx.PHASE_CLOSED_FORM)
        p.set_phase_form(smx.PHASE_BATCHES)
        assert p.describe()["phase_launches"] > 1
        p.set_phase_form(smx.PHASE_AUTO)
        assert p.describe()["phase_launches"] == d["phase_launches"]
        with pytest.raises(smx.SmxError, match="EINVAL"):
            p.set_phase_form(4)
        p.run(2, perturb=True, graph=True)
        p.sync()
        p.close()


FUSED_SHAPES = [(8, 4, 0, 0), (8, 8, 0, 0), (16, 4, 0, 0), (16, 4, 4, 0), (16, 8, 0, 0), (16, 8, 2, 0), (32, 4, 0, 0),
                (32, 4, 2, 0), (32, 8, 0, 0), (32, 8, 1, 0), (8, 4, 0, 1), (8, 8, 0, 1), (16, 4, 0, 1), (32, 8, 0, 1),
                (8, 4, 4, 1), (8, 8, 2, 1), (16, 4, 4, 1), (16, 8, 2, 1), (32, 4, 4, 1), (32, 8, 2, 1)]


@pytest.mark.parametrize("case", ["rt", "long_rows"])
def test_every_fused_shape(smx, case):
    """Each launch shape of the fused pass (entries re-read or kept in
    registers, 8-32 lanes per row, z gathered from memory or from LDS)
    against the oracle; the long-row case has rows beyond the entries the
    register-cached shapes hold (256, or 16 a lane with z in LDS)."""
    if case == "rt":
        w = W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=60, K=12)
        storage, vr = "bf16", "bf16"
    else:
        w = W.random_sparse(1500, 3000, 40, seed=61, empty_frac=0.1, long_rows=6, long_len=700,
                            obj=W.OBJ_SQNORM, K=10)
        storage, vr = "f32", None
    xo, sto, ho, P = oracle_run(w, w.K, value_round=vr)
    storage_deviation(w, w.K, value_round=vr)
    te = max(RTOL, 30 * storage_deviation.elem)
    for lpr, vec, cap, zl in FUSED_SHAPES:
        say(f"{case} fused shape lpr={lpr} vec={vec} cap={cap} z_in_lds={zl}")
        p = smx.problem_from_workload(w, storage=storage, history_cap=w.K, refine_iters=0)
        p.set_fused_shape(lpr, vec, cap, zl)
        info = p.describe()[storage]["fused"]
        assert info["in_use"] and (info["lpr"], info["vec"], info["cap"], info["zl"]) == (lpr, vec, cap, zl)
        p.run(w.K)
        p.sync()
        x = p.get_x().cpu().numpy()[:, 0].astype(np.float64)
        h = p.history()
        p.close()
        assert np.array_equal(h["trials"][:, 0], ho.trials)
        r = rel(x, xo)
        assert r <= RTOL and elem(x, xo) <= te, (lpr, vec, cap, zl, r, elem(x, xo), te)
        np.testing.assert_allclose(h["prox"][:, 0], ho.prox, rtol=RTOL, atol=1e-6 * abs(ho.prox[0]))
    p = smx.problem_from_workload(w, storage=storage)
    with pytest.raises(smx.SmxError):
        p.set_fused_shape(8, 4, 8)
    with pytest.raises(smx.SmxError):
        p.set_fused_shape(8, 4, 8, 1)
    with pytest.raises(smx.SmxError):
        smx.check(smx.lib().smx_set_fused_shape(p.handle, 8, 4, 0, 2))
    p.close()


# ---------------------------------------------------------------------------
# adaptive step size (Section 2.1.2; the sixth strategy of the CT experiment)
# ---------------------------------------------------------------------------

ADAPTIVE_CASES = {
    "dense_sqnorm": lambda: W.dense_small(K=60),
    "ct_tv_emr": lambda: W.ct(N=48, n_angles=36, seed=7, K=40).with_params(basic=W.BASIC_EMR),
    "ct_tv": lambda: W.ct(N=48, n_angles=36, seed=8, K=40),
    "rt_linear": lambda: W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=10, K=30),
    "edge_rows_l1": lambda: W.random_sparse(3000, 2000, 12, seed=44, empty_frac=0.08, long_rows=2, obj=W.OBJ_L1,
                                            K=25),
}


@pytest.mark.parametrize("case", list(ADAPTIVE_CASES))
def test_adaptive_step_parity(smx, case):
    """The adaptive step (beta = (f(x^k) - f_ref)/||g|| toward where the last
    phase ended) against the oracle: decisions, iterate, proximities; TV and
    EMR with the conditioning-aware tolerance.  Then two slices at once."""
    w = ADAPTIVE_CASES[case]().with_params(step_rule=W.STEP_ADAPTIVE)
    sensitive = w.obj == W.OBJ_TV2D or getattr(w, "basic", 0) == W.BASIC_EMR
    x, h = check_parity(smx, w, w.K, sensitive=sensitive)
    assert h["trials"][0, 0] == 0 and np.all(h["trials"] <= 1)
    if case == "ct_tv":
        wb = W.ct(N=48, n_angles=36, seed=8, K=40, B=2).with_params(step_rule=W.STEP_ADAPTIVE)
        check_parity(smx, wb, wb.K, sensitive=True)


def test_adaptive_step_lockstep(smx):
    """Oracle-driven single iterations (CT-48, TV, EMR, adaptive step): every
    iterate, proximity, decision and the reference value f_ref at 1e-5."""
    w = W.ct(N=48, n_angles=36, seed=7, K=30).with_params(basic=W.BASIC_EMR, step_rule=W.STEP_ADAPTIVE)
    say("ct48 lockstep, EMR, adaptive step")
    p = smx.problem_from_workload(w, history_cap=w.K)
    P = oracle.from_workload(w)
    x = w.x0[:, 0].astype(np.float32).astype(np.float64)
    so = oracle.State()
    po = []
    for k in range(w.K):
        xg, sg, xo, so1, pk = step_from_oracle(p, P, x, so)
        check_step(xg, sg, xo, so1, False, RTOL, k)
        if not np.isnan(so1.f_ref):
            assert abs(sg["f_ref"] - so1.f_ref) <= RTOL * abs(so1.f_ref), (k, sg["f_ref"], so1.f_ref)
        po.append(pk)
        x, so = xo.astype(np.float32).astype(np.float64), so1
    check_step_proximities(p, range(w.K), po, RTOL)
    p.close()


# ---------------------------------------------------------------------------
# other basic algorithms (DROP, CQ, EL, EMR)
# ---------------------------------------------------------------------------

BASIC_CASES = {"drop": W.BASIC_DROP, "cq": W.BASIC_CQ, "el": W.BASIC_EL, "emr": W.BASIC_EMR}


def _with_basic(w, method):
    kw = dict(basic=BASIC_CASES[method])
    if method == "drop":  # inside DROP's range (0, 2/max w]: lambda = m for uniform weights
        kw["lam"] = float(w.m) if w.weights is None else 1.0 / float(np.max(w.weights / w.weights.sum()))
    return w.with_params(**kw)


@pytest.mark.parametrize("method", ["drop", "cq", "el", "emr"])
@pytest.mark.parametrize("case", ["rt", "edge_rows", "ct_tv"])
def test_basic_algorithm_parity(smx, method, case):
    """Each basic algorithm against the oracle (fused pass where it applies,
    the two passes otherwise, and the two passes forced)."""
    if case == "rt":
        w = W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=70, K=15)
    elif case == "edge_rows":
        w = W.random_sparse(2000, 1500, 25, seed=71, empty_frac=0.05, long_rows=3, long_len=1400,
                            obj=W.OBJ_SQNORM, K=12)
    else:
        w = W.ct(N=32, n_angles=24, seed=72, K=15)
    w = _with_basic(w, method)
    info = _fused_info(smx, w)
    assert info is not None and info["in_use"]
    # the extrapolated steps multiply y by sigma >> 1 on inconsistent sets (the
    # paper notes EL's fluctuation there), amplifying float32 rounding: they take
    # the conditioning-aware tolerance, and their per-iteration check is the
    # lockstep test below
    sens = w.obj == W.OBJ_TV2D or method in ("el", "emr")
    check_parity(smx, w, w.K, sensitive=sens)
    check_parity(smx, w, w.K, sensitive=sens, fused=False)


@pytest.mark.parametrize("method", ["el", "emr"])
@pytest.mark.parametrize("case", ["rt", "ct_tv"])
def test_extrapolated_steps_lockstep(smx, method, case):
    """Each iteration of EL / EMR from the oracle's iterate and state agrees
    with the oracle's to 1e-5, with the same decisions."""
    if case == "rt":
        w = W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=70, K=15)
    else:
        w = W.ct(N=32, n_angles=24, seed=72, K=15)
    w = _with_basic(w, method)
    say(f"{case} {method} lockstep")
    worst = lockstep(smx, w, w.K)
    print(f"  worst per-iteration rel err {worst:.3e}", flush=True)


@pytest.mark.parametrize("tiles", [False, True])
@pytest.mark.parametrize("method", ["el", "emr", "drop"])
def test_basic_algorithm_batched(smx, method, tiles, monkeypatch):
    """Several slices (multi-slice kernels, per-slice sigma) against the oracle;
    with tiles, pass 2 (kept y for EL and EMR, column factors for DROP) runs
    over the image-tile layout."""
    monkeypatch.setenv("SMX_TILES", "1" if tiles else "0")
    w = _with_basic(W.ct(N=32, n_angles=24, seed=73, B=4, K=12), method)
    p = smx.problem_from_workload(w)
    assert (p.describe()["f32"]["pass2"]["mode"] == "tiles") == tiles
    p.close()
    check_parity(smx, w, w.K, sensitive=True)
    if method == "drop":
        check_parity(smx, w, w.K, sensitive=True, fused=False)


@pytest.mark.parametrize("method", ["el", "emr", "cq"])
def test_basic_algorithm_bf16(smx, method):
    w = _with_basic(W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=74, K=12), method)
    check_parity(smx, w, w.K, storage="bf16", value_round="bf16", refine_iters=0, sensitive=method != "cq")


def test_basic_algorithm_args(smx):
    w = W.random_sparse(200, 100, 8, seed=75, obj=W.OBJ_NONE, K=3)
    with pytest.raises(smx.SmxError):
        smx.problem_from_workload(w.with_params(basic=W.BASIC_DROP, lam=2.0 * w.m + 1.0))
    with pytest.raises(smx.SmxError):
        smx.problem_from_workload(w.with_params(basic=W.BASIC_EL, lam=2.5))
    with pytest.raises(smx.SmxError):
        smx.problem_from_workload(w.with_params(basic=7))
    p = smx.problem_from_workload(w.with_params(basic=W.BASIC_DROP, lam=2.0 * w.m))
    assert p.describe()["basic"] == "drop"
    p.close()


# ---------------------------------------------------------------------------
# stopping rules (device-side, per slice)
# ---------------------------------------------------------------------------

def _log_mid(a, b):
    return float(np.sqrt(a * b))


def _margin_ok(values, thr, rel=1e-4):
    v = np.asarray(values, float)
    v = v[np.isfinite(v) & (v > 0)]
    return np.all(np.abs(np.log(v / thr)) > rel)


def _stop_compare(smx, w, K, perturb=True):
    """GPU run with w.stop against the oracle's: same iterations, reason, and
    iterate within the usual tolerance."""
    P = oracle.from_workload(w)
    xo, so, ho = P.run(w.x0[:, 0], K, perturb=perturb)
    p = smx.problem_from_workload(w, history_cap=K, fused=False)
    p.run(K, perturb=perturb)
    p.sync()
    st, x = p.get_state()
    reason = p.stop_status()
    p.close()
    print(f"  oracle k={so.k} reason={so.stop_reason}; gpu k={st[0]['k']} reason={reason[0]}", flush=True)
    assert so.stop_reason != 0, "the oracle did not stop: pick other thresholds"
    assert st[0]["k"] == so.k and reason[0] == so.stop_reason
    assert st[0]["dp_run"] == so.dp_run and st[0]["feas_ok"] == so.feas_ok
    if not perturb:  # (TV-perturbed iterates: the parity and lockstep tests above)
        assert rel(x[:, 0], xo) <= max(RTOL, 10 * storage_deviation(w, so.k, perturb)[0])
    return so


def test_stop_proximity_threshold(smx):
    w = W.ct(N=32, n_angles=24, seed=80, K=60)
    P = oracle.from_workload(w)
    _, _, h = P.run(w.x0[:, 0], 40, perturb=False)
    thr = _log_mid(h.prox[14], h.prox[15])
    assert _margin_ok(h.prox, thr)
    say("stop on P*")
    so = _stop_compare(smx, w.with_params(stop=dict(prox=thr, dprox=-1.0, n=5, max_iters=0, dobj=-1.0)), 40,
                       perturb=False)
    assert so.k == 16 and so.stop_reason == oracle.STOP_PROX


def test_stop_stalled_proximity_and_cap(smx):
    w = W.random_sparse(1500, 800, 15, seed=81, obj=W.OBJ_NONE, K=80)
    P = oracle.from_workload(w)
    _, _, h = P.run(w.x0[:, 0], 80, perturb=False)
    dp = np.abs(np.diff(h.prox)) / np.maximum(1.0, h.prox[:-1])
    thr = _log_mid(dp[19], dp[20])
    assert _margin_ok(dp, thr)
    say("stop on Delta P")
    _stop_compare(smx, w.with_params(stop=dict(prox=-1.0, dprox=thr, n=3, max_iters=0, dobj=-1.0)), 80,
                  perturb=False)
    say("stop on N_max")
    so = _stop_compare(smx, w.with_params(stop=dict(prox=-1.0, dprox=-1.0, n=3, max_iters=9, dobj=-1.0)), 80,
                       perturb=False)
    assert so.k == 9 and so.stop_reason == oracle.STOP_MAXIT


def test_stop_iterate_variance(smx):
    w = W.random_sparse(1500, 800, 15, seed=82, obj=W.OBJ_NONE, K=60)
    w = w.with_params(x0=np.zeros_like(w.x0))  # omega_1 = 1, then small: the variance falls
    P = oracle.from_workload(w)
    xs = [w.x0[:, 0].astype(np.float64)]
    st = None
    for _ in range(60):
        x, st, _ = P.run(xs[-1], 1, perturb=False, state=st)
        xs.append(x)
    om = [np.linalg.norm(xs[i] - xs[i - 1]) / np.linalg.norm(xs[i]) for i in range(1, 61)]
    var = [np.var(om[:k], ddof=1) for k in range(2, 61)]
    thr = _log_mid(var[24], var[25])
    assert _margin_ok(var, thr)
    say("stop on the iterate-change variance")
    so = _stop_compare(smx, w.with_params(stop=dict(prox=-1.0, dprox=-1.0, n=3, max_iters=0, dobj=-1.0, var=thr)),
                       60, perturb=False)
    assert so.stop_reason == oracle.STOP_VAR


def test_stop_superiorized(smx):
    """Superiorized CT: a proximity rule and a small objective change."""
    w = W.ct(N=32, n_angles=24, seed=83, K=80)
    P = oracle.from_workload(w)
    _, _, h = P.run(w.x0[:, 0], 80)
    dp = np.abs(np.diff(h.prox)) / np.maximum(1.0, h.prox[:-1])
    df = np.abs(np.diff(h.f_start)) / np.maximum(1.0, h.f_start[:-1])
    srt = np.sort(df[10:])
    tp, tf = _log_mid(dp[29], dp[30]), _log_mid(srt[len(srt) // 2], srt[len(srt) // 2 + 1])
    assert _margin_ok(dp, tp) and _margin_ok(df, tf)
    say("superiorized stop")
    so = _stop_compare(smx, w.with_params(stop=dict(prox=-1.0, dprox=tp, n=2, max_iters=0, dobj=tf)), 80)
    assert so.stop_reason == oracle.STOP_SM


def test_stop_batched_and_resume(smx):
    """Slices stop at their own iterations; a checkpoint taken after some have
    stopped resumes to the uninterrupted result bitwise."""
    w = W.ct(N=32, n_angles=24, seed=84, B=4, K=60)
    stop = dict(prox=-1.0, dprox=5e-3, n=3, max_iters=0, dobj=-1.0)
    w = w.with_params(stop=stop)
    for s in range(4):
        _, _, h = oracle.from_workload(w.with_params(stop=None), s).run(w.x0[:, s], 60, perturb=False)
        assert _margin_ok(np.abs(np.diff(h.prox)) / np.maximum(1.0, h.prox[:-1]), 5e-3)
    p = smx.problem_from_workload(w, history_cap=0)
    p.run(60, perturb=False)
    p.sync()
    full, xfull = p.get_state()
    reasons = p.stop_status()
    p.close()
    for s in range(4):
        P = oracle.from_workload(w, s)
        _, so, _ = P.run(w.x0[:, s], 60, perturb=False)
        assert full[s]["k"] == so.k and reasons[s] == so.stop_reason, s
    q = smx.problem_from_workload(w, history_cap=0)
    q.run(min(f["k"] for f in full), perturb=False)
    q.sync()
    mid, xmid = q.get_state()
    q.close()
    r = smx.problem_from_workload(w, history_cap=0)
    r.set_state(mid, xmid)
    r.run(60, perturb=False)
    r.sync()
    end, xend = r.get_state()
    r.close()
    assert np.array_equal(xend, xfull) and end == full


# ---------------------------------------------------------------------------
# dose-volume constraints (split problem, Section 2.3.3)
# ---------------------------------------------------------------------------

def _dvc_random(B=1, K=20, obj=W.OBJ_SQNORM, seed=81):
    """A random operator with two dose-volume constraints on (overlapping)
    row sets, their doses between the true point's values."""
    import scipy.sparse as sp

    w = W.random_sparse(2000, 1500, 25, seed=seed, B=B, empty_frac=0.05, long_rows=2, long_len=1400, obj=obj, K=K)
    A = sp.csr_matrix((w.val.astype(np.float64), w.col_idx, w.row_ptr), shape=(w.m, w.n))
    r = A @ np.asarray(w.x_true, np.float64).reshape(w.n, -1)[:, 0]
    rows1, rows2 = np.arange(0, 500), np.arange(300, 900)
    return W.with_dvc(w, [(rows1, W.DVC_MAX, 0.2, float(np.quantile(r[rows1], 0.6))),
                          (rows2, W.DVC_MIN, 0.8, float(np.quantile(r[rows2], 0.4)))])


def _dvc_rt(basic, K=30):
    """The small radiotherapy case with the horseshoe plan's constraints from
    a seeded starting point: the phantom and beams are symmetric, so from
    x0 = 0 the first perturbed point gives mirror voxels doses equal in exact
    arithmetic that rounding alone orders (a tie either nearest point
    resolves); this starting point keeps every ranking of the run clear of
    float32 near-ties (checked by check_parity)."""
    w = W.rt_with_dvc(W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=70, K=K), basic=basic)
    return w.with_params(x0=W.synthetic_iterate(w, seed=79, spread=0.3))


@pytest.mark.parametrize("fused", [True, False])
def test_dvc_random_parity(smx, fused):
    """Two dose-volume constraints beside ordinary bands, squared-norm
    perturbations: the iterate, every proximity and the decisions match, with
    the fused pass (z in LDS: the constraint rows' values stored during the
    pass, their c_i a_i added by a second kernel after the ranking) and with
    the two passes."""
    w = _dvc_random()
    info = _fused_info(smx, w)
    assert info is not None and info["zl"] == 1  # only the shapes that store the rows' values
    check_parity(smx, w, w.K, fused=fused)


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("method", ["simult", "emr"])
def test_dvc_rt_parity(smx, method, fused):
    """The radiotherapy case with the horseshoe plan's dose-volume constraints,
    the linear objective, and the weighted simultaneous or the EMR step, with
    the fused pass and with the two passes."""
    w = _dvc_rt(BASIC_CASES.get(method, W.BASIC_SIMULT))
    check_parity(smx, w, w.K, sensitive=method == "emr", fused=fused)


def test_dvc_rt_emr_lockstep(smx):
    w = _dvc_rt(W.BASIC_EMR, K=20)
    say("rt dose-volume lockstep (EMR)")
    worst = lockstep(smx, w, w.K)
    print(f"  worst per-iteration rel err {worst:.3e}", flush=True)


def test_dvc_batched(smx):
    """Two slices (multi-slice pass kernels, a selection per slice)."""
    check_parity(smx, _dvc_random(B=2, K=15, seed=82), 15)


def test_dvc_bf16(smx):
    w = _dvc_random(K=20, seed=83)
    check_parity(smx, w, w.K, storage="bf16", value_round="bf16")


def test_dvc_query_and_graph(smx):
    """The proximity at a loaded point counts the constraints' projections;
    graph replay equals eager bitwise (two passes)."""
    w = _dvc_random(K=25, seed=84)
    say("dose-volume query and graph replay")
    x = W.synthetic_iterate(w, seed=85)
    p = smx.problem_from_workload(w, history_cap=0)
    p.set_x(x)
    prox, _ = p.query()
    p.close()
    P = oracle.from_workload(w)
    assert prox[0] == pytest.approx(P.proximity(x[:, 0].astype(np.float64)), rel=2e-6)
    xe, _, _, he, _ = gpu_run(smx, w, w.K, graph=False, fused=False)  # the two passes: sums in a fixed order
    xg, _, _, hg, _ = gpu_run(smx, w, w.K, graph=True, fused=False)
    assert np.array_equal(xe, xg) and np.array_equal(he["prox"], hg["prox"])


def test_dvc_invalid_args(smx):
    w = _dvc_random(K=2, seed=86)
    op = smx.Operator(w.m, w.n, w.row_ptr, w.col_idx, w.val)
    g0, g1 = w.dvc
    bad = [
        [dict(g0, row_end=g0["row_begin"])],                   # empty block
        [dict(g0, row_end=w.m + 1)],                           # beyond m
        [g0, dict(g1, row_begin=g1["row_begin"] + 1)],         # not consecutive
        [dict(g0, fraction=1.5)], [dict(g0, fraction=-0.1)],
        [dict(g0, sense=2)], [dict(g0, dose=float("nan"))],
        [g0] * 17,
    ]
    for tab in bad:
        with pytest.raises(smx.SmxError) as e:
            smx.Problem(op, lower=w.lower, upper=w.upper, dvc=tab)
        assert e.value.code == smx.EINVAL, tab
    op.close()


# ---------------------------------------------------------------------------
# image operators: A^T over 8 x 8 pixel tiles with each tile's rows in LDS
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_image_tiles_pass(smx, storage, monkeypatch):
    """An image operator's one-slice problems take pass 2 over the tile layout
    (ragged edge tiles: a 30 x 60 image); the results match the oracle and,
    to float32 rounding, the column copy's pass."""
    w = W.seismic(rows=30, cols=60, n_src=15, n_rec=30, seed=9, K=40, variant="paper")
    info = smx.problem_from_workload(w, storage=storage)
    d = info.describe()[storage]["pass2"]
    info.close()
    assert d["mode"] == "tiles" and d["format"].endswith("+u16"), d
    vr = None if storage == "f32" else storage
    xt, ht = check_parity(smx, w, w.K, storage=storage, value_round=vr, sensitive=True)
    monkeypatch.setenv("SMX_TILES", "0")
    p = smx.problem_from_workload(w, storage=storage)
    assert p.describe()[storage]["pass2"]["mode"] != "tiles"
    p.close()
    xc, hc = check_parity(smx, w, w.K, storage=storage, value_round=vr, sensitive=True)
    assert np.array_equal(ht["trials"], hc["trials"])
    assert rel(xt, xc) < 1e-5


def test_image_tiles_autotuned_ct(smx):
    """CT-64 with the autotuner choosing among tile and column shapes."""
    w = W.ct(N=64, n_angles=48, seed=12, K=30)
    p = smx.problem_from_workload(w, history_cap=w.K)
    shapes = p.autotune(reps=2)
    p.run(w.K)
    p.sync()
    x = p.get_x().cpu().numpy().astype(np.float64)
    p.close()
    say(f"ct64 autotuned pass 2: {shapes['f32']['pass2']}")
    xo, _, _, _ = oracle_run(w, w.K)
    assert rel(x[:, 0], xo) < max(RTOL, 10 * storage_deviation(w, w.K)[0])


def test_image_tiles_absent_when_a_tile_has_too_many_rows(smx):
    """A tile touched by more rows than its LDS copy holds (16,384) leaves the
    operator without the tile layout; pass 2 reads the column copy."""
    m, R, C = 20000, 8, 8
    rng = np.random.default_rng(48)
    cols = rng.integers(0, R * C, size=(m, 2))
    cols.sort(axis=1)
    cols[:, 1] = np.where(cols[:, 1] == cols[:, 0], (cols[:, 0] + 1) % (R * C), cols[:, 1])
    cols.sort(axis=1)
    row_ptr = np.arange(0, 2 * m + 1, 2, dtype=np.int32)
    val = rng.uniform(0.5, 1.5, 2 * m).astype(np.float32)
    xs = rng.uniform(0, 1, R * C)
    A = np.zeros((m, R * C))
    A[np.repeat(np.arange(m), 2), cols.reshape(-1)] = val
    b = A @ xs
    w = W.Workload(name="dense_rows", m=m, n=R * C, row_ptr=row_ptr, col_idx=cols.reshape(-1).astype(np.int32),
                   val=val, lower=(b - 0.05).astype(np.float32)[:, None], upper=(b + 0.05).astype(np.float32)[:, None],
                   box_lo=np.zeros(R * C, np.float32), box_hi=np.ones(R * C, np.float32),
                   x0=np.full((R * C, 1), 0.5, np.float32), obj=W.OBJ_SQNORM, K=10, image=(R, C))
    p = smx.problem_from_workload(w)
    d = p.describe()
    p.close()
    assert d["tiles"] is None and d["f32"]["pass2"]["mode"] != "tiles"
    check_parity(smx, w, w.K)
