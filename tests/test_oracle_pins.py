"""Pins of the FP64 oracle to facts fixed outside the oracle itself.

Each test ties one part of the oracle to a closed form, a theorem, a textbook
routine or brute force, so that a plausible slip (a dropped term, a sign, an
index, a transposed operand) fails at least one of them.  CPU only.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _single_row(orc, a, lo, up, lam=1.0, box=None, obj=0, **kw):
    a = np.asarray(a, float)
    n = a.size
    blo, bhi = (None, None) if box is None else box
    return orc.Problem(
        1, n, [0, n], np.arange(n), a, [lo], [up], box_lo=blo, box_hi=bhi, lam=lam, obj=obj, **kw
    )


def _dense_problem(orc, A, lo, up, **kw):
    A = np.asarray(A, float)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    rp = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    return orc.Problem(m, n, rp, cols, A[rows, cols], lo, up, **kw)


# ---------------------------------------------------------------------------
# Projection onto one band (Section 2.1.1) and its relaxation
# ---------------------------------------------------------------------------

def test_golden_halfspace_cases(orc):
    """Hand-derived projections from the half-space formula (golden file)."""
    path = os.path.join(GOLDEN, "halfspace_projection.txt")
    n_cases = 0
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, a, lo, up, lam, x, tx, prox = [f.strip() for f in line.split(";")]
        a = np.array(a.split(), float)
        P = _single_row(orc, a, float(lo), float(up), lam=float(lam))
        x = np.array(x.split(), float)
        Tx, p = P.step(x)
        np.testing.assert_allclose(Tx, np.array(tx.split(), float), rtol=0, atol=1e-14, err_msg=name)
        assert p == pytest.approx(float(prox), abs=1e-14), name
        n_cases += 1
    assert n_cases == 6


@pytest.mark.parametrize("seed", range(6))
def test_single_band_is_euclidean_projection(orc, seed):
    """For one row, lambda = 1 and no box, T(x) is the nearest point of the band:
    compared with a generic constrained least-distance solve (SLSQP)."""
    rng = np.random.default_rng(seed)
    n = 5
    a = rng.standard_normal(n)
    x = rng.standard_normal(n) * 3
    r = a @ x
    lo, up = sorted(rng.uniform(-2, 2, 2))
    if seed % 3 == 0:
        lo = -np.inf
    P = _single_row(orc, a, lo, up)
    Tx, _ = P.step(x)
    cons = []
    if np.isfinite(lo):
        cons.append({"type": "ineq", "fun": lambda y: a @ y - lo, "jac": lambda y: a})
    cons.append({"type": "ineq", "fun": lambda y: up - a @ y, "jac": lambda y: -a})
    res = minimize(
        lambda y: 0.5 * np.sum((y - x) ** 2),
        x,
        jac=lambda y: y - x,
        constraints=cons,
        method="SLSQP",
        options={"ftol": 1e-14, "maxiter": 200},
    )
    assert res.success
    np.testing.assert_allclose(Tx, res.x, atol=1e-7)
    # lands exactly on the violated bound, or stays put
    assert a @ Tx == pytest.approx(min(max(r, lo), up), abs=1e-12)


def test_reflection_lambda2_is_involution(orc):
    """With l = u (a hyperplane) and lambda = 2, T is the reflection: T(T(x)) = x."""
    rng = np.random.default_rng(11)
    for _ in range(5):
        a = rng.standard_normal(4)
        b = rng.standard_normal()
        P = _single_row(orc, a, b, b, lam=2.0)
        x = rng.standard_normal(4)
        y, _ = P.step(x)
        z, _ = P.step(y)
        np.testing.assert_allclose(z, x, atol=1e-13)
        assert a @ (0.5 * (x + y)) == pytest.approx(b, abs=1e-13)


def test_proximity_is_half_weighted_squared_distance(orc):
    """Proximity equals 1/2 sum_i w_i dist(x, C_i)^2 with each distance measured
    by a generic least-distance solve, and weights normalised to sum 1."""
    rng = np.random.default_rng(5)
    m, n = 4, 3
    A = rng.standard_normal((m, n))
    lo = rng.uniform(-1.0, 0.0, m)
    up = lo + rng.uniform(0.1, 0.5, m)
    wts = rng.uniform(0.5, 2.0, m)
    P = _dense_problem(orc, A, lo, up, weights=wts)
    x = rng.standard_normal(n) * 2
    total = 0.0
    for i in range(m):
        a = A[i]
        cons = [
            {"type": "ineq", "fun": lambda y, a=a, l=lo[i]: a @ y - l},
            {"type": "ineq", "fun": lambda y, a=a, u=up[i]: u - a @ y},
        ]
        res = minimize(lambda y: 0.5 * np.sum((y - x) ** 2), x, constraints=cons, method="SLSQP",
                       options={"ftol": 1e-15, "maxiter": 300})
        total += wts[i] / wts.sum() * np.sum((res.x - x) ** 2)
    assert P.proximity(x) == pytest.approx(0.5 * total, rel=1e-6)


# ---------------------------------------------------------------------------
# The simultaneous step
# ---------------------------------------------------------------------------

def test_weighted_least_squares_limit(orc):
    """l = u = b, no box, full column rank: the simultaneous iteration is a
    gradient method on 1/2 ||D^(1/2)(Ax - b)||^2, D = diag(w_i/||a_i||^2), so it
    converges to the weighted least-squares solution (numpy lstsq)."""
    rng = np.random.default_rng(3)
    m, n = 8, 3
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)  # inconsistent
    P = _dense_problem(orc, A, b, b, lam=1.5)
    x, _, _ = P.run(np.zeros(n), 20000, perturb=False)
    D = (1.0 / m) / np.sum(A * A, axis=1)
    ref = np.linalg.lstsq(np.sqrt(D)[:, None] * A, np.sqrt(D) * b, rcond=None)[0]
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("lam", [0.5, 1.0, 1.9])
def test_proximity_nonincreasing_unperturbed(orc, lam):
    """Projected gradient on P with step lambda <= 2/L, L <= sum w_i = 1:
    the proximity never increases, on consistent and inconsistent systems."""
    for seed in range(3):
        w = W.random_sparse(60, 40, 6, seed=100 + seed, empty_frac=0.1)
        P = orc.from_workload(w.with_params(lam=lam))
        _, _, h = P.run(w.x0[:, 0], 200, perturb=False)
        d = np.diff(h.prox)
        assert np.all(d <= 1e-12 * h.prox[:-1] + 1e-300), (seed, d.max())


def test_box_feasible_after_each_step(orc):
    w = W.random_sparse(50, 30, 5, seed=7)
    P = orc.from_workload(w)
    x = w.x0[:, 0].astype(float) * 4 - 2
    for _ in range(10):
        x, _ = P.step(x)
        assert np.all(x >= w.box_lo - 0) and np.all(x <= w.box_hi + 0)


# ---------------------------------------------------------------------------
# Brute-force LP feasibility on tiny instances
# ---------------------------------------------------------------------------

def _vertices(A, lo, up, box):
    """All vertices of {lo <= Ax <= up, -box <= x <= box} by enumeration of
    n-subsets of the bounding hyperplanes."""
    m, n = A.shape
    H, h = [], []
    for i in range(m):
        if np.isfinite(lo[i]):
            H.append(A[i]); h.append(lo[i])
        if np.isfinite(up[i]):
            H.append(A[i]); h.append(up[i])
    for j in range(n):
        e = np.zeros(n); e[j] = 1
        H.append(e); h.append(box); H.append(e); h.append(-box)
    H, h = np.array(H), np.array(h)
    out = []
    for idx in itertools.combinations(range(len(h)), n):
        M = H[list(idx)]
        if abs(np.linalg.det(M)) < 1e-9:
            continue
        out.append(np.linalg.solve(M, h[list(idx)]))
    return out


def _feasible(A, lo, up, box, tol=1e-9):
    for v in _vertices(A, lo, up, box):
        r = A @ v
        if np.all(r >= lo - tol) and np.all(r <= up + tol) and np.all(np.abs(v) <= box + tol):
            return True
    return False


def test_lp_feasibility_brute_force(orc):
    """Vertex enumeration decides feasibility of tiny systems; the unperturbed
    simultaneous method must drive the proximity to 0 exactly on the feasible
    ones, and to the box-constrained minimum of the proximity otherwise.
    Runs the oracle on one thread: its parallel loops only add overhead to
    systems of a few rows (results do not depend on the thread count)."""
    threads = orc.max_threads()
    orc.set_threads(1)
    try:
        _lp_cases(orc)
    finally:
        orc.set_threads(threads)


def _lp_cases(orc):
    n_feas = n_infeas = 0
    for seed in range(100, 140):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 4))
        m = int(rng.integers(2, 7))
        A = rng.integers(-3, 4, size=(m, n)).astype(float)
        A[np.all(A == 0, axis=1), 0] = 1.0
        box = 2.0
        if seed % 2 == 0:  # feasible with a margin around a centre point
            xc = rng.uniform(-1.5, 1.5, n)
            r = A @ xc
            marg = 0.05 * np.linalg.norm(A, axis=1) + rng.uniform(0, 0.5, m)
            lo, up = r - marg, r + marg
        else:
            lo = rng.uniform(-4, 4, m)
            up = lo + rng.uniform(0.0, 0.5, m)
        feas = _feasible(A, lo, up, box)
        P = _dense_problem(orc, A, lo, up, box_lo=np.full(n, -box), box_hi=np.full(n, box), lam=1.0)
        x, _, _ = P.run(np.zeros(n), 100000, perturb=False)
        pk = P.proximity(x)
        if feas:
            n_feas += 1
            if seed % 2 == 0:
                assert pk <= 1e-10, (seed, pk)
            else:
                assert pk <= 1e-5, (seed, pk)
        else:
            n_infeas += 1
            best = np.inf
            for s in range(8):
                x0 = np.random.default_rng(s).uniform(-box, box, n)
                res = minimize(P.proximity, x0, method="L-BFGS-B", bounds=[(-box, box)] * n,
                               options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 2000})
                best = min(best, res.fun)
            assert best > 1e-8
            assert pk == pytest.approx(best, rel=1e-5, abs=1e-9), (seed, pk, best)
    assert n_feas >= 15 and n_infeas >= 5


# ---------------------------------------------------------------------------
# Perturbation schedule (Section 2.1.2, Algorithm 1)
# ---------------------------------------------------------------------------

def _unconstrained(orc, n, obj, **kw):
    """A problem whose feasibility step is the identity (no finite bound)."""
    return orc.Problem(1, n, [0, 0], [], [], [-np.inf], [np.inf], obj=obj, **kw)


def test_sqnorm_norm_dynamics_closed_form(orc):
    """f = ||x||^2 with the direction v = -u, u = x^k/||x^k||, fixed for the
    phase: inside a phase x = s u for a signed scalar s (s = ||x^k|| at the
    start), a trial beta is accepted iff (s - beta)^2 <= s^2, i.e. iff s > 0 and
    beta <= 2 s, and then s <- s - beta.  beta = gamma alpha^ell with ell
    advancing once per trial.  The final x is the product of the per-phase
    factors s_end / s_start times x0."""
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal(7)
    gamma, alpha, n_red, J, K = 1.3, 0.9, 2, 40, 30
    P = _unconstrained(orc, 7, W.OBJ_SQNORM, gamma=gamma, alpha=alpha, n_red=n_red, max_trials=J)
    x, st, h = P.run(x0, K)
    rho, ell, scale, trials, caps = np.linalg.norm(x0), 0, 1.0, 0, 0
    for _ in range(K):
        if rho == 0:
            continue
        s = rho
        for _ in range(n_red):
            ok = False
            for _ in range(J):
                beta = gamma * alpha**ell
                ell += 1
                trials += 1
                if s > 0 and beta <= 2 * s:
                    s -= beta
                    ok = True
                    break
            if not ok:
                caps += 1
                break
        scale *= s / rho
        rho = abs(s)
    assert st.ell == ell and st.trials == trials and st.cap_hits == caps
    assert caps > 0  # the overshoot case is exercised
    np.testing.assert_allclose(x, scale * x0, rtol=1e-12, atol=1e-14)


def test_linear_objective_always_accepts(orc):
    """f = c^T x: f(x + beta v) - f(x) = -beta ||c|| < 0, so every trial is
    accepted, trials = accepts = n_red in each iteration."""
    w = W.random_sparse(40, 25, 5, seed=9, obj=W.OBJ_LINEAR)
    P = orc.from_workload(w.with_params(n_red=3, gamma=0.1))
    _, st, h = P.run(w.x0[:, 0], 15)
    assert np.all(h.trials == 3) and np.all(h.accepts == 3)
    assert st.cap_hits == 0
    assert np.all(h.f_end < h.f_start)


def test_linear_objective_is_summed_dose(orc):
    """With c = A^T 1 the linear objective is the summed 'dose' sum_i (Ax)_i."""
    w = W.random_sparse(30, 20, 4, seed=10)
    A = w.dense()
    c = A.sum(axis=0)
    P = orc.from_workload(w.with_params(obj=W.OBJ_LINEAR, linear_c=c.astype(np.float32)))
    x = np.random.default_rng(1).uniform(0, 1, 20)
    assert P.objective(x) == pytest.approx(np.sum(A @ x), rel=1e-6)


def test_restart_schedule(orc):
    """Restarts at k = n_rs, 2 n_rs, ...: r grows by one and ell <- r.  With every
    trial accepted, ell after K iterations is r + (K - k_last) * n_red."""
    n_red, n_rs, K = 2, 7, 30
    P = _unconstrained(orc, 5, W.OBJ_SQNORM, gamma=1e-3, alpha=0.9, n_red=n_red, restart_every=n_rs)
    x0 = np.full(5, 100.0)
    _, st, h = P.run(x0, K)
    r = (K - 1) // n_rs
    assert st.restarts == r
    assert st.ell == r + (K - r * n_rs) * n_red
    assert np.all(h.accepts == n_red)


def test_bounded_perturbations(orc):
    """The accepted perturbations are summable: their total length is at most
    gamma * sum_{q=0..R} alpha^q / (1 - alpha) for R restarts."""
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(6) * 50
    gamma, alpha, n_rs, K = 2.0, 0.8, 10, 45
    P = _unconstrained(orc, 6, W.OBJ_SQNORM, gamma=gamma, alpha=alpha, n_red=3, restart_every=n_rs)
    x, st, _ = P.run(x0, K)
    R = st.restarts
    bound = gamma * sum(alpha**q for q in range(R + 1)) / (1 - alpha)
    assert np.linalg.norm(x - x0) <= bound + 1e-12


def test_phase_never_increases_objective(orc):
    """Acceptance rule: every accepted trial satisfies f(z) <= f(x^{k,n})."""
    w = W.random_sparse(40, 36, 5, seed=12, obj=W.OBJ_TV2D, tv_shape=(6, 6))
    P = orc.from_workload(w)
    x, _, h = P.run(w.x0[:, 0], 25)
    ok = ~np.isnan(h.f_start)
    assert np.all(h.f_end[ok] <= h.f_start[ok])
    assert np.all(h.accepts <= h.trials)


# ---------------------------------------------------------------------------
# Adaptive step size (Section 2.1.2): beta = (f(x^k) - f_ref)/||g|| when
# f(x^k) > f_ref, else no step; f_ref is f after the previous phase, f(x^0)
# before the first
# ---------------------------------------------------------------------------

def test_adaptive_step_sqnorm_closed_form(orc):
    """f = ||x||^2: g = 2x, v = -x/||x||, so the step to f_ref = c lands on
    z = x (||x||^2 + c) / (2 ||x||^2), always accepted (f(z) <= f(x) iff
    c <= ||x||^2), and f_ref becomes f(z).  The first phase (no reference
    yet) does not move; a point already at or below the reference is not
    moved, and the reference becomes its value."""
    P = _unconstrained(orc, 5, W.OBJ_SQNORM, step_rule=orc.STEP_ADAPTIVE)
    x0 = np.array([1.0, -2.0, 0.5, 3.0, -1.5])
    z, st = P.perturb(x0)
    assert np.array_equal(z, x0) and st.f_ref == np.dot(x0, x0) and st.ell == 0
    r2 = float(np.dot(x0, x0))
    for c in (0.0, 0.3 * r2, 0.99 * r2):
        st = orc.State()
        st.f_ref = c
        z, s1 = P.perturb(x0, st)
        np.testing.assert_allclose(z, x0 * (r2 + c) / (2 * r2), rtol=1e-14)
        assert s1.f_ref == pytest.approx((r2 + c) ** 2 / (4 * r2), rel=1e-14) and s1.ell == 1
    st = orc.State()
    st.f_ref = 2 * r2
    z, s1 = P.perturb(x0, st)
    assert np.array_equal(z, x0) and s1.f_ref == r2 and s1.ell == 0


def test_adaptive_step_linear_reaches_the_reference(orc):
    """f = c^T x: g = c, so the step beta = (c^T x - f_ref)/||c|| along
    -c/||c|| lands exactly on the level f_ref (f decreases by beta ||c||)."""
    rng = np.random.default_rng(3)
    c = rng.uniform(0.1, 1.0, 6)
    P = _unconstrained(orc, 6, W.OBJ_LINEAR, linear_c=c, step_rule=orc.STEP_ADAPTIVE)
    x = rng.uniform(0.0, 2.0, 6)
    st = orc.State()
    st.f_ref = 0.25 * float(c @ x)
    z, s1 = P.perturb(x, st)
    assert float(c @ z) == pytest.approx(0.25 * float(c @ x), rel=1e-13)
    np.testing.assert_allclose(z, x - (0.75 * float(c @ x) / float(c @ c)) * c, rtol=1e-13)
    assert s1.f_ref == pytest.approx(float(c @ z), rel=1e-15)


def test_adaptive_step_run(orc):
    """A superiorized run with the adaptive step (TV on a small CT image): at
    most one trial per iteration, none in the first; every phase ends at or
    below where it started; each phase's reference is where the previous
    phase ended (the first step aims at f(x^0)), checked by replaying each
    phase alone from the run's states; the run is resumable."""
    w = W.ct(N=24, n_angles=16, seed=5, K=25).with_params(step_rule=W.STEP_ADAPTIVE)
    P = orc.from_workload(w)
    x, st, h = P.run(w.x0[:, 0], 25)
    assert h.trials[0] == 0 and np.all(h.trials <= 1) and h.trials.sum() > 5 and h.accepts.sum() > 0
    ok = ~np.isnan(h.f_start)
    assert np.all(h.f_end[ok] <= h.f_start[ok])
    xs, ss = w.x0[:, 0].astype(np.float64), None
    for k in range(25):
        ref = (ss.f_ref if ss is not None else np.nan)
        z, sz = P.perturb(xs, ss)
        assert sz.f_ref == pytest.approx(h.f_end[k], rel=1e-14)
        if k > 0 and h.trials[k]:
            assert h.f_start[k] > ref
        xs, ss, _ = P.run(xs, 1, state=ss)
    assert np.array_equal(xs, x)
    x1, s1, _ = P.run(w.x0[:, 0], 10)
    x2, _, _ = P.run(x1, 15, state=s1)
    assert np.array_equal(x2, x)


def test_perturb_then_step_is_one_iteration(orc):
    """The perturbation phase alone, then the feasibility step, is one outer
    iteration (bitwise); on f = ||x||^2 the phase of the first iteration is
    x (1 - beta/||x||) with beta = gamma (ell = 0), as in the closed form."""
    w = W.random_sparse(40, 36, 5, seed=14, obj=W.OBJ_TV2D, tv_shape=(6, 6))
    P = orc.from_workload(w.with_params(n_red=2, restart_every=3))
    x, st, _ = P.run(w.x0[:, 0], 7)
    z, sz = P.perturb(x, st)
    x2, _ = P.step(z)
    x1, s1, _ = P.run(x, 1, state=st)
    assert np.array_equal(x1, x2) and sz.ell == s1.ell and sz.restarts == s1.restarts
    Q = _unconstrained(orc, 5, W.OBJ_SQNORM, gamma=0.3, alpha=0.9)
    x0 = np.arange(1.0, 6.0)
    z, sz = Q.perturb(x0)
    np.testing.assert_allclose(z, x0 * (1 - 0.3 / np.linalg.norm(x0)), rtol=1e-15)
    assert sz.ell == 1 and sz.k == 0


def _proximity_objective_path(P, x0, K, perturb):
    """(P(x^k), f(x^k)) for k = 1..K along one run."""
    x, st, out = np.asarray(x0, np.float64), None, []
    for _ in range(K):
        x, st, _ = P.run(x, 1, perturb=perturb, state=st)
        out.append((P.proximity(x), P.objective(x)))
    return np.array(out)


def _best_objective_at_levels(path, levels):
    """min f(x^k) over the iterates with P(x^k) <= level, per level (NaN where
    no iterate reaches the level)."""
    return np.array([path[path[:, 0] <= e, 1].min() if np.any(path[:, 0] <= e) else np.nan for e in levels])


@pytest.mark.parametrize("case", ["dense", "ct_tv", "seismic_tv", "rt_linear"])
def test_superiorized_beats_unperturbed_at_equal_proximity(orc, case):
    """'Superior' in the sense of Section 2.1.2: from the same x0, at every
    proximity level on a log grid between the levels both runs reach, the
    lowest objective of the superiorized run is at most that of the
    feasibility-seeking run alone, and strictly lower at the finest level.
    This is the method's aim rather than a theorem; the cases are the small
    dense, CT, seismic and radiotherapy problems (the dense one over 1000
    iterations, once beta has decayed enough for its proximity to fall)."""
    w, K = {"dense": (W.dense_small(), 1000), "ct_tv": (W.ct(N=32, n_angles=24, seed=5, K=60), 60),
            "seismic_tv": (W.seismic(rows=30, cols=60, n_src=15, n_rec=30, seed=9, K=80, variant="paper"), 80),
            "rt_linear": (W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=10, K=40), 40)}[case]
    P = orc.from_workload(w)
    sm = _proximity_objective_path(P, w.x0[:, 0], K, True)
    fe = _proximity_objective_path(P, w.x0[:, 0], K, False)
    hi = min(sm[:, 0].max(), fe[:, 0].max())
    lo = max(sm[:, 0].min(), fe[:, 0].min())
    assert lo < hi
    levels = np.geomspace(hi, lo, 8)
    a, b = _best_objective_at_levels(sm, levels), _best_objective_at_levels(fe, levels)
    assert np.all(a <= b * (1 + 1e-12)), (levels, a, b)
    assert a[-1] < b[-1]


def test_checkpoint_resume_bitwise(orc):
    w = W.random_sparse(40, 36, 5, seed=13, obj=W.OBJ_TV2D, tv_shape=(6, 6))
    P = orc.from_workload(w)
    xa, sa, _ = P.run(w.x0[:, 0], 20)
    x1, s1, _ = P.run(w.x0[:, 0], 8)
    xb, sb, _ = P.run(x1, 12, state=s1)
    assert np.array_equal(xa, xb) and sa.as_dict() == sb.as_dict()


# ---------------------------------------------------------------------------
# Total variation (Section 2.3.1)
# ---------------------------------------------------------------------------

def _tv_problem(orc, R, C, eps):
    n = R * C
    return orc.Problem(1, n, [0, 0], [], [], [-np.inf], [np.inf], obj=W.OBJ_TV2D, tv_rows=R, tv_cols=C, tv_eps=eps)


def test_tv_constant_and_ramps(orc):
    R, C, eps = 5, 8, 0.3
    P = _tv_problem(orc, R, C, eps)
    assert P.objective(np.full(R * C, 2.5)) == pytest.approx((R - 1) * (C - 1) * eps, rel=1e-14)
    I, J = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    a, b = 0.7, -1.9
    X = (a * I + b * J).reshape(-1)
    assert P.objective(X) == pytest.approx((R - 1) * (C - 1) * math.sqrt(a * a + b * b + eps * eps), rel=1e-13)
    # variation along rows only, on a non-square grid: pins the row-major layout
    X = (1.0 * I).reshape(-1)
    assert P.objective(X) == pytest.approx((R - 1) * (C - 1) * math.sqrt(1 + eps * eps), rel=1e-13)
    # a single bright pixel in the interior
    P0 = _tv_problem(orc, R, C, 0.0)
    X = np.zeros((R, C)); X[2, 3] = 1.0
    # terms touching (2,3): its own (sqrt 2), from above (i=1,j=3: dx=1), from the left (i=2,j=2: dy=1)
    assert P0.objective(X.reshape(-1)) == pytest.approx(math.sqrt(2) + 2.0, rel=1e-14)


def test_tv_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(4)
    R, C, eps = 7, 9, 0.05
    P = _tv_problem(orc, R, C, eps)
    x = rng.uniform(0, 1, R * C)
    g = P.gradient(x)
    h = 1e-6
    fd = np.empty_like(x)
    for p in range(x.size):
        e = np.zeros_like(x); e[p] = h
        fd[p] = (P.objective(x + e) - P.objective(x - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_tv_transpose_invariance_and_zero_subgradient(orc):
    rng = np.random.default_rng(6)
    N = 6
    P = _tv_problem(orc, N, N, 0.01)
    X = rng.uniform(0, 1, (N, N))
    assert P.objective(X.reshape(-1)) == pytest.approx(P.objective(X.T.reshape(-1)), rel=1e-14)
    gX = P.gradient(X.reshape(-1)).reshape(N, N)
    gXt = P.gradient(X.T.reshape(-1)).reshape(N, N)
    np.testing.assert_allclose(gX.T, gXt, atol=1e-14)
    P0 = _tv_problem(orc, N, N, 0.0)
    assert np.all(P0.gradient(np.ones(N * N)) == 0.0)


# ---------------------------------------------------------------------------
# Products and storage rounding
# ---------------------------------------------------------------------------

def test_products_match_dense(orc):
    w = W.random_sparse(70, 50, 8, seed=21, long_rows=2)
    A = w.dense()
    P = orc.from_workload(w)
    x = np.random.default_rng(0).standard_normal(50)
    c = np.random.default_rng(1).standard_normal(70)
    np.testing.assert_allclose(P.matvec(x), A @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(P.matvec_t(c), A.T @ c, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(P.row_sqnorms(), np.sum(A * A, axis=1), rtol=1e-14)


def test_bf16_rounding_matches_torch(orc):
    import torch

    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(20000), rng.uniform(-1e-30, 1e-30, 1000), [0.0, -0.0, 1.0, 65504.0]])
    v = v.astype(np.float32)
    # ties: mantissa ending exactly in 0x8000
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000 | (0x3F800000)).view(np.float32)
    v = np.concatenate([v, ties])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    out = orc.round_bf16(v.astype(np.float64))
    assert np.array_equal(out, ref)


def test_f16_scaled_rounding_matches_numpy(orc):
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(20000) * np.exp(rng.uniform(-12, 2, 20000))).astype(np.float32).astype(np.float64)
    out, s = orc.round_f16_scaled(v)
    amax = np.abs(v).max()
    e = math.ceil(math.log2(amax))
    assert s == 2.0 ** (14 - e)
    ref = (v * s).astype(np.float16).astype(np.float64) / s
    assert np.array_equal(out, ref)


# ---------------------------------------------------------------------------
# Other basic algorithms (appendix table of methods; CQ of Section 2.1.1)
# ---------------------------------------------------------------------------

BASIC = {"simult": W.BASIC_SIMULT, "drop": W.BASIC_DROP, "cq": W.BASIC_CQ, "el": W.BASIC_EL, "emr": W.BASIC_EMR}


def test_golden_basic_operators(orc):
    """Hand-derived single steps of each basic algorithm (golden file)."""
    from fractions import Fraction

    n_cases = 0
    for line in open(os.path.join(GOLDEN, "basic_operators.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, method, rows, b, lam, tx = [f.strip() for f in line.split(";")]
        A = np.array([[float(v) for v in r.split()] for r in rows.split("|")])
        b = np.array(b.split(), float)
        P = _dense_problem(orc, A, b, b, lam=float(lam), basic=BASIC[method])
        Tx, _ = P.step(np.zeros(A.shape[1]))
        want = np.array([float(Fraction(v)) for v in tx.split()])
        np.testing.assert_allclose(Tx, want, rtol=1e-14, atol=1e-15, err_msg=name)
        n_cases += 1
    assert n_cases == 10


@pytest.mark.parametrize("method", ["drop", "cq", "el", "emr"])
def test_basic_single_band_is_projection(orc, method):
    """With one band every basic algorithm at lambda = 1 is the Euclidean
    projection onto it (Section 2.1.1 formula); DROP's column factors are 1
    on the row's support and zero columns stay put."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        a = rng.normal(size=6)
        a[rng.random(6) < 0.3] = 0.0
        if not np.any(a):
            continue
        x = rng.normal(size=6) * 3
        r = a @ x
        lo, up = sorted(rng.normal(size=2))
        t = min(max(r, lo), up) - r
        want = x + (t / (a @ a)) * a
        P = _single_row(orc, a, lo, up, basic=BASIC[method])
        Tx, _ = P.step(x)
        np.testing.assert_allclose(Tx, want, rtol=1e-12, atol=1e-12)


def test_emr_residual_orthogonal_to_search_image(orc):
    """EMR's step length minimises the W-weighted residual along y (equality
    bands, no box): the new residual b - A x' is W-orthogonal to A y."""
    rng = np.random.default_rng(8)
    A = rng.normal(size=(9, 5))
    b = rng.normal(size=9)
    w = rng.random(9) + 0.5
    w = w / w.sum()
    x = rng.normal(size=5)
    P = _dense_problem(orc, A, b, b, weights=w, basic=W.BASIC_EMR)
    Tx, _ = P.step(x)
    y = A.T @ (w * (b - A @ x))
    r_new = b - A @ Tx
    assert abs((A @ y) @ (w * r_new)) <= 1e-12 * np.linalg.norm(A @ y) * np.linalg.norm(b - A @ x)


def test_el_extrapolation_at_least_one(orc):
    """EL's extrapolation sigma = t^T D t / ||A^T D t||^2 is >= 1 when the
    weights sum to 1 (Cauchy-Schwarz / convexity of the squared norm), so its
    step is never shorter than the simultaneous projection's."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        A = rng.normal(size=(12, 6))
        b = rng.normal(size=12)
        x = rng.normal(size=6)
        Ps = _dense_problem(orc, A, b, b, basic=W.BASIC_SIMULT)
        Pe = _dense_problem(orc, A, b, b, basic=W.BASIC_EL)
        ds = Ps.step(x)[0] - x
        de = Pe.step(x)[0] - x
        ratio = (de @ ds) / (ds @ ds)
        assert ratio >= 1 - 1e-12
        np.testing.assert_allclose(de, ratio * ds, rtol=1e-10, atol=1e-12)


def _consistent_dense(orc, method, lam):
    rng = np.random.default_rng(40)
    A = rng.normal(size=(40, 15))
    A[rng.random((40, 15)) < 0.5] = 0.0
    xs = rng.uniform(0, 1, 15)
    r = A @ xs
    P = _dense_problem(orc, A, r - 0.1, r + 0.1, basic=BASIC[method], lam=lam, box_lo=np.full(15, -1.0),
                       box_hi=np.full(15, 2.0))
    return P, xs


@pytest.mark.parametrize("method,lam", [("simult", 1.0), ("drop", 40.0), ("cq", 1.0), ("el", 1.0)])
def test_basic_fejer_monotone(orc, method, lam):
    """SIMULT, DROP (lambda = 1/max w, inside its range), CQ and EL are
    Fejer-monotone on a consistent system: the distance to any point of the
    bands and the box never grows."""
    P, xs = _consistent_dense(orc, method, lam)
    x = np.full(15, 1.8)
    d = [np.linalg.norm(x - xs)]
    for _ in range(40):
        x, _ = P.step(x)
        d.append(np.linalg.norm(x - xs))
    assert np.all(np.diff(d) <= 1e-12)
    assert d[-1] < 0.5 * d[0]


def test_emr_reduces_proximity(orc):
    P, _ = _consistent_dense(orc, "emr", 1.0)
    x = np.full(15, 1.8)
    p0 = P.proximity(x)
    for _ in range(40):
        x, _ = P.step(x)
    assert P.proximity(x) < 1e-6 * p0


def test_drop_counts_nonzeros_before_rounding(orc):
    """DROP's column factors count the nonzeros of A as given: an explicit
    column count overrides counting the (possibly rounded) values."""
    A = np.array([[1.0, 1.0, 0.0], [2.0, 0.0, 1.0]])
    b = np.array([2.0, 4.0])
    P = _dense_problem(orc, A, b, b, basic=W.BASIC_DROP, col_nnz=np.array([1.0, 1.0, 1.0]))
    Tx, _ = P.step(np.zeros(3))
    np.testing.assert_allclose(Tx, [1.3, 0.5, 0.4], rtol=1e-14)


# ---------------------------------------------------------------------------
# Stopping rules (Section 2.2.1; superiorized rule of Section 2.2.3; variance
# rule of Section 2.3.2)
# ---------------------------------------------------------------------------

NEVER = dict(prox=-1.0, dprox=-1.0, n=5, max_iters=0, dobj=-1.0, var=0.0)


def test_stop_on_proximity_threshold(orc):
    """One band, lambda = 1: x^1 is its projection, so P(x^1) = 0 <= P* and the
    run stops after iteration 1 (k = 2) however large K is."""
    P = _single_row(orc, [3.0, 4.0], -np.inf, 0.0, stop=dict(NEVER, prox=1e-12))
    x, st, h = P.run(np.array([3.0, 4.0]), 50, perturb=False)
    assert st.k == 2 and st.stop_reason == orc.STOP_PROX
    assert h.prox[0] == pytest.approx(12.5) and h.prox[1] <= 1e-24
    assert np.all(np.isnan(h.prox[2:]))


def test_stop_on_stalled_proximity(orc):
    """Two contradictory bands on one unknown (x >= 1, x <= 0) from x = 1/2:
    the simultaneous step is 0, P stays 1/8, Delta P = 0 from iteration 1 on,
    so N = 5 consecutive small changes end the run at k = 6."""
    P = _dense_problem(orc, [[1.0], [1.0]], [1.0, -np.inf], [np.inf, 0.0], stop=dict(NEVER, dprox=1e-8, n=5))
    x, st, h = P.run(np.array([0.5]), 40, perturb=False)
    assert st.k == 6 and st.stop_reason == orc.STOP_DPROX
    np.testing.assert_allclose(h.prox[:6], 0.125, rtol=1e-15)


def test_stop_on_iteration_cap(orc):
    P = _dense_problem(orc, [[1.0], [1.0]], [1.0, -np.inf], [np.inf, 0.0], stop=dict(NEVER, max_iters=7))
    x, st, h = P.run(np.array([0.5]), 40, perturb=False)
    assert st.k == 7 and st.stop_reason == orc.STOP_MAXIT


def test_stop_on_iterate_variance(orc):
    """x^k = b (1 - 2^-k) for one equality band with lambda = 1/2 from 0, so
    omega_k = 2^-k / (1 - 2^-k); the run stops at the first k whose sample
    variance of omega_1..omega_k is below the threshold."""
    b, thr = 3.0, 0.05
    P = _single_row(orc, [1.0], b, b, lam=0.5, stop=dict(NEVER, var=thr))
    x, st, h = P.run(np.array([0.0]), 100, perturb=False)
    k = np.arange(1, 101)
    om = 0.5 ** k / (1.0 - 0.5 ** k)
    want = next(kk for kk in range(2, 101) if np.var(om[:kk], ddof=1) < thr)
    assert st.stop_reason == orc.STOP_VAR and st.k == want


def test_stop_superiorized_needs_objective_change(orc):
    """f = x^2 on the band [1, 2] from x = 1.5, gamma = 1, alpha = 0.9, one trial
    per phase (always accepted): x^k = 1 for k >= 1, the recorded proximity is
    P^0 = 1/8, P^k = 0.81^k / 2, and f^k = 1.  With Delta P* = 1e-3, N = 3 the
    proximity rule first holds after N consecutive iterations with
    0.095 * 0.81^(k-1) < 1e-3; the next phase sees Delta f = 0 and stops."""
    P = _single_row(orc, [1.0], 1.0, 2.0, obj=W.OBJ_SQNORM, gamma=1.0, alpha=0.9, n_red=1,
                    stop=dict(NEVER, dprox=1e-3, n=3, dobj=1e-6))
    x, st, h = P.run(np.array([1.5]), 200, perturb=True)
    pk = [0.125] + [0.5 * 0.81 ** k for k in range(1, 200)]
    run, k_feas = 0, None
    for k in range(1, 200):
        run = run + 1 if abs(pk[k] - pk[k - 1]) / max(1.0, pk[k - 1]) < 1e-3 else 0
        if run >= 3:
            k_feas = k
            break
    # iteration k_feas completes (k = k_feas + 1); the next one stops at its phase
    assert st.stop_reason == orc.STOP_SM and st.k == k_feas + 1
    np.testing.assert_allclose(h.prox[:st.k], pk[:st.k], rtol=1e-12)


# ---------------------------------------------------------------------------
# L1 perturbation (Section 2.3.1)
# ---------------------------------------------------------------------------

def test_l1_value_and_subgradient(orc):
    """f = sum |x_j|; its (sub)gradient sign(x) (0 at 0) satisfies the
    subgradient inequality f(y) >= f(x) + g.(y - x) everywhere."""
    rng = np.random.default_rng(12)
    P = _unconstrained(orc, 9, W.OBJ_L1)
    for _ in range(50):
        x = rng.normal(size=9)
        x[rng.random(9) < 0.3] = 0.0
        y = rng.normal(size=9)
        assert P.objective(x) == pytest.approx(np.abs(x).sum(), rel=1e-15)
        g = P.gradient(x)
        assert np.array_equal(g, np.sign(x))
        assert P.objective(y) >= P.objective(x) + g @ (y - x) - 1e-12


def test_l1_perturbation_closed_form(orc):
    """Unconstrained, x = (3, -4, 0), gamma = 1, alpha = 1/2, one reduction
    step: v = -sign(x)/sqrt(2); beta = 1 shrinks both nonzero entries by
    1/sqrt(2) (f drops by sqrt(2)), accepted; the next phase uses beta = 1/2."""
    P = _unconstrained(orc, 3, W.OBJ_L1, gamma=1.0, alpha=0.5, n_red=1)
    x, st, h = P.run(np.array([3.0, -4.0, 0.0]), 2)
    r2 = 1.0 / math.sqrt(2.0)
    np.testing.assert_allclose(x, [3.0 - r2 - 0.5 * r2, -4.0 + r2 + 0.5 * r2, 0.0], rtol=1e-15, atol=1e-15)
    assert list(h.trials) == [1, 1] and st.ell == 2
    np.testing.assert_allclose(h.f_start, [7.0, 7.0 - math.sqrt(2.0)], rtol=1e-15)


# ---------------------------------------------------------------------------
# Dose-volume constraints (Section 2.3.3) as output-space sets of the split
# problem: the projection is the nearest point of a nonconvex set
# ---------------------------------------------------------------------------

def _identity_dvc(orc, N, sense, frac, dose, basic=0, lam=1.0, extra_rows=0):
    """N unit rows e_j (the row value is x_j), one dose-volume group over the
    first N rows, and `extra_rows` plain bands [-1, 1] on the same unknowns."""
    m = N + extra_rows
    cols = np.concatenate([np.arange(N), np.arange(extra_rows) % N])
    lo = np.concatenate([np.full(N, -np.inf), -np.ones(extra_rows)])
    up = np.concatenate([np.full(N, np.inf), np.ones(extra_rows)])
    return orc.Problem(m, N, np.arange(m + 1), cols, np.ones(m), lo, up, lam=lam, basic=basic,
                       dvc=[dict(row_begin=0, row_end=N, sense=sense, fraction=frac, dose=dose)])


def _dvc_brute_force(d, sense, k, dose):
    """Nearest point of {at most k values above dose} (MAX) or {at least k
    values at or above dose} (MIN) to d, by enumerating which values change."""
    N = d.size
    best, arg = np.inf, None
    for T in itertools.chain.from_iterable(itertools.combinations(range(N), r) for r in range(N + 1)):
        T = list(T)
        p = d.copy()
        if sense == W.DVC_MAX:
            if len(T) > k:  # T = the values allowed above dose
                continue
            keep = np.zeros(N, bool)
            keep[T] = True
            p[~keep] = np.minimum(p[~keep], dose)
        else:
            if len(T) < k:  # T = the values required at or above dose
                continue
            p[T] = np.maximum(p[T], dose)
        dist = float(np.sum((p - d) ** 2))
        if dist < best - 1e-15:
            best, arg = dist, p
    return best, arg


@pytest.mark.parametrize("sense", [0, 1])
def test_dvc_projection_is_nearest_point(orc, sense):
    """The proximity of a dose-volume group of unit rows is half the weighted
    squared distance to the nearest point of its set, found by brute force over
    which values change; one DROP step with lambda = N (unit columns, D = 1/N)
    lands on that point exactly."""
    rng = np.random.default_rng(90 + sense)
    for trial in range(40):
        N = int(rng.integers(1, 8))
        frac = float(rng.choice([0.0, 0.05, 0.3, 0.5, 0.95, 1.0, rng.uniform()]))
        dose = float(rng.uniform(0.2, 0.8))
        d = rng.uniform(0.0, 1.0, N)
        P = _identity_dvc(orc, N, sense, frac, dose)
        k = P.dvc_count(0)
        assert k == (math.floor(frac * N) if sense == W.DVC_MAX else math.ceil(frac * N))
        best, p = _dvc_brute_force(d, sense, k, dose)
        assert 2 * N * P.proximity(d) == pytest.approx(best, rel=1e-12, abs=1e-15), (trial, N, frac)
        Pd = _identity_dvc(orc, N, sense, frac, dose, basic=W.BASIC_DROP, lam=float(N))
        x1, _ = Pd.step(d)
        np.testing.assert_allclose(x1, p, rtol=0, atol=1e-15)


def test_dvc_ties_rank_by_row_index(orc):
    """Equal values rank by row index: at x = 0 a 'at least 3 of 6 at or above
    1' group raises the first three rows; 'at most 2 of 6 above 0.5' at equal
    values 0.8 keeps the first two."""
    P = _identity_dvc(orc, 6, W.DVC_MIN, 0.5, 1.0, basic=W.BASIC_DROP, lam=6.0)
    x1, prox = P.step(np.zeros(6))
    np.testing.assert_array_equal(x1, [1, 1, 1, 0, 0, 0])
    assert prox == pytest.approx(0.5 * 3 / 6)
    P = _identity_dvc(orc, 6, W.DVC_MAX, 2 / 6, 0.5, basic=W.BASIC_DROP, lam=6.0)
    x1, _ = P.step(np.full(6, 0.8))
    np.testing.assert_allclose(x1, [0.8, 0.8, 0.5, 0.5, 0.5, 0.5], rtol=0, atol=1e-15)
    lo, up = P.bands_at(np.full(6, 0.8))
    np.testing.assert_array_equal(up, [np.inf, np.inf, 0.5, 0.5, 0.5, 0.5])
    assert np.all(lo == -np.inf)


def test_dvc_limits_reduce_to_bands(orc):
    """V = 0 of 'at most' is the plain band (-inf, d]; V = 1 of 'at least' is
    [d, +inf); V = 1 of 'at most' and V = 0 of 'at least' constrain nothing.
    Compared against plain band rows through a whole perturbed run on a
    random operator with other band rows."""
    rng = np.random.default_rng(95)
    m0, n, N = 30, 12, 10
    A = rng.uniform(0, 1, (m0 + N, n)) * (rng.uniform(size=(m0 + N, n)) < 0.5)
    A[m0:] = A[:N]  # the group's rows repeat rows 0..N-1
    lo0 = rng.uniform(0.5, 1.0, m0)
    up0 = lo0 + rng.uniform(0.1, 1.0, m0)
    x0 = rng.uniform(0, 1, n)
    for sense, frac, blo, bup in ((W.DVC_MAX, 0.0, -np.inf, 0.7), (W.DVC_MIN, 1.0, 0.7, np.inf),
                                  (W.DVC_MAX, 1.0, -np.inf, np.inf), (W.DVC_MIN, 0.0, -np.inf, np.inf)):
        lo = np.concatenate([lo0, np.full(N, -np.inf)])
        up = np.concatenate([up0, np.full(N, np.inf)])
        kw = dict(obj=W.OBJ_SQNORM, box_lo=np.zeros(n), box_hi=np.full(n, 2.0), lam=1.5, n_red=2)
        Pg = _dense_problem(orc, A, lo, up, dvc=[dict(row_begin=m0, row_end=m0 + N, sense=sense, fraction=frac,
                                                      dose=0.7)], **kw)
        Pb = _dense_problem(orc, A, np.concatenate([lo0, np.full(N, blo)]), np.concatenate([up0, np.full(N, bup)]),
                            **kw)
        xg, sg, hg = Pg.run(x0, 15)
        xb, sb, hb = Pb.run(x0, 15)
        np.testing.assert_allclose(xg, xb, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(hg.prox, hb.prox, rtol=1e-13)
        assert sg.trials == sb.trials


def test_dvc_rank_uses_exact_values(orc):
    """The ranking compares exact values: 0.6 and 0.6 + 1e-12 (equal in
    float32) on rows 0 and 1 of an 'at most 1 of 2 above 0.5' group keep row 1,
    the higher value, which is the unique nearest point: lowering row 0 costs
    0.1^2, lowering row 1 (0.1 + 1e-12)^2.  The same holds with the rows'
    order reversed, and the boundary query reports the two values."""
    P = _identity_dvc(orc, 2, W.DVC_MAX, 0.5, 0.5)
    lo, up = P.bands_at(np.array([0.6, 0.6 + 1e-12]))
    np.testing.assert_array_equal(up, [0.5, np.inf])
    lo, up = P.bands_at(np.array([0.6 + 1e-12, 0.6]))
    np.testing.assert_array_equal(up, [np.inf, 0.5])
    best, _ = _dvc_brute_force(np.array([0.6, 0.6 + 1e-12]), W.DVC_MAX, 1, 0.5)
    assert 2 * 2 * P.proximity(np.array([0.6, 0.6 + 1e-12])) == pytest.approx(best, rel=1e-12)
    kth, nxt = P.dvc_boundary(np.array([0.6, 0.6 + 1e-12]))
    assert kth[0] == 0.6 + 1e-12 and nxt[0] == 0.6
    # 'at least 1 of 2 at or above 0.9' raises the higher of two near-equal values
    Q = _identity_dvc(orc, 2, W.DVC_MIN, 0.5, 0.9)
    lo, up = Q.bands_at(np.array([0.3, 0.3 + 1e-13]))
    np.testing.assert_array_equal(lo, [-np.inf, 0.9])


# ---------------------------------------------------------------------------
# Sequential projections (Kaczmarz / ART, table of methods): the oracle only
# ---------------------------------------------------------------------------

def test_art_orthogonal_rows_one_sweep(orc):
    """Rows orthogonal to each other: one sweep with lambda = 1 lands on the
    solution of the square system (each projection leaves the others' values)."""
    rng = np.random.default_rng(110)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    A = Q * rng.uniform(0.5, 2.0, 6)[:, None]
    xs = rng.standard_normal(6)
    b = A @ xs
    P = _dense_problem(orc, A, b, b, basic=orc.BASIC_ART)
    x1, prox = P.step(np.zeros(6))
    np.testing.assert_allclose(x1, xs, rtol=1e-12, atol=1e-12)
    assert prox == pytest.approx(0.5 * np.mean((b / np.linalg.norm(A, axis=1)) ** 2), rel=1e-12)


def test_art_converges_on_consistent_system(orc):
    """Kaczmarz sweeps converge to the solution of a consistent nonsingular
    system (numpy solve) and each sweep equals the rows' projections applied
    in order by hand."""
    rng = np.random.default_rng(111)
    A = rng.standard_normal((8, 8)) + 4 * np.eye(8)
    xs = rng.uniform(-1, 1, 8)
    b = A @ xs
    P = _dense_problem(orc, A, b, b, basic=orc.BASIC_ART, lam=1.2)
    x = np.zeros(8)
    by_hand = x.copy()
    for i in range(8):
        a = A[i]
        by_hand = by_hand + 1.2 * (b[i] - a @ by_hand) / (a @ a) * a
    x1, _ = P.step(x)
    np.testing.assert_allclose(x1, by_hand, rtol=1e-13, atol=1e-14)
    xK, _, h = P.run(x, 300, perturb=False)
    np.testing.assert_allclose(xK, np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)
    assert h.prox[-1] < 1e-18


def test_art_single_row_equals_simultaneous(orc):
    """With one row the sweep is the simultaneous step (w = 1)."""
    a = np.array([1.0, -2.0, 0.5])
    Pa = _single_row(orc, a, 0.3, 0.6, lam=1.5, basic=orc.BASIC_ART)
    Ps = _single_row(orc, a, 0.3, 0.6, lam=1.5)
    x = np.array([0.7, 0.1, -0.4])
    np.testing.assert_allclose(Pa.step(x)[0], Ps.step(x)[0], rtol=1e-15, atol=1e-15)
