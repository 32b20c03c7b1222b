"""Full-size configurations on the GPU, checked at sampled iterations.

The GPU runs in the benchmark's launch configuration (autotuned passes, graph
replay).  At each sampled iteration index k, a seeded point near the true
solution and an iteration state for k (ell, restarts) are loaded into the
device, which runs one iteration; the oracle runs the same iteration from the
same point, and the two iterates must agree to 1e-5 with the same decisions.
The oracle cannot afford whole runs at these sizes, but it can afford single
iterations.  The whole run from x0 is then checked by properties that hold at
any size (every iteration done, finite values, the proximity reduced).
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import RTOL, check_step, check_step_proximities, elem, near_tie_step, rel, say, step_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd as smx

    smx.lib()
    return smx


def sampled_lockstep(smx, w, K, samples, storage="f32"):
    """At each sampled index: the device's iteration from the oracle's point
    against the oracle's (check_step: decisions, the iterate norm-wise and
    element-wise to 1e-5 unless a dose-volume ranking meets a float32
    near-tie), and every step's proximity to 1e-5."""
    t0 = time.time()
    p = smx.problem_from_workload(w, storage=storage, refine_iters=0, history_cap=max(samples) + 1)
    p.autotune(reps=3)
    print(f"  setup {time.time() - t0:.1f}s shapes {p.describe()}", flush=True)
    P = oracle.from_workload(w, value_round=None if storage == "f32" else storage)
    worst, ks_done, po = 0.0, [], []
    for ks in sorted(samples):
        x = W.synthetic_iterate(w, seed=1000 + ks)[:, 0].astype(np.float64)
        so = oracle.State()
        so.k = ks
        so.restarts = ks // w.restart_every if w.restart_every > 0 else 0
        so.ell = ks + so.restarts
        so.trials = so.accepts = so.ell
        t = time.time()
        tie = near_tie_step(P, w, x, so)
        xg, sg, xo, so1, pk = step_from_oracle(p, P, x, so, graph=True)
        r = check_step(xg, sg, xo, so1, tie, RTOL, ks)
        worst = max(worst, r)
        ks_done.append(ks)
        po.append(pk)
        print(f"  k={ks}: rel {r:.2e} trials {sg['trials'] - so.trials} (oracle {so1.trials - so.trials}), "
              f"oracle {time.time() - t:.1f}s", flush=True)
    check_step_proximities(p, ks_done, po, RTOL)
    p.reset(w.x0)
    p.run(1)
    p.sync()
    prox1, _ = p.query()
    p.reset(w.x0)
    p.run(K, graph=True)
    p.sync()
    prox, obj = p.query()
    states, _ = p.get_state()
    p.close()
    print(f"  full run: proximity after one iteration {prox1[0]:.4e}, after {K} {prox[0]:.4e}", flush=True)
    assert states[0]["k"] == K and np.isfinite(prox[0]) and np.isfinite(obj[0])
    assert prox[0] < prox1[0]
    return worst


def test_seismic_full_size(smx):
    w = W.seismic(seed=3, K=500)
    say(f"seismic full m={w.m} n={w.n} nnz={w.nnz}")
    sampled_lockstep(smx, w, w.K, [0, 1, 250, 499])


def test_seismic_full_size_bf16(smx):
    w = W.seismic(seed=3, K=500)
    say("seismic full bf16")
    sampled_lockstep(smx, w, w.K, [0, 250, 499], storage="bf16")


@pytest.fixture(scope="module")
def rt_case():
    """The radiotherapy configuration (160 x 160 x 80 voxels, 9 beams of 47 x 47
    beamlets, ~400M nonzeros) and the oracle's first 120 iterations from x0 on
    the float32 operator.  From x0 = 0 the perturbation (beta = 0.99^k along
    the normalised negative dose gradient) outweighs the feasibility step and
    the box keeps x at 0 for about 85 iterations; by 120 about 1,200
    beamlets are open."""
    t = time.time()
    w = W.rt_large(seed=4, K=300)
    say(f"rt full m={w.m} n={w.n} nnz={w.nnz} (generated in {time.time() - t:.1f}s)")
    t = time.time()
    P = oracle.from_workload(w)
    K = 120
    xo, so, ho = P.run(w.x0[:, 0], K)
    assert np.count_nonzero(xo) > 500
    print(f"  oracle: {K} iterations in {time.time() - t:.1f}s ({oracle.max_threads()} threads)", flush=True)
    return w, P, K, xo, so, ho


def full_run(smx, w, K, storage):
    """K iterations from x0 in the benchmark's launch configuration (autotuned,
    graph replay, no refinement tail): iterate, proximity, objective, history,
    state."""
    p = smx.problem_from_workload(w, storage=storage, refine_iters=0, history_cap=K)
    p.autotune(reps=3)
    p.run(K, graph=True)
    p.sync()
    x = p.get_x().cpu().numpy()[:, 0].astype(np.float64)
    prox, obj = p.query()
    h = p.history()
    st, _ = p.get_state()
    p.close()
    return x, prox[0], obj[0], h, st[0]


def test_rt_full_size(smx, rt_case):
    w, _, _, _, _, _ = rt_case
    sampled_lockstep(smx, w, w.K, [0, 150, 299])


def test_rt_full_size_end_to_end(smx, rt_case):
    """120 iterations from x0 on the full radiotherapy configuration, float32:
    the iterate norm-wise and element by element, every per-iteration
    proximity and the final proximity and objective within 1e-5 of the
    oracle, with the same decisions."""
    w, P, K, xo, so, ho = rt_case
    x, prox, obj, h, st = full_run(smx, w, K, "f32")
    r, re = rel(x, xo), elem(x, xo)
    po, fo = P.proximity(xo), P.objective(xo)
    print(f"  iterate rel {r:.2e} element-wise {re:.2e}; proximity {prox:.6e} (oracle {po:.6e}), "
          f"objective {obj:.6e} (oracle {fo:.6e})", flush=True)
    assert np.array_equal(h["trials"][:, 0], ho.trials) and np.array_equal(h["accepts"][:, 0], ho.accepts)
    assert st["ell"] == so.ell and st["k"] == K
    assert r <= RTOL and re <= RTOL
    np.testing.assert_allclose(h["prox"][:, 0], ho.prox, rtol=RTOL)
    assert abs(prox - po) <= RTOL * abs(po) and abs(obj - fo) <= RTOL * abs(fo)


def test_rt_full_size_bf16_against_float32_oracle(smx, rt_case):
    """bf16-stored A (packed with 16-bit indices), 120 iterations from x0 without
    the refinement tail: proximity and objective within 2e-2 of the oracle on
    the float32 operator."""
    w, P, K, xo, _, _ = rt_case
    x, prox, obj, _, _ = full_run(smx, w, K, "bf16")
    po, fo = P.proximity(xo), P.objective(xo)
    ep, ef = abs(prox - po) / abs(po), abs(obj - fo) / abs(fo)
    print(f"  bf16: proximity rel err {ep:.2e}, objective rel err {ef:.2e}, iterate rel {rel(x, xo):.2e}",
          flush=True)
    assert ep <= 2e-2 and ef <= 2e-2


def test_seismic_full_size_bf16_against_float32_oracle(smx):
    """The straight-ray seismic configuration (200 x 400 cells, 20,000 rays,
    TV), bf16-stored A, all 500 iterations from x0 without the refinement
    tail: proximity and objective within 2e-2 of the oracle on the float32
    operator."""
    w = W.seismic(seed=3, K=500)
    say(f"seismic full bf16 against the float32 oracle, K={w.K}")
    t = time.time()
    P = oracle.from_workload(w)
    xo, _, _ = P.run(w.x0[:, 0], w.K)
    print(f"  oracle: {w.K} iterations in {time.time() - t:.1f}s", flush=True)
    x, prox, obj, _, _ = full_run(smx, w, w.K, "bf16")
    po, fo = P.proximity(xo), P.objective(xo)
    ep, ef = abs(prox - po) / abs(po), abs(obj - fo) / abs(fo)
    print(f"  bf16: proximity rel err {ep:.2e}, objective rel err {ef:.2e}, iterate rel {rel(x, xo):.2e}",
          flush=True)
    assert ep <= 2e-2 and ef <= 2e-2


def test_seismic_fresnel_paper_shape(smx):
    t = time.time()
    w = W.seismic_fresnel(K=200)
    say(f"seismic fresnel paper shape m={w.m} n={w.n} nnz={w.nnz} DROP L1 "
        f"(generated in {time.time() - t:.1f}s)")
    sampled_lockstep(smx, w, w.K, [0, 100, 199])


def test_rt_dose_volume_full_size(smx):
    t = time.time()
    w = W.rt_with_dvc(W.rt_large(seed=4, K=100), basic=W.BASIC_EMR)
    say(f"rt full with dose-volume constraints m={w.m} n={w.n} nnz={w.nnz} EMR "
        f"(generated in {time.time() - t:.1f}s)")
    sampled_lockstep(smx, w, w.K, [0, 50, 99])
