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
from test_gpu_parity import rel, say, step_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd as smx

    smx.lib()
    return smx


def sampled_lockstep(smx, w, K, samples, storage="f32"):
    t0 = time.time()
    p = smx.problem_from_workload(w, storage=storage, refine_iters=0)
    p.autotune(reps=3)
    print(f"  setup {time.time() - t0:.1f}s shapes {p.describe()}", flush=True)
    P = oracle.from_workload(w, value_round=None if storage == "f32" else storage)
    worst = 0.0
    for ks in sorted(samples):
        x = W.synthetic_iterate(w, seed=1000 + ks)[:, 0].astype(np.float64)
        so = oracle.State()
        so.k = ks
        so.restarts = ks // w.restart_every if w.restart_every > 0 else 0
        so.ell = ks + so.restarts
        so.trials = so.accepts = so.ell
        t = time.time()
        xg, sg, xo, so1 = step_from_oracle(p, P, x, so, graph=True)
        r = rel(xg, xo)
        worst = max(worst, r)
        print(f"  k={ks}: rel {r:.2e} trials {sg['trials'] - so.trials} (oracle {so1.trials - so.trials}), "
              f"oracle {time.time() - t:.1f}s", flush=True)
        assert sg["trials"] == so1.trials and sg["ell"] == so1.ell and sg["accepts"] == so1.accepts, ks
        assert r <= 1e-5, (ks, r)
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


def test_rt_full_size(smx):
    t = time.time()
    w = W.rt_large(seed=4, K=300)
    say(f"rt full m={w.m} n={w.n} nnz={w.nnz} (generated in {time.time() - t:.1f}s)")
    sampled_lockstep(smx, w, w.K, [0, 150, 299])


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
