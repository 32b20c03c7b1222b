"""Full-size configurations on the GPU, checked at sampled iterations.

The GPU runs the whole configuration (the benchmark's launch shapes: graph
replay, autotuned passes).  At sampled iterations k the oracle starts from the
GPU's own iterate and state and runs one iteration; the GPU's next iterate
must agree to 1e-5 with the same decisions.  The oracle cannot afford the
whole run at these sizes, but it can afford single iterations.
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import rel, say

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
    k = 0
    worst = 0.0
    for ks in sorted(samples):
        if ks > k:
            p.run(ks - k, graph=True)
            k = ks
        states, xk = p.get_state()
        assert states[0]["k"] == ks
        so = oracle.State()
        for f in ("k", "ell", "restarts", "trials", "accepts", "cap_hits"):
            setattr(so, f, states[0][f])
        t = time.time()
        xo, so1, _ = P.run(xk[:, 0].astype(np.float64), 1, state=so)
        p.run(1, graph=True)
        k += 1
        states1, xg = p.get_state()
        r = rel(xg[:, 0].astype(np.float64), xo)
        worst = max(worst, r)
        print(f"  k={ks}: rel {r:.2e} trials {states1[0]['trials'] - states[0]['trials']} "
              f"(oracle {so1.trials - so.trials}), oracle {time.time() - t:.1f}s", flush=True)
        assert states1[0]["trials"] == so1.trials and states1[0]["ell"] == so1.ell, ks
        assert r <= 1e-5, (ks, r)
    if k < K:
        p.run(K - k, graph=True)
    p.sync()
    prox, obj = p.query()
    states, _ = p.get_state()
    p.close()
    assert states[0]["k"] == K and np.isfinite(prox[0]) and np.isfinite(obj[0])
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
