"""Continuous-batching server: results equal a solo run bitwise, match the
oracle, admission respects the HBM budget, and latency statistics come out."""
import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import rel, say, storage_deviation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd.serve as srv

    return srv


def _specs(srv, ops):
    return {k: srv.OperatorSpec(key=k, m=o["m"], n=o["n"], row_ptr=o["row_ptr"], col_idx=o["col_idx"],
                                val=o["val"], params=o["params"]) for k, o in ops.items()}


def _requests(srv, reqs):
    return [srv.Request(rid=r["rid"], op_key=r["op_key"], lower=r["lower"], upper=r["upper"], x0=r["x0"], K=r["K"],
                        t_arrival=r["t_arrival"]) for r in reqs]


def test_mix_equals_solo_and_oracle(srv):
    ops, reqs, pools = W.serving_mix(sizes=(24, 32), n_requests=10, slices=(2, 5), pool=6, K=12, seed=7,
                                     n_angles=20, rate_hz=400.0)
    say("serving mix")
    specs = _specs(srv, ops)
    server = srv.Server(specs, hbm_budget=1 << 34, slots=8, chunk=4, storage="f32", autotune=False)
    stats = server.run(_requests(srv, reqs))
    server.close()
    print(f"  {stats}", flush=True)
    assert stats["requests"] == len(reqs) and stats["rejected"] == 0
    assert stats["p50_ms"] is not None and stats["p99_ms"] >= stats["p50_ms"]
    done = {r.rid: r for r in server.done}
    # alone: one request at a time through a fresh server of the same capacity
    for rid in (0, 3, 7):
        solo = srv.Server(specs, hbm_budget=1 << 34, slots=8, chunk=4, storage="f32", autotune=False)
        solo.run(_requests(srv, [dict(reqs[rid], t_arrival=0.0)]))
        r_solo = solo.done[0]
        solo.close()
        assert np.array_equal(r_solo.result, done[rid].result), rid
    # every slice of two requests against the oracle
    for rid in (1, 5):
        r = reqs[rid]
        w = pools[r["op_key"]]
        for j, s in enumerate(r["pool_index"]):
            ws = w.slice(int(s))
            P = oracle.from_workload(ws)
            xo, _, _ = P.run(ws.x0[:, 0], r["K"])
            dx, _, _ = storage_deviation(ws, r["K"])
            assert rel(done[rid].result[:, j], xo) <= max(1e-5, 10 * dx)


def test_footprint_admission_and_eviction(srv):
    ops, reqs, _ = W.serving_mix(sizes=(24, 32), n_requests=6, slices=(2, 3), pool=4, K=6, seed=8, n_angles=16)
    specs = _specs(srv, ops)
    probe = srv.Server(specs, hbm_budget=1 << 34, slots=4, storage="f32", autotune=False)
    need = {k: probe.group_bytes(s) for k, s in specs.items()}
    budget = max(need.values()) + min(need.values()) // 2  # room for one group at a time
    server = srv.Server(specs, hbm_budget=budget, slots=4, chunk=3, storage="f32", autotune=False)
    stats = server.run(_requests(srv, reqs))
    assert stats["requests"] == len(reqs)
    assert server.resident_bytes() <= budget
    server.close()
    tiny = srv.Server(specs, hbm_budget=min(need.values()) - 1, slots=4, storage="f32", autotune=False)
    stats = tiny.run(_requests(srv, reqs))
    assert stats["requests"] == 0 and stats["rejected"] == len(reqs)
    tiny.close()


def test_mix_bf16_against_float32_oracle(srv):
    """The served path as the benchmark runs it (bf16-stored A, no refinement
    tail): each result equals its solo run bitwise, and every slice's
    proximity and objective are within 2e-2 of the oracle's run on the
    float32 operator."""
    ops, reqs, pools = W.serving_mix(sizes=(24, 32), n_requests=8, slices=(2, 4), pool=6, K=30, seed=9,
                                     n_angles=20, rate_hz=400.0)
    say("serving mix, bf16")
    specs = _specs(srv, ops)
    server = srv.Server(specs, hbm_budget=1 << 34, slots=8, chunk=5, storage="bf16", autotune=False)
    stats = server.run(_requests(srv, reqs))
    server.close()
    print(f"  {stats}", flush=True)
    assert stats["requests"] == len(reqs) and stats["rejected"] == 0
    done = {r.rid: r for r in server.done}
    for rid in (0, 5):
        solo = srv.Server(specs, hbm_budget=1 << 34, slots=8, chunk=5, storage="bf16", autotune=False)
        solo.run(_requests(srv, [dict(reqs[rid], t_arrival=0.0)]))
        assert np.array_equal(solo.done[0].result, done[rid].result), rid
        solo.close()
    worst = 0.0
    for r in reqs:
        w = pools[r["op_key"]]
        for j, s in enumerate(r["pool_index"]):
            ws = w.slice(int(s))
            P = oracle.from_workload(ws)
            xo, _, _ = P.run(ws.x0[:, 0], r["K"])
            xs = done[r["rid"]].result[:, j].astype(np.float64)
            po, fo = P.proximity(xo), P.objective(xo)
            ep = abs(P.proximity(xs) - po) / abs(po)
            ef = abs(P.objective(xs) - fo) / abs(fo)
            worst = max(worst, ep, ef)
            assert ep <= 2e-2 and ef <= 2e-2, (r["rid"], j, ep, ef)
    print(f"  worst proximity/objective rel err against the float32 oracle: {worst:.2e}", flush=True)
