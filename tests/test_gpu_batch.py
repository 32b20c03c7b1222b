"""Multi-slice (SpMM) passes and slots: B right-hand sides sharing one A.

Each slice must match the FP64 oracle as if it ran alone; a slot's result must
be bitwise identical whether the other slots of the same problem are active,
idle or loaded at other times; per-slot iteration budgets must stop a slot at
exactly its budget.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import check_parity, oracle_run, rel, say, storage_deviation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd as smx

    smx.lib()
    return smx


@pytest.mark.parametrize("B", [2, 8, 32])
def test_batched_ct_slices_match_oracle(smx, B):
    w = W.ct(N=32, n_angles=24, seed=30 + B, B=B, K=20)
    check_parity(smx, w, w.K, sensitive=True)


@pytest.mark.parametrize("obj", [W.OBJ_SQNORM, W.OBJ_LINEAR, W.OBJ_NONE])
def test_batched_random_sparse(smx, obj):
    w = W.random_sparse(1500, 900, 14, seed=33 + obj, B=4, empty_frac=0.05, long_rows=2, obj=obj, K=15)
    check_parity(smx, w, w.K, perturb=obj != W.OBJ_NONE)


@pytest.mark.parametrize("storage,B", [("f32", 2), ("f32", 4), ("bf16", 4), ("f32", 8)])
def test_batched_image_tiles(smx, storage, B, monkeypatch):
    """Several slices of an image operator take pass 2 over the tile layout (a
    44 x 44 image: ragged edge tiles); each slice matches the oracle, and the
    column copy's pass to float32 rounding with the same trial decisions."""
    w = W.ct(N=44, n_angles=30, seed=38, B=B, K=20)
    monkeypatch.setenv("SMX_TILES", "1")
    p = smx.problem_from_workload(w, storage=storage)
    d = p.describe()[storage]["pass2"]
    p.close()
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


def test_batched_tiles_only_where_lds_holds_them(smx, monkeypatch):
    """A tile's staged rows take B floats each: with 180 angles a tile of a
    64 x 64 image is crossed by some 1,800 rays, which fit 64 KB of LDS for 8
    slices but not for 32, where pass 2 keeps the column copy."""
    monkeypatch.setenv("SMX_TILES", "1")
    w8 = W.ct(N=64, n_angles=180, seed=39, B=8, K=5)
    p = smx.problem_from_workload(w8)
    assert p.describe()["f32"]["pass2"]["mode"] == "tiles"
    p.close()
    w32 = W.ct(N=64, n_angles=180, seed=39, B=32, K=5)
    p = smx.problem_from_workload(w32)
    assert p.describe()["f32"]["pass2"]["mode"] != "tiles"
    p.close()


def test_batched_bf16(smx):
    w = W.ct(N=32, n_angles=24, seed=36, B=4, K=20)
    check_parity(smx, w, w.K, storage="bf16", value_round="bf16", sensitive=True)


def _run_slots(smx, w, active, K, budgets=None, graph=False):
    """A problem of capacity w.B where only the slots in `active` are loaded."""
    p = smx.problem_from_workload(w, history_cap=0)
    for s in range(w.B):
        if s in active:
            b = K if budgets is None else budgets[s]
            p.slot_load(s, w.lower[:, s], w.upper[:, s], w.x0[:, s], b)
        else:
            p.slot_load(s, w.lower[:, s], w.upper[:, s], w.x0[:, s], 0)
    p.run(K, graph=graph)
    p.sync()
    xs = {s: p.slot_x(s).cpu().numpy() for s in range(w.B)}
    k, live = p.slot_status()
    p.close()
    return xs, k, live


def test_slot_alone_equals_full_batch_bitwise(smx):
    w = W.ct(N=32, n_angles=24, seed=37, B=8, K=25)
    say("slot alone vs full batch")
    full, _, _ = _run_slots(smx, w, set(range(8)), w.K)
    for s in (0, 3, 7):
        alone, k, live = _run_slots(smx, w, {s}, w.K)
        assert np.array_equal(alone[s], full[s]), s
        assert k[s] == w.K and all(k[q] == 0 for q in range(8) if q != s)


def test_slot_budgets_stop_exactly(smx):
    w = W.ct(N=32, n_angles=24, seed=38, B=4, K=30)
    budgets = [30, 10, 0, 21]
    say("slot budgets")
    xs, k, live = _run_slots(smx, w, {0, 1, 2, 3}, 30, budgets=budgets)
    assert list(k) == budgets and not any(live)
    for s, b in enumerate(budgets):
        if b == 0:
            assert np.array_equal(xs[s], w.x0[:, s])
            continue
        alone, k1, _ = _run_slots(smx, w, {s}, b)
        assert np.array_equal(alone[s], xs[s]), s
        xo, _, _, _ = oracle_run(w.slice(s), b)
        dx, _, _ = storage_deviation(w.slice(s), b)
        assert rel(xs[s], xo) <= max(1e-5, 10 * dx)


def test_slot_reload_mid_run(smx):
    """A slot reloaded with a new problem while others keep iterating ends
    exactly as if it had run alone, and the others are unaffected."""
    w = W.ct(N=32, n_angles=24, seed=39, B=4, K=20)
    say("slot reload")
    p = smx.problem_from_workload(w, history_cap=0)
    for s in range(4):
        p.slot_load(s, w.lower[:, s], w.upper[:, s], w.x0[:, s], 20 if s != 2 else 5)
    p.run(5)
    # slot 2 finished its 5 iterations; give it slot 1's problem for 15 iterations
    p.slot_load(2, w.lower[:, 1], w.upper[:, 1], w.x0[:, 1], 15)
    p.run(15)
    p.sync()
    k, live = p.slot_status()
    x2 = p.slot_x(2).cpu().numpy()
    x1 = p.slot_x(1).cpu().numpy()
    p.close()
    assert list(k) == [20, 20, 15, 20]
    w1 = w.with_params(lower=np.repeat(w.lower[:, 1:2], 4, 1), upper=np.repeat(w.upper[:, 1:2], 4, 1),
                       x0=np.repeat(w.x0[:, 1:2], 4, 1))
    alone15, _, _ = _run_slots(smx, w1, {2}, 15)
    assert np.array_equal(alone15[2], x2)
    alone20, _, _ = _run_slots(smx, w, {1}, 20)
    assert np.array_equal(alone20[1], x1)


def test_batched_graph_equals_eager(smx):
    w = W.ct(N=32, n_angles=24, seed=40, B=8, K=23)
    say("batched graph vs eager")
    a, _, _ = _run_slots(smx, w, set(range(8)), w.K, graph=False)
    b, _, _ = _run_slots(smx, w, set(range(8)), w.K, graph=True)
    for s in range(8):
        assert np.array_equal(a[s], b[s])


def test_slot_load_rejects_bad_input(smx):
    w = W.ct(N=16, n_angles=8, seed=41, B=2, K=3)
    p = smx.problem_from_workload(w)
    with pytest.raises(smx.SmxError):
        p.slot_load(2, w.lower[:, 0], w.upper[:, 0], w.x0[:, 0], 3)
    lo = w.lower[:, 0].copy()
    lo[0] = w.upper[0, 0] + 1
    with pytest.raises(smx.SmxError):
        p.slot_load(0, lo, w.upper[:, 0], w.x0[:, 0], 3)
    with pytest.raises(smx.SmxError):
        p.slot_load(0, w.lower[:, 0], w.upper[:, 0], w.x0[:, 0], -1)
    p.close()
