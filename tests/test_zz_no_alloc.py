"""smx_slot_load_noalloc, the slot load that allocates nothing (its staging in
the library's fixed device scratch), against smx_slot_load: two problems with
the same operator and parameters get the same slot loaded by each entry point,
run the same iterations, and must hold bitwise equal iterates and states; two
calls in a row, the second with a smaller problem (so the scratch still holds
the first call's larger contents), host then device input.  Invalid bands are
rejected before anything changes, sizes beyond the scratch are rejected, and
the call leaves the device's free memory unchanged (the scratch array is
resident once a problem exists on the device)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd as smx

    smx.lib()
    return smx


def _pair(smx, w, B):
    op = smx.Operator(w.m, w.n, w.row_ptr, w.col_idx, w.val)
    kw = smx.workload_kwargs(w)
    kw.update(B=B, lower=np.zeros((w.m, B), np.float32), upper=np.zeros((w.m, B), np.float32))
    probs = [smx.Problem(op, **kw) for _ in range(2)]
    for p in probs:
        for s in range(B):
            p.slot_disable(s)
    return op, probs


def _compare(smx, w, B, slot, device_input):
    import torch

    print(f"[case] no-alloc slot load {w.name} m={w.m} n={w.n} B={B} slot={slot} device_input={device_input}",
          flush=True)
    op, (pa, pb) = _pair(smx, w, B)
    lo, up, x0 = w.lower[:, 0], w.upper[:, 0], w.x0[:, 0]
    pa.slot_load(slot, lo, up, x0, w.K)
    if device_input:
        args = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (lo, up, x0)]
    else:
        args = [lo, up, x0]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    pb.slot_load_noalloc(slot, *args, w.K)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0, "the no-alloc slot load changed the device's free memory"
    for p in (pa, pb):
        p.run(w.K, perturb=True)
        p.sync()
    ka, la = pa.slot_status()
    kb, lb = pb.slot_status()
    assert np.array_equal(ka, kb) and np.array_equal(la, lb)
    assert ka[slot] == w.K
    for s in range(B):
        xa, xb = pa.slot_x_host(s), pb.slot_x_host(s)
        assert np.array_equal(xa, xb), s
    sa, xa_all = pa.get_state()
    sb, xb_all = pb.get_state()
    assert sa == sb and np.array_equal(xa_all, xb_all)
    for p in (pa, pb):
        p.close()
    op.close()


def test_noalloc_slot_load_matches_slot_load(smx):
    big = W.ct(N=64, n_angles=48, seed=12, K=15)
    small = W.random_sparse(700, 300, 9, seed=44, obj=W.OBJ_SQNORM, K=12)
    assert small.m < big.m and small.n < big.n
    _compare(smx, big, 4, 2, device_input=False)
    _compare(smx, small, 2, 1, device_input=True)


def test_noalloc_slot_load_rejects_invalid_bands_unchanged(smx):
    w = W.random_sparse(500, 200, 6, seed=45, obj=W.OBJ_SQNORM, K=5)
    print("[case] no-alloc slot load: invalid bands", flush=True)
    op, (pa, _) = _pair(smx, w, 2)
    pa.slot_load_noalloc(0, w.lower[:, 0], w.upper[:, 0], w.x0[:, 0], 3)
    k0, live0 = pa.slot_status()
    x0 = pa.slot_x_host(0)
    for bad_row, kind in ((17, "nan"), (311, "order")):
        lo, up = w.lower[:, 0].copy(), w.upper[:, 0].copy()
        if kind == "nan":
            up[bad_row] = np.nan
        else:
            lo[bad_row], up[bad_row] = 2.0, 1.0
        with pytest.raises(smx.SmxError) as e:
            pa.slot_load_noalloc(0, lo, up, np.zeros(w.n, np.float32), 9)
        assert e.value.code == smx.EINVAL and str(bad_row) in str(e.value), str(e.value)
        k1, live1 = pa.slot_status()
        assert np.array_equal(k0, k1) and np.array_equal(live0, live1)
        assert np.array_equal(pa.slot_x_host(0), x0)
    pa.close()
    op.close()


def test_noalloc_slot_load_rejects_sizes_beyond_scratch(smx):
    """2m + n floats beyond the 32 MiB scratch: a 4.2M-row operator."""
    m, n = 4_200_000, 2
    print(f"[case] no-alloc slot load beyond the scratch m={m}", flush=True)
    row_ptr = np.arange(m + 1, dtype=np.int32)
    col = (np.arange(m) % n).astype(np.int32)
    val = np.ones(m, np.float32)
    op = smx.Operator(m, n, row_ptr, col, val)
    b = np.zeros((m, 1), np.float32)
    p = smx.Problem(op, lower=b, upper=b, B=1)
    with pytest.raises(smx.SmxError) as e:
        p.slot_load_noalloc(0, b[:, 0], b[:, 0], np.zeros(n, np.float32), 1)
    assert e.value.code == smx.EINVAL and "scratch" in str(e.value)
    p.close()
    op.close()
