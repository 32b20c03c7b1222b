"""smx_footprint against what the library allocates: the problem's bytes equal
the sum of the buffers smx_problem_create allocates (exactly, over the
configurations that change the plan), the operator's bound holds, and both
agree with the device's own free-memory count around creation on the
radiotherapy and CT-512 shapes."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _dvc_random, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27086_amd as smx

    smx.lib()
    return smx


def _planned(smx, w, storage, history_cap=0):
    kw = smx.workload_kwargs(w, history_cap=history_cap)
    return smx.problem_footprint(w.m, w.n, w.nnz, storage, keep_f32=True, image=getattr(w, "image", None), **kw)


CASES = [
    ("ct64 f32 (fused pass)", lambda: W.ct(N=64, n_angles=48, seed=12, K=10), "f32", 0),
    ("ct64 bf16 8 slices, history", lambda: W.ct(N=64, n_angles=48, seed=12, K=10, B=8), "bf16", 25),
    ("random EMR", lambda: W.random_sparse(3000, 2000, 12, seed=40, obj=W.OBJ_SQNORM, K=5).with_params(basic=4),
     "f32", 7),
    ("random EL bf16", lambda: W.random_sparse(3000, 2000, 12, seed=41, obj=W.OBJ_L1, K=5).with_params(basic=3),
     "bf16", 0),
    ("random CQ, variance rule", lambda: W.random_sparse(3000, 2000, 12, seed=42, obj=W.OBJ_LINEAR, K=5)
     .with_params(basic=2, stop=dict(var=1e-9, n=3)), "f32", 0),
    ("dose-volume, two slices", lambda: _dvc_random(B=2, K=5, seed=82), "f32", 5),
    ("row panels (m > 40,448)", lambda: W.random_sparse(100001, 700, 6, seed=50, obj=W.OBJ_SQNORM, K=5), "bf16", 0),
]


@pytest.mark.parametrize("name,make,storage,hc", CASES, ids=[c[0] for c in CASES])
def test_problem_footprint_equals_allocation(smx, name, make, storage, hc):
    w = make()
    say(f"footprint {name} m={w.m} n={w.n} B={w.B}")
    ob, pb = _planned(smx, w, storage, hc)
    p = smx.problem_from_workload(w, storage=storage, history_cap=hc)
    d = p.describe()
    p.close()
    print(f"  planned problem {pb} allocated {d['device_bytes']}; operator bound {ob} allocated "
          f"{d['operator_bytes']}", flush=True)
    assert pb == d["device_bytes"]
    assert d["operator_bytes"] <= ob


@pytest.mark.parametrize("shape", ["rt_160x160x80", "ct512_8_slices"])
def test_footprint_against_device_free_memory(smx, shape):
    """The drop in the device's free memory across operator and problem
    creation (torch's cached blocks released before each reading) against
    the footprint: the problem's share within 2 % + 16 MiB (allocation
    granularity), the operator's below its bound."""
    import torch

    w = W.rt_large(seed=4, K=20) if shape.startswith("rt") else W.ct(N=512, seed=2, K=20, B=8)
    storage = "f32" if shape.startswith("rt") else "bf16"
    say(f"footprint vs free memory {shape} m={w.m} n={w.n} nnz={w.nnz} B={w.B} {storage}")
    ob, pb = _planned(smx, w, storage)

    def free():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return torch.cuda.mem_get_info()[0]

    tiny = W.random_sparse(50, 40, 4, seed=3, K=1)  # a first problem makes the library's fixed scratch resident
    smx.problem_from_workload(tiny).close()
    f0 = free()
    op = smx.Operator(w.m, w.n, w.row_ptr, w.col_idx, w.val, storage=storage, image=getattr(w, "image", None))
    f1 = free()
    p = smx.problem_from_workload(w, storage=storage, op=op)
    f2 = free()
    d = p.describe()
    p.close()
    op.close()
    d_op, d_pb = f0 - f1, f1 - f2
    print(f"  operator: free-memory drop {d_op / 2**20:.1f} MiB, allocated {d['operator_bytes'] / 2**20:.1f}, "
          f"bound {ob / 2**20:.1f}; problem: drop {d_pb / 2**20:.1f} MiB, planned {pb / 2**20:.1f}", flush=True)
    assert pb == d["device_bytes"]
    assert abs(d_pb - pb) <= 0.02 * pb + (16 << 20)
    assert d_op <= ob + (16 << 20)


def test_release_panels(smx):
    """An operator's row-panel layout freed before any problem uses it: the
    operator holds fewer bytes, problems on it run the column pass 2 instead
    and still match the oracle; refused while a problem exists; a second
    release frees nothing and succeeds."""
    from test_gpu_parity import RTOL, oracle_run, rel

    w = W.random_sparse(100001, 700, 6, seed=50, obj=W.OBJ_SQNORM, K=5)
    say(f"release panels m={w.m} n={w.n}")
    op = smx.Operator(w.m, w.n, w.row_ptr, w.col_idx, w.val, storage="bf16")
    p = smx.problem_from_workload(w, storage="bf16", op=op, fused=False)
    before = p.describe()["operator_bytes"]
    with pytest.raises(smx.SmxError, match="ESTATE"):
        op.release_panels()
    p.close()
    op.release_panels()
    op.release_panels()
    q = smx.problem_from_workload(w, storage="f32", op=op, fused=False, history_cap=w.K)
    d = q.describe()
    assert d["operator_bytes"] < before
    assert all(d[st]["pass2"]["mode"] != "panels" for st in ("f32", "bf16") if st in d)
    q.autotune(reps=2)
    assert all(q.describe()[st]["pass2"]["mode"] != "panels" for st in ("f32", "bf16") if st in d)
    q.run(w.K)
    q.sync()
    x = q.get_x().cpu().numpy()[:, 0].astype(np.float64)
    q.close()
    op.close()
    xo, _, _, _ = oracle_run(w, w.K)
    assert rel(x, xo) <= RTOL


def test_read_rate_probe(smx):
    """The read-only stream of the measurement aid reads every word: its
    per-workgroup sums add up to the buffer's sum; misaligned or ragged
    buffers and bad grids are refused."""
    import torch

    g = torch.Generator().manual_seed(5)
    buf = torch.rand(1 << 20 | 4, generator=g).cuda()  # 16-byte multiple with a ragged tail
    part = torch.zeros(300, dtype=torch.float32, device="cuda")
    smx.read_rate_probe(buf, part, 300)
    torch.cuda.synchronize()
    assert abs(float(part.double().sum()) - float(buf.double().sum())) <= 1e-5 * float(buf.double().sum())
    with pytest.raises(smx.SmxError, match="EINVAL"):
        smx.read_rate_probe(buf[1:-3], part, 300)  # 4-byte offset
    with pytest.raises(smx.SmxError, match="EINVAL"):
        smx.read_rate_probe(buf[:-1], part, 300)  # not a multiple of 16 bytes
    with pytest.raises(smx.SmxError, match="EINVAL"):
        smx.check(smx.lib().smx_read_rate_probe(buf.data_ptr(), 64, part.data_ptr(), 0, None))
