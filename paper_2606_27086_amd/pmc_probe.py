"""Workload for hardware-counter runs (rocprofv3 --pmc): one device copy of a
known size (the normalising reference for FETCH_SIZE / WRITE_SIZE), then a few
eagerly launched iterations of the CT 256x256 workload (float32 and bf16
storage, autotuned launch shapes), a smaller copy that marks the boundary, and
a few iterations of the 160x160x80 radiotherapy workload (fused pass and two
passes), so every pass launch is its own dispatch."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 512 * 1024 * 1024
MARK_BYTES = 64 * 1024 * 1024


def _copy(nbytes):
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy {nbytes} bytes done", flush=True)


def _iterate(smx, w, storage, iters, reps, fused=True):
    p = smx.problem_from_workload(w, storage=storage, refine_iters=0, fused=fused)
    p.autotune(reps=reps)
    p.run(iters, perturb=True, graph=False)
    p.sync()
    print(w.name, storage, "fused" if fused else "two passes", p.describe(), flush=True)
    p.close()


def main(iters: int = 5):
    import torch

    import paper_2606_27086_amd as smx
    import workloads as W

    torch.cuda.set_device(0)
    _copy(COPY_BYTES)
    w = W.ct(N=256, seed=2, K=200)
    for storage in ("f32", "bf16"):
        _iterate(smx, w, storage, iters, 3)
    _copy(MARK_BYTES)
    w = W.rt_large(seed=4, K=300)
    for storage in ("f32", "bf16"):
        for fused in (True, False):
            _iterate(smx, w, storage, 3, 2, fused)


if __name__ == "__main__":
    main()
