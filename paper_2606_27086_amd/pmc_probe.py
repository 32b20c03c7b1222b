"""Workload for hardware-counter runs (rocprofv3 --pmc): one device copy of a
known size (the normalising reference for FETCH_SIZE / WRITE_SIZE), then a few
eagerly launched iterations of the CT 256x256 workload (float32 and bf16
storage, autotuned launch shapes), so every pass launch is its own dispatch."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 512 * 1024 * 1024


def main(iters: int = 5):
    import torch

    import paper_2606_27086_amd as smx
    import workloads as W

    torch.cuda.set_device(0)
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy {COPY_BYTES} bytes done", flush=True)
    w = W.ct(N=256, seed=2, K=200)
    for storage in ("f32", "bf16"):
        p = smx.problem_from_workload(w, storage=storage, refine_iters=0)
        p.autotune(reps=3)
        p.run(iters, perturb=True, graph=False)
        p.sync()
        print(storage, p.describe(), flush=True)
        p.close()


if __name__ == "__main__":
    main()
