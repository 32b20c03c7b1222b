"""Reference HBM rates on this device: torch's device copy (read + write)
and sum reduction (read) over buffers of 64 MiB to 4 GiB, timed with CUDA
events.  Context for the pass kernels' roofline fraction.

    python paper_2606_27086_amd/copy_bandwidth.py
"""
import torch


def main():
    torch.cuda.set_device(0)
    for mb in (64, 256, 1024, 4096):
        n = mb * (1 << 20) // 4
        a = torch.rand(n, device="cuda")
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        for _ in range(3):
            b.copy_(a)
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        t_copy = e0.elapsed_time(e1) / reps * 1e-3
        for _ in range(3):
            a.sum()
        e0.record()
        for _ in range(reps):
            a.sum()
        e1.record()
        torch.cuda.synchronize()
        t_sum = e0.elapsed_time(e1) / reps * 1e-3
        print(f"{mb} MiB: copy {2 * n * 4 / t_copy / 1e9:.0f} GB/s, sum {n * 4 / t_sum / 1e9:.0f} GB/s", flush=True)
        del a, b


if __name__ == "__main__":
    main()
