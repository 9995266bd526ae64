"""A plain device-to-device copy of known size (256 MiB, three times), run
under rocprofv3 to calibrate the FETCH_SIZE / WRITE_SIZE counters against
known bytes (the factors that turn counter readings into HBM traffic); and
copy_bandwidth(), the achieved device copy rate that the benchmark reports
beside the datasheet peak.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2405_05155_amd.hbm_copy
    python3 -m paper_2405_05155_amd.hbm_copy --small

--small times back-to-back copies of a few MB (the per-launch floor of a
short kernel over a few hundred thousand particles).
"""
import sys

import torch

N = 64 * 1024 * 1024  # floats (256 MiB)


def copy_bandwidth(nbytes=1 << 30, reps=20):
    """Bytes moved (read + written) per second by a device copy of nbytes,
    the best of `reps` timed copies after one untimed."""
    n = nbytes // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * 4 * n / best


def small_copies(sizes=(4 << 20, 16 << 20, 64 << 20), reps=500):
    """Microseconds per launch of `reps` back-to-back copies of each size."""
    out = {}
    for nbytes in sizes:
        a = torch.ones(nbytes // 4, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        out[nbytes] = e0.elapsed_time(e1) * 1e3 / reps
        del a, b
    return out


def main():
    if "--small" in sys.argv:
        for nbytes, us in small_copies().items():
            print(f"copy of {nbytes >> 20} MiB: {us:.2f} us per launch ({2 * nbytes / us / 1e6:.2f} TB/s read + write)",
                  flush=True)
        return
    a = torch.ones(N, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied bytes per dispatch", 4 * N, flush=True)


if __name__ == "__main__":
    main()
