"""A plain device-to-device copy of known size (256 MiB, three times), run
under rocprofv3 to calibrate the FETCH_SIZE / WRITE_SIZE counters against
known bytes (the factors that turn counter readings into HBM traffic); and
copy_bandwidth(), the achieved device copy rate that the benchmark reports
beside the datasheet peak.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2405_05155_amd.hbm_copy
"""
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


def main():
    a = torch.ones(N, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied bytes per dispatch", 4 * N, flush=True)


if __name__ == "__main__":
    main()
