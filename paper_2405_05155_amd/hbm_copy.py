"""A plain device-to-device copy of known size (256 MiB, three times), run
under rocprofv3 to calibrate the FETCH_SIZE / WRITE_SIZE counters against
known bytes (the factors that turn counter readings into HBM traffic).

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2405_05155_amd.hbm_copy
"""
import torch

N = 64 * 1024 * 1024  # floats (256 MiB)


def main():
    a = torch.ones(N, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied bytes per dispatch", 4 * N, flush=True)


if __name__ == "__main__":
    main()
