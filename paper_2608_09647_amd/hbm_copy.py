"""Calibration workload for rocprofv3's HBM counters: three device copies of
2^27 float64 values (1 GiB read and 1 GiB written per copy).  The FETCH_SIZE
and WRITE_SIZE the counters report per copy, against 1,048,576 KiB, give the
scale factors applied to the solver kernels' counters.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2608_09647_amd.hbm_copy
"""
import torch


def main() -> None:
    a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB", flush=True)


if __name__ == "__main__":
    main()
