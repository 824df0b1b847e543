"""Plain device-to-device copy of a known size, run under rocprofv3 --pmc to
calibrate the FETCH_SIZE / WRITE_SIZE counters: HBM bytes per counter unit
= bytes copied / counter reading.

    rocprofv3 --pmc FETCH_SIZE -- python3 paper_2410_15080_amd/copy_calibration.py
"""

import sys

import torch

MIB = 64


def main():
    n = MIB * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n * 8} bytes per launch, 3 launches", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
