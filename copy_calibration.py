"""A plain device-to-device copy of a known size, for scaling the
FETCH_SIZE / WRITE_SIZE hardware counters to bytes: run it under the same
`rocprofv3 --pmc` pass as the kernel being measured and divide.

usage: python3 copy_calibration.py [MiB]   (from the repository root)
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * 1024 * 1024 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB three times ({n * 8} bytes read and written per copy)", flush=True)


if __name__ == "__main__":
    main()
