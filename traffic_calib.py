"""Known-size copy for calibrating the HBM byte counters of rocprofv3.

Runs an elementwise kernel that reads exactly `GIB` GiB of binary32 data and
writes the same amount (y = 1.0 * x, both tensors resident in HBM), a few
times, one dispatch each (torch splits larger elementwise launches; 1 GiB is
one dispatch, grid 2^26 work-items of four elements).  Under `rocprofv3 --pmc FETCH_SIZE` (then
`WRITE_SIZE`) the counter value of one dispatch, in KiB, divided into the
known byte count gives the scale factor applied to the counters of the
streaming kernels.

Usage: python traffic_calib.py [--gib 1] [--reps 3]   (from the repository root)
"""
import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=int, default=1, choices=[1])
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        print("needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.gib * (1 << 30) // 4  # 2^28 elements: torch issues one dispatch
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"copied {args.reps} x {args.gib} GiB (read {n * 4} bytes, write {n * 4} bytes per dispatch)")


if __name__ == "__main__":
    main()
