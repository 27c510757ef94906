"""Measure the row-transform variant of every length in a range, and the
segmentation of the tridiagonal solve of every row count, on this device and
append the choices to the tuning table (FDS_TUNE_FILE format: "n precision
variant" and "tri rows precision mpb ls").  Entries already in the table are
skipped by the library itself.

    python -m paper_2509_23180_amd.tune_table --nmin 1 --nmax 2048 --tri-max 2049 --out paper_2509_23180_amd/tune_gfx950.txt
"""

import argparse
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--nmin", type=int, default=1)
    ap.add_argument("--nmax", type=int, default=2048)
    ap.add_argument("--tri-max", type=int, default=0, help="also tune the tridiagonal solve for rows 1..tri-max")
    ap.add_argument("--skip-dst", action="store_true")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    os.environ["FDS_TUNE_FILE"] = os.path.abspath(args.out)
    import torch
    import paper_2509_23180_amd as fds
    torch.cuda.set_device(0)
    t0 = time.time()
    for n in range(args.nmin, args.nmax + 1):
        if args.skip_dst:
            break
        for dtype in (torch.float64, torch.float32):
            x = torch.zeros((1, n), dtype=dtype, device="cuda")
            fds.dst_rows(x, x)      # first use of (n, precision): the tuner measures it
        if n % 64 == 0:
            print(f"n={n} ({time.time() - t0:.0f} s)", flush=True)
    for rows in range(1, args.tri_max + 1):
        for dtype in (torch.float64, torch.float32):
            d = torch.zeros((rows, 16), dtype=dtype, device="cuda")
            fds.tridiag_modes(d, 1.0 / (rows + 1), 0.0)   # first use of (rows, precision): measured
        if rows % 64 == 0:
            print(f"tri rows={rows} ({time.time() - t0:.0f} s)", flush=True)
    print(f"done in {time.time() - t0:.0f} s", file=sys.stderr)


if __name__ == "__main__":
    main()
