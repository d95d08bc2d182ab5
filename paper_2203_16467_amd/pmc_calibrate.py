"""Copy kernel of known size for calibrating the HBM traffic counters.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2203_16467_amd.pmc_calibrate [bytes]

Copies a device buffer of `bytes` (default 256 MiB) three times; a counter
that reads R KiB per copy dispatch for B bytes moved in that direction gives
the scale factor B / (1024 R) applied to the solver kernels' readings.
"""

import sys


def main(argv=None):
    import torch
    argv = sys.argv[1:] if argv is None else argv
    n = int(argv[0]) if argv else 256 << 20
    a = torch.empty(n // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n} bytes x3", flush=True)


if __name__ == "__main__":
    main()
