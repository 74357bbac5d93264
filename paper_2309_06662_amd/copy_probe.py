"""A plain device-to-device copy of known size, for calibrating memory-traffic
counters: run it under a counter collector and compare the bytes the counters
report for the copy kernel with the bytes it must move (n floats read, n
floats written).

    python -m paper_2309_06662_amd.copy_probe [--mib 1024] [--repeat 3]
"""
import argparse
import json


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024, help="size of each buffer in MiB")
    ap.add_argument("--repeat", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(a.repeat):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_floats": n, "bytes_read": 4 * n, "bytes_written": 4 * n, "repeat": a.repeat}))


if __name__ == "__main__":
    main()
