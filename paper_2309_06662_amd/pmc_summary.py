"""Summarise rocprofv3 counter runs into the per-launch traffic record of the
tendency kernel.

Inputs are the counter_collection.csv files of four runs: FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) of the benchmark, and the same two counters of
copy_probe. The copy kernel must read and write a known number of bytes; the
ratio of those bytes to what the counters report for it scales the
tendency kernel's counters into bytes. The record also keeps the hash of the
kernel source so that a reader can tell whether it still applies.

    python -m paper_2309_06662_amd.pmc_summary --workload latlon_4320x1800x100 --precision fp32 \
        --fetch BENCH_FETCH.csv --write BENCH_WRITE.csv --copy-fetch COPY_FETCH.csv \
        --copy-write COPY_WRITE.csv --copy-bytes N --command "..." --out profiles/...json
"""
import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def per_dispatch(path, counter, name_part):
    """Counter values per dispatch of kernels whose name contains name_part, in dispatch order."""
    vals = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter or name_part not in r.get("Kernel_Name", ""):
                continue
            d = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
            vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    return [vals[d] for d in sorted(vals)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--precision", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=float, required=True, help="bytes the copy kernel reads (= writes)")
    ap.add_argument("--kernel", default="k_tend")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    cf = per_dispatch(a.copy_fetch, "FETCH_SIZE", "copy")
    cw = per_dispatch(a.copy_write, "WRITE_SIZE", "copy")
    kf = per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    kw = per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    if not (cf and cw and kf and kw):
        raise SystemExit("missing dispatches in the counter files")
    # the largest copy dispatch is the probe's copy; the last kernel dispatch is a steady step
    f_scale = a.copy_bytes / (max(cf) * 1024.0)
    w_scale = a.copy_bytes / (max(cw) * 1024.0)
    fetch_b = kf[-1] * 1024.0 * f_scale
    write_b = kw[-1] * 1024.0 * w_scale
    with open(os.path.join(HERE, "csrc", "k_tend.hip"), "rb") as f:
        src = hashlib.sha256(f.read()).hexdigest()[:16]
    rec = {"kernel": a.kernel, "workload": a.workload, "precision": a.precision,
           "source_sha256_16": src,
           "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
           "copy_fetch_kib": max(cf), "copy_write_kib": max(cw), "copy_bytes": a.copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_fetch_bytes_per_launch": fetch_b, "hbm_write_bytes_per_launch": write_b,
           "hbm_bytes_per_launch": fetch_b + write_b, "commands": a.command}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("fetch_scale", "write_scale", "hbm_bytes_per_launch")}))


if __name__ == "__main__":
    main()
