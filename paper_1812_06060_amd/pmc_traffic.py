"""HBM bytes per launch from rocprofv3 PMC runs: reduces FETCH_SIZE and
WRITE_SIZE counter CSVs to profiles/traffic.json, which bench.py reads into
its roofline line.

FETCH_SIZE and WRITE_SIZE are read from one run each (rocprofv3 collects
them in separate passes).  Each is scaled by what the same counter reads for
a device-to-device copy of known size (bench.py --copy-calib: five copies of
1 GiB), so the result is in bytes.  Per kernel the mean over its dispatches
is kept, together with the sha256 of the source file it came from: bench.py
drops a record whose source has changed since.

    python -m paper_1812_06060_amd.pmc_traffic \\
        --fetch <dir of the FETCH_SIZE run> --write <dir of the WRITE_SIZE run> \\
        --calib-fetch <dir> --calib-write <dir> [--out profiles/traffic.json]

Each directory is searched for ``*counter_collection.csv`` files.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# record name -> (kernel name fragment, source file, launches per diffusion
# pass or None); the fragments end at the template bracket so that
# k_patch_pass does not also match k_patch_pass_ov
KERNELS = {
    "k_admm_edge_tiled": ("k_admm_edge_tiled<", "paper_1812_06060_amd/csrc/kernels_admm.hip", None),
    "k_patch_pass": ("k_patch_pass<", "paper_1812_06060_amd/csrc/kernels_patch.hip", "colours"),
    "k_patch_pass_ov": ("k_patch_pass_ov<", "paper_1812_06060_amd/csrc/kernels_patch.hip", None),
}
COPY_KERNEL = "copyBuffer"


def per_dispatch(run_dir: str, counter: str) -> dict:
    """{kernel name: [value per dispatch]} for one counter (KiB as reported)."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    acc: dict = {}
    for path in files:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = (path, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                acc.setdefault(row["Kernel_Name"], {}).setdefault(key, 0.0)
                acc[row["Kernel_Name"]][key] += float(row["Counter_Value"])
    return {k: list(v.values()) for k, v in acc.items()}


def mean_for(data: dict, fragment: str):
    vals = [x for name, xs in data.items() if fragment in name for x in xs]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--calib-fetch", required=True)
    ap.add_argument("--calib-write", required=True)
    ap.add_argument("--calib-bytes", type=float, default=float(1 << 30),
                    help="bytes each calibration copy reads and writes (bench.py --copy-calib: 1 GiB)")
    ap.add_argument("--colours", type=int, default=5, help="diffusion tile colours (launches per pass)")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    a = ap.parse_args(argv)

    cf, _ = mean_for(per_dispatch(a.calib_fetch, "FETCH_SIZE"), COPY_KERNEL)
    cw, _ = mean_for(per_dispatch(a.calib_write, "WRITE_SIZE"), COPY_KERNEL)
    if not cf or not cw:
        raise SystemExit("calibration copy kernel not found in the calibration runs")
    sf = a.calib_bytes / (cf * 1024.0)
    sw = a.calib_bytes / (cw * 1024.0)
    fetch = per_dispatch(a.fetch, "FETCH_SIZE")
    write = per_dispatch(a.write, "WRITE_SIZE")
    out = {"_scale": {"fetch": sf, "write": sw, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
                      "copy_kernel": COPY_KERNEL}}
    for key, (frag, src, per_pass) in KERNELS.items():
        f, nf = mean_for(fetch, frag)
        w, nw = mean_for(write, frag)
        if f is None or w is None:
            continue
        rec = {"bytes_per_launch": f * 1024.0 * sf + w * 1024.0 * sw, "fetch_kib_raw": f, "write_kib_raw": w,
               "launches": min(nf, nw), "src": src,
               "src_sha256": hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()}
        if per_pass:
            rec["launches_per_pass"] = a.colours
            rec["bytes_per_pass"] = rec["bytes_per_launch"] * a.colours
        out[key] = rec
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    json.dump(out, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
