"""Turns rocprofv3 output into the HBM-traffic record the benchmark reports.

Counter runs (one counter set per run, as the profiler requires):

    rocprofv3 --pmc FETCH_SIZE -d DIR_F -o fetch --output-format csv -- python3 bench.py ...
    rocprofv3 --pmc WRITE_SIZE -d DIR_W -o write --output-format csv -- python3 bench.py ...

FETCH_SIZE / WRITE_SIZE are the L2-to-memory read / write volumes in KiB per
dispatch.  Each is scaled by the ratio (known bytes / counter reading) of a
plain device-to-device copy of known size profiled the same way
(``bench.py --workload copy``), which corrects for what the counters do not
see or see twice.  The result is written as JSON together with a hash of the
kernel sources, so that the benchmark reports it only while the kernel is
unchanged.

    python -m paper_1310_1537_amd.profiling FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV \\
        COPY_BYTES KERNEL_SUBSTRING OUT_JSON [plain|batched|diff]
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_CSRC = os.path.join(ROOT, "paper_1310_1537_amd", "csrc")
# the sources each measured kernel is built from
KERNEL_SOURCES = {
    "plain": ("tr_math.hpp", "rng.hpp", "publish.hpp", "fg_kernel.hpp", "glm_plain.hip"),
    "batched": ("tr_math.hpp", "rng.hpp", "publish.hpp", "fg_kernel.hpp", "fg_batched.hpp",
                "glm_batched.hip"),
    "diff": ("tr_math.hpp", "elem.hpp", "publish.hpp", "glm_diff.hip"),
    "mx": ("tr_math.hpp", "rng.hpp", "publish.hpp", "fg_kernel.hpp", "fg_mfma.hpp",
           "glm_multi_mx.hip"),
}


def kernel_source_hash(kind: str = "plain") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(_CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def per_dispatch(path: str, counter: str, kernel_sub: str) -> list[float]:
    """Counter values (KiB) of each dispatch whose kernel name contains kernel_sub."""
    vals: dict[str, float] = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name", "")
            if kernel_sub not in name or row.get("Counter_Name") != counter:
                continue
            d = row.get("Dispatch_Id") or row.get("Correlation_Id")
            vals[d] = vals.get(d, 0.0) + float(row["Counter_Value"])
    return list(vals.values())


def main(argv: list[str]) -> int:
    fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, ksub, out = argv[:7]
    kind = argv[7] if len(argv) > 7 else "plain"
    copy_bytes = float(copy_bytes)
    cf = per_dispatch(cfetch_csv, "FETCH_SIZE", "copy")
    cw = per_dispatch(cwrite_csv, "WRITE_SIZE", "copy")
    f = per_dispatch(fetch_csv, "FETCH_SIZE", ksub)
    w = per_dispatch(write_csv, "WRITE_SIZE", ksub)
    if not (cf and cw and f and w):
        print("missing dispatches", len(cf), len(cw), len(f), len(w), file=sys.stderr)
        return 1
    k_f = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    k_w = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    fetch = sum(f) / len(f) * 1024.0 * k_f
    write = sum(w) / len(w) * 1024.0 * k_w
    rec = {"kernel": ksub, "sources": kind, "kernel_source_hash": kernel_source_hash(kind),
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write, "dispatches": [len(f), len(w)],
           "copy_scale_fetch": k_f, "copy_scale_write": k_w, "copy_bytes": copy_bytes}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
