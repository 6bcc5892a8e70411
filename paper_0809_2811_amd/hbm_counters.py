"""HBM traffic of the step kernels from two rocprofv3 counter passes.

`rocprofv3 --kernel-trace --pmc FETCH_SIZE` and then `--pmc WRITE_SIZE` (each
its own run, CSV output) over

    python3 bench.py --forms liquid4096 --no-cpu --steps 300 --warmup 10 --copy-mib 1024 --graph-steps 0

give per-dispatch KiB for every launch.  The run starts with a plain copy
(`out = -in` over 1024 MiB of fp32: 1 GiB read, 1 GiB written), whose
readings scale each counter to bytes.  `reduce()` averages the scaled
counters over the launches of the NVE phase (every `k_forces<L, 2, false>`
launch and each `k_moments<L, false>` launch directly followed by one) of the
4096-atom liquid (L = 32) and the 262144-atom box (L = 8) and writes the
record next to this file, keyed by a digest of the kernel sources so that the
benchmark reports it only while they are unchanged:

    python -m paper_0809_2811_amd.hbm_counters <fetch_dir> <write_dir> [out.json]
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
RECORD = os.path.join(PKG, "hbm_counters.json")
KERNEL_SOURCES = ("sw_kernels.hip", "sw_device.h", "sw_internal.h")
COPY_KIB = 1024 * 1024
WORKLOADS = ((32, "liquid4096"), (8, "liquid262144"))


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) recorded for this
    kernel and workload, or None when there is no record or the kernel
    sources changed since the counters were taken."""
    try:
        with open(RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != kernel_sources_digest():
        return None
    ent = rec.get("kernels", {}).get(f"{workload}/{kernel}")
    if not ent:
        return None
    return ent["fetch_bytes"] * rec["fetch_scale"] + ent["write_bytes"] * rec["write_scale"]


def _rows(directory: str, counter: str):
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    with open(files[0]) as fh:
        r = [x for x in csv.DictReader(fh) if x["Counter_Name"] == counter]
    r.sort(key=lambda x: int(x["Dispatch_Id"]))
    return r


def _durations(directory: str):
    """Kernel durations (us) by dispatch id from the same run's kernel trace, if any."""
    files = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        return {}
    with open(files[0]) as fh:
        return {x["Dispatch_Id"]: (int(x["End_Timestamp"]) - int(x["Start_Timestamp"])) / 1e3
                for x in csv.DictReader(fh)}


def _per_kernel(rows, dur=None):
    """Mean counter per launch of each NVE-phase kernel; k_moments launches
    are also split into those that rebuilt rows and those that did not (the
    launch durations are bimodal: split at the midpoint of their range)."""
    acc = collections.defaultdict(list)
    mom = collections.defaultdict(list)
    for k, x in enumerate(rows):
        name = x["Kernel_Name"]
        for lpa, wl in WORKLOADS:
            fk, mk = f"k_forces<{lpa}, 2, false>", f"k_moments<{lpa}, false>"
            if fk in name:
                acc[f"{wl}/{fk}"].append(float(x["Counter_Value"]))
            elif mk in name and k + 1 < len(rows) and fk in rows[k + 1]["Kernel_Name"]:
                acc[f"{wl}/{mk}"].append(float(x["Counter_Value"]))
                if dur and x["Dispatch_Id"] in dur:
                    mom[f"{wl}/{mk}"].append((dur[x["Dispatch_Id"]], float(x["Counter_Value"])))
    for key, lst in mom.items():
        lo, hi = min(d for d, _ in lst), max(d for d, _ in lst)
        cut = 0.5 * (lo + hi)
        for part, sel in (("rebuild", [c for d, c in lst if d > cut]), ("plain", [c for d, c in lst if d <= cut])):
            if sel and hi > 1.5 * lo:
                acc[f"{key}/{part}"] = sel
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def reduce(fetch_dir: str, write_dir: str, out: str = RECORD) -> dict:
    per, cal = {}, {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _rows(d, counter)
        copy = [float(x["Counter_Value"]) for x in rows if "neg_kernel" in x["Kernel_Name"]]
        if not copy:
            raise ValueError(f"{counter}: no calibration copy launch in the trace")
        cal[counter] = sum(copy) / len(copy)
        per[counter] = _per_kernel(rows, _durations(d))
    rec = {
        "kernel_sources_sha256": kernel_sources_digest(),
        "fetch_scale": COPY_KIB / cal["FETCH_SIZE"],
        "write_scale": COPY_KIB / cal["WRITE_SIZE"],
        "calibration": {"kernel": "out = -in over 1024 MiB of fp32 (reads 1024 MiB, writes 1024 MiB)",
                        "fetch_KiB": cal["FETCH_SIZE"], "write_KiB": cal["WRITE_SIZE"], "expected_KiB": COPY_KIB},
        "command": "rocprofv3 --kernel-trace --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 "
                   "bench.py --forms liquid4096 --no-cpu --steps 300 --warmup 10 --copy-mib 1024 --graph-steps 0",
        "selection": "launches of the NVE phase only: every k_forces<L, 2, false> launch and each k_moments<L, false> "
                     "launch directly followed by one; k_moments also split by duration into launches that "
                     "rebuilt rows and plain ones",
        "kernels": {},
    }
    for k in sorted(per["FETCH_SIZE"]):
        f, n = per["FETCH_SIZE"][k]
        w, _ = per["WRITE_SIZE"][k]
        rec["kernels"][k] = {"fetch_bytes": f * 1024, "write_bytes": w * 1024, "launches": n}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def main(argv):
    if len(argv) < 2:
        print(__doc__)
        return 2
    rec = reduce(argv[0], argv[1], argv[2] if len(argv) > 2 else RECORD)
    for k, v in rec["kernels"].items():
        f = v["fetch_bytes"] * rec["fetch_scale"]
        w = v["write_bytes"] * rec["write_scale"]
        print(f"{k}: {v['launches']} launches, fetch {f / 1e6:.3f} MB, write {w / 1e6:.3f} MB, "
              f"traffic {(f + w) / 1e6:.3f} MB")
    print("scales", rec["fetch_scale"], rec["write_scale"])
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
