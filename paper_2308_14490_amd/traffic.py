"""HBM traffic per launch from the hardware counters, for bench.py's roofline.

Runs ``bench.py --profile-only --calibrate`` twice under rocprofv3, once
with FETCH_SIZE and once with WRITE_SIZE (one counter group per pass), then
averages each library kernel's counters per dispatch.  The calibration
kernel is an elementwise product over 2^27 doubles (1 GiB read, 1 GiB
written); each counter is scaled by known bytes / counted bytes on it.  The
result goes to profiles/traffic.json together with a hash of the kernel
sources: bench.py reports it only while the sources are unchanged.

Run on the GPU machine from the repository root:
    python3 -m paper_2308_14490_amd.traffic
(this process starts rocprofv3 as a child and never touches the GPU itself).
"""
import csv
import glob
import json
import os
import re
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CAL_BYTES = float(1 << 30)


def source_hash():
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2308_14490_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def prof_name(kernel):
    """rocprofv3 kernel name -> the library's per-launch profile name."""
    m = re.search(r"az::k_row<(\d+), \w+, \d+, (\d+)", kernel)
    if m:   # the row pass: template arguments N2, 1D, lines per row, mode (A, Z*, A Z*, A Z* with rows)
        mode = ("row_A", "row_Z", "row_AZ", "row_AZ")[int(m.group(2))]
        return f"{mode} n2={m.group(1)}"
    m = re.search(r"az::k_(\w+)<(\d+)", kernel)
    if m:
        base, n = m.group(1), m.group(2)
        if base.startswith("col_"):
            return f"{base} n1={n}"
        if base.startswith("row_"):
            return f"{base} n2={n}"
        if base.startswith("fused_"):
            return f"{base} n={n}"
        return base
    m = re.search(r"az::(?:\(anonymous namespace\)::)?k_(\w+)", kernel)
    if not m:
        return None
    return {"tsqr_reg": "tsqr_block"}.get(m.group(1), m.group(1))


def counters(csvpath, counter):
    """{kernel name: [values per dispatch]} (rocprofv3 reports KiB)."""
    out = {}
    for r in csv.DictReader(open(csvpath)):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
    return out


def run_pass(counter, outdir, extra):
    cmd = ["rocprofv3", "--pmc", counter, "--output-format", "csv", "-d", outdir, "-o", "p", "--",
           sys.executable, "-u", "bench.py", "--profile-only", "--calibrate", "--steps", "2", "--warmup", "1"] + extra
    env = dict(os.environ, TMPDIR="/tmp")
    subprocess.run(cmd, cwd=ROOT, env=env, check=True, timeout=300)
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter output for {counter}")
    return counters(files[0], counter), cmd


def main():
    tmp = tempfile.mkdtemp(prefix="azrbf_pmc_", dir="/tmp")
    fetch, cmd_f = run_pass("FETCH_SIZE", os.path.join(tmp, "fetch"), [])
    write, cmd_w = run_pass("WRITE_SIZE", os.path.join(tmp, "write"), [])
    cal = [k for k in fetch if "elementwise" in k and "Mul" in k]
    if not cal:
        raise RuntimeError("calibration kernel not found")
    cf = CAL_BYTES / max(fetch[cal[0]])
    cw = CAL_BYTES / max(write.get(cal[0], [CAL_BYTES]))
    kernels = {}
    for name in set(fetch) | set(write):
        pn = prof_name(name)
        if not pn:
            continue
        f = fetch.get(name, [])
        w = write.get(name, [])
        e = kernels.setdefault(pn, {"dispatches": 0, "fetch_sum": 0.0, "write_sum": 0.0})
        e["dispatches"] += max(len(f), len(w))
        e["fetch_sum"] += sum(f) * cf
        e["write_sum"] += sum(w) * cw
    for e in kernels.values():
        n = max(e["dispatches"], 1)
        e["fetch_bytes"] = e.pop("fetch_sum") / n
        e["write_bytes"] = e.pop("write_sum") / n
        e["bytes_per_launch"] = e["fetch_bytes"] + e["write_bytes"]
    out = {"source_hash": source_hash(),
           "commands": [" ".join(cmd_f), " ".join(cmd_w)],
           "calibration": {"kernel": cal[0][:120], "bytes_read": CAL_BYTES, "bytes_written": CAL_BYTES,
                           "fetch_scale": cf, "write_scale": cw},
           "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(path)
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"])[:12]:
        print(f"{k:28s} {v['dispatches']:4d} fetch {v['fetch_bytes']/1e6:9.2f} MB write {v['write_bytes']/1e6:9.2f} MB")


if __name__ == "__main__":
    main()
