"""HBM traffic per launch from the hardware counters, for bench.py's roofline.

Runs ``bench.py --profile-only --calibrate`` four times under rocprofv3:
FETCH_SIZE, WRITE_SIZE, and two passes of the raw TCC request counters behind
them (request sizes, and the requests destined for DRAM), then averages each
library kernel's counters per dispatch.  The calibration
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


def counters(csvpath, names):
    """{counter: {kernel name: [values per dispatch]}} (FETCH_SIZE and
    WRITE_SIZE are reported in KiB and converted to bytes; raw counters are
    request counts)."""
    out = {n: {} for n in names}
    for r in csv.DictReader(open(csvpath)):
        n = r["Counter_Name"]
        if n not in out:
            continue
        v = float(r["Counter_Value"]) * (1024.0 if n in ("FETCH_SIZE", "WRITE_SIZE") else 1.0)
        out[n].setdefault(r["Kernel_Name"], []).append(v)
    return out


def run_pass(names, outdir, extra):
    cmd = ["rocprofv3", "--pmc", *names, "--output-format", "csv", "-d", outdir, "-o", "p", "--",
           sys.executable, "-u", "bench.py", "--profile-only", "--calibrate", "--steps", "2", "--warmup", "1"] + extra
    env = dict(os.environ, TMPDIR="/tmp")
    subprocess.run(cmd, cwd=ROOT, env=env, check=True, timeout=300)
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter output for {names}")
    return counters(files[0], names), cmd


# The passes (each within the per-block limits: at most 4 TCC counters, a
# derived counter's sum counting once).  FETCH_SIZE and WRITE_SIZE are the
# derived byte counts; the raw passes give the request sizes behind them and
# how many requests went to DRAM (as opposed to other memory) so that the
# scale factor of FETCH_SIZE can be explained rather than only calibrated.
PASSES = [
    ["FETCH_SIZE"],
    ["WRITE_SIZE"],
    ["TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_DRAM_sum"],
    ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_WRREQ_DRAM_sum"],
]


def main():
    tmp = tempfile.mkdtemp(prefix="azrbf_pmc_", dir="/tmp")
    data, cmds = {}, []
    for i, names in enumerate(PASSES):
        d, cmd = run_pass(names, os.path.join(tmp, f"p{i}"), [])
        data.update(d)
        cmds.append(" ".join(cmd))
    fetch, write = data["FETCH_SIZE"], data["WRITE_SIZE"]
    cal = [k for k in fetch if "elementwise" in k and "Mul" in k]
    if not cal:
        raise RuntimeError("calibration kernel not found")
    cf = CAL_BYTES / max(fetch[cal[0]])
    cw = CAL_BYTES / max(write.get(cal[0], [CAL_BYTES]))

    def total(counter, name):
        return sum(data[counter].get(name, []))

    kernels = {}
    for name in set(fetch) | set(write) | set(data["TCC_EA0_RDREQ_sum"]):
        pn = prof_name(name) if name not in cal else "calibration (elementwise, 1 GiB in, 1 GiB out)"
        if not pn:
            continue
        f = fetch.get(name, [])
        w = write.get(name, [])
        e = kernels.setdefault(pn, {"dispatches": 0, "fetch_sum": 0.0, "write_sum": 0.0, "rd": 0.0, "rd128": 0.0,
                                    "rd32": 0.0, "rddram": 0.0, "wr": 0.0, "wr64": 0.0, "wrdram": 0.0})
        e["dispatches"] += max(len(f), len(w))
        e["fetch_sum"] += sum(f) * cf
        e["write_sum"] += sum(w) * cw
        e["rd"] += total("TCC_EA0_RDREQ_sum", name)
        e["rd128"] += total("TCC_EA0_RDREQ_128B_sum", name)
        e["rd32"] += total("TCC_EA0_RDREQ_32B_sum", name)
        e["rddram"] += total("TCC_EA0_RDREQ_DRAM_sum", name)
        e["wr"] += total("TCC_EA0_WRREQ_sum", name)
        e["wr64"] += total("TCC_EA0_WRREQ_64B_sum", name)
        e["wrdram"] += total("TCC_EA0_WRREQ_DRAM_sum", name)
    for e in kernels.values():
        n = max(e["dispatches"], 1)
        e["fetch_bytes"] = e.pop("fetch_sum") / n
        e["write_bytes"] = e.pop("write_sum") / n
        e["bytes_per_launch"] = e["fetch_bytes"] + e["write_bytes"]
        rd, rd128, rd32, wr, wr64 = e.pop("rd"), e.pop("rd128"), e.pop("rd32"), e.pop("wr"), e.pop("wr64")
        rddram, wrdram = e.pop("rddram"), e.pop("wrdram")
        # request sizes: 128, 64 or 32 bytes for reads, 64 or 32 for writes
        e["read_bytes_by_request_size"] = (128.0 * rd128 + 64.0 * (rd - rd128 - rd32) + 32.0 * rd32) / n
        e["write_bytes_by_request_size"] = (64.0 * wr64 + 32.0 * (wr - wr64)) / n
        e["read_requests_128B_frac"] = rd128 / rd if rd else None
        e["read_requests_to_dram_frac"] = rddram / rd if rd else None
        e["write_requests_to_dram_frac"] = wrdram / wr if wr else None
    out = {"source_hash": source_hash(),
           "commands": cmds,
           "calibration": {"kernel": cal[0][:120], "bytes_read": CAL_BYTES, "bytes_written": CAL_BYTES,
                           "fetch_scale": cf, "write_scale": cw},
           "note": "FETCH_SIZE's expression (rocprofv3 --list-avail) counts TCC_BUBBLE requests as 128 bytes and "
                   "every other non-32-byte read request as 64 bytes; on gfx950 the 128-byte reads are counted by "
                   "TCC_EA0_RDREQ_128B instead, so FETCH_SIZE counts them at half their size. "
                   "read_bytes_by_request_size counts them at 128 bytes.",
           "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(path)
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"])[:16]:
        print(f"{k:34s} {v['dispatches']:4d} fetch {v['fetch_bytes']/1e6:9.2f} MB write {v['write_bytes']/1e6:9.2f} MB"
              f" | by size: read {v['read_bytes_by_request_size']/1e6:9.2f} MB write "
              f"{v['write_bytes_by_request_size']/1e6:9.2f} MB, 128B reads {v['read_requests_128B_frac']}, "
              f"DRAM rd {v['read_requests_to_dram_frac']} wr {v['write_requests_to_dram_frac']}", flush=True)


if __name__ == "__main__":
    main()
