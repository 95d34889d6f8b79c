"""Summarise rocprofv3 CSV output into the text tables kept beside the
benchmark numbers, and record the dominant kernel's measured HBM traffic.

Usage:
  python -m paper_1904_01201_amd.rocprof_summary --trace DIR --pmc DIR [DIR ...]
      --copy-fetch DIR --copy-write DIR --kernel 'k_raster<8>' --steps N
      [--traffic-out FILE] [--command TEXT]

--trace is a `rocprofv3 --kernel-trace --stats --output-format csv` output
directory, --pmc are `rocprofv3 --pmc ... --output-format csv` directories
(FETCH_SIZE and WRITE_SIZE among them), --copy-fetch/--copy-write are the
same two counters taken over `bench.py --copy-calibration` (plain 256 MiB
device copies): the counters' KiB per dispatch for the copy, against the
256 MiB it moves, give the scale applied to every kernel's counts.

Per kernel the trace gives the average duration over the last N launches
(the timed steps); the counter runs give per-dispatch averages.  VALU issue
utilisation is SQ_INSTS_VALU * 4 / (SIMDs * cycles): a wave64 VALU
instruction holds a 16-lane SIMD for 4 cycles; cycles are GRBM_GUI_ACTIVE
over the 8 XCDs.  Occupancy (waves resident per SIMD, averaged over the
dispatch) is 4 * SQ_WAVE_CYCLES / (SIMDs * cycles): the counter advances once
per 4 cycles per resident wave (checked against the raster, launched
persistently at 6 waves per SIMD).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

SIMDS = 256 * 4
XCDS = 8
COPY_BYTES = 256 << 20
HERE = os.path.dirname(os.path.abspath(__file__))


def kname(full: str) -> str:
    n = full.split("(")[0].replace("void ", "").replace("habmi::", "")
    return n.strip()


def _csv(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def trace_durations(d: str):
    rows = _csv(d, "kernel_trace.csv")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    out = collections.defaultdict(list)
    for r in rows:
        out[kname(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    return out


def counters(dirs):
    """kernel -> counter -> list of per-dispatch values."""
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in _csv(d, "counter_collection.csv"):
            out[kname(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def copy_scale(d: str, counter: str) -> float:
    vals = [float(r["Counter_Value"]) for r in _csv(d, "counter_collection.csv")
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise ValueError(f"no copy dispatch with {counter} in {d}")
    kib = sum(vals) / len(vals)
    return (COPY_BYTES / 1024.0) / kib


# the sources the render kernels are compiled from: a change to any of them
# invalidates recorded traffic
KERNEL_SOURCES = ("kernels.hip", "kernels.h", "raster_math.h", "dtypes.h")


def source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--pmc", nargs="+", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--kernel", required=True, help="dominant kernel, e.g. 'k_raster<8>'")
    ap.add_argument("--steps", type=int, required=True, help="timed launches at the end of the trace")
    ap.add_argument("--traffic-out")
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)

    dur = trace_durations(a.trace)
    cnt = counters(a.pmc)
    sf, sw = copy_scale(a.copy_fetch, "FETCH_SIZE"), copy_scale(a.copy_write, "WRITE_SIZE")

    lines = []
    if a.command:
        lines += ["Commands:", "", *[f"    {c}" for c in a.command.split(" ;; ")], ""]
    lines += [f"Copy calibration: FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f} "
              f"(256 MiB device copy = 262144 KiB each way)", ""]
    lines += ["| kernel | launches (timed) | avg us (timed) | VALU instr | VALU issue util | waves/SIMD | SALU instr | "
              "LDS instr | LDS bank-conflict cycles | HBM read MB | HBM write MB |",
              "|---|---|---|---|---|---|---|---|---|---|---|"]
    order = sorted(dur, key=lambda k: -sum(dur[k][-a.steps:]))
    traffic = None
    for k in order:
        if k.startswith("__amd") or k.startswith("at::"):
            continue
        d = dur[k][-a.steps:]
        c = cnt.get(k, {})
        avg = lambda n: (sum(c[n]) / len(c[n])) if n in c and c[n] else None
        valu, salu, lds = avg("SQ_INSTS_VALU"), avg("SQ_INSTS_SALU"), avg("SQ_INSTS_LDS")
        gui = avg("GRBM_GUI_ACTIVE")
        util = valu * 4 / (SIMDS * gui / XCDS) if valu and gui else None
        wcyc = avg("SQ_WAVE_CYCLES")
        occ = wcyc * 4 / (SIMDS * gui / XCDS) if wcyc and gui else None
        conf = avg("SQ_LDS_BANK_CONFLICT")
        fetch, write = avg("FETCH_SIZE"), avg("WRITE_SIZE")
        rd = fetch * 1024 * sf / 1e6 if fetch is not None else None
        wr = write * 1024 * sw / 1e6 if write is not None else None
        f = lambda x, p=3: "-" if x is None else (f"{x:.{p}g}" if isinstance(x, float) else str(x))
        lines.append(f"| `{k}` | {len(d)} | {sum(d) / len(d):.1f} | {f(valu)} | {f(util, 2)} | {f(occ, 2)} | {f(salu)} | "
                     f"{f(lds)} | {f(conf)} | {f(rd, 4)} | {f(wr, 4)} |")
        if k == a.kernel and rd is not None and wr is not None:
            traffic = {"kernel": k, "avg_launch_us": sum(d) / len(d), "hbm_read_bytes": rd * 1e6,
                       "hbm_write_bytes": wr * 1e6, "bytes_per_launch": (rd + wr) * 1e6,
                       "fetch_scale": sf, "write_scale": sw, "source_sha256": source_hash()}
    print("\n".join(lines))
    if a.traffic_out and traffic:
        with open(a.traffic_out, "w") as fo:
            json.dump(traffic, fo, indent=1)
            fo.write("\n")


if __name__ == "__main__":
    main()
