"""Summaries of rocprofv3 output for the committed profiles.

Two kinds of summary, both markdown on stdout:

  stats    a --kernel-trace --stats run: calls, average and total time per kernel;
  traffic  two --pmc runs (FETCH_SIZE, then WRITE_SIZE) of the same program, which also ran one
           plain elementwise kernel over a known number of bytes (bench.py --copy-calib): each
           counter is scaled by (known bytes / what that counter read for the plain kernel), and
           one machine-readable ``traffic-record`` line per kernel gives the calibrated HBM bytes
           per launch, tagged with the hash of the kernel sources they were measured on.

    python -m paper_2311_03096_amd.prof_summary stats RUN_kernel_stats.csv --title T --command C
    python -m paper_2311_03096_amd.prof_summary traffic FETCH_counter_collection.csv \\
        WRITE_counter_collection.csv --calib-bytes N --workload W --command-fetch C1 --command-write C2
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


PROBE_SOURCES = ("wsr_lds_probe.hip",)  # measurement probes, not kernels of the prox path


def source_hash() -> str:
    """Hash of the HIP kernel sources of the prox library (the files under csrc/ other than the
    measurement probes), so a stored counter reading can be matched to the code it was taken on."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")) and name not in PROBE_SOURCES:
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def short_name(full: str) -> str:
    """rocprof kernel name -> the name the library's own launch trace uses."""
    n = re.sub(r"\(.*", "", full).replace("void ", "").strip()
    m = re.match(r"wsr::k_(prox_(?:fwd|bwd)_small)<(\d+),", n)
    if m:
        return "%s_%s" % (m.group(1), m.group(2))
    n = re.sub(r"<.*", "", n)
    return n.replace("wsr::k_", "") if n.startswith("wsr::k_") else n


def stats(path, title, command):
    rows = list(csv.DictReader(open(path)))
    out = ["# %s" % title, "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| %s | %s | %.2f | %.3f | %.1f |" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    return "\n".join(out) + "\n"


def _per_kernel(path, counter):
    acc = collections.defaultdict(lambda: [0, 0.0])
    calib = None
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if "AUnaryFunctor" in r["Kernel_Name"]:  # the calibration kernel: out = in * 1
            calib = v
            continue
        a = acc[short_name(r["Kernel_Name"])]
        a[0] += 1
        a[1] += v
    return {k: (n, s / n) for k, (n, s) in acc.items()}, calib


def traffic(fetch_csv, write_csv, calib_bytes, workload, cmd_fetch, cmd_write):
    fk, fcal = _per_kernel(fetch_csv, "FETCH_SIZE")
    wk, wcal = _per_kernel(write_csv, "WRITE_SIZE")
    if not fcal or not wcal:
        raise SystemExit("calibration kernel not found in the counter files")
    ff = calib_bytes / (fcal * 1024.0)
    fw = calib_bytes / (wcal * 1024.0)
    src = source_hash()
    out = ["# HBM traffic per launch: %s" % workload, "",
           "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 --pmc runs, scaled by what "
           "the same counters read for one plain elementwise kernel over %d bytes in and %d bytes out "
           "(fetch factor %.4f, write factor %.4f)." % (calib_bytes, calib_bytes, ff, fw), "",
           "Commands:", "", "```", cmd_fetch, cmd_write, "```", "",
           "Kernel sources hash: `%s`" % src, "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB | total MB |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    recs = []
    for k in sorted(set(fk) | set(wk)):
        n = fk.get(k, wk.get(k))[0]
        f = fk.get(k, (0, 0.0))[1]
        w = wk.get(k, (0, 0.0))[1]
        rb, wb = f * 1024.0 * ff, w * 1024.0 * fw
        out.append("| %s | %d | %.1f | %.1f | %.2f | %.2f | %.2f |" % (k, n, f, w, rb / 1e6, wb / 1e6,
                                                                   (rb + wb) / 1e6))
        if not k.startswith(("radix_", "big_", "prox_", "zero_")):
            continue  # framework kernels (input set-up) get a row but no record
        recs.append("traffic-record: workload=%s kernel=%s src=%s read_bytes=%.0f write_bytes=%.0f" % (
            workload, k, src, rb, wb))
    out += ["", "```"] + recs + ["```"]
    return "\n".join(out) + "\n"


def read_traffic(path, workload, kernel):
    """Calibrated bytes per launch of `kernel` stored in a traffic summary, or None when the
    summary is missing, has no such kernel, or was measured on other kernel sources."""
    if not os.path.exists(path):
        return None
    src = source_hash()
    for line in open(path):
        if not line.startswith("traffic-record:"):
            continue
        kv = dict(t.split("=", 1) for t in line.split()[1:])
        if kv.get("workload") == workload and kv.get("kernel") == kernel:
            if kv.get("src") != src:
                return None
            return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


INSTR_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_WAVES")


def instr_counters(csv_path, workload, command):
    """Per-launch wave-instruction counts (VALU, LDS, SALU) and waves of every library kernel
    from one rocprofv3 --pmc run, with counter records that the bench matches by source hash."""
    per = {c: _per_kernel(csv_path, c)[0] for c in INSTR_COUNTERS}
    src = source_hash()
    out = ["# Instruction counters per launch: %s" % workload, "",
           "Wave-level instruction counts per dispatch (`SQ_INSTS_*` sum over the dispatch's waves) "
           "from one rocprofv3 --pmc run.", "", "Command:", "", "```", command, "```", "",
           "Kernel sources hash: `%s`" % src, "",
           "| kernel | dispatches | VALU | LDS | SALU | waves | VALU / wave | LDS / wave |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    recs = []
    for k in sorted(per["SQ_INSTS_VALU"]):
        n, valu = per["SQ_INSTS_VALU"][k]
        lds = per["SQ_INSTS_LDS"].get(k, (0, 0.0))[1]
        salu = per["SQ_INSTS_SALU"].get(k, (0, 0.0))[1]
        waves = per["SQ_WAVES"].get(k, (0, 0.0))[1]
        out.append("| %s | %d | %.4g | %.4g | %.4g | %.0f | %.0f | %.0f |" % (
            k, n, valu, lds, salu, waves, valu / max(waves, 1), lds / max(waves, 1)))
        if k.startswith(("radix_", "big_", "prox_")):
            recs.append("counter-record: workload=%s kernel=%s src=%s valu=%.0f lds=%.0f salu=%.0f waves=%.0f" % (
                workload, k, src, valu, lds, salu, waves))
    out += ["", "```"] + recs + ["```"]
    return "\n".join(out) + "\n"


def read_counters(path, workload, kernel):
    """{valu, lds, salu, waves} per launch of `kernel` from an instruction-counter summary, or None
    when missing or measured on other kernel sources."""
    if not os.path.exists(path):
        return None
    src = source_hash()
    for line in open(path):
        if not line.startswith("counter-record:"):
            continue
        kv = dict(t.split("=", 1) for t in line.split()[1:])
        if kv.get("workload") == workload and kv.get("kernel") == kernel:
            if kv.get("src") != src:
                return None
            return {c: float(kv[c]) for c in ("valu", "lds", "salu", "waves")}
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--calib-bytes", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--workload", required=True)
    c.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        print(stats(a.csv, a.title, a.command), end="")
    elif a.cmd == "counters":
        print(instr_counters(a.csv, a.workload, a.command), end="")
    else:
        print(traffic(a.fetch_csv, a.write_csv, a.calib_bytes, a.workload, a.command_fetch, a.command_write),
              end="")


if __name__ == "__main__":
    main()
