"""Short text summaries of rocprofv3 output, for keeping next to the results.

    python -m paper_2205_14741_amd.profsum stats --csv RUN_kernel_stats.csv \
        --cmd "<the profiled command>" --out SUMMARY.txt
    python -m paper_2205_14741_amd.profsum traffic --fetch FETCH_counter_collection.csv \
        --write WRITE_counter_collection.csv --copy-bytes B --cmd-fetch "..." \
        --cmd-write "..." --out SUMMARY.txt
    python -m paper_2205_14741_amd.profsum mfma --csv MOPS_counter_collection.csv \
        --cmd "<the profiled command>" --out SUMMARY.txt
    python -m paper_2205_14741_amd.profsum counters --csv A.csv B.csv --cmd "<cmd A>" "<cmd B>" \
        [--kernels ns_gemm] --out SUMMARY.txt

`stats` lists the kernels of a kernel-trace run by total time (calls, average,
total, share); with `--trace RUN_kernel_trace.csv --tail KERNEL=N` it also
averages the last N dispatches of KERNEL (a benchmark's timed steps come
last, after its set-up launches of the same kernel).  `traffic --tail` does the
same for the counters.  `traffic` averages the FETCH_SIZE and WRITE_SIZE counters (KiB
per dispatch) of every GEMM kernel over two counter runs, and scales each by
what the same counter reads for a plain copy kernel of known size (the
elementwise negation of a float32 buffer of B bytes, run by the profiled
command first): factor = B / counter bytes.  The traffic lines carry a hash
of the GEMM sources, so a reader can tell whether the kernel has changed since.
`mfma` gives the matrix-core flops per dispatch of every kernel from the
SQ_INSTS_VALU_MFMA_MOPS_* counters (512 flops per unit), by precision.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
GEMM_SOURCES = ("csrc/k_gemm.hip", "csrc/device_common.h", "csrc/smsign_internal.h")


def gemm_source_hash() -> str:
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel name without its argument list: 'sm::ns_gemm_kernel<4, 0, 1, true>'."""
    m = re.match(r"\s*(?:void\s+)?([^(]*)", name)
    return (m.group(1) if m else name).strip()


def parse_tails(specs) -> list:
    """'KERNEL=N' items: the last N dispatches of KERNEL (a short name)."""
    out = []
    for spec in specs or []:
        name, _, n = spec.rpartition("=")
        out.append((name.strip(), int(n)))
    return out


def stats_summary(path: str, cmd: str, top: int = 25, trace: str | None = None, tails=()) -> str:
    """Kernels by total time; with the per-dispatch trace, also the average
    duration of the last N dispatches of each kernel in `tails` (the
    profiled benchmark's timed steps come last)."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 --kernel-trace --stats", f"# command: {cmd}",
           f"# {'kernel':64s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        out.append(f"  {short_name(r['Name'])[:64]:64s} {int(r['Calls']):7d} "
                   f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                   f"{float(r['Percentage']):6.2f}")
    if trace and tails:
        out.append("# tail <kernel> | last N dispatches | their average duration (us)")
        disp = collections.defaultdict(list)
        for r in csv.DictReader(open(trace)):
            disp[short_name(r["Kernel_Name"])].append(
                (int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for name, n in tails:
            d = sorted(disp.get(name, []))[-n:]
            if d:
                out.append(f"tail {name} | {len(d)} | {sum(x[1] for x in d) / len(d) / 1e3:.2f}")
    return "\n".join(out) + "\n"


def counter_means(path: str, counter: str, tails: dict | None = None) -> dict:
    """{kernel short name: (dispatches, mean counter value per dispatch)};
    for a kernel in `tails` ({name: N}) only its last N dispatches count."""
    acc = collections.defaultdict(list)
    for i, r in enumerate(csv.DictReader(open(path))):
        if r["Counter_Name"] != counter:
            continue
        order = int(r["Dispatch_Id"]) if r.get("Dispatch_Id") else i
        acc[short_name(r["Kernel_Name"])].append((order, float(r["Counter_Value"])))
    out = {}
    for k, v in acc.items():
        v.sort()
        if tails and k in tails:
            v = v[-tails[k]:]
        out[k] = (len(v), sum(x[1] for x in v) / len(v))
    return out


def traffic_summary(fetch_csv: str, write_csv: str, copy_bytes: float, cmd_f: str, cmd_w: str,
                    tails=()) -> str:
    fe = counter_means(fetch_csv, "FETCH_SIZE")
    wr = counter_means(write_csv, "WRITE_SIZE")
    copy_f = [v for k, v in fe.items() if "neg" in k]
    copy_w = [v for k, v in wr.items() if "neg" in k]
    if not copy_f or not copy_w:
        raise SystemExit("no copy-kernel dispatches found in the counter runs")
    ff = copy_bytes / (copy_f[0][1] * 1024.0)
    fw = copy_bytes / (copy_w[0][1] * 1024.0)
    out = ["# rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (KiB per dispatch)",
           f"# command (FETCH_SIZE): {cmd_f}", f"# command (WRITE_SIZE): {cmd_w}",
           f"# copy kernel: {copy_bytes:.0f} bytes read and written; it reads FETCH {copy_f[0][1]:.1f} KiB, "
           f"WRITE {copy_w[0][1]:.1f} KiB per dispatch",
           f"copy_fetch_factor {ff:.4f}", f"copy_write_factor {fw:.4f}",
           f"gemm_source_sha {gemm_source_hash()}",
           "# traffic <kernel> | dispatches | fetch_kib | write_kib | scaled_bytes_per_dispatch"]
    for k in sorted(fe):
        if "gemm" not in k or k not in wr:
            continue
        n, f = fe[k]
        _, w = wr[k]
        out.append(f"traffic {k} | {n} | {f:.1f} | {w:.1f} | {f * 1024 * ff + w * 1024 * fw:.0f}")
    if tails:
        # the profiled benchmark's timed steps come last: the same kernel
        # averaged over its last N dispatches only
        td = dict(tails)
        fe_t, wr_t = counter_means(fetch_csv, "FETCH_SIZE", td), counter_means(write_csv, "WRITE_SIZE", td)
        out.append("# traffic_tail <kernel> | last N dispatches | fetch_kib | write_kib | scaled_bytes_per_dispatch")
        for k, _ in tails:
            if k in fe_t and k in wr_t:
                n, f = fe_t[k]
                _, w = wr_t[k]
                out.append(f"traffic_tail {k} | {n} | {f:.1f} | {w:.1f} | {f * 1024 * ff + w * 1024 * fw:.0f}")
    return "\n".join(out) + "\n"


MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F16",
                 "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64")


def mfma_summary(csv_path: str, cmd: str) -> str:
    """Matrix-core flops per dispatch of every kernel that issues any, from
    the SQ_INSTS_VALU_MFMA_MOPS_* counters (units of 512 flops)."""
    means = {c: counter_means(csv_path, c) for c in MFMA_COUNTERS}
    names = sorted({k for m in means.values() for k, (_, v) in m.items() if v > 0})
    out = ["# rocprofv3 --pmc " + " ".join(c for c in MFMA_COUNTERS if means[c]),
           "# command: " + cmd,
           "# mfma <kernel> | dispatches | flops per dispatch: bf16 | f16 | f32 | f64"]
    for k in names:
        n = max(m.get(k, (0, 0.0))[0] for m in means.values())
        vals = [means[c].get(k, (0, 0.0))[1] * 512.0 for c in MFMA_COUNTERS]
        out.append(f"mfma {k} | {n} | " + " | ".join(f"{v:.4g}" for v in vals))
    return "\n".join(out) + "\n"


def counters_summary(csv_paths: list, cmds: list, kernels_like: str = "", tails=()) -> str:
    """Mean value per dispatch of every counter in the given counter-collection
    CSVs (one rocprofv3 --pmc pass each), by kernel: one line per (kernel,
    counter).  kernels_like: keep only kernels whose name contains it.  For a
    kernel in `tails` ((name, N) pairs) only its last N dispatches count."""
    td = dict(tails)
    rows = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in csv_paths:
        for i, r in enumerate(csv.DictReader(open(path))):
            k = short_name(r["Kernel_Name"])
            if kernels_like and kernels_like not in k:
                continue
            order = int(r["Dispatch_Id"]) if r.get("Dispatch_Id") else i
            rows[k][r["Counter_Name"]].append((order, float(r["Counter_Value"])))
    out = ["# rocprofv3 --pmc, one pass per command (counters summed over the chip, mean per dispatch)"]
    out += [f"# command (pass {i + 1}): {c}" for i, c in enumerate(cmds)]
    if td:
        out.append("# last dispatches only: " + ", ".join(f"{k} (last {n})" for k, n in td.items()))
    out.append("# counter <kernel> | dispatches | counter | mean per dispatch")
    for k in sorted(rows):
        for cn in sorted(rows[k]):
            v = sorted(rows[k][cn])
            if k in td:
                v = v[-td[k]:]
            out.append(f"counter {k} | {len(v)} | {cn} | {sum(x[1] for x in v) / len(v):.6g}")
    return "\n".join(out) + "\n"


def read_traffic(path: str, symbol: str):
    """Scaled HBM bytes per dispatch of `symbol` from a traffic summary, or
    None when the summary is missing, lacks the kernel, or was taken on GEMM
    sources other than the current ones."""
    if not os.path.exists(path):
        return None
    sha, val, tail = None, None, None
    for line in open(path):
        if line.startswith("gemm_source_sha "):
            sha = line.split()[1]
        elif line.startswith("traffic ") and line[8:].split(" | ")[0].strip() == symbol:
            val = float(line.rsplit("|", 1)[1])
        elif line.startswith("traffic_tail ") and line[13:].split(" | ")[0].strip() == symbol:
            tail = float(line.rsplit("|", 1)[1])
    if sha != gemm_source_hash():
        return None
    return tail if tail is not None else val


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--cmd", dest="command", required=True)
    s.add_argument("--trace", default=None, help="the run's kernel_trace.csv (for --tail)")
    s.add_argument("--tail", nargs="*", default=[], metavar="KERNEL=N")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--tail", nargs="*", default=[], metavar="KERNEL=N")
    t.add_argument("--out", required=True)
    cn = sub.add_parser("counters")
    cn.add_argument("--csv", nargs="+", required=True)
    cn.add_argument("--cmd", dest="commands", nargs="+", required=True)
    cn.add_argument("--kernels", default="")
    cn.add_argument("--tail", nargs="*", default=[], metavar="KERNEL=N")
    cn.add_argument("--out", required=True)
    mf = sub.add_parser("mfma")
    mf.add_argument("--csv", required=True)
    mf.add_argument("--cmd", dest="command", required=True)
    mf.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        text = stats_summary(a.csv, a.command, trace=a.trace, tails=parse_tails(a.tail))
    elif a.cmd == "mfma":
        text = mfma_summary(a.csv, a.command)
    elif a.cmd == "counters":
        text = counters_summary(a.csv, a.commands, a.kernels, parse_tails(a.tail))
    else:
        text = traffic_summary(a.fetch, a.write, a.copy_bytes, a.cmd_fetch, a.cmd_write, parse_tails(a.tail))
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
