"""Summaries of rocprofv3 runs of bench.py: kernel times and HBM traffic.

    python -m paper_2205_05982_amd.profile_summary KT_DIR FETCH_CSV WRITE_CSV OUT_MD "COMMANDS" "TITLE" [COPY_BYTES]

KT_DIR holds the ``--kernel-trace --stats`` CSV files (kt_kernel_stats.csv,
kt_kernel_trace.csv); FETCH_CSV and WRITE_CSV are the counter_collection.csv files
of a ``--pmc FETCH_SIZE`` and a ``--pmc WRITE_SIZE`` run of the same command.
Counter values are KiB per dispatch; they are scaled by what the same counter reads
for the device-to-device copies of the input buffers that bench.py makes (a copy of
B bytes reads and writes B bytes; COPY_BYTES, default 8e8, is the size of the
input).  Writes OUT_MD and, beside it, a JSON file with the level kernel's average
HBM bytes per launch and the hash of the kernel sources they were measured on
(bench.py reports the traffic only while the hash matches).  Runs that include the
learned splitter also get the time and traffic of its histogram and scatter
kernels against their algorithmic bytes (one read; one read and one write of the
keys).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """sha256 of the HIP sources of the sorting kernels."""
    d = os.path.join(HERE, "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip", ".inc")) and "learned" not in f:
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _is_level(name: str) -> bool:
    """The device-wide partition kernel (either placement of its output)."""
    return "level_kernel" in name or "level_runs_kernel" in name


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _short(n: str) -> str:
    import re
    n = n.replace("void ", "")
    n = re.sub(r"vqs::KeyL<(\d+), (\d+)> ?", lambda m: f"k{m.group(1)},I{m.group(2)}", n)
    n = re.sub(r"vqs::Key<(\d+)> ?", lambda m: f"k{m.group(1)}", n)
    for a, b in (("(vqs::Params)", ""), ("vqs::", "")):
        n = n.replace(a, b)
    return n[:60]


def summarize(kt_dir, fetch_csv, write_csv, commands, title, copy_bytes=800_000_000):
    out = [f"# {title}\n",
           "Commands (from the repository root on the MI355X box, after `cd /tmp && export TMPDIR=/tmp`):\n"]
    out += [f"    {c.strip()}" for c in commands.split(";;")]
    out.append("")
    stats = _rows(os.path.join(kt_dir, "kt_kernel_stats.csv"))
    out.append("## Kernel time (rocprofv3 --kernel-trace --stats)\n")
    out.append("| kernel | calls | total ms | average us | min us | max us | % |")
    out.append("|---|---|---|---|---|---|---|")
    for r in stats[:8]:
        out.append(f"| {_short(r['Name'])} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {int(r['MinNs']) / 1e3:.1f} | {int(r['MaxNs']) / 1e3:.1f} | "
                   f"{r['Percentage']} |")
    tr = _rows(os.path.join(kt_dir, "kt_kernel_trace.csv"))
    lv = [r for r in tr if _is_level(r["Kernel_Name"])]
    kname = "level_runs_kernel" if any("level_runs_kernel" in r["Kernel_Name"] for r in lv) else "level_kernel"
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in lv]
    lv_avg_us = statistics.mean(durs) if durs else 0.0
    out.append("")
    out.append(f"{kname} launches: {len(durs)}, average {lv_avg_us:.1f} us; the last step's launches (us): "
               + ", ".join(f"{d:.0f}" for d in durs[-20:]))

    f, w = _rows(fetch_csv), _rows(write_csv)
    alg_kib = copy_bytes / 1024

    def copies(rows):
        vals = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        big = max(vals)
        return [v for v in vals if v > 0.9 * big]

    fc, wc = copies(f), copies(w)
    ff, wf = alg_kib / statistics.mean(fc), alg_kib / statistics.mean(wc)
    out.append("\n## HBM traffic (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE; KiB per dispatch)\n")
    out.append(f"Calibration: the {copy_bytes / 1e6:.0f} MB device-to-device copies of the input "
               f"(`__amd_rocclr_copyBuffer`) read and write {alg_kib:.0f} KiB each; they report FETCH_SIZE = "
               f"{statistics.mean(fc):.0f} KiB (factor {ff:.3f}) and WRITE_SIZE = {statistics.mean(wc):.0f} KiB "
               f"(factor {wf:.3f}).\n")
    lvf = [float(r["Counter_Value"]) for r in f if _is_level(r["Kernel_Name"])]
    lvw = [float(r["Counter_Value"]) for r in w if _is_level(r["Kernel_Name"])]
    full_f = [v for v in lvf if v > 0.9 * max(lvf)]
    full_w = [v for v in lvw if v > 0.9 * max(lvw)]
    mf, mw = statistics.mean(full_f) * ff, statistics.mean(full_w) * wf
    out.append(f"{kname} on a full level (every key once; algorithmic {alg_kib:.0f} KiB read + "
               f"{alg_kib:.0f} KiB written): read {mf:.0f} KiB ({mf / alg_kib:.3f} of algorithmic), written "
               f"{mw:.0f} KiB ({mw / alg_kib:.3f}).")
    per_launch = (statistics.mean(lvf) * ff + statistics.mean(lvw) * wf) * 1024
    out.append(f"Average over all {len(lvf)} {kname} dispatches: {per_launch / 1e6:.1f} MB per launch "
               f"(read + written, scaled).")
    def solo(name, inplace):
        return "solo_kernel" in name and (", true>" in name) == inplace

    sf = [float(r["Counter_Value"]) for r in f if solo(r["Kernel_Name"], False)]
    sw = [float(r["Counter_Value"]) for r in w if solo(r["Kernel_Name"], False)]
    if sf:
        out.append(f"\nsolo_kernel per launch: read {statistics.mean(sf) * ff:.0f} KiB, written "
                   f"{statistics.mean(sw) * wf:.0f} KiB (scaled).")
    # in-place mode (bench.py's in-place record), if the run has it
    ipk = [("ip_count_kernel", 1, 0), ("ip_scatter_kernel", 1, 1)]
    if any("ip_count_kernel" in r["Kernel_Name"] for r in tr):
        out.append("\n## In-place mode (the bench's in-place sorts)\n")
        for lk, reads, writes in ipk:
            kf = [float(r["Counter_Value"]) for r in f if lk in r["Kernel_Name"]]
            kw = [float(r["Counter_Value"]) for r in w if lk in r["Kernel_Name"]]
            kd = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr if lk in r["Kernel_Name"]]
            if not (kf and kw and kd):
                continue
            full_d = [d for d in kd if d > 0.8 * max(kd)]
            full_f = [v for v in kf if v > 0.9 * max(kf)]
            full_w = [v for v in kw if v > 0.9 * max(kw)] if max(kw) > 0 else [0.0]
            rd, wr = statistics.mean(full_f) * ff, statistics.mean(full_w) * wf
            wtxt = (f"writes {wr:.0f} KiB ({wr / alg_kib:.3f} of one pass)" if writes else
                    f"writes {wr:.0f} KiB (block counts and their look-back words)")
            out.append(f"{lk}: {len(kd)} launches, {sum(kd) / 1e3:.3f} ms in all; on a full level "
                       f"(about {statistics.mean(full_d):.0f} us) it reads {rd:.0f} KiB ({rd / alg_kib:.3f} of "
                       f"one pass over the keys) and {wtxt}; "
                       f"{(rd + wr) * 1024 / (statistics.mean(full_d) * 1e-6) / 1e9:.0f} GB/s measured traffic.")
        isf = [float(r["Counter_Value"]) for r in f if solo(r["Kernel_Name"], True)]
        isw = [float(r["Counter_Value"]) for r in w if solo(r["Kernel_Name"], True)]
        isd = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr
               if solo(r["Kernel_Name"], True)]
        if isf and isd:
            out.append(f"solo_kernel (in place): {statistics.mean(isd):.0f} us per launch, read "
                       f"{statistics.mean(isf) * ff:.0f} KiB, written {statistics.mean(isw) * wf:.0f} KiB (scaled).")
    # the learned splitter's one-pass kernels, if the run has them
    def learned(name, lk):
        return lk in name and "ip_" + lk not in name

    for lk, reads, writes in (("histogram_kernel", 1, 0), ("scatter_kernel", 1, 1)):
        kf = [float(r["Counter_Value"]) for r in f if learned(r["Kernel_Name"], lk)]
        kw = [float(r["Counter_Value"]) for r in w if learned(r["Kernel_Name"], lk)]
        kd = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr
              if learned(r["Kernel_Name"], lk)]
        if not (kf and kw and kd):
            continue
        big = [d for d in kd if d > 0.5 * max(kd)]    # the launches over the whole input
        nbytes = max(kf) * ff * 1024 / max(reads, 1)  # one read of the keys
        out.append(f"\n{lk}: {len(kd)} launches, the large ones average {statistics.mean(big):.1f} us; on the "
                   f"largest input it reads {max(kf) * ff:.0f} KiB and writes {max(kw) * wf:.0f} KiB "
                   f"(algorithmic: {reads} read{'' if not writes else ' + 1 write'} of the keys, "
                   f"{(reads + writes) * nbytes / 1e6:.0f} MB); achieved "
                   f"{(max(kf) * ff + max(kw) * wf) * 1024 / (statistics.mean(big) * 1e-6) / 1e9:.0f} GB/s measured "
                   f"traffic.")
    js = {"kernel": kname, "traffic_bytes_per_launch": per_launch, "launches": len(lvf),
          "avg_launch_us_trace": lv_avg_us, "fetch_factor": ff, "write_factor": wf,
          "full_level_read_frac": mf / alg_kib, "full_level_write_frac": mw / alg_kib,
          "source_hash": kernel_source_hash()}
    return "\n".join(out) + "\n", js


def main(argv):
    kt_dir, fetch_csv, write_csv, out_md, commands, title = argv[1:7]
    copy_bytes = int(float(argv[7])) if len(argv) > 7 else 800_000_000
    md, js = summarize(kt_dir, fetch_csv, write_csv, commands, title, copy_bytes)
    with open(out_md, "w") as f:
        f.write(md)
    with open(os.path.splitext(out_md)[0] + ".traffic.json", "w") as f:
        json.dump(js, f, indent=1)
    print(md)


if __name__ == "__main__":
    main(sys.argv)
