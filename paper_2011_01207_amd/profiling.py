"""Summaries of rocprofv3 output for the committed profiles, and the HBM traffic lookup of the
benchmark's roofline entry.

  python -m paper_2011_01207_amd.profiling stats <kernel_stats.csv> <title> <command> [top] [kernel_trace.csv]
  python -m paper_2011_01207_amd.profiling traffic <fetch.csv> <write.csv> <title> <fetch command> <write command>
  python -m paper_2011_01207_amd.profiling counters <counter_collection.csv> <title> <command>

Traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, from two separate --pmc runs of the same
command) are scaled by what the same counters read for the plain 256 MiB device-to-device
copies the command ends with (__amd_rocclr_copyBuffer): bytes = KiB x 1024 x (copy bytes /
copy counter KiB x 1024).  Each kernel's row carries a SHA-256 of the sources it is built from;
the benchmark reports the traffic only while that hash still matches.
"""
import csv
import hashlib
import os
import re
import statistics as st
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 256 * 1024 * 1024
# sources of each profiled kernel family (the .hip file and the headers it includes)
HEADERS = ["common.h", "reduce.h", "spline.h"]
KERNEL_SOURCES = {
    "k_block_tiles": ["realspace.hip"], "k_real_reduce": ["realspace.hip"], "k_perm_assemble": ["realspace.hip"],
    "k_pme_": ["plane.hip"], "k_plane_": ["plane.hip"], "k_xybin": ["plane.hip"],
    "k_update": ["pcg.hip"], "k_direction": ["pcg.hip"], "k_init_residual": ["pcg.hip"],
    "k_filter": ["blocklist.hip"], "k_tile_refresh": ["blocklist.hip"], "k_rev_sort": ["blocklist.hip"],
}


def short(name):
    n = re.sub(r"\(.*", "", name).replace("void ", "").replace("amoeba::", "")
    return n.strip()[:90]


def sources_of(kernel):
    for prefix, files in KERNEL_SOURCES.items():
        if kernel.startswith(prefix):
            return files + HEADERS
    return None


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def streams_md(trace_csv, prefixes=("k_block_tiles",), short_us=5.0):
    """Per-stream durations of the named kernels from a --kernel-trace CSV: all dispatches, and
    those of at least short_us (the ones that return at entry after convergence excluded)."""
    d = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        k = short(r["Kernel_Name"])
        if any(k.startswith(p) for p in prefixes):
            d[(k, r["Stream_Id"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["\nPer stream (from the kernel trace of the same run; stream 1 is the second stream of the "
           "products, where the tiles run beside the reciprocal passes, stream 0 the stage pass that runs "
           f"every stage alone; 'working' excludes dispatches under {short_us:g} us):\n",
           "| kernel | stream | dispatches | avg us | working dispatches | working avg us |", "|---|---|---|---|---|---|"]
    for (k, sid), v in sorted(d.items()):
        w = [x for x in v if x >= short_us]
        out.append(f"| `{k}` | {sid} | {len(v)} | {st.mean(v):.2f} | {len(w)} | {st.mean(w) if w else 0:.2f} |")
    return "\n".join(out) + "\n"


def stats_md(path, title, cmd, top=30):
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}\n", f"Command (repository root on the profiled machine, R = its path):\n\n```\n{cmd}\n```\n",
           "Kernel durations in microseconds from `rocprofv3 --kernel-trace --stats` (all dispatches of the run).\n",
           "| kernel | calls | total us | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _per_kernel(path):
    d = defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[(short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return d


def _copy_factor(d):
    vals = [v for (k, g), vs in d.items() if k.startswith(COPY_KERNEL) for v in vs if v * 1024 > COPY_BYTES / 4]
    if not vals:
        raise SystemExit("no 256 MiB copy dispatch found for the calibration")
    return COPY_BYTES / (st.median(vals) * 1024.0), len(vals)


def traffic_md(fetch_csv, write_csv, title, fcmd, wcmd, top=20):
    f, w = _per_kernel(fetch_csv), _per_kernel(write_csv)
    ff, nf = _copy_factor(f)
    fw, nw = _copy_factor(w)
    rows = []
    for k in f:
        if k not in w or k[0].startswith("__amd_rocclr"):
            continue
        fk, wk = st.median(f[k]), st.median(w[k])
        rows.append((k[0], k[1], len(f[k]), fk, wk, fk * 1024 * ff + wk * 1024 * fw))
    rows.sort(key=lambda r: -r[5] * r[2])
    out = [f"# {title}\n",
           "Commands (repository root on the profiled machine, R = its path), FETCH_SIZE and WRITE_SIZE in separate runs:\n",
           f"```\n{fcmd}\n{wcmd}\n```\n",
           f"Copy calibration (the run's three 256 MiB `{COPY_KERNEL}` dispatches): FETCH_SIZE factor "
           f"{ff:.4f} ({nf} dispatches), WRITE_SIZE factor {fw:.4f} ({nw} dispatches); HBM bytes = "
           f"FETCH KiB x 1024 x {ff:.4f} + WRITE KiB x 1024 x {fw:.4f}.\n",
           "Per dispatch, median over the run's dispatches of the same kernel and grid; `sources` is the "
           "SHA-256 prefix of the files the kernel is built from at the time of the run.\n",
           "| kernel | grid | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes | sources |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        files = sources_of(r[0])
        hs = source_hash(files) if files else "-"
        out.append(f"| `{r[0]}` | {r[1]} | {r[2]} | {r[3]:.1f} | {r[4]:.1f} | {r[5]:.0f} | {hs} |")
    return "\n".join(out) + "\n"


def counters_md(path, title, cmd, kernels=None):
    d = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        d[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in d.values() for c in v})
    out = [f"# {title}\n", f"Command (repository root on the profiled machine, R = its path):\n\n```\n{cmd}\n```\n",
           "Median per dispatch.\n", "| kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
    for k, v in sorted(d.items(), key=lambda kv: -st.median(kv[1].get("SQ_WAVES", [0]))):
        if kernels and not any(k.startswith(p) for p in kernels):
            continue
        out.append(f"| `{k}` | " + " | ".join(f"{st.median(v[c]):.3g}" if c in v else "-" for c in names) + " |")
    return "\n".join(out) + "\n"


def traffic_lookup(md_path, kernel):
    """HBM bytes per dispatch of `kernel` from a committed traffic summary, or None when the
    summary is missing, has no row for it, or the kernel's sources changed since."""
    if not os.path.exists(md_path):
        return None
    files = sources_of(kernel)
    if not files:
        return None
    want = source_hash(files)
    for line in open(md_path):
        m = re.match(r"\| `([^`]*)` \| \d+ \| \d+ \| [\d.]+ \| [\d.]+ \| (\d+) \| (\w+) \|", line)
        if m and m.group(1) == kernel:
            return float(m.group(2)) if m.group(3) == want else None
    return None


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        print(stats_md(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]) if len(sys.argv) > 5 else 30), end="")
        if len(sys.argv) > 6:
            print(streams_md(sys.argv[6]), end="")
    elif mode == "traffic":
        print(traffic_md(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6]), end="")
    elif mode == "counters":
        print(counters_md(sys.argv[2], sys.argv[3], sys.argv[4]), end="")
    else:
        raise SystemExit(__doc__)
