"""Summaries of rocprofv3 output as short Markdown files.

    python -m paper_2007_08555_amd.prof stats KERNEL_STATS_CSV OUT.md "COMMAND" "TITLE"
    python -m paper_2007_08555_amd.prof traffic FETCH_CSV WRITE_CSV OUT.md "FETCH COMMAND" "WRITE COMMAND" \\
        "TITLE" CALIB_MIB KERNEL_REGEX SOURCE_FILE

`stats` tabulates `*_kernel_stats.csv` of `rocprofv3 --kernel-trace --stats`.

`traffic` turns two counter runs (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`,
both in KiB per dispatch) into HBM bytes.  Each run also executed one plain
device copy of CALIB_MIB MiB (read and written once); the copy dispatch is
the one with the largest WRITE_SIZE, and each counter is scaled by
(CALIB_MIB MiB) / (what it read for that copy).  Kernels whose names match
KERNEL_REGEX are summed per dispatch round (one launch of each per step).
The summary ends with two lines that bench.py reads:
`traffic_bytes_per_launch: <bytes>` and `kernel_part_sha256: <hash of the
FP64 evaluation part of SOURCE_FILE>` (the lines that part 1 of the build
compiles: the counters only describe the kernels built from them).
"""
import collections
import csv
import hashlib
import re
import sys


def _short(name):
    name = name.replace("(anonymous namespace)::", "").replace("|", "/")
    for cut in ("(mtp::", "(long", "(int", "(float", "(double"):
        name = name.split(cut)[0]
    return name


def stats(src, out, cmd, title):
    rows = list(csv.DictReader(open(src)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {title}", "", "Command (from the repository root on the MI355X):", "", "```",
             "cd /tmp && export TMPDIR=/tmp && cd $GRAFT_REPO_ROOT", cmd, "```", "",
             "rocprofv3 kernel statistics (`*_kernel_stats.csv`), kernels above 1 us average:", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        avg = float(r["AverageNs"]) / 1000
        if avg < 1:
            continue
        lines.append(f"| `{_short(r['Name'])[:90]}` | {r['Calls']} | {avg:.1f} | {float(r['MinNs']) / 1000:.1f} | "
                     f"{float(r['MaxNs']) / 1000:.1f} | {float(r['Percentage']):.1f}% |")
    open(out, "w").write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    """{kernel: [value per dispatch in dispatch order]} and the dispatch list."""
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    d = collections.defaultdict(list)
    for r in rows:
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return d, rows


def eval_part_digest(source_file):
    """SHA-256 of the lines of a generated kernel file that the FP64
    evaluation part of the build compiles."""
    from .build import _part_text
    with open(source_file, "rb") as fh:
        return hashlib.sha256(_part_text(fh.read(), 1)).hexdigest()


def traffic(fetch_csv, write_csv, out, cmd_fetch, cmd_write, title, calib_mib, kernel_regex, source_file):
    calib = float(calib_mib) * 2 ** 20
    fetch, frows = _per_kernel(fetch_csv, "FETCH_SIZE")
    write, wrows = _per_kernel(write_csv, "WRITE_SIZE")
    # the copy: largest WRITE_SIZE among copy dispatches; same position in the fetch run
    copies_w = [r for r in wrows if "copyBuffer" in r["Kernel_Name"]]
    copies_f = [r for r in frows if "copyBuffer" in r["Kernel_Name"]]
    k = max(range(len(copies_w)), key=lambda t: float(copies_w[t]["Counter_Value"]))
    f_copy = float(copies_f[k]["Counter_Value"]) * 1024
    w_copy = float(copies_w[k]["Counter_Value"]) * 1024
    sf, sw = calib / f_copy, calib / w_copy
    pat = re.compile(kernel_regex)
    names = sorted((n for n in set(fetch) | set(write) if pat.search(n)), key=_short)
    lines = [f"# {title}", "", "Commands (from the repository root on the MI355X):", "", "```",
             "cd /tmp && export TMPDIR=/tmp && cd $GRAFT_REPO_ROOT", cmd_fetch, cmd_write, "```", "",
             f"Calibration: one plain device copy of {calib_mib} MiB per run read FETCH_SIZE "
             f"{f_copy / 2 ** 20:.1f} MiB and WRITE_SIZE {w_copy / 2 ** 20:.1f} MiB; scale factors "
             f"{sf:.3f} (fetch) and {sw:.3f} (write).", "",
             "| kernel | dispatches | HBM read per dispatch (MB) | HBM write per dispatch (MB) |", "|---|---|---|---|"]
    tot_r = tot_w = 0.0
    for n in names:
        fr = fetch.get(n, [0.0])
        wr = write.get(n, [0.0])
        r_b = sum(fr) / len(fr) * 1024 * sf
        w_b = sum(wr) / len(wr) * 1024 * sw
        tot_r += r_b
        tot_w += w_b
        lines.append(f"| `{_short(n)[:90]}` | {len(fr)} | {r_b / 1e6:.1f} | {w_b / 1e6:.1f} |")
    lines += ["", f"Sum over the matched kernels (one launch each per step): read {tot_r / 1e9:.3f} GB, "
              f"written {tot_w / 1e9:.3f} GB.", ""]
    lines += [f"traffic_bytes_per_launch: {tot_r + tot_w:.6e}", f"kernel_part_sha256: {eval_part_digest(source_file)}"]
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:6])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:11])
    else:
        raise SystemExit(__doc__)
