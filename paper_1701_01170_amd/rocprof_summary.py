"""Summaries of rocprofv3 output for the committed profiles/ directory.

  python -m paper_1701_01170_amd.rocprof_summary stats <rocpd_dir> <out.md> "<command>" \
          [<label>=<kernel-regex> ...]
      per-kernel call counts and durations (from --kernel-trace --stats runs);
      each label=regex adds a line for all kernels whose name matches
  python -m paper_1701_01170_amd.rocprof_summary traffic <fetch_dir> <write_dir> <kernel-regex> \
          <copy_bytes> <out.json> "<command>"
      bytes per launch that the kernels matching the regex move between the
      L2 caches and the memory fabric, from a FETCH_SIZE run and a WRITE_SIZE
      run, each scaled by what the same counter reads for the calibration copy
      kernel (k_copy16, copy_bytes read and copy_bytes written per launch).
      These counters sit at the L2's fabric side: reads the Infinity Cache
      serves count too, so the figure bounds HBM traffic from above; for a
      streaming kernel the two agree, for a random gather they need not.
  python -m paper_1701_01170_amd.rocprof_summary counters <out.md> "<command>" \
          <label>=<kernel-regex> <pmc_dir> [<pmc_dir> ...]
      per-dispatch averages of every counter found in the --pmc runs, over
      the dispatches of the kernels matching the regex, plus the ratios the
      kernel analysis uses (wait share of wave cycles, L2 hit rate)

rocprofv3 writes a rocpd SQLite database; only its `kernels` and
`counters_collection` views are read here.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _db(d: str) -> sqlite3.Connection:
    files = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no rocpd database under {d}")
    return sqlite3.connect(files[0])


def short_name(n: str) -> str:
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*\)$", "", n)
    return n.replace("gr::", "").replace("void ", "")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1701_01170_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def stats(d: str, out: str, command: str, groups=()) -> None:
    c = _db(d)
    agg = {}
    for name, dur in c.execute("select name, duration from kernels"):
        k = short_name(name)
        a = agg.setdefault(k, [0, 0.0, float("inf"), 0.0])
        a[0] += 1
        a[1] += dur
        a[2] = min(a[2], dur)
        a[3] = max(a[3], dur)
    total = sum(a[1] for a in agg.values())
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             f"Kernel source hash: `{kernel_source_hash()}`", "",
             "| kernel | calls | total us | avg us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k, (n, tot, mn, mx) in sorted(agg.items(), key=lambda x: -x[1][1]):
        lines.append(f"| `{k}` | {n} | {tot / 1e3:.1f} | {tot / 1e3 / n:.2f} | {mn / 1e3:.2f} | "
                     f"{mx / 1e3:.2f} | {100 * tot / total:.1f} |")
    if groups:
        lines += ["", "| group (kernel regex) | calls | total us | avg us |", "|---|---:|---:|---:|"]
        for g in groups:
            label, rx = g.split("=", 1)
            sel = [(n, tot) for k, (n, tot, _, _) in agg.items() if re.search(rx, k)]
            n = sum(x[0] for x in sel)
            tot = sum(x[1] for x in sel)
            if n:
                lines.append(f"| {label} (`{rx}`) | {n} | {tot / 1e3:.1f} | {tot / 1e3 / n:.2f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:20] + lines[-4:]))


def _counter_per_dispatch(d: str, counter: str):
    c = _db(d)
    rows = c.execute("select dispatch_id, kernel_name, value from counters_collection "
                     "where counter_name = ?", (counter,))
    return [(did, short_name(kn), v) for did, kn, v in rows]


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int, out: str,
            command: str) -> None:
    res = {}
    for label, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _counter_per_dispatch(d, counter)
        copy = [v for _, n, v in rows if "k_copy16" in n]
        kern = [v for _, n, v in rows if re.search(kernel, n)]
        if not copy or not kern:
            raise RuntimeError(f"{counter}: no copy-kernel or '{kernel}' dispatches in {d}")
        # counter values are KiB per dispatch; the copy kernel moves copy_bytes each way
        scale = (copy_bytes / 1024.0) / (sum(copy) / len(copy))
        res[label] = dict(kib_per_launch=sum(kern) / len(kern), launches=len(kern),
                          copy_kib_per_launch=sum(copy) / len(copy), scale=scale)
    fabric = 1024.0 * (res["fetch"]["kib_per_launch"] * res["fetch"]["scale"]
                       + res["write"]["kib_per_launch"] * res["write"]["scale"])
    raw = 1024.0 * (res["fetch"]["kib_per_launch"] + res["write"]["kib_per_launch"])
    j = dict(kernel=kernel, command=command, kernel_source_hash=kernel_source_hash(),
             fetch=res["fetch"], write=res["write"],
             l2_fabric_bytes_per_launch=round(fabric), unscaled_bytes_per_launch=round(raw),
             meaning="L2 <-> fabric bytes per launch (FETCH_SIZE + WRITE_SIZE, each scaled by "
                     "its reading for the copy kernel); Infinity Cache hits included, so an "
                     "upper bound of HBM bytes")
    with open(out, "w") as f:
        json.dump(j, f, indent=1)
    print(json.dumps(j, indent=1))


def counters(out: str, command: str, group: str, dirs) -> None:
    label, rx = group.split("=", 1)
    vals = {}
    for d in dirs:
        c = _db(d)
        for kn, name, v in c.execute("select kernel_name, counter_name, value from counters_collection"):
            if re.search(rx, short_name(kn)):
                vals.setdefault(name, []).append(v)
    if not vals:
        raise RuntimeError(f"no dispatches of '{rx}' in {dirs}")
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    lines = ["# rocprofv3 counters", "", f"Command: `{command}`", "",
             f"Kernel source hash: `{kernel_source_hash()}`", "",
             f"Kernels: {label} (`{rx}`)", "",
             "| counter | dispatches | average per dispatch |", "|---|---:|---:|"]
    for k in sorted(avg):
        lines.append(f"| `{k}` | {len(vals[k])} | {avg[k]:.6g} |")
    ratios = []
    if "SQ_WAIT_ANY" in avg and avg.get("SQ_WAVE_CYCLES"):
        ratios.append(("waves waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES)",
                       avg["SQ_WAIT_ANY"] / avg["SQ_WAVE_CYCLES"]))
    if avg.get("SQ_WAVE_CYCLES") and avg.get("SQ_WAVES"):
        ratios.append(("average wave lifetime in cycles (SQ_WAVE_CYCLES / SQ_WAVES)",
                       avg["SQ_WAVE_CYCLES"] / avg["SQ_WAVES"]))
    if "TCC_HIT_sum" in avg and "TCC_MISS_sum" in avg and avg["TCC_HIT_sum"] + avg["TCC_MISS_sum"] > 0:
        ratios.append(("L2 hit rate (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum))",
                       avg["TCC_HIT_sum"] / (avg["TCC_HIT_sum"] + avg["TCC_MISS_sum"])))
    if ratios:
        lines += ["", "| ratio | value |", "|---|---:|"]
        lines += [f"| {n} | {v:.4g} |" for n, v in ratios]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6], sys.argv[7])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:])
    else:
        raise SystemExit(__doc__)
