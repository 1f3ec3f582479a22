"""Summaries of rocprofv3 CSV output for ``profiles/``.

``python -m paper_2303_12873_amd.profsum stats <kernel_stats.csv> [N]``
    Markdown table of the N most expensive kernels (calls, mean and total
    duration, share of GPU time).

``python -m paper_2303_12873_amd.profsum traffic <fetch.csv> <write.csv>
  <copy_fetch.csv> <copy_write.csv> <copy_bytes> <kernel substring>``
    HBM traffic per launch of one kernel from two ``--pmc FETCH_SIZE`` /
    ``--pmc WRITE_SIZE`` runs (KiB per dispatch), each scaled by what the
    same counter reads for a plain device copy of ``copy_bytes`` bytes (runs
    of ``python -m paper_2303_12873_amd.microbench copy``).
"""
from __future__ import annotations

import csv
import re
import sys


def _short(name: str) -> str:
    name = name.replace("pic::(anonymous namespace)::", "")
    m = re.search(r"(k_\w+(<[^()]*>)?)\(", name)
    return m.group(1) if m else name[:60]


def stats(path: str, top: int = 15) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | mean ms | total ms | share % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str, match: str):
    vals = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, match):
    copy_bytes = float(copy_bytes)
    cf = _per_dispatch(copy_fetch_csv, "FETCH_SIZE", "k_copy16")
    cw = _per_dispatch(copy_write_csv, "WRITE_SIZE", "k_copy16")
    kf = _per_dispatch(fetch_csv, "FETCH_SIZE", match)
    kw = _per_dispatch(write_csv, "WRITE_SIZE", match)
    if not (cf and cw and kf and kw):
        raise SystemExit("missing dispatches in the counter files")
    sf = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    sw = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    fetch = sum(kf) / len(kf) * 1024.0 * sf
    write = sum(kw) / len(kw) * 1024.0 * sw
    return {"fetch_scale": sf, "write_scale": sw, "fetch_bytes": fetch, "write_bytes": write,
            "traffic_bytes_per_launch": int(round(fetch + write)), "dispatches": (len(kf), len(kw))}


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        print(stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 15))
    elif len(sys.argv) == 8 and sys.argv[1] == "traffic":
        for k, v in traffic(*sys.argv[2:]).items():
            print(f"- {k}: {v}")
    else:
        print(__doc__)
        sys.exit(2)
