"""Summarise rocprofv3 output.

  python -m paper_1712_08872_amd.profsummary <results.db> "<command>" [top]
      markdown table of a --kernel-trace --stats database (rocpd SQLite)
  python -m paper_1712_08872_amd.profsummary traffic <fetch.csv> <write.csv>
      <copy_fetch.csv> <copy_write.csv> <copy_bytes> <sha256> name=regex ...
      per-launch HBM traffic of each named kernel (matched by regex) from
      FETCH_SIZE and WRITE_SIZE counter passes (KiB per dispatch), each
      scaled by what the same counter reads for a plain copy of copy_bytes
      bytes; JSON out
"""
import csv
import json
import re
import sqlite3
import sys


def summary(db, command, top=12):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["# rocprofv3 --kernel-trace --stats summary", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows[:top]:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {calls} | {tot / 1e3:.1f} | {avg:.1f} | {pct:.3f} |")
    return "\n".join(out) + "\n"


def _per_dispatch(path, regex):
    vals = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if re.search(regex, row["Kernel_Name"]):
                vals[row["Dispatch_Id"]] = vals.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
    return vals


def traffic(fetch, write, cfetch, cwrite, copy_bytes, sha, named):
    # the copy probe: the largest dispatch is the copy of copy_bytes
    cf = max(_per_dispatch(cfetch, ".").values())
    cw = max(_per_dispatch(cwrite, ".").values())
    ff = copy_bytes / (cf * 1024.0)
    fw = copy_bytes / (cw * 1024.0)
    out = {"source_sha256": sha, "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": ff, "write_scale": fw, "kernels": {}}
    for name, regex in named:
        f = _per_dispatch(fetch, regex)
        w = _per_dispatch(write, regex)
        fk = sum(f.values()) / len(f)
        wk = sum(w.values()) / len(w)
        out["kernels"][name] = {"regex": regex, "dispatches": len(f), "fetch_kib_per_dispatch": fk,
                                "write_kib_per_dispatch": wk,
                                "traffic_bytes_per_launch": fk * 1024.0 * ff + wk * 1024.0 * fw}
    return out


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        a = sys.argv[2:]
        named = [tuple(x.split("=", 1)) for x in a[6:]]
        print(json.dumps(traffic(a[0], a[1], a[2], a[3], float(a[4]), a[5], named), indent=1))
    else:
        print(summary(sys.argv[1], sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 12))
