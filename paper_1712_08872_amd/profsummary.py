"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as markdown.

Usage: python -m paper_1712_08872_amd.profsummary <results.db> "<command>" [top]
"""
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


if __name__ == "__main__":
    print(summary(sys.argv[1], sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 12))
