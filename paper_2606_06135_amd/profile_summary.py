"""Turn a rocprofv3 --kernel-trace --stats result database into a short
markdown summary (per-kernel calls, total and average duration).

    python -m paper_2606_06135_amd.profile_summary DB OUT.md "COMMAND" "TITLE"
"""

import sqlite3
import sys


def main(db, out, cmd, title):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    tot = sum(r[2] for r in rows)
    with open(out, "w") as f:
        f.write(f"# {title}\n\nCommand (from the repository root, on one MI355X):\n\n```\n{cmd}\n```\n\n")
        f.write("rocprofv3 kernel-trace summary (durations in microseconds); total GPU kernel time "
                f"{tot / 1e3:.2f} ms over the whole run, set-up included.\n\n")
        f.write("| kernel | calls | total us | avg us | % |\n|---|---:|---:|---:|---:|\n")
        for n, c, t, a, p in rows:
            short = n.split("(")[0].replace("hfdib::", "").replace("void ", "")
            f.write(f"| {short} | {c} | {t:.1f} | {a:.2f} | {p:.2f} |\n")


if __name__ == "__main__":
    main(*sys.argv[1:5])
