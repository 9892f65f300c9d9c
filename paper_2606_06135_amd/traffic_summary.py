"""Per-launch memory traffic of one kernel from two rocprofv3 counter runs
(FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch), each scaled by what
the same counter reads for the plain copy kernel k_copy of the same run (N
doubles read and N doubles written per dispatch).  Writes a short markdown
summary that bench.py reads (with the SHA-256 of the kernel's sources at the
time of the measurement).

    python -m paper_2606_06135_amd.traffic_summary FETCH.csv WRITE.csv KERNEL N WORKLOAD "COMMAND" OUT.md
"""

import csv
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def per_dispatch(path, counter):
    vals = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] != counter:
                continue
            name = row["Kernel_Name"].split("(")[0].replace("void ", "").replace("hfdib::", "").split("<")[0]
            vals.setdefault(name, []).append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}


def main(fetch_csv, write_csv, kernel, ncells, workload, cmd, out):
    from bench import kernel_source_hash
    n = int(ncells)
    f, fcount = per_dispatch(fetch_csv, "FETCH_SIZE")
    w, _ = per_dispatch(write_csv, "WRITE_SIZE")
    copy_bytes = 8.0 * n
    kf = copy_bytes / (f["k_copy"] * 1024.0)
    kw = copy_bytes / (w["k_copy"] * 1024.0)
    fetch_b = f[kernel] * 1024.0 * kf
    write_b = w[kernel] * 1024.0 * kw
    total = fetch_b + write_b
    with open(out, "w") as fh:
        fh.write(f"# Memory traffic of {kernel}, {workload}\n\n")
        fh.write("Counters from two runs of the same command (from the repository root, one MI355X), "
                 "the first with `--pmc FETCH_SIZE`, the second with `--pmc WRITE_SIZE`:\n\n")
        fh.write(f"```\n{cmd}\n```\n\n")
        fh.write("FETCH_SIZE and WRITE_SIZE count the traffic between the L2 caches and the memory "
                 "fabric (last-level cache or HBM).  Each is scaled by the reading of the same counter "
                 f"for the copy kernel k_copy of that run, which reads and writes {n} doubles per dispatch.\n\n")
        fh.write("| quantity | value |\n|---|---:|\n")
        fh.write(f"| dispatches of {kernel} | {fcount[kernel]} |\n")
        fh.write(f"| FETCH_SIZE per dispatch (KiB) | {f[kernel]:.1f} |\n")
        fh.write(f"| WRITE_SIZE per dispatch (KiB) | {w[kernel]:.1f} |\n")
        fh.write(f"| k_copy FETCH_SIZE / WRITE_SIZE (KiB) | {f['k_copy']:.1f} / {w['k_copy']:.1f} |\n")
        fh.write(f"| calibration factors fetch / write | {kf:.4f} / {kw:.4f} |\n")
        fh.write(f"| bytes read per launch | {fetch_b:.0f} ({fetch_b / n:.2f} B/cell) |\n")
        fh.write(f"| bytes written per launch | {write_b:.0f} ({write_b / n:.2f} B/cell) |\n\n")
        fh.write(f"- traffic_bytes_per_launch: {total:.0f}\n")
        fh.write(f"- source_sha256: `{kernel_source_hash(kernel)}`\n")


if __name__ == "__main__":
    main(*sys.argv[1:8])
