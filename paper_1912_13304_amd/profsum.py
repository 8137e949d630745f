"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_1912_13304_amd.profsum stats KERNEL_STATS_CSV --title T --cmd C
      Markdown table of the per-kernel statistics of a --kernel-trace --stats run.

  python -m paper_1912_13304_amd.profsum traffic --fetch CSV --write CSV --cmd-fetch C --cmd-write C
      JSON of the HBM traffic per dispatch from two --pmc runs (FETCH_SIZE, then
      WRITE_SIZE), per kernel, each counter scaled by what it reads for the plain
      1 GiB device copy that the benchmark runs (the largest copy dispatch).  The
      JSON records a hash of the HIP sources: the benchmark reports the traffic
      only while the sources are unchanged.
"""
import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30   # the benchmark's calibration copy: 2^27 float64 read and written


def source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.replace("fde::", "").replace("bat::", "")
    return name.split("(")[0] if "(" in name else name


def stats(path, title, cmd, top=30):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", cmd, "```", "",
           f"Total kernel time: {tot / 1e6:.1f} ms", "",
           "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def per_kernel(path, counter):
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = r["Kernel_Name"]
        a = acc.setdefault(k, [0.0, 0, 0.0])
        v = float(r["Counter_Value"])
        a[0] += v
        a[1] += 1
        a[2] = max(a[2], v)
    return acc


def traffic(fetch_csv, write_csv, cmd_fetch, cmd_write):
    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    copies = [k for k in f if "copy" in k.lower()]
    if not copies:
        raise SystemExit("no copy kernel in the FETCH_SIZE run")
    ck = max(copies, key=lambda k: f[k][2])
    fetch_kib, write_kib = f[ck][2], w.get(ck, [0, 0, 0.0])[2]
    ff = COPY_BYTES / (fetch_kib * 1024.0)
    wf = COPY_BYTES / (write_kib * 1024.0) if write_kib else 1.0
    kernels = {}
    for k in f:
        if k not in w:
            continue
        fa = f[k][0] / f[k][1]
        wa = w[k][0] / w[k][1]
        kernels[k] = {"dispatches": f[k][1], "fetch_kib_avg": fa, "write_kib_avg": wa,
                      "traffic_bytes_avg": ff * fa * 1024.0 + wf * wa * 1024.0}
    return {"source_hash": source_hash(), "commands": [cmd_fetch, cmd_write],
            "calibration": {"copy_kernel": ck, "copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                            "fetch_kib": fetch_kib, "write_kib": write_kib, "fetch_factor": ff,
                            "write_factor": wf},
            "kernels": kernels}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        sys.stdout.write(stats(a.csv, a.title, a.cmd))
    else:
        json.dump(traffic(a.fetch, a.write, a.cmd_fetch, a.cmd_write), sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()
