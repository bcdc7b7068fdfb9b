"""Summaries of rocprofv3 output for the kernels of this package.

  python -m paper_2606_04882_amd.profsum kernels RESULTS_DB OUT.md --cmd "..."
      per-kernel calls / total / average duration table (markdown) from a
      --kernel-trace --stats run
  python -m paper_2606_04882_amd.profsum pmc RESULTS_DB COUNTER [--match S]
      per-kernel dispatch count and average counter value from a --pmc run
  python -m paper_2606_04882_amd.profsum sha KERNEL
      hash of the sources a kernel is built from (stored with counter
      records, so a record is used only while the kernel is unchanged)

RESULTS_DB is the SQLite database rocprofv3 writes (<pid>_results.db).
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def _code_only(text: bytes) -> bytes:
    """Source text without // comments and blank lines, so that a record
    survives edits of comments but not of code."""
    out = []
    for line in text.decode("utf-8", "replace").splitlines():
        if '"' not in line and "//" in line:
            line = line[:line.index("//")]
        line = line.rstrip()
        if line:
            out.append(line)
    return "\n".join(out).encode()


def kernel_sources_sha(kernel: str) -> str:
    """sha256 (16 hex digits) over what a kernel is built from, comments
    aside: its .hip file (k_fwd2d<...> -> k_fwd2d.hip, k_fwd3d_cross<...> ->
    k_fwd3d.hip), every header of csrc/ and the build script with its flags."""
    base = kernel.split("<")[0].split("::")[-1].replace("void ", "").strip()
    hip = os.path.join(CSRC, base + ".hip")
    while not os.path.exists(hip) and "_" in base:
        base = base.rsplit("_", 1)[0]
        hip = os.path.join(CSRC, base + ".hip")
    if not os.path.exists(hip):
        raise FileNotFoundError(f"no source file for kernel {kernel!r}")
    files = [hip] + sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
    files.append(os.path.join(HERE, "build.py"))
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(_code_only(fh.read()))
    return h.hexdigest()[:16]


def kernel_rows(db: str):
    """(name, calls, total us, average us, percent) per kernel, from the
    top_kernels view of the results database."""
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    con.close()
    return rows


def write_kernels(db: str, out: str, cmd: str):
    rows = kernel_rows(db)
    with open(out, "w") as f:
        f.write("# rocprofv3 kernel trace summary\n\nCommand (run from the repository root on one MI355X):\n\n")
        f.write(f"```\n{cmd}\n```\n\n")
        f.write("| kernel | calls | total (us) | average (us) | % |\n|---|---|---|---|---|\n")
        for n, c, t, a, p in rows:
            f.write(f"| `{n}` | {c} | {t:.1f} | {a:.3f} | {p:.2f} |\n")
    print(open(out).read())


def pmc_averages(db: str, counter: str):
    """{kernel name: [values per dispatch]} for one counter."""
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
    ci = {c: i for i, c in enumerate(cols)}
    name_col = "kernel_name" if "kernel_name" in ci else "name"
    agg = collections.defaultdict(list)
    for r in con.execute("select * from counters_collection"):
        if r[ci["counter_name"]] == counter:
            agg[r[ci[name_col]]].append(float(r[ci["value"]]))
    con.close()
    return agg


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="action", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("out")
    k.add_argument("--cmd", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("db")
    p.add_argument("counter")
    p.add_argument("--match", default="")
    s = sub.add_parser("sha")
    s.add_argument("kernel")
    a = ap.parse_args(argv)
    if a.action == "kernels":
        write_kernels(a.db, a.out, a.cmd)
    elif a.action == "pmc":
        agg = pmc_averages(a.db, a.counter)
        for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
            if a.match in name:
                print(f"{len(v):6d} dispatches  avg {sum(v) / len(v):14.1f}  {name}")
    else:
        print(kernel_sources_sha(a.kernel))


if __name__ == "__main__":
    sys.exit(main())
