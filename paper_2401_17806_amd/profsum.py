"""Short text summaries of rocprofv3 results (SQLite databases written with -d DIR -o NAME).

  python -m paper_2401_17806_amd.profsum kernels DB [--top N]
      per-kernel calls / mean / total duration from a --kernel-trace --stats run
  python -m paper_2401_17806_amd.profsum counters DB KERNEL_SUBSTRING
      mean per dispatch of every counter of a --pmc run, over the matching dispatches
  python -m paper_2401_17806_amd.profsum traffic FETCH_DB WRITE_DB --workload W --bytes B
      HBM bytes per CG-iteration launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of
      k_cg_step, each divided by the same counter's reading per byte on the calibration kernel
      (bench.py --copy-calibration: torch's elementwise multiply by a scalar, whose kernel name
      carries AUnaryFunctor, reading and writing B bytes).  Prints the markdown lines bench.py
      reads back.
"""
from __future__ import annotations

import argparse
import collections
import glob
import os
import sqlite3
import statistics


def _db(path: str) -> str:
    if os.path.isdir(path):
        hits = sorted(glob.glob(os.path.join(path, "**", "*results.db"), recursive=True))
        if not hits:
            raise SystemExit(f"no *results.db under {path}")
        return hits[0]
    return path


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if "(" in name else name


def kernels(db: str, top: int) -> None:
    con = sqlite3.connect(_db(db))
    rows = list(con.execute("select name, total_calls, average, total_duration, percentage "
                            "from top_kernels"))
    print(f"| kernel | calls | mean us | total ms | % |")
    print(f"|---|---|---|---|---|")
    # top_kernels holds durations in microseconds
    for name, calls, avg, tot, pct in rows[:top]:
        print(f"| `{_short(str(name))[:90]}` | {calls} | {avg:.3f} | {tot / 1e3:.3f} | "
              f"{pct:.1f} |")


def counter_means(db: str, substr: str) -> dict:
    con = sqlite3.connect(_db(db))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for d, kn, c, v in con.execute(
            "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        if substr in str(kn):
            per[d][c] += v
    if not per:
        raise SystemExit(f"no dispatch of a kernel matching {substr!r} in {db}")
    names = sorted({c for d in per.values() for c in d})
    return {c: statistics.fmean(per[d][c] for d in per) for c in names} | {"_dispatches": len(per)}


def traffic(fetch_db: str, write_db: str, workload: str, copy_bytes: int) -> None:
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for name in ("kernels_cg.hip", "kernels_mx.hip", "mx.h", "device_common.h", "refops.h",
                 "sld_internal.h"):
        with open(os.path.join(root, "csrc", name), "rb") as f:
            h.update(f.read())
    f_cg = counter_means(fetch_db, "k_cg_step")
    w_cg = counter_means(write_db, "k_cg_step")
    f_cp = counter_means(fetch_db, "AUnaryFunctor")
    w_cp = counter_means(write_db, "AUnaryFunctor")
    ff = f_cp["FETCH_SIZE"] * 1024.0 / copy_bytes
    wf = w_cp["WRITE_SIZE"] * 1024.0 / copy_bytes
    hbm = f_cg["FETCH_SIZE"] * 1024.0 / ff + w_cg["WRITE_SIZE"] * 1024.0 / wf
    print(f"- workload: `{workload}`")
    print(f"- kernel_source_sha256: `{h.hexdigest()}`")
    print(f"- k_cg_step_dispatches: {f_cg['_dispatches']} (FETCH run), {w_cg['_dispatches']} (WRITE run)")
    print(f"- fetch_kib_per_dispatch: {f_cg['FETCH_SIZE']:.1f}")
    print(f"- write_kib_per_dispatch: {w_cg['WRITE_SIZE']:.1f}")
    print(f"- copy_bytes: {copy_bytes}")
    print(f"- copy_fetch_kib_per_dispatch: {f_cp['FETCH_SIZE']:.1f}")
    print(f"- copy_write_kib_per_dispatch: {w_cp['WRITE_SIZE']:.1f}")
    print(f"- fetch_scale: {ff:.4f}")
    print(f"- write_scale: {wf:.4f}")
    print(f"- hbm_fetch_bytes_per_launch: {f_cg['FETCH_SIZE'] * 1024.0 / ff:.0f}")
    print(f"- hbm_write_bytes_per_launch: {w_cg['WRITE_SIZE'] * 1024.0 / wf:.0f}")
    print(f"- hbm_bytes_per_launch: {hbm:.0f}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--top", type=int, default=12)
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("kernel")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--workload", required=True)
    t.add_argument("--bytes", type=int, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        kernels(a.db, a.top)
    elif a.cmd == "counters":
        for name, v in counter_means(a.db, a.kernel).items():
            print(f"- {name}: {v:.1f}")
    else:
        traffic(a.fetch_db, a.write_db, a.workload, a.bytes)


if __name__ == "__main__":
    main()
