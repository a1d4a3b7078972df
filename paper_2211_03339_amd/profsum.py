"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2211_03339_amd.profsum stats KERNEL_STATS_CSV OUT_TXT "COMMAND"
      per-kernel calls / total / average / min / max duration from `rocprofv3 --kernel-trace --stats`.
  python -m paper_2211_03339_amd.profsum stats-db DB_DIR OUT_TXT "COMMAND"
      the same table from the rocpd database (*_results.db) of a `rocprofv3 --kernel-trace` run.
  python -m paper_2211_03339_amd.profsum traffic FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV COPY_BYTES
      OUT_JSON SOURCES "COMMANDS"
  python -m paper_2211_03339_amd.profsum traffic-db FETCH_DB_DIR WRITE_DB_DIR COPY_FETCH_DB_DIR COPY_WRITE_DB_DIR
      COPY_BYTES OUT_JSON SOURCES "COMMANDS"
      the same from the rocpd databases of the four `rocprofv3 --pmc` runs (for a run that ends with
      the profiler's own fault after a cooperative launch, when no CSV is written)
      mean FETCH_SIZE / WRITE_SIZE per dispatch and kernel from two `rocprofv3 --pmc` runs, each
      scaled by bytes / counter of a plain device copy of COPY_BYTES bytes measured with the same
      counter, with the sha256 of each kernel source in SOURCES (comma-separated; bench.py reports
      the traffic only while they are unchanged).
"""
from __future__ import annotations

import csv
import hashlib
import json
import sys
from collections import defaultdict


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    name = name.strip()
    return name.split("(")[0] if "(" in name else name


def stats(csv_path: str, out_path: str, command: str):
    rows = _rows(csv_path)
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))
    total = sum(float(r.get("TotalDurationNs", 0) or 0) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'kernel':70s} {'calls':>7s} {'total ms':>10s} {'avg us':>9s} {'min us':>9s} {'max us':>9s} {'share':>6s}"]
    for r in rows:
        tot = float(r["TotalDurationNs"])
        lines.append(f"{_short(r['Name'])[:70]:70s} {int(r['Calls']):7d} {tot / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {tot / total:6.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def stats_db(db_dir: str, out_path: str, command: str):
    """The same table from the rocpd database rocprofv3 writes (*_results.db): rocprofv3 can end
    with a fault of its own after a cooperative launch, before it writes the statistics CSV, while
    the database of the finished run is complete."""
    import glob
    import sqlite3
    db = sorted(glob.glob(db_dir.rstrip("/") + "/*.db"))[0]
    cur = sqlite3.connect(db).cursor()
    durs = defaultdict(list)
    for name, st, en in cur.execute("select s.display_name, d.start, d.end from rocpd_kernel_dispatch d "
                                    "join rocpd_info_kernel_symbol s on d.kernel_id = s.id"):
        durs[_short(name)].append(en - st)
    total = sum(sum(v) for v in durs.values())
    lines = [f"# rocprofv3 kernel statistics (from the kernel-trace database)", f"# command: {command}", "",
             f"{'kernel':70s} {'calls':>7s} {'total ms':>10s} {'avg us':>9s} {'min us':>9s} {'max us':>9s} {'share':>6s}"]
    for k, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        tot = float(sum(v))
        lines.append(f"{k[:70]:70s} {len(v):7d} {tot / 1e6:10.3f} {tot / len(v) / 1e3:9.2f} {min(v) / 1e3:9.2f} "
                     f"{max(v) / 1e3:9.2f} {tot / total:6.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    acc = defaultdict(list)
    for r in _rows(path):
        if r.get("Counter_Name", counter) != counter:
            continue
        acc[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def _per_kernel_db(db_dir, counter):
    """Mean counter value per dispatch and kernel from a rocpd database (counters_collection view:
    one row per dispatch and counter, the value summed over the counter's instances)."""
    import glob
    import sqlite3
    db = sorted(glob.glob(db_dir.rstrip("/") + "/*.db"))[0]
    cur = sqlite3.connect(db).cursor()
    acc = defaultdict(list)
    for name, value in cur.execute("select kernel_name, value from counters_collection where counter_name = ?",
                                   (counter,)):
        acc[_short(name)].append(float(value))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def traffic(fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, out_json, sources, command, reader=None):
    reader = reader or _per_kernel
    fetch, nf = reader(fetch_csv, "FETCH_SIZE")
    write, nw = reader(write_csv, "WRITE_SIZE")
    cf, _ = reader(cfetch_csv, "FETCH_SIZE")
    cw, _ = reader(cwrite_csv, "WRITE_SIZE")
    # the copy kernel is the one whose mean counter is largest in the copy runs
    ck = max(cf, key=cf.get)
    sf = float(copy_bytes) / (cf[ck] * 1024.0)
    sw = float(copy_bytes) / (cw[max(cw, key=cw.get)] * 1024.0)
    out = {"sources": {src: hashlib.sha256(open(src, "rb").read()).hexdigest() for src in sources.split(",")},
           "command": command, "copy_kernel": ck, "copy_bytes": int(copy_bytes),
           "scale_fetch": sf, "scale_write": sw, "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        fb = fetch.get(k, 0.0) * 1024.0 * sf
        wb = write.get(k, 0.0) * 1024.0 * sw
        out["kernels"][k] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb,
                             "dispatches": max(nf.get(k, 0), nw.get(k, 0))}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "stats-db":
        stats_db(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    elif sys.argv[1] == "traffic-db":
        traffic(*sys.argv[2:10], reader=_per_kernel_db)
    else:
        raise SystemExit(__doc__)
