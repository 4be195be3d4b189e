"""Summaries of rocprofv3 output databases (rocpd SQLite) as short text.

    python -m paper_1703_01325_amd.profiling trace <run_results.db> <out.md> <command>
    python -m paper_1703_01325_amd.profiling traffic <fetch.db> <write.db> <copy_fetch.db> \
        <copy_write.db> <kernel substring> <algorithmic bytes per launch> <out.json> <workload> <command>

`trace` tabulates per-kernel launches and durations.  `traffic` scales the
FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of one kernel by what
the same counters read for a plain device copy of known size, and reports
HBM bytes per launch beside the algorithmic bytes.
"""
from __future__ import annotations

import hashlib
import json
import os
import sqlite3
import sys

COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 8 * 64 * 1024 * 1024     # bench.py --copy-calibration moves 512 MiB each way


def kernel_table(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    con.close()
    return rows


def counter_avg(db, counter, selector):
    """Average of `counter` over the dispatches whose kernel name contains
    the selector; "name@even" / "name@odd" keep every other such dispatch
    (two sweeps that share one kernel and strictly alternate); "name@run"
    keeps the dispatches that did work (a value of at least a tenth of the
    largest), leaving out launches that a solver's device flag turned into
    no-ops (the gated true-residual SpMV, the step queued after the exit);
    "name@even+run" / "name@odd+run" apply both, in that order."""
    substring, _, flags = selector.partition("@")
    parts = set(flags.split("+")) if flags else set()
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value from counters_collection where counter_name = ? "
                       "order by dispatch_id", (counter,)).fetchall()
    con.close()
    vals = [v for name, v in rows if substring in name]
    if "even" in parts:
        vals = vals[0::2]
    elif "odd" in parts:
        vals = vals[1::2]
    if "run" in parts and vals:
        top = max(vals)
        vals = [v for v in vals if v >= 0.1 * top]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def short(name, width=70):
    name = name.replace("bilu::dev::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def write_trace(db, out, command):
    rows = kernel_table(db)
    total = sum(r[2] for r in rows)
    lines = [f"# rocprofv3 kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | launches | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, n, tot, avg in rows[:20]:
        lines.append(f"| `{short(name)}` | {n} | {tot / 1e6:.2f} | {avg / 1e3:.1f} | {100 * tot / total:.1f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_traffic(fetch_db, write_db, cfetch_db, cwrite_db, substring, alg_bytes, out, workload, command):
    f_kib, nf = counter_avg(fetch_db, "FETCH_SIZE", substring)
    w_kib, nw = counter_avg(write_db, "WRITE_SIZE", substring)
    cf_kib, _ = counter_avg(cfetch_db, "FETCH_SIZE", COPY_KERNEL)
    cw_kib, _ = counter_avg(cwrite_db, "WRITE_SIZE", COPY_KERNEL)
    sf = COPY_BYTES / (cf_kib * 1024.0)
    sw = COPY_BYTES / (cw_kib * 1024.0)
    fetch = f_kib * 1024.0 * sf
    write = w_kib * 1024.0 * sw
    here = os.path.dirname(os.path.abspath(__file__))
    hsh = hashlib.sha256()
    for name in ("kernels.h", "sweep_kernels.h", "kernels_batch.h"):     # as bench.kernels_hash
        with open(os.path.join(here, "csrc", name), "rb") as fh:
            hsh.update(fh.read())
    sha = hsh.hexdigest()[:16]
    rec = {"kernel": substring, "workload": workload, "dispatches": [nf, nw],
           "fetch_kib_raw": f_kib, "write_kib_raw": w_kib,
           "copy_scale_fetch": sf, "copy_scale_write": sw,
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write, "algorithmic_bytes_per_launch": alg_bytes,
           "traffic_over_algorithmic": (fetch + write) / alg_bytes if alg_bytes else None,
           "kernels_sha": sha, "command": command}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        write_trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == "traffic":
        write_traffic(*sys.argv[2:7], float(sys.argv[7]), sys.argv[8], sys.argv[9], sys.argv[10])
    else:
        raise SystemExit(__doc__)
