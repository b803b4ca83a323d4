"""Summaries of rocprofv3 output databases (SQLite, the default rocpd format).

  python -m paper_2605_31419_amd.profsum kernels  <db>      per-kernel dispatch durations
  python -m paper_2605_31419_amd.profsum counters <db>      per-kernel average counter values
  python -m paper_2605_31419_amd.profsum traffic --fetch <db> --write <db> --kernel <name>

`traffic` scales the kernel's per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) by what the same
counters read for the 256 MiB device-to-device copy that `bench.py --copy-calibration` runs
(the copy dispatch with the largest WRITE_SIZE), and prints one `traffic:` line (bytes per
launch, plus the source fingerprint of the current build) that bench.py reads back.
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3

COPY_BYTES = 256 << 20


def _short(name: str) -> str:
    m = re.search(r"(k_[a-z_0-9]+)(<\d+>)?", name or "")
    if m:
        return m.group(1) + (m.group(2) or "")
    return (name or "")[:40]


def _rows(db, table):
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [r[1] for r in cur.execute(f"pragma table_info({table})")]
    rows = [dict(zip(cols, r)) for r in cur.execute(f"select * from {table}").fetchall()]
    con.close()
    return rows


def kernel_durations(db):
    out = collections.defaultdict(list)
    for d in _rows(db, "kernels"):
        out[_short(d.get("kernel_name") or d.get("name"))].append((d["end"] - d["start"]) / 1e3)
    return out


def counter_values(db):
    out = collections.defaultdict(list)
    for d in _rows(db, "counters_collection"):
        out[(_short(d.get("kernel_name")), d.get("counter_name"))].append(float(d.get("value")))
    return out


def print_kernels(db):
    out = kernel_durations(db)
    print(f"{'kernel':<28} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_us':>11}")
    for k, v in sorted(out.items(), key=lambda kv: -sum(kv[1])):
        print(f"{k:<28} {len(v):>6} {sum(v) / len(v):>10.2f} {min(v):>10.2f} {max(v):>10.2f} {sum(v):>11.1f}")


def print_counters(db):
    out = counter_values(db)
    print(f"{'kernel':<28} {'counter':<12} {'calls':>6} {'avg':>14}")
    for (k, c), v in sorted(out.items()):
        print(f"{k:<28} {c:<12} {len(v):>6} {sum(v) / len(v):>14.1f}")


def traffic(fetch_db, write_db, kernel):
    f = counter_values(fetch_db)
    w = counter_values(write_db)
    copy_w = max(w[("__amd_rocclr_copyBuffer", "WRITE_SIZE")])
    copies_f = f[("__amd_rocclr_copyBuffer", "FETCH_SIZE")]
    # the calibration copy is the largest dispatch of the copy kernel in each pass
    copy_f = max(copies_f)
    ff = COPY_BYTES / (copy_f * 1024.0)
    fw = COPY_BYTES / (copy_w * 1024.0)
    kf = f[(kernel, "FETCH_SIZE")]
    kw = w[(kernel, "WRITE_SIZE")]
    fb = sum(kf) / len(kf) * 1024.0 * ff
    wb = sum(kw) / len(kw) * 1024.0 * fw
    return {"fetch_factor": ff, "write_factor": fw, "fetch_bytes": fb, "write_bytes": wb,
            "dispatches": (len(kf), len(kw))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["kernels", "counters", "traffic"])
    ap.add_argument("db", nargs="?")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", action="append", help="kernel name (repeatable); default k_train_fused<1>")
    a = ap.parse_args()
    if a.mode == "kernels":
        print_kernels(a.db)
    elif a.mode == "counters":
        print_counters(a.db)
    else:
        from .build import source_fingerprint

        fp = source_fingerprint()
        for i, k in enumerate(a.kernel or ["k_train_fused<1>"]):
            t = traffic(a.fetch, a.write, k)
            if i == 0:
                print(f"calibration: fetched bytes = {t['fetch_factor']:.3f} x FETCH_SIZE, "
                      f"written bytes = {t['write_factor']:.3f} x WRITE_SIZE")
            print(f"traffic: kernel={k} fetch_bytes={t['fetch_bytes']:.0f} write_bytes={t['write_bytes']:.0f} "
                  f"sources={fp}")


if __name__ == "__main__":
    main()
