"""Summarise rocprofv3 --pmc databases (FETCH_SIZE / WRITE_SIZE, KiB per dispatch).

usage: python profiles/pmc_summary.py <fetch_db> <write_db> <kernel-substring> [calib-substring]
Prints, per matching kernel, the mean FETCH_SIZE and WRITE_SIZE per dispatch and,
for the calibration kernel (a plain device copy of known size), the figures of its
largest dispatch (the calibration copy; other dispatches of that kernel are small
runtime copies).
"""
import sqlite3
import sys
from collections import defaultdict


def per_kernel(db, counter):
    cur = sqlite3.connect(db).cursor()
    out = defaultdict(list)
    for name, val in cur.execute("select kernel_name, value from counters_collection where counter_name=?",
                                 (counter,)):
        out[name].append(val)
    return out


def main():
    fdb, wdb, pat = sys.argv[1:4]
    calib = sys.argv[4] if len(sys.argv) > 4 else None
    f, w = per_kernel(fdb, "FETCH_SIZE"), per_kernel(wdb, "WRITE_SIZE")
    for label, sub in (("kernel", pat), ("calibration", calib)):
        if sub is None:
            continue
        for name in sorted(set(f) | set(w)):
            if sub in name:
                fv, wv = f.get(name, []), w.get(name, [])
                if label == "calibration":
                    fm = max(fv) if fv else float("nan")
                    wm = max(wv) if wv else float("nan")
                else:
                    fm = sum(fv) / len(fv) if fv else float("nan")
                    wm = sum(wv) / len(wv) if wv else float("nan")
                print(f"{label}\t{name[:90]}\tdispatches={len(fv)}/{len(wv)}\t"
                      f"FETCH_KiB={fm:.1f}\tWRITE_KiB={wm:.1f}\tFETCH_MB={fm * 1024 / 1e6:.2f}\t"
                      f"WRITE_MB={wm * 1024 / 1e6:.2f}")


if __name__ == "__main__":
    main()
