"""Text summaries of rocprofv3 output for the library's kernels.

Reads the SQLite database that rocprofv3 writes (``-d DIR -o run`` gives
``DIR/run_results.db``) and prints:

* ``trace``: per-kernel dispatch count and duration statistics of a
  ``--kernel-trace --stats`` run;
* ``traffic``: HBM bytes per dispatch of the sweep kernels from one ``--pmc FETCH_SIZE``
  run and one ``--pmc WRITE_SIZE`` run of ``bench.py --calibration-copy-mib M``. Both
  counters are scaled by what they read for the calibration copy, whose true traffic is
  M MiB read and M MiB written. The result ends with a ``traffic_json:`` line that
  bench.py reads back, tagged with a hash of the sweep kernel sources;
* ``kernels``: the same scaled HBM bytes per dispatch for every kernel whose name starts
  with one of the given prefixes, also per cell of the grid;
* ``counters``: the mean per dispatch of every counter of one or more ``--pmc`` runs, for
  the kernels whose names start with the given prefixes.

Usage::

    python -m paper_2001_03477_amd.profsum trace DB --command CMD > summary.txt
    python -m paper_2001_03477_amd.profsum traffic --fetch DB1 --write DB2 --calib-mib M \\
        --workload leveque3d_128 --command-fetch CMD1 --command-write CMD2 > traffic.txt
"""
import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_SOURCES = ("sweep.hip", "common.h", "geom.h", "geom32.h", "kernels.h")
SWEEP_KERNELS = ("k_sweep_x", "k_sweep_t<1>", "k_sweep_t<2>")  # axis order
SWEEP_KERNELS_MIXED = ("k_sweep_x_mixed", "k_sweep_t_mixed<1>", "k_sweep_t_mixed<2>")


def sweep_source_hash():
    """Hash of the sources the sweep kernels are built from."""
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    n = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("pcv::", "")
    return n.split("(")[0]


def sweep_axis(name, kernels=SWEEP_KERNELS):
    n = short_name(name)
    for a, k in enumerate(kernels):
        if n == k:
            return a
    return None


def kernel_rows(db):
    con = sqlite3.connect(db)
    return con.execute("select name, duration from kernels order by start").fetchall()


def counter_rows(db):
    """Per dispatch: kernel name and the sum of each counter over its instances."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value "
                       "from counters_collection").fetchall()
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for did, kn, cn, v in rows:
        per[did][cn] += v
        names[did] = kn
    return [(names[d], dict(per[d])) for d in sorted(per)]


def trace_summary(db, command):
    stats = collections.OrderedDict()
    for name, dur in kernel_rows(db):
        stats.setdefault(short_name(name), []).append(dur / 1e3)
    total = sum(sum(v) for v in stats.values())
    lines = [f"command: {command}", "",
             f"{'kernel':44s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'total_%':>8s}"]
    for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k[:44]:44s} {len(v):6d} {sum(v) / len(v):9.2f} {min(v):9.2f} {max(v):9.2f} "
                     f"{100 * sum(v) / total:8.2f}")
    return "\n".join(lines)


def calib_value(rows, counter):
    """The counter of the calibration copy: the first copy kernel of the run (bench.py
    copies the calibration buffer before anything else is copied)."""
    for n, c in rows:
        if "copy" in n.lower() and counter in c:
            return c[counter]
    raise SystemExit(f"no copy kernel with {counter} in the run")


def _sweep_traffic(frows, wrows, kernels, f_fetch, f_write):
    """Per axis: (launches, mean FETCH KiB, mean WRITE KiB, read bytes, write bytes) of
    the sweep kernels named in kernels, or None for an axis without dispatches."""
    per = {a: {"fetch": [], "write": []} for a in range(3)}
    for n, c in frows:
        a = sweep_axis(n, kernels)
        if a is not None and "FETCH_SIZE" in c:
            per[a]["fetch"].append(c["FETCH_SIZE"])
    for n, c in wrows:
        a = sweep_axis(n, kernels)
        if a is not None and "WRITE_SIZE" in c:
            per[a]["write"].append(c["WRITE_SIZE"])
    out = []
    for a in range(3):
        fe, wr = per[a]["fetch"], per[a]["write"]
        if not fe or not wr:
            out.append(None)
            continue
        fk, wk = sum(fe) / len(fe), sum(wr) / len(wr)
        out.append((len(fe), fk, wk, fk * 1024 * f_fetch, wk * 1024 * f_write))
    return out


def traffic_summary(fetch_db, write_db, calib_mib, workload, cmd_fetch, cmd_write):
    frows, wrows = counter_rows(fetch_db), counter_rows(write_db)
    true_bytes = calib_mib * (1 << 20)
    f_fetch = true_bytes / (calib_value(frows, "FETCH_SIZE") * 1024.0)
    f_write = true_bytes / (calib_value(wrows, "WRITE_SIZE") * 1024.0)
    lines = [f"fetch run: {cmd_fetch}", f"write run: {cmd_write}", "",
             f"calibration copy: {calib_mib} MiB read + {calib_mib} MiB written",
             f"scale factors (true bytes / counter bytes): FETCH_SIZE {f_fetch:.4f}, "
             f"WRITE_SIZE {f_write:.4f}", "",
             f"{'kernel':20s} {'n':>3s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'read_MB':>10s} "
             f"{'write_MB':>10s} {'total_MB':>10s}"]
    rec = {"workload": workload}
    for key, kernels in (("bytes_per_launch", SWEEP_KERNELS), ("bytes_per_launch_mixed", SWEEP_KERNELS_MIXED)):
        rows = _sweep_traffic(frows, wrows, kernels, f_fetch, f_write)
        if all(r is None for r in rows):
            continue
        bpl = []
        for a, r in enumerate(rows):
            if r is None:
                bpl.append(None)
                continue
            n, fk, wk, rb, wb = r
            bpl.append(rb + wb)
            lines.append(f"{kernels[a]:20s} {n:3d} {fk:12.0f} {wk:12.0f} {rb / 1e6:10.2f} "
                         f"{wb / 1e6:10.2f} {(rb + wb) / 1e6:10.2f}")
        rec[key] = bpl
    rec.update({"fetch_scale": f_fetch, "write_scale": f_write, "source_hash": sweep_source_hash()})
    lines += ["", "traffic_json: " + json.dumps(rec)]
    return "\n".join(lines)


def kernels_summary(fetch_db, write_db, calib_mib, cells, prefixes, cmd_fetch, cmd_write):
    """HBM bytes per dispatch of every kernel whose short name starts with one of the
    prefixes, scaled like the sweep summary, with bytes per cell for a grid of cells."""
    frows, wrows = counter_rows(fetch_db), counter_rows(write_db)
    true_bytes = calib_mib * (1 << 20)
    f_fetch = true_bytes / (calib_value(frows, "FETCH_SIZE") * 1024.0)
    f_write = true_bytes / (calib_value(wrows, "WRITE_SIZE") * 1024.0)
    per = collections.OrderedDict()
    for rows, cn in ((frows, "FETCH_SIZE"), (wrows, "WRITE_SIZE")):
        for n, c in rows:
            k = short_name(n)
            if cn in c and any(k.startswith(p) for p in prefixes):
                per.setdefault(k, {"FETCH_SIZE": [], "WRITE_SIZE": []})[cn].append(c[cn])
    lines = [f"fetch run: {cmd_fetch}", f"write run: {cmd_write}", "",
             f"calibration copy: {calib_mib} MiB read + {calib_mib} MiB written",
             f"scale factors (true bytes / counter bytes): FETCH_SIZE {f_fetch:.4f}, "
             f"WRITE_SIZE {f_write:.4f}; bytes per cell over {cells} cells", "",
             f"{'kernel':24s} {'n':>5s} {'read_MB':>10s} {'write_MB':>10s} {'read_B/cell':>12s} "
             f"{'write_B/cell':>13s}"]
    for k, v in per.items():
        fe, wr = v["FETCH_SIZE"], v["WRITE_SIZE"]
        if not fe or not wr:
            continue
        rb = sum(fe) / len(fe) * 1024 * f_fetch
        wb = sum(wr) / len(wr) * 1024 * f_write
        lines.append(f"{k[:24]:24s} {len(fe):5d} {rb / 1e6:10.2f} {wb / 1e6:10.2f} {rb / cells:12.2f} "
                     f"{wb / cells:13.2f}")
    return "\n".join(lines)


def counters_summary(dbs, prefixes, command):
    """Mean of every collected counter per dispatch, for the kernels whose short name
    starts with one of the prefixes (several --pmc runs may be given; their counters are
    merged by kernel name)."""
    per = collections.OrderedDict()
    for db in dbs:
        for n, c in counter_rows(db):
            k = short_name(n)
            if not any(k.startswith(p) for p in prefixes):
                continue
            slot = per.setdefault(k, collections.OrderedDict())
            for cn, v in c.items():
                slot.setdefault(cn, []).append(v)
    names = []
    for slot in per.values():
        for cn in slot:
            if cn not in names:
                names.append(cn)
    lines = [f"command: {command}", "", "mean per dispatch", ""]
    lines.append(f"{'counter':28s} " + " ".join(f"{k[:18]:>18s}" for k in per))
    for cn in names:
        vals = []
        for slot in per.values():
            v = slot.get(cn)
            vals.append(f"{sum(v) / len(v):18.4g}" if v else f"{'-':>18s}")
        lines.append(f"{cn[:28]:28s} " + " ".join(vals))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", required=True)
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--calib-mib", type=int, required=True)
    f.add_argument("--workload", required=True)
    f.add_argument("--command-fetch", required=True)
    f.add_argument("--command-write", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("--fetch", required=True)
    k.add_argument("--write", required=True)
    k.add_argument("--calib-mib", type=int, required=True)
    k.add_argument("--cells", type=int, required=True)
    k.add_argument("--prefixes", required=True, help="comma-separated kernel name prefixes")
    k.add_argument("--command-fetch", required=True)
    k.add_argument("--command-write", required=True)
    cn = sub.add_parser("counters")
    cn.add_argument("dbs", nargs="+")
    cn.add_argument("--prefixes", required=True, help="comma-separated kernel name prefixes")
    cn.add_argument("--command", required=True)
    args = ap.parse_args(argv)
    if args.what == "counters":
        print(counters_summary(args.dbs, args.prefixes.split(","), args.command))
    elif args.what == "kernels":
        print(kernels_summary(args.fetch, args.write, args.calib_mib, args.cells, args.prefixes.split(","),
                              args.command_fetch, args.command_write))
    elif args.what == "trace":
        print(trace_summary(args.db, args.command))
    else:
        print(traffic_summary(args.fetch, args.write, args.calib_mib, args.workload,
                              args.command_fetch, args.command_write))


if __name__ == "__main__":
    sys.exit(main())
