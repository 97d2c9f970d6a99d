"""Summaries of rocprofv3 result databases (SQLite files written by
`rocprofv3 -d DIR -o NAME ...`).

    python -m paper_2509_12494_amd.profile_summary kernels RESULTS.db [--match mw::] [--top N]
    python -m paper_2509_12494_amd.profile_summary counters FETCH.db WRITE.db --copy-bytes BYTES [--match mw::] [--top N]
    python -m paper_2509_12494_amd.profile_summary valu VALU.db [--match mw::] [--top N]
    python -m paper_2509_12494_amd.profile_summary sq A.db [B.db ...] [--match mw::]

`kernels` lists every kernel (grouped by name and grid size) with its launch
count and average / min / max duration.  `sq` lists every counter of one or more counter runs per kernel (name, grid
size), averaged over dispatches.  `counters` reads FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) from two separate counter runs and converts them
to bytes with the factor that makes the largest single device-to-device copy
dispatch of the run (`__amd_rocclr_copyBuffer`, BYTES long) read and write
exactly BYTES.
"""
import argparse
import sqlite3
import sys


def _short(name):
    n = name.split("(")[0]
    return n.replace("void ", "")


def kernels(db, match=None):
    con = sqlite3.connect(db)
    q = ("select name, grid_x, workgroup_x, count(*), avg(duration), min(duration), max(duration) "
         "from kernels group by name, grid_x order by avg(duration)*count(*) desc")
    rows = []
    for name, grid, wg, n, avg, mn, mx in con.execute(q):
        if match and match not in name:
            continue
        rows.append((_short(name), grid // max(wg, 1), wg, n, avg / 1e3, mn / 1e3, mx / 1e3))
    return rows


def _counter(db, counter):
    con = sqlite3.connect(db)
    q = ("select kernel_name, grid_size, workgroup_size, avg(value), count(*) from counters_collection "
         "where counter_name = ? group by kernel_name, grid_size")
    return [(k, g // max(w, 1), v * 1024.0, n) for k, g, w, v, n in con.execute(q, (counter,))]


def _largest_copy(db, counter):
    """Counter value (bytes) of the single largest device copy dispatch: the
    calibration copy of known size (other copies of the run are smaller)."""
    con = sqlite3.connect(db)
    q = ("select max(value) from counters_collection "
         "where counter_name = ? and kernel_name like '%copyBuffer%'")
    (v,), = con.execute(q, (counter,))
    return v * 1024.0


def counters(fetch_db, write_db, copy_bytes, match=None):
    fetch = _counter(fetch_db, "FETCH_SIZE")
    write = _counter(write_db, "WRITE_SIZE")
    fraw = _largest_copy(fetch_db, "FETCH_SIZE")
    wraw = _largest_copy(write_db, "WRITE_SIZE")
    fs, ws = copy_bytes / fraw, copy_bytes / wraw
    wmap = {(k, g): v for k, g, v, _ in write}
    out = []
    for k, g, v, n in fetch:
        if match and match not in k:
            continue
        w = wmap.get((k, g))
        out.append((_short(k), g, n, v * fs, (w or 0) * ws))
    out.sort(key=lambda r: -(r[3] + r[4]) * r[2])
    return {"fetch_factor": fs, "write_factor": ws, "copy_fetch_raw": fraw, "copy_write_raw": wraw, "rows": out}


def valu(db, match=None):
    """Per kernel (name, grid): VALU wave-instructions, waves and the share
    of cycles the SQ had work (SQ_BUSY_CYCLES / SQ_CYCLES), averaged over
    dispatches."""
    con = sqlite3.connect(db)
    q = ("select kernel_name, grid_size, workgroup_size, counter_name, avg(value), count(*) "
         "from counters_collection group by kernel_name, grid_size, counter_name")
    rows = {}
    for k, g, w, c, v, n in con.execute(q):
        if match and match not in k:
            continue
        rows.setdefault((_short(k), g // max(w, 1)), {})[c] = (v, n)
    out = []
    for (k, g), d in rows.items():
        insts, n = d.get("SQ_INSTS_VALU", (0, 0))
        waves = d.get("SQ_WAVES", (0, 0))[0]
        busy = d.get("SQ_BUSY_CYCLES", (0, 0))[0]
        cyc = d.get("SQ_CYCLES", (1, 0))[0] or 1
        out.append((k, g, n, insts, waves, busy / cyc))
    out.sort(key=lambda r: -r[3] * r[2])
    return out


def sq(dbs, match=None):
    """{(kernel, workgroups): {counter: (average per dispatch, dispatches)}} over several runs."""
    rows = {}
    for db in dbs:
        con = sqlite3.connect(db)
        q = ("select kernel_name, grid_size, workgroup_size, counter_name, avg(value), count(*) "
             "from counters_collection group by kernel_name, grid_size, counter_name")
        for k, g, w, c, v, n in con.execute(q):
            if match and match not in k:
                continue
            rows.setdefault((_short(k), g // max(w, 1)), {})[c] = (v, n)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernels")
    a.add_argument("db")
    a.add_argument("--match", default=None)
    a.add_argument("--top", type=int, default=None)
    b = sub.add_parser("counters")
    b.add_argument("fetch_db")
    b.add_argument("write_db")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--match", default=None)
    b.add_argument("--top", type=int, default=None)
    c = sub.add_parser("valu")
    c.add_argument("db")
    c.add_argument("--match", default=None)
    c.add_argument("--top", type=int, default=None)
    d = sub.add_parser("sq")
    d.add_argument("dbs", nargs="+")
    d.add_argument("--match", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "sq":
        rows = sq(args.dbs, args.match)
        names = sorted({c for r in rows.values() for c in r})
        print("| kernel | workgroups | dispatches | " + " | ".join(names) + " |")
        print("|---|---|---|" + "---|" * len(names))
        for (k, g), r in sorted(rows.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
            n = max(v[1] for v in r.values())
            vals = " | ".join(f"{r[c][0]:.0f}" if c in r else "" for c in names)
            print(f"| `{k}` | {g} | {n} | {vals} |")
        return 0
    if args.cmd == "kernels":
        print("| kernel | workgroups | threads | launches | avg us | min us | max us |")
        print("|---|---|---|---|---|---|---|")
        for r in kernels(args.db, args.match)[:args.top]:
            print(f"| `{r[0]}` | {r[1]} | {r[2]} | {r[3]} | {r[4]:.3f} | {r[5]:.3f} | {r[6]:.3f} |")
    elif args.cmd == "valu":
        print("| kernel | workgroups | dispatches | VALU wave-instructions | waves | SQ busy share |")
        print("|---|---|---|---|---|---|")
        for k, g, n, i, w, b in valu(args.db, args.match)[:args.top]:
            print(f"| `{k}` | {g} | {n} | {i:.0f} | {w:.0f} | {b:.3f} |")
    else:
        c = counters(args.fetch_db, args.write_db, args.copy_bytes, args.match)
        print(f"calibration copy of {args.copy_bytes} B: FETCH_SIZE read {c['copy_fetch_raw']:.0f} B "
              f"(factor {c['fetch_factor']:.3f}), WRITE_SIZE read {c['copy_write_raw']:.0f} B "
              f"(factor {c['write_factor']:.3f})")
        print()
        print("| kernel | workgroups | dispatches | fetch bytes (scaled) | write bytes (scaled) |")
        print("|---|---|---|---|---|")
        for k, g, n, f, w in c["rows"][:args.top]:
            print(f"| `{k}` | {g} | {n} | {f:.0f} | {w:.0f} |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
