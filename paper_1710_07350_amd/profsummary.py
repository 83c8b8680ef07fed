"""Summarise a rocprofv3 kernel-trace database into a short text table.

  python -m paper_1710_07350_amd.profsummary <results.db> [--title T] [--cmd C]

Prints, per kernel: calls, total and average duration (from the dispatch
records), and the last dispatch sequence of the trace.
"""
import argparse
import sqlite3
import sys


def summary(db: str, last: int = 0):
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, grid_x, workgroup_x, lds_size, vgpr_count, "
                       "sgpr_count from kernels order by start").fetchall()
    stats = {}
    for name, s, e, gx, wx, lds, vg, sg in rows:
        short = name.split("(")[0].replace("void ", "")
        st = stats.setdefault(short, [0, 0.0, gx // max(wx, 1), wx, lds])
        st[0] += 1
        st[1] += (e - s) / 1e3
    out = []
    tot = sum(v[1] for v in stats.values())
    out.append("| kernel | calls | total us | avg us | % | grid x block | LDS B |")
    out.append("|---|---|---|---|---|---|---|")
    for k, (c, t, g, w, lds) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {c} | {t:.1f} | {t / c:.2f} | {100 * t / tot:.1f} | {g}x{w} | {lds} |")
    if last:
        trk = [r for r in rows if "trk::" in r[0]][-last:]
        if trk:
            out.append("")
            out.append(f"last {len(trk)} library dispatches (us from the first):")
            t0 = trk[0][1]
            prev = None
            for name, s, e, *_ in trk:
                short = name.split("(")[0].replace("void ", "").replace("trk::", "")
                gap = (s - prev) / 1e3 if prev else 0.0
                out.append(f"  {short:26s} start {(s - t0) / 1e3:9.1f}  dur {(e - s) / 1e3:8.1f}"
                           f"  gap {gap:5.1f}")
                prev = e
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--title", default="")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--last", type=int, default=0)
    a = ap.parse_args()
    if a.title:
        print(f"# {a.title}\n")
    if a.cmd:
        print(f"command: `{a.cmd}`\n")
    print(summary(a.db, a.last))


if __name__ == "__main__":
    sys.exit(main())
