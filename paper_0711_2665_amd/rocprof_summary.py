"""Text summaries of rocprofv3 results (the SQLite databases rocprofv3 writes)
for the profiles folder.

    # kernel table of a --kernel-trace --stats run (with --json, the mean of
    # the selected dispatches and the kernel source hash for bench.py)
    python -m paper_0711_2665_amd.rocprof_summary trace --db DB --out profiles/X.md \
        --command "the rocprofv3 command" [--kernel k_lb --last 200 --json profiles/X.json --layout '{...}']

    # one coupled step as a timeline (kernel starts relative to the end of the
    # previous step, sub-step durations summarised)
    python -m paper_0711_2665_amd.rocprof_summary timeline --db DB --out profiles/X.md \
        --command "the rocprofv3 command" --step -5

    # HBM bytes of the sweep from one FETCH_SIZE run and one WRITE_SIZE run
    python -m paper_0711_2665_amd.rocprof_summary counters --fetch-db DB1 --write-db DB2 \
        --meta META.json --kernel k_lb --out profiles/lb_sweep_fp32dev_c3 --command "..."

The counters are calibrated against a plain device-to-device copy of known
size run in the same process after the sweeps: factor = copied bytes /
counter bytes, for reads and writes separately.
"""
import argparse
import json
import re
import sqlite3


def short(name):
    """Kernel name without argument list and return type."""
    n = re.sub(r"\(.*$", "", name)
    n = re.sub(r"^void ", "", n)
    return n


def kernel_rows(db):
    c = sqlite3.connect(db)
    return c.execute("select name, start, end, duration, grid_x, workgroup_x from kernels order by start").fetchall()


def trace(a):
    rows = kernel_rows(a.db)
    agg = {}
    for name, st, en, dur, gx, wx in rows:
        k = short(name)
        e = agg.setdefault(k, [0, 0.0, float("inf"), 0.0])
        e[0] += 1
        e[1] += dur
        e[2] = min(e[2], dur)
        e[3] = max(e[3], dur)
    total = sum(e[1] for e in agg.values())
    lines = [f"# rocprofv3 kernel trace: {a.title}", "", "Command (from the repository root):", "",
             "```", a.command, "```", "",
             f"Summary: `python -m paper_0711_2665_amd.rocprof_summary trace --db <results.db> ...`", "",
             "| kernel | calls | avg us | min us | max us | total ms | % of GPU time |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k, e in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{k}` | {e[0]} | {e[1] / e[0] / 1e3:.2f} | {e[2] / 1e3:.2f} | {e[3] / 1e3:.2f} | "
                     f"{e[1] / 1e6:.3f} | {100 * e[1] / total:.2f} |")
    if a.kernel:
        sel = [r for r in rows if a.kernel in short(r[0])]
        if a.skip_last:
            sel = sel[:-a.skip_last]
        if a.last:
            sel = sel[-a.last:]
        d = [r[3] for r in sel]
        if d and a.json:
            from .build import kernel_source_hash
            rec = dict(kernel=a.kernel, dispatches=len(d), mean_launch_ms=sum(d) / len(d) / 1e6,
                       min_launch_ms=min(d) / 1e6, max_launch_ms=max(d) / 1e6, grid=sel[-1][4],
                       workgroup=sel[-1][5], command=a.command, kernel_source_hash=kernel_source_hash(),
                       layout=json.loads(a.layout) if a.layout else None)
            with open(a.json, "w") as fh:
                json.dump(rec, fh, indent=1)
        if d:
            lines += ["", f"{len(d)} dispatches of `{a.kernel}` in the timed region"
                      f"{f' (the last {a.skip_last} dispatches, later in the run, excluded)' if a.skip_last else ''}: "
                      f"mean {sum(d) / len(d) / 1e3:.2f} us, min {min(d) / 1e3:.2f} us, max {max(d) / 1e3:.2f} us, "
                      f"grid {sel[-1][4]} x workgroup {sel[-1][5]}."]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def timeline(a):
    """Kernels of one coupled step (between two k_step_end dispatches), in
    start order, with start and end relative to the end of the previous step;
    the MD sub-step launches are summarised (count, median, while the sweep
    runs and after it)."""
    rows = kernel_rows(a.db)
    ends = [i for i, r in enumerate(rows) if short(r[0]).endswith("k_step_end")]
    i0, i1 = ends[a.step - 1], ends[a.step]
    t0 = rows[i0][2]
    lines = [f"# rocprofv3 timeline of one coupled step: {a.title}", "", "Command (from the repository root):", "",
             "```", a.command, "```", "",
             f"Summary: `python -m paper_0711_2665_amd.rocprof_summary timeline --db <results.db> --step {a.step}`", "",
             "| kernel | start us | end us | duration us |", "|---|---:|---:|---:|"]
    md, sweep_end = [], None
    for name, st, en, dur, gx, wx in rows[i0 + 1:i1 + 1]:
        k = short(name)
        if k.endswith("k_md_substep") or k.endswith("k_md_substep<false>"):   # uniform sub-steps
            md.append((st - t0, en - t0, dur))
            continue
        if "k_lb<" in k:
            sweep_end = en - t0
        lines.append(f"| `{k}` | {(st - t0) / 1e3:.1f} | {(en - t0) / 1e3:.1f} | {dur / 1e3:.1f} |")
    if md:
        d = sorted(x[2] for x in md)
        during = [x[2] for x in md if sweep_end is not None and x[1] <= sweep_end]
        after = [x[2] for x in md if sweep_end is not None and x[0] >= sweep_end]
        med = lambda v: sorted(v)[len(v) // 2] / 1e3 if v else float("nan")
        lines += ["", f"{len(md)} MD sub-step launches from {md[0][0] / 1e3:.1f} us to {md[-1][1] / 1e3:.1f} us: "
                  f"median {med(d):.2f} us, max {d[-1] / 1e3:.1f} us; median {med(during):.2f} us over the "
                  f"{len(during)} that ran beside the sweep, {med(after):.2f} us over the {len(after)} after it."]
    lines += ["", f"Step span: {(rows[i1][2] - t0) / 1e3:.1f} us."]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counter_rows(db, counter):
    c = sqlite3.connect(db)
    return c.execute("select name, start, counter_value from pmc_events where counter_name=? order by start",
                     (counter,)).fetchall()


def counters(a):
    meta = json.load(open(a.meta))
    layouts, n = meta["layouts"], meta["sweeps"]
    per = [dict(layout=l) for l in layouts]
    res = {}
    for counter, db in (("FETCH_SIZE", a.fetch_db), ("WRITE_SIZE", a.write_db)):
        rows = counter_rows(db, counter)
        sweep = [(st, v) for nm, st, v in rows if a.kernel in short(nm)]
        last = sweep[-1][0]
        copy = [v for nm, st, v in rows if "copyBuffer" in nm and st > last]
        sweep = sweep[-len(layouts) * n:]
        copy_kib = sum(copy)
        factor = meta["copy_bytes"] / (copy_kib * 1024.0)
        res[counter] = dict(copy_kib=copy_kib, copy_dispatches=len(copy), factor=factor)
        for k, e in enumerate(per):
            kib = sum(v for _, v in sweep[k * n:(k + 1) * n]) / n
            e[counter] = dict(kib_per_launch=kib, bytes_per_launch=kib * 1024.0 * factor)
    alg = meta["algorithmic_bytes_per_launch"]
    for e in per:
        e["bytes_per_launch"] = e["FETCH_SIZE"]["bytes_per_launch"] + e["WRITE_SIZE"]["bytes_per_launch"]
        e["traffic_over_algorithmic"] = e["bytes_per_launch"] / alg
    out = dict(meta, counters=res, per_layout=per, command=a.command)
    with open(a.out + "_counters.json", "w") as fh:
        json.dump(out, fh, indent=1)
    f, w = res["FETCH_SIZE"], res["WRITE_SIZE"]
    variant = f", fluctuating fluid (kT = {meta['fluid_kT']:g})" if meta.get("fluid_kT", 0.0) > 0 else ""
    lines = [f"# HBM traffic of the LB sweep: {meta['workload']} {meta['precision']}{variant}", "",
             "Commands (from the repository root):", "", "```", a.command, "```", "",
             f"Lattice {meta['shape']} ({meta['nodes']} nodes, {meta['nfluid']} fluid), kernel source hash "
             f"`{meta['kernel_source_hash']}`, {n} sweeps per layout.  Counters are calibrated against a "
             f"device-to-device copy of {meta['copy_bytes']} B: factor (bytes / counter bytes) "
             f"{f['factor']:.4f} for FETCH_SIZE ({f['copy_dispatches']} copy dispatches), {w['factor']:.4f} "
             f"for WRITE_SIZE.", "",
             f"Algorithmic bytes per launch: {alg:.4e}.", "",
             "| tile nodes | order | grid | cap | FETCH_SIZE KiB/launch (raw) | WRITE_SIZE KiB/launch (raw) | "
             "HBM bytes per launch | / algorithmic |",
             "|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for e in per:
        l = e["layout"]
        lines.append(f"| {l['tile_nodes']} | {l['order']} | {l['grid']} | {l['cap']} | "
                     f"{e['FETCH_SIZE']['kib_per_launch']:.1f} | "
                     f"{e['WRITE_SIZE']['kib_per_launch']:.1f} | {e['bytes_per_launch']:.4e} | "
                     f"{e['traffic_over_algorithmic']:.4f} |")
    with open(a.out + "_counters.md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--db", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--kernel", default="")
    t.add_argument("--last", type=int, default=0)
    t.add_argument("--skip-last", type=int, default=0)
    t.add_argument("--json", default="", help="also write the selected dispatches' mean here")
    t.add_argument("--layout", default="", help="the sweep layout of the run, as JSON (recorded in --json)")
    tl = sub.add_parser("timeline")
    tl.add_argument("--db", required=True)
    tl.add_argument("--out", required=True)
    tl.add_argument("--command", required=True)
    tl.add_argument("--title", default="")
    tl.add_argument("--step", type=int, default=-5)
    c = sub.add_parser("counters")
    c.add_argument("--fetch-db", required=True)
    c.add_argument("--write-db", required=True)
    c.add_argument("--meta", required=True)
    c.add_argument("--kernel", default="k_lb<")
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    a = ap.parse_args()
    {"trace": trace, "timeline": timeline, "counters": counters}[a.mode](a)


if __name__ == "__main__":
    main()
