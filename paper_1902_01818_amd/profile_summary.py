"""Summarize rocprofv3 output of a benchmark run into a short markdown table.

    python -m paper_1902_01818_amd.profile_summary stats <kernel_trace.csv> [--title T] [--cmd C]
    python -m paper_1902_01818_amd.profile_summary traffic <fetch.csv> <write.csv>
        --kernel NAME [--grid G | --sweep-total G] --copy-bytes B [--copy-kernel NAME]
        [--copy-last]

`stats` groups the kernel trace by kernel name and grid size (a grid size
identifies the level) and prints calls, total and average durations.
`traffic` takes two --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch), averages them over the dispatches of one kernel at one grid size,
and scales by what the same counters read for a plain device copy of
copy-bytes bytes (first dispatch of the copy kernel whose grid is the largest).
"""
import argparse
import collections
import csv
import json
import re
import sys


def short_name(name):
    m = re.search(r"::(\w+?)(<[^(]*>)?\(", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0][-60:]


def grid_of(r):
    g = 1
    for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Grid_Size"):
        if k in r and r[k]:
            g *= int(r[k])
    return g


def stats(path, title, cmd, top=16):
    rows = list(csv.DictReader(open(path)))
    tot = collections.defaultdict(float)
    calls = collections.Counter()
    per = collections.defaultdict(list)
    for r in rows:
        n = short_name(r["Kernel_Name"])
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        tot[n] += dt
        calls[n] += 1
        per[(n, grid_of(r))].append(dt)
    T = sum(tot.values())
    out = ["# %s" % title, "", "Command: `%s`" % cmd, "",
           "| kernel | calls | total us | avg us | share |", "|---|---|---|---|---|"]
    for n in sorted(tot, key=lambda k: -tot[k])[:top]:
        out.append("| %s | %d | %.1f | %.2f | %.1f%% |" % (n, calls[n], tot[n], tot[n] / calls[n],
                                                         100 * tot[n] / T))
    out += ["", "Per grid size (grid = work-items; one grid size per level):", "",
            "| kernel | grid | calls | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for (n, g) in sorted(per, key=lambda k: (k[0], k[1])):
        if tot[n] < 0.02 * T:
            continue
        v = per[(n, g)]
        out.append("| %s | %d | %d | %.2f | %.2f | %.2f |" % (n, g, len(v), sum(v) / len(v), min(v),
                                                           max(v)))
    return "\n".join(out)


def pmc_rows(path):
    rows = list(csv.DictReader(open(path)))
    return rows


def counter_per_dispatch(rows, kernel, grid, counter, sweep_total=None):
    """Counter value per dispatch of `kernel`; with sweep_total, only dispatches in
    runs of consecutive `kernel` dispatches whose grid sizes sum to sweep_total
    (this identifies the launches of one grid level)."""
    per = collections.OrderedDict()
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        if r.get("Counter_Name") != counter:
            continue
        d = r["Dispatch_Id"]
        if d not in per:
            per[d] = [r["Kernel_Name"], grid_of(r), 0.0]
        per[d][2] += float(r["Counter_Value"])
    seq = list(per.values())
    vals = []
    if sweep_total is None:
        grids = None if grid is None else {int(x) for x in str(grid).split(",")}
        for name, g, v in seq:
            if kernel in name and (grids is None or g in grids):
                vals.append(v)
        return vals
    run = []
    for name, g, v in seq + [["", 0, 0.0]]:
        if kernel in name:
            run.append((g, v))
            continue
        if run and sum(x[0] for x in run) == sweep_total:
            vals.extend(x[1] for x in run)
        run = []
    return vals


def traffic(fetch, write, kernel, grid, copy_bytes, copy_kernel, sweep_total=None, copy_last=False,
            per_launch=1):
    fr, wr = pmc_rows(fetch), pmc_rows(write)
    f = counter_per_dispatch(fr, kernel, grid, "FETCH_SIZE", sweep_total)
    w = counter_per_dispatch(wr, kernel, grid, "WRITE_SIZE", sweep_total)
    # calibration: the copy dispatch with the largest grid (copy_last: the
    # last dispatch of the copy kernel, the run's final calibration copy)
    def biggest(rows, counter):
        best = None
        for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
            if r.get("Counter_Name") != counter or copy_kernel not in r["Kernel_Name"]:
                continue
            g = grid_of(r)
            if best is None or g > best[0] or copy_last:
                best = (g, r["Dispatch_Id"])
        if best is None:
            return None
        return sum(float(r["Counter_Value"]) for r in rows
                   if r.get("Counter_Name") == counter and r["Dispatch_Id"] == best[1])
    cf, cw = biggest(fr, "FETCH_SIZE"), biggest(wr, "WRITE_SIZE")
    sf = copy_bytes / (cf * 1024.0) if cf else None
    sw = copy_bytes / (cw * 1024.0) if cw else None
    res = dict(kernel=kernel, grid=grid, dispatches=[len(f), len(w)],
               fetch_kib=sum(f) / max(len(f), 1), write_kib=sum(w) / max(len(w), 1),
               copy_fetch_kib=cf, copy_write_kib=cw, scale_fetch=sf, scale_write=sw)
    if sf and sw:
        # per launch of the timed unit: per_launch dispatches of the kernel
        res["dispatches_per_launch"] = per_launch
        res["traffic_bytes"] = per_launch * (res["fetch_kib"] * 1024 * sf
                                             + res["write_kib"] * 1024 * sw)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode")
    ap.add_argument("files", nargs="+")
    ap.add_argument("--title", default="rocprofv3 kernel trace")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--grid", default=None, help="grid size, or a comma-separated list of them")
    ap.add_argument("--copy-bytes", type=float, default=0)
    ap.add_argument("--copy-kernel", default="copy")
    ap.add_argument("--sweep-total", type=int, default=None)
    ap.add_argument("--source-hash", default="")
    ap.add_argument("--per-launch", type=int, default=1,
                    help="dispatches of the kernel per launch of the timed unit")
    ap.add_argument("--copy-last", action="store_true",
                    help="calibrate on the last dispatch of the copy kernel")
    a = ap.parse_args()
    if a.mode == "stats":
        print(stats(a.files[0], a.title, a.cmd))
    else:
        res = traffic(a.files[0], a.files[1], a.kernel, a.grid, a.copy_bytes, a.copy_kernel,
                      a.sweep_total, a.copy_last, a.per_launch)
        res["source_hash"] = a.source_hash
        print(json.dumps(res, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
