"""Summarise rocprofv3 CSV output into small text tables (measurement helper,
not part of the library).

    python3 rocprof_csv_summary.py trace <rocprofv3 -d dir> <out.txt>   # kernel_trace.csv: calls, total/avg/min/max us
    python3 rocprof_csv_summary.py stats <dir> <out.txt>                # the kernel_stats.csv files, concatenated
    python3 rocprof_csv_summary.py pmc   <dir> <out.txt>                # counter_collection.csv: sum per kernel and counter

Rows are keyed by kernel name and grid size (the grid tells pyramid levels
apart).  The raw output of a run can be large; keep it outside the folders
that are copied back and keep only these tables.
"""
import csv, glob, os, sys
from collections import defaultdict

def find(d, pat):
    r = glob.glob(os.path.join(d, "**", pat), recursive=True)
    return r

def kernel_stats(d, out):
    fs = find(d, "*kernel_stats.csv")
    with open(out, "w") as o:
        for f in fs:
            o.write(f"# {os.path.relpath(f, d)}\n")
            with open(f) as fh:
                for row in csv.reader(fh):
                    o.write(",".join(row) + "\n")

def kernel_trace(d, out):
    fs = find(d, "*kernel_trace.csv")
    agg = defaultdict(lambda: [0, 0.0, 1e30, 0.0, None])
    for f in fs:
        with open(f) as fh:
            r = csv.DictReader(fh)
            for row in r:
                name = row.get("Kernel_Name", "?")
                dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
                grid = row.get("Grid_Size", row.get("Grid_Size_X", ""))
                key = (name, grid)
                a = agg[key]
                a[0] += 1; a[1] += dur; a[2] = min(a[2], dur); a[3] = max(a[3], dur)
                a[4] = (row.get("VGPR_Count"), row.get("LDS_Block_Size"), row.get("Workgroup_Size"))
    with open(out, "w") as o:
        o.write("kernel|grid|calls|total_us|avg_us|min_us|max_us|vgpr,lds,wg\n")
        for (name, grid), a in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            o.write(f"{name}|{grid}|{a[0]}|{a[1]:.1f}|{a[1]/a[0]:.2f}|{a[2]:.2f}|{a[3]:.2f}|{a[4]}\n")

def counters(d, out):
    fs = find(d, "*counter_collection.csv")
    agg = defaultdict(lambda: [0, 0.0])
    for f in fs:
        with open(f) as fh:
            r = csv.DictReader(fh)
            for row in r:
                key = (row.get("Kernel_Name", "?"), row.get("Grid_Size", ""), row.get("Counter_Name", "?"))
                agg[key][0] += 1
                agg[key][1] += float(row.get("Counter_Value", 0))
    with open(out, "w") as o:
        o.write("kernel|grid|counter|dispatches|sum|per_dispatch\n")
        for k, a in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            o.write(f"{k[0]}|{k[1]}|{k[2]}|{a[0]}|{a[1]:.1f}|{a[1]/a[0]:.1f}\n")

if __name__ == "__main__":
    mode, d, out = sys.argv[1:4]
    {"stats": kernel_stats, "trace": kernel_trace, "pmc": counters}[mode](d, out)
