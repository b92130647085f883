"""Summary of rocprofv3 CSV output for a bench.py run.

usage: python -m paper_1210_2536_amd.prof_summary TRACE_CSV BENCH_LOG [FETCH_CSV [WRITE_CSV]]

TRACE_CSV is the kernel trace (--kernel-trace -f csv) of the bench command,
BENCH_LOG that run's output (its last JSON line names the dominant kernel;
"a<..> + b<..>" means one launch of each per SpMV).  The timed region is the
dispatches between the two 16-byte marker copies the bench issues around its
timed steps.  FETCH_CSV / WRITE_CSV are --pmc FETCH_SIZE and --pmc WRITE_SIZE
runs of the same launches (bench.py --replay); both counters are scaled by
what they read for the bench's 1 GiB copy probe, which moves exactly 1 GiB
each way.
"""
import collections
import csv
import json
import re
import sys


def short(n):
    n = n.replace('smat::(anonymous namespace)::', '').replace('void ', '')
    return n.split('(')[0]


def matches(name, pat):
    """A kernel name against one kernel of a plan's symbol ("false|true"
    stands for either value of that template argument)."""
    return re.fullmatch(re.escape(pat).replace(r'false\|true', '(?:false|true)'), name) is not None


def dominant_runs(reg, dom):
    """The dominant plan's runs: a dispatch of its first kernel followed, in
    dispatch order, by its other kernels in order (kernels that other plans
    also launch are counted only inside these runs)."""
    names = [short(r['Kernel_Name']) for r in reg]
    out, i = [], 0
    while i < len(reg):
        if i + len(dom) <= len(reg) and all(matches(names[i + j], d) for j, d in enumerate(dom)):
            out.append(reg[i:i + len(dom)])
            i += len(dom)
        else:
            i += 1
    return out


def region(rows, grid_key):
    """Dispatches between the two 16-byte marker copies, and all rows."""
    rows.sort(key=lambda r: int(r['Start_Timestamp']))
    marks = [i for i, r in enumerate(rows)
             if 'k_stream_copy' in r['Kernel_Name'] and int(r[grid_key]) <= 256]
    return rows[marks[0] + 1:marks[1]], rows


def trace_summary(trace_csv, B, dom):
    rows = list(csv.DictReader(open(trace_csv)))
    reg, _ = region(rows, 'Grid_Size_X')
    stats = collections.defaultdict(lambda: [0, 0.0])
    for r in reg:
        d = (int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1e6
        s = stats[short(r['Kernel_Name'])]
        s[0] += 1
        s[1] += d
    out = [f"timed region: {len(reg)} dispatches between the two marker copies; "
           f"bench steps={B['steps']}",
           f"{'kernel':48s} {'calls':>7s} {'total_ms':>10s} {'avg_ms':>9s}"]
    for k, (c, t) in sorted(stats.items(), key=lambda kv: -kv[1][1])[:15]:
        out.append(f"{k:48s} {c:7d} {t:10.3f} {t / c:9.5f}")
    runs = dominant_runs(reg, dom)
    C = len(runs)
    T = sum((int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1e6 for g in runs for r in g)
    out.append(f"dominant kernel {' + '.join(dom)}: {C} launches, avg {T / C:.5f} ms per launch "
               f"(bench live events over the same launches: "
               f"{B['roofline']['avg_launch_ms']:.5f} ms)")
    return out


def pmc(path, dom):
    """(KiB the 1 GiB copy reads, dominant launches, their KiB) of a counter run."""
    rs = list(csv.DictReader(open(path)))
    reg, allr = region(rs, 'Grid_Size')
    big = [r for r in allr if 'k_stream_copy' in r['Kernel_Name'] and int(r['Grid_Size']) > 256]
    cal = float(big[-1]['Counter_Value'])
    runs = dominant_runs(reg, dom)
    return cal, len(runs), sum(float(r['Counter_Value']) for g in runs for r in g)


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    trace_csv, bench_log = argv[0], argv[1]
    fetch_csv = argv[2] if len(argv) > 2 else None
    write_csv = argv[3] if len(argv) > 3 else None
    line = [l for l in open(bench_log) if l.startswith('{')][-1]
    B = json.loads(line)
    dom = [s.strip() for s in B['roofline']['kernel'].split(' + ')]
    print("\n".join(trace_summary(trace_csv, B, dom)))
    if fetch_csv and write_csv:
        cf, nf, tf = pmc(fetch_csv, dom)
        cw, nw, tw = pmc(write_csv, dom)
        ff = (1 << 30) / (cf * 1024.0)
        fw = (1 << 30) / (cw * 1024.0)
        fb = tf / nf * ff * 1024.0
        wb = tw / nw * fw * 1024.0
        print(f"copy calibration: the 1 GiB copy reads FETCH_SIZE {cf:.0f} KiB (factor {ff:.4f}), "
              f"WRITE_SIZE {cw:.0f} KiB (factor {fw:.4f})")
        print(f"dominant kernel traffic: {nf} / {nw} launches in the counter runs' timed regions, "
              f"{fb + wb:.0f} bytes per launch (fetch {fb:.0f} + write {wb:.0f}); "
              f"algorithmic {B['roofline']['bytes_per_launch']} bytes per launch")
        print(json.dumps({"traffic_bytes_per_launch": int(fb + wb), "fetch_factor": ff,
                          "write_factor": fw}))
    elif fetch_csv:
        # reads only: no traffic figure (that needs both counters)
        cf, nf, tf = pmc(fetch_csv, dom)
        ff = (1 << 30) / (cf * 1024.0)
        fb = tf / nf * ff * 1024.0
        print(f"copy calibration: the 1 GiB copy reads FETCH_SIZE {cf:.0f} KiB (factor {ff:.4f})")
        print(f"dominant kernel reads: {nf} launches in the counter run's timed region, "
              f"{fb:.0f} bytes fetched per launch (no WRITE_SIZE run); algorithmic "
              f"{B['roofline']['bytes_per_launch']} bytes per launch")


if __name__ == "__main__":
    main()
