"""The rocprofv3 summary tool on small hand-made CSV files: timed region
between the marker copies, the dominant plan's launches found in dispatch
order, and the counter bytes scaled by the copy probe's calibration."""
import csv
import json

from paper_1210_2536_amd import prof_summary as PS

DOM = "void smat::(anonymous namespace)::k_a<float, false>(long)"
DOM2 = "void smat::(anonymous namespace)::k_b<float>(long)"
OTHER = "void smat::(anonymous namespace)::k_c<double>(long)"
MARK = "smat::(anonymous namespace)::k_stream_copy(long, int4 const*, int4*)"


def _write(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _trace(path):
    # (name, start, end, grid): the first dominant pair lies before the first
    # marker and must not count; inside, two pairs (3 + 1 and 5 + 1 us) and
    # an unrelated kernel, a lone k_a that is not followed by k_b
    seq = [(DOM, 0, 9000, 1024), (DOM2, 9000, 10000, 1024),
           (MARK, 20000, 21000, 16),
           (DOM, 30000, 33000, 1024), (DOM2, 33000, 34000, 1024),
           (OTHER, 40000, 47000, 1024),
           (DOM, 50000, 55000, 1024), (DOM2, 55000, 56000, 1024),
           (DOM, 60000, 62000, 1024), (OTHER, 62000, 63000, 1024),
           (MARK, 70000, 71000, 16)]
    _write(path, ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"],
           [dict(Kernel_Name=n, Start_Timestamp=s, End_Timestamp=e, Grid_Size_X=g)
            for n, s, e, g in seq])


def _counters(path, copy_kib, vals):
    seq = [(DOM, 10, 4096, 999.0),                      # before the region
           (MARK, 20, 16, 1.0),
           (DOM, 30, 4096, vals[0]), (DOM2, 31, 4096, vals[1]),
           (DOM, 40, 4096, vals[2]), (DOM2, 41, 4096, vals[3]),
           (MARK, 50, 16, 1.0),
           (MARK, 60, 1 << 20, copy_kib)]               # the 1 GiB copy probe
    _write(path, ["Kernel_Name", "Start_Timestamp", "Grid_Size", "Counter_Value"],
           [dict(Kernel_Name=n, Start_Timestamp=s, Grid_Size=g, Counter_Value=v)
            for n, s, g, v in seq])


def _bench_log(path):
    rec = {"steps": 2, "roofline": {"kernel": "k_a<float, false|true> + k_b<float>",
                                    "avg_launch_ms": 0.005, "bytes_per_launch": 4096}}
    with open(path, "w") as fh:
        fh.write("[bench] not json\n")
        fh.write(json.dumps(rec) + "\n")


def test_kernel_pattern_matching():
    assert PS.matches("k_a<float, true>", "k_a<float, false|true>")
    assert PS.matches("k_a<float, false>", "k_a<float, false|true>")
    assert not PS.matches("k_a<double, false>", "k_a<float, false|true>")
    assert PS.short(DOM) == "k_a<float, false>"


def test_trace_and_counter_summary(tmp_path, capsys):
    tr, log = tmp_path / "t.csv", tmp_path / "b.log"
    fe, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    _trace(tr)
    _bench_log(log)
    # FETCH: the copy reads 2^19 KiB for 1 GiB (factor 2); WRITE: 2^20 KiB (factor 1)
    _counters(fe, float(1 << 19), [10.0, 2.0, 14.0, 4.0])
    _counters(wr, float(1 << 20), [1.0, 3.0, 5.0, 7.0])
    PS.main([str(tr), str(log), str(fe), str(wr)])
    out = capsys.readouterr().out
    # two dominant runs inside the region: (3 + 1) and (5 + 1) us -> 5 us each
    assert "dominant kernel k_a<float, false|true> + k_b<float>: 2 launches, avg 0.00500 ms" in out
    assert "timed region: 7 dispatches" in out
    rec = json.loads([l for l in out.splitlines() if l.startswith("{")][-1])
    fetch = (10 + 2 + 14 + 4) / 2 * 2.0 * 1024
    write = (1 + 3 + 5 + 7) / 2 * 1.0 * 1024
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["traffic_bytes_per_launch"] == int(fetch + write)


def test_fetch_only_summary(tmp_path, capsys):
    tr, log, fe = tmp_path / "t.csv", tmp_path / "b.log", tmp_path / "f.csv"
    _trace(tr)
    _bench_log(log)
    _counters(fe, float(1 << 19), [10.0, 2.0, 14.0, 4.0])
    PS.main([str(tr), str(log), str(fe)])
    out = capsys.readouterr().out
    assert f"{(10 + 2 + 14 + 4) / 2 * 2.0 * 1024:.0f} bytes fetched per launch" in out
    assert "traffic_bytes_per_launch" not in out
