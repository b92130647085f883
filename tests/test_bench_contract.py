"""The bench entry point's command-line contract that holds without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_defaults_finish_within_minutes():
    sys.path.insert(0, ROOT)
    import bench
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.gpus == 1 and a.workload == "sweep"
    assert 1 <= a.steps <= 50 and 0 <= a.warmup <= 10
    assert a.cpu_seconds <= 30


def test_profile_summary_attributes_shared_kernels_to_the_dominant_plan():
    """A kernel that several plans launch (the long-row kernels) counts for
    the dominant plan only inside that plan's runs: its first kernel followed
    by its other kernels in dispatch order."""
    from paper_1210_2536_amd.prof_summary import dominant_runs, matches

    def row(name, t0, t1):
        return {"Kernel_Name": f"void smat::(anonymous namespace)::{name}(long)",
                "Start_Timestamp": str(t0), "End_Timestamp": str(t1)}
    dom = ["k_csr_adaptive_rest<float, false>", "k_long_tiles<float>",
           "k_long_tiles_reduce<float>"]
    reg = [row("k_csr_adaptive_rest<float, false>", 0, 5), row("k_long_tiles<float>", 5, 9),
           row("k_long_tiles_reduce<float>", 9, 10),
           row("k_csr_panel_xcd_rest<float, false>", 10, 20), row("k_panel_reduce_rest<float>", 20, 21),
           row("k_long_tiles<float>", 21, 30), row("k_long_tiles_reduce<float>", 30, 31),
           row("k_csr_adaptive_rest<float, false>", 31, 33), row("k_ell<float, 2, false, 1>", 33, 34)]
    runs = dominant_runs(reg, dom)
    assert len(runs) == 1 and [r["Start_Timestamp"] for r in runs[0]] == ["0", "5", "9"]
    assert matches("k_csr_panel_rest<float, false, true>", "k_csr_panel_rest<float, false, false|true>")
    assert not matches("k_csr_panel_rest<double, false, true>",
                       "k_csr_panel_rest<float, false, false|true>")
