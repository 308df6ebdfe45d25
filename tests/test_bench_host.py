"""Host logic of bench.py that needs no GPU: the one-GPU guard and the
rocprofv3 kernel-trace summary the committed profiles are made with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_trace_summary_counts_full_and_early_exit_launches(tmp_path):
    """Three kernels on a made-up timeline (ns): kernel A has four full
    launches of 10 us and two early exits of 1 us; the span, busy share, mean
    gap, averages and the full-launch count follow by hand."""
    rows = [("k_a", 0, 10000), ("k_a", 12000, 22000), ("k_b", 22000, 27000), ("k_a", 30000, 40000),
            ("k_a", 40000, 50000), ("k_a", 50000, 51000), ("k_a", 52000, 53000), ("k_c", 53000, 55000)]
    csv = tmp_path / "trace.csv"
    with open(csv, "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for k, s0, s1 in rows:
            f.write(f"{k},{s0},{s1}\n")
    r = subprocess.run([sys.executable, BENCH, "--summarize-trace", str(csv)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().splitlines()
    # span 55 us, busy 10+10+5+10+10+1+1+2 = 49 us, idle 6 us over 8 launches
    assert lines[0] == "traced span 0.06 ms, kernels running 89.1% of it, 8 launches, mean gap 0.75 us"
    table = {ln.split()[0]: ln.split()[1:] for ln in lines[2:]}
    assert list(table) == ["k_a", "k_b", "k_c"]            # by total time
    launches, worked, avg_all, avg_worked, mn, mx = table["k_a"]
    assert (int(launches), int(worked)) == (6, 4)
    assert abs(float(avg_all) - 42.0 / 6) < 1e-3 and abs(float(avg_worked) - 10.0) < 1e-3
    assert (float(mn), float(mx)) == (1.0, 10.0)
    assert table["k_b"][:2] == ["1", "1"] and float(table["k_b"][2]) == 5.0
