"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the pmc and trace summary
modes read rocprofv3 CSVs without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_torus_goes_with_the_batched_section():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--torus"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--torus goes with --only batched" in r.stderr


def test_pmc_summary_reads_a_counter_csv(tmp_path):
    rows = [
        "Correlation_Id,Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value",
        '1,1,"gb::bfs_round_kernel(gb::BfsArgs, unsigned int)",FETCH_SIZE,100.0',
        '2,2,"gb::bfs_round_kernel(gb::BfsArgs, unsigned int)",FETCH_SIZE,300.0',
        '3,3,"__amd_rocclr_copyBuffer",FETCH_SIZE,524300.0',
    ]
    (tmp_path / "x_counter_collection.csv").write_text("\n".join(rows) + "\n")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--pmc-summary",
                        str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    line = [l for l in r.stdout.splitlines() if "bfs_round_kernel" in l][0]
    assert "dispatches=     2" in line and "200.0" in line


def test_trace_summary_concurrency(tmp_path):
    """Kernels A [0, 4) and B [2, 6) ms overlap for 2 ms, then C [10, 11) ms
    runs alone: 9 ms of kernel time while the device was busy 7 ms, so the
    mean concurrency is 9/7 = 1.29 and the device is busy 7/11 of the span."""
    ms = 1_000_000
    rows = ["Kernel_Name,Start_Timestamp,End_Timestamp",
            f'"gb::a(int)",{0},{4 * ms}',
            f'"gb::b(int)",{2 * ms},{6 * ms}',
            f'"gb::a(int)",{10 * ms},{11 * ms}']
    (tmp_path / "x_kernel_trace.csv").write_text("\n".join(rows) + "\n")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--trace-summary",
                        str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = r.stdout
    assert "3 kernels over 0.011 s, 0.009 s of kernel time" in out
    assert "device busy 0.007 s (63.6 % of the span), mean concurrency 1.29" in out
    a = [l for l in out.splitlines() if "gb::a" in l][0]
    assert "calls=       2" in a and "total=      5.00 ms" in a


def test_segments_split_searches_and_total_steps(tmp_path):
    """Dispatches cut at each start kernel; a step log totals the weighted
    step dispatches of each logged search by kind."""
    rows = ["Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp"]
    t = 0
    seq = ["gb::wbfs_init_kernel", "gb::wbfs_step_kernel", "gb::wbfs_step_kernel",
           "gb::wbfs_step_kernel", "gb::wbfs_init_kernel", "gb::wbfs_step_kernel"]
    for i, k in enumerate(seq):
        rows.append(f'{i + 1},"{k}(int)",{t},{t + 1000 * (i + 1)}')
        t += 100000
    (tmp_path / "x_kernel_trace.csv").write_text("\n".join(rows) + "\n")
    log = tmp_path / "run.log"
    log.write_text('{"metric": "wbfs_section", "step_logs": {"7": [[0, 1, 2, 0], [3, 4, 5, 1], '
                   '[3, 4, 5, 2]], "9": [[0, 1, 1, 0]]}}\n')
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--segments", str(tmp_path),
                        "--start", "wbfs_init_kernel", "--kernel", "wbfs_step_kernel",
                        "--step-log", str(log), "--segment", "0"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = r.stdout
    assert "2 searches starting at wbfs_init_kernel; values in us" in out
    assert "search 0: 3 dispatches, total 9.0" in out      # 2 + 3 + 4 us
    assert "source 7: 3 steps; push 1 steps 2.0, mark 1 steps 3.0, pull 1 steps 4.0" in out
    assert "source 9: 1 steps; push 1 steps 6.0" in out
