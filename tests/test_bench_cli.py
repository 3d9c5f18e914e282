"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the pmc summary mode reads a
counter CSV without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


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
