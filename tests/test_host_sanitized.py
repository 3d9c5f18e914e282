"""Host code under address and undefined-behaviour sanitizers (CPU only):

* the input generator (graphgen.c) and every oracle function (oracle.c) on
  small RMAT, Erdos-Renyi and torus graphs (sanitize_check.c);
* the query server's scheduling rules (paper_1805_05208_amd/csrc/admission.h:
  first-fit arena, admission with bit-packing and halving, head-of-line
  waiting for memory, overflow re-queue and learned bucket capacity) with
  fake graphs and footprints (sched_check.cpp);
* the grid-barrier protocol of the single-launch forms
  (paper_1805_05208_amd/csrc/gridbar_protocol.h), the same code run by
  threads standing for workgroups on uneven dies (gridbar_model.cpp).

Each driver is compiled here with gcc / g++ and run as a child process; a
sanitizer report makes it exit non-zero.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def build_and_run(cmd, exe):
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("compiler without sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, \
        run.stderr[-4000:]
    return run.stdout


def test_oracle_and_generator_under_sanitizers(tmp_path):
    out = build_and_run(["gcc", "-std=c11", *SAN, "-fopenmp",
                         os.path.join(HERE, "sanitize_check.c"),
                         os.path.join(ROOT, "oracle", "oracle.c"),
                         os.path.join(ROOT, "graphgen", "graphgen.c"), "-lm"],
                        str(tmp_path / "sanitize_check"))
    assert "generator and oracle checks passed" in out


def test_server_scheduling_rules_under_sanitizers(tmp_path):
    out = build_and_run(["g++", "-std=c++17", *SAN,
                         "-I" + os.path.join(ROOT, "include"),
                         "-I" + os.path.join(ROOT, "paper_1805_05208_amd", "csrc"),
                         os.path.join(HERE, "sched_check.cpp")],
                        str(tmp_path / "sched_check"))
    assert "scheduler checks passed" in out


def test_grid_barrier_protocol_on_threads(tmp_path):
    out = build_and_run(["g++", "-std=c++17", *SAN, "-pthread",
                         "-I" + os.path.join(ROOT, "paper_1805_05208_amd", "csrc"),
                         os.path.join(HERE, "gridbar_model.cpp")],
                        str(tmp_path / "gridbar_model"))
    assert "grid barrier model checks passed" in out
