"""Host logic of the tile work plans: compile the checks in tests/host/ (which
include the library's headers) with the host compiler and run them.

plan_check.cpp: the level kernel's grid and XCD remap cover every tile of
every plane exactly once; the batched level kernel's plan covers every tile
of every image once and keeps every LL band inside its ping-pong buffer.
persist_check.cpp: a replay of the persistent forward's work queue (one
thread per work-group, the kernel's ticket loop, dependency waits and
publication, built on dwt2_batch_plan.h) on random batches and plane stacks
of every tile shape: no wait runs out, every tile runs once, every tile reads
only finished tiles of the level before (checked by brute force over the
rows it reads), and the tables and LL bands stay inside the workspace."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

needs_tools = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                                 reason="needs g++ and the ROCm headers")


def build_and_run(tmp_path, name):
    exe = tmp_path / name
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "paper_1704_08657_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", name + ".cpp"), "-o", str(exe)], check=True)
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)


@needs_tools
def test_level_grid_covers_every_tile_once(tmp_path):
    r = build_and_run(tmp_path, "plan_check")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout


@needs_tools
def test_persistent_work_queue_replay(tmp_path):
    r = build_and_run(tmp_path, "persist_check")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout
