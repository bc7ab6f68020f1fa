"""Host-side checks of the benchmark script (no GPU): the algorithmic byte
counts behind its roofline figures, and its refusal of more than one GPU."""
import os
import subprocess
import sys

import bench
from paper_2207_14256_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N3 = 512 ** 3


def test_push_bytes_c3():
    # FP32, psi != phi, phi-dot = 0: 6 bf16 slots (12-byte cells), all data
    cfg = workloads.preset("c3")
    assert bench.mesh_slots(cfg) == (6, 6)
    assert bench.bytes_per_launch(cfg, N3, True) == N3 * (36 + 24) + N3 * 6 * 2
    assert bench.bytes_per_launch(cfg, N3, False) == N3 * (36 + 12) + N3 * 6 * 2
    assert bench.bytes_per_push_sort(cfg, N3) == N3 * 92 + N3 * 6 * 2
    assert bench.mesh_padding_bytes(cfg) == 0
    cfg = workloads.preset("c3", pad_mesh=True)       # 16-byte cells: 8 stored, 6 data
    assert bench.mesh_slots(cfg) == (8, 6)
    assert bench.mesh_padding_bytes(cfg) == N3 * 2 * 2


def test_push_bytes_fp64_no_slip_and_time_dependent():
    cfg = workloads.preset("c3", precision="fp64")   # phi-dot = 0 with slip: 6 binary64 slots
    assert bench.mesh_slots(cfg) == (6, 6)
    assert bench.bytes_per_launch(cfg, N3, True) == N3 * (72 + 48) + N3 * 6 * 8
    cfg = workloads.preset("c3", slip_amp=0.0)       # psi = phi: 4 bf16 slots, 3 with data
    assert bench.mesh_slots(cfg) == (4, 3)
    assert bench.bytes_per_launch(cfg, N3, True) == N3 * 60 + N3 * 3 * 2
    assert bench.bytes_per_push_sort(cfg, N3) == N3 * 92 + N3 * 3 * 2
    cfg = workloads.preset("c3", model="radmat")     # phi-dot carries data: 7 of 8
    assert bench.mesh_slots(cfg) == (8, 7)


def test_refuses_several_gpus():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""
