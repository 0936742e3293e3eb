"""Host logic of the measurement scripts (no GPU): the benchmark refuses more than one GPU before it
touches a device, its algorithmic byte counts follow the pass model, and the traffic summary weights
one step's launches as stated."""
import os
import subprocess
import sys

import bench
import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_of_the_fused_pass():
    """conv_z_fused per step: 4 launches over 6 component solves; each component reads its N nonzero
    inputs and writes its N kept outputs of every z column, one column per (x frequency, y frequency)
    pair, (P/2 + 1) x P columns of complex values (16 B in FP64); each launch reads the real spectrum
    (P/2 + 1)^3 once."""
    N, P, es = 256, 512, 8
    b = bench.alg_bytes_per_step(N, P, es)
    nh = P // 2 + 1
    per_comp = 2 * (2 * es) * N * nh * P  # read + write
    spec = es * nh ** 3
    assert b["conv_z_fused"] == 6 * per_comp + 4 * spec
    assert all(v > 0 for v in b.values())
    # FP32 halves every count
    b32 = bench.alg_bytes_per_step(N, P, 4)
    assert all(abs(b32[k] * 2 - b[k]) <= 1 for k in b)


def test_traffic_step_average():
    """Dispatches are grouped by grid size (a launch over c components has c times the grid) and
    averaged with the step's mix (one 3-component launch, three 1-component launches)."""
    g = 1000
    vals = [(g, 10.0)] * 6 + [(3 * g, 40.0)] * 2
    avg, det = traffic.step_average("conv_z_fused", vals)
    assert avg == (1 * 40.0 + 3 * 10.0) / 4
    assert det["launches_by_components"] == {"1": 6, "3": 2}
    avg, det = traffic.step_average("if_xy", [(5, 1.0), (7, 3.0)])
    assert avg == 2.0 and det["launches"] == 2
