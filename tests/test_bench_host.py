"""Host logic of bench.py (no GPU): the one-GPU guard and the algorithmic bytes per
launch of the 2D sweeps on the 512 x 256 workload."""
import os
import subprocess
import sys

import pytest

import fixtures as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("kind,mb", [("background", 235.1), ("born", 235.7), ("adjoint", 268.6)])
def test_kernel_bytes_of_the_512x256_workload(kind, mb):
    import bench
    w = F.c2()
    # 552 x 296 propagation cells, 512 x 256 model cells, 64 shots
    assert (w.prop_cells, w.model_cells, w.ns) == (163392, 131072, 64)
    assert round(bench.kernel_bytes(kind, w) / 1e6, 1) == mb
    # one step per launch moves fewer bytes per launch but more per step
    one, two = bench.kernel_bytes(kind, w, s=1), bench.kernel_bytes(kind, w, s=2)
    assert one < two < 2 * one
