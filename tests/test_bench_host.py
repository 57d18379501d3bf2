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


def test_kernel_bytes_of_the_256_cube_launch():
    """The fused 3D launch of a wave of 8 shots at 296^3: 28 B per cell and shot plus
    kappa and the perturbation once, the figure the benchmark divides by the launch time."""
    import bench
    w = F.c5()
    assert w.prop_cells == 296 ** 3 and w.model_cells == 256 ** 3
    assert bench.kernel_bytes3d("fused", w, 8) == (28 * 8 + 8) * 296 ** 3 == 6016765952
    assert bench.kernel_bytes3d("background", w, 8) == (16 * 8 + 4) * 296 ** 3 + 4 * 8 * 256 ** 3
    assert bench.kernel_bytes3d("adjoint", w, 8) == (12 * 8 + 4) * 296 ** 3 + 12 * 8 * 256 ** 3


def test_counter_traffic_only_for_the_launch_shape_and_source_it_was_taken_on(monkeypatch):
    """profiles/traffic*.json hold HBM bytes per launch for one workload, one shot count
    per launch and one kernel source: any other shape or source reads as unmeasured."""
    import json

    import bench
    for dims, w in (("3d", F.c5()), ("c3", F.c3()), ("2d", F.c2())):
        rec_name, _ = bench.TRAFFIC[dims]
        rec = json.load(open(os.path.join(ROOT, "profiles", rec_name)))
        assert rec["workload"] == w.name and rec["launch_shots"] == bench.LAUNCH_SHOTS[dims]
        nsh = rec["launch_shots"]
        kind = next(iter(rec["kernels"]))
        got = bench.traffic_for(kind, w, nsh)
        assert got is None or got == rec["kernels"][kind]["bytes_per_launch"]
        if got is not None:
            assert bench.traffic_for(kind, w, nsh * 2) is None
            assert bench.traffic_for(kind, w.with_(name="other"), nsh) is None
            monkeypatch.setattr(bench, "_sha", lambda path: "0" * 64)
            assert bench.traffic_for(kind, w, nsh) is None
            monkeypatch.undo()
