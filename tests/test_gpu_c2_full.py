"""Full-size parity of the 512 x 256, 64-shot, 3000-step FP32 workload.

The expected values were written by tests/golden/make_c2_golden.py, which calls
only the FP64 oracle: H y0 over the whole model grid, and the Born traces of
two shots at every second time step (sampled outputs of F y0).  The GPU runs
the same launch configuration as the benchmark.
"""
import os

import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_golden.npz")


def test_c2_full_size_apply_H_and_F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    g = np.load(GOLDEN)
    w = F.c2()
    c = F.medium(w)
    y = F.trials(w, c)[0]
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    Hy = P.apply_H(torch.from_numpy(y)).double().cpu().numpy()
    err_H = np.linalg.norm(Hy - g["H_y0"]) / np.linalg.norm(g["H_y0"])
    d = P.apply_F(torch.from_numpy(y))
    shots = [int(s) for s in g["F_shots"]]
    got = d[shots][:, ::2].double().cpu().numpy()
    ref = g["F_y0"].astype(np.float64)
    err_F = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"full-size 512x256 fp32: apply_H rel L2 = {err_H:.3e}, apply_F (2 shots) rel L2 = {err_F:.3e}")
    assert err_H <= 1e-5
    assert err_F <= 1e-5
