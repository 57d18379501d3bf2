"""Full-length parity of the 1024 x 512, 4000-step workload against the FP64 oracle.

The expected values were written by tests/golden/make_c3_golden.py, which calls
only the oracle: for eight of the workload's 128 shots (every 16th), H y and
F* d summed over those shots, and F y at every 16th receiver.  The GPU runs the
same eight shots at the full grid and record length, with the workload's own
snapshot mode (BF16 checkpoints every 4 steps with FP32 scales, recomputation
between them) and with the FP32 full g history.  Bounds: 1e-2 relative L2 for
the BF16-checkpointed H and F*, 1e-5 for everything in FP32 (F never reads a
checkpoint, so it is held to 1e-5 in both modes).
"""
import os

import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_golden.npz")
DATA_SEED = 19


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def golden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = np.load(GOLDEN)
    w = F.c3()
    w = w.with_(src=w.src[[int(s) for s in g["shots"]]])
    c = F.medium(w)
    y = F.trials(w, c)[0]
    d = F.bandlimited_data((w.ns, w.nt, w.nr), DATA_SEED, w.dt, w.f_peak)
    return g, w, c, y, d


@pytest.mark.parametrize("snap", ["ckpt_bf16", "full"])
def test_c3_full_length_against_oracle(golden, snap):
    import paper_1101_3615_amd as M
    g, w, c, y, d = golden
    P = M.Problem.from_spec(w, snap=snap, ckpt_every=(4 if snap == "ckpt_bf16" else 0))
    P.set_background(torch.from_numpy(c))
    Hy = P.apply_H(torch.from_numpy(y)).cpu().numpy()
    dF = P.apply_F(torch.from_numpy(y))
    rec = [int(r) for r in g["F_rec"]]
    Fy = dF[:, :, rec].cpu().numpy()
    del dF
    img = P.apply_Fadj(torch.from_numpy(d)).cpu().numpy()
    eH, eF, eA = rel(Hy, g["H_y"]), rel(Fy, g["F_y"]), rel(img, g["Fadj_d"])
    print(f"1024x512, 8 shots, 4000 steps, {snap}: apply_H {eH:.3e}, apply_F {eF:.3e}, apply_Fadj {eA:.3e}")
    assert eF <= 1e-5
    tol = 1e-2 if snap == "ckpt_bf16" else 1e-5
    assert eH <= tol
    assert eA <= tol
