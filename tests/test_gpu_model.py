"""Nonlinear modelling on the GPU path (the map from m = 1/c^2 to data, Sec. 1.1) against
the FP64 oracle's background traces, and its pairing with the Born operator.

Tolerances as for the linear operators: relative L2 <= 1e-10 (FP64), <= 1e-5 (FP32)."""
import numpy as np
import pytest

import fixtures as F
from oracle import Problem as Oracle
from test_gpu_wave import ragged
from test_gpu_wave3d import cube

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"f64": 1e-10, "f32": 1e-5}


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    return M


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_traces(w, c):
    O = Oracle(w, c)
    return np.stack([O.background(s, keep_g=False)[1] for s in range(w.ns)])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_model_matches_oracle(dim, dtype):
    """Ragged strips, chunks and tiles; 2D with three shots (one null shot pads the group)."""
    M = _gpu()
    w = ragged(dtype) if dim == 2 else cube(dtype)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    d = P.model().cpu().numpy()
    assert d.shape == (w.ns, w.nt, w.nr)
    assert rel(d, _oracle_traces(w, c)) <= TOL[dtype]


def test_model_keeps_the_cache_and_ignores_the_snapshot_mode():
    """Modelling stores no history: a cached background survives it bit for bit, and the
    traces are the same bits whatever the snapshot mode of the context."""
    M = _gpu()
    w = ragged("f32")
    c = F.medium(w)
    dm = torch.from_numpy(F.normal_field(w.model_shape, 61))
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    first = P.apply_F(dm).cpu().numpy()
    d = P.model().cpu().numpy()
    again = P.apply_F(dm).cpu().numpy()
    assert P.stats()["background_cached"]
    assert np.array_equal(first, again)
    Q = M.Problem.from_spec(w.with_(snap="ckpt_bf16", ckpt_every=4))
    Q.set_background(torch.from_numpy(c))
    Q.apply_H(dm)
    assert np.array_equal(Q.model().cpu().numpy(), d)


def test_born_is_the_derivative_of_modelling_full_size():
    """On the 128 x 128 FP64 workload: (F[m0 + e dm] - F[m0 - e dm]) / 2e -> F dm with an
    O(e^2) error, for a smooth interior perturbation that leaves c_max (hence the damping)
    and the layer's edge velocity unchanged."""
    M = _gpu()
    w = F.c1()
    c0 = F.medium(w).astype(np.float64)
    nz, nx = w.model_shape
    z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    m0 = 1.0 / c0 ** 2
    dm = 0.02 * float(np.mean(m0)) * np.exp(-((z - 0.3 * nz) ** 2 + (x - 0.5 * nx) ** 2) / (2 * 6.0 ** 2))
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c0))
    born = P.apply_F(torch.from_numpy(dm)).cpu().numpy()
    errs = []
    for eps in (1.0, 0.5):
        cp, cm = 1.0 / np.sqrt(m0 + eps * dm), 1.0 / np.sqrt(m0 - eps * dm)
        assert np.max(cp) == np.max(cm) == np.max(c0)
        P.set_background(torch.from_numpy(cp))
        dp = P.model().cpu().numpy()
        P.set_background(torch.from_numpy(cm))
        dmn = P.model().cpu().numpy()
        errs.append(rel((dp - dmn) / (2 * eps), born))
    print("Taylor errors", errs)
    assert errs[1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0
