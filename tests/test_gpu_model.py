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


def test_model_full_size_sampled_shots():
    """512 x 256 FP32 workload (64 shots, 3000 steps, the launch configuration of the
    benchmark): the traces of a sampled shot against the oracle's background sweep of it."""
    M = _gpu()
    w = F.c2()
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    d = P.model()
    O = Oracle(w, c)
    for s in (37,):
        ref = O.background(s, keep_g=False)[1]
        err = rel(d[s].double().cpu().numpy(), ref)
        print(f"shot {s}: rel L2 {err:.3e}")
        assert err <= TOL["f32"]


def test_gauss_newton_lowers_the_misfit_full_size():
    """On the 128 x 128 FP64 workload, from the smooth background towards it plus a weak
    reflectivity: one Gauss-Newton step with three CG iterations lowers the misfit."""
    M = _gpu()
    from paper_1101_3615_amd import inversion as I
    w = F.c1()
    c0 = F.medium(w).astype(np.float64)
    m_true = 1.0 / c0 ** 2 + 0.5 * F.reflectivity(w, c0, seed=3).astype(np.float64)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(1.0 / np.sqrt(m_true)))
    d_obs = P.model().clone()
    cs, Js = I.gauss_newton(P, torch.from_numpy(c0), d_obs, 1, 3)
    print("misfits", Js)
    assert Js[1] < 0.5 * Js[0]
    err0 = np.linalg.norm(1.0 / c0 ** 2 - m_true)
    err1 = np.linalg.norm(1.0 / cs[1].cpu().numpy() ** 2 - m_true)
    assert err1 < err0
