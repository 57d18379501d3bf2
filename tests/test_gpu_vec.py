"""The solvers' vector kernels (dot with FP64 accumulation in a fixed order, axpby, the
Gauss-Newton velocity update) against numpy."""
import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problem(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    w = F.tiny(n=16, nr=16, dtype=dtype).with_(nx=64, nz=32)
    return M, M.Problem.from_spec(w), w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [0, 1, 1000, 262144 + 77, 3_000_001])
def test_dot(dtype, n):
    M, P, _ = _problem(dtype)
    npdt = np.float64 if dtype == "f64" else np.float32
    a = F.normal_field((n,), 1, npdt)
    b = F.normal_field((n,), 2, npdt)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    got = P.dot(ta, tb)
    ref = float(np.sum(a.astype(np.float64) * b.astype(np.float64)))
    scale = float(np.sum(np.abs(a.astype(np.float64) * b.astype(np.float64)))) or 1.0
    assert abs(got - ref) <= 1e-13 * scale
    assert P.dot(ta, tb) == got      # fixed order: the same bits every call


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_axpby(dtype):
    M, P, _ = _problem(dtype)
    npdt = np.float64 if dtype == "f64" else np.float32
    n = 100_003
    x = F.normal_field((n,), 3, npdt)
    y = F.normal_field((n,), 4, npdt)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    P.axpby(0.75, tx, -1.25, ty)
    ref = 0.75 * x.astype(np.float64) - 1.25 * y.astype(np.float64)
    got = ty.cpu().numpy().astype(np.float64)
    # FP64 arithmetic (possibly fused), then one rounding to the field precision
    terms = 0.75 * np.abs(x.astype(np.float64)) + 1.25 * np.abs(y.astype(np.float64))
    rnd = 0.0 if dtype == "f64" else 6e-8
    assert np.all(np.abs(got - ref) <= 4e-16 * terms + rnd * np.abs(ref))
    # beta = 0 overwrites y without reading it
    tz = torch.full_like(tx, float("nan"))
    P.axpby(-0.5, tx, 0.0, tz)
    assert torch.equal(tz, (-0.5 * tx.double()).to(tx.dtype))
    with pytest.raises(M.MatprobeError) as e:
        P.axpby(float("nan"), tx, 1.0, ty)
    assert e.value.code == -5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_velocity_update(dtype):
    M, P, w = _problem(dtype)
    c = F.medium(w).astype(np.float64 if dtype == "f64" else np.float32)
    dm = 0.01 * F.normal_field(w.model_shape, 5, np.float64) / np.mean(c.astype(np.float64)) ** 2
    dm = dm.astype(c.dtype)
    tc, tdm = torch.from_numpy(c.copy()).cuda(), torch.from_numpy(dm).cuda()
    P.velocity_update(tc, tdm)
    ref = 1.0 / np.sqrt(1.0 / c.astype(np.float64) ** 2 + dm.astype(np.float64))
    tol = 1e-15 if dtype == "f64" else 1.2e-7
    np.testing.assert_allclose(tc.cpu().numpy().astype(np.float64), ref, rtol=tol)
    # a step that makes m non-positive somewhere is refused and c is left as it was
    before = tc.clone()
    bad = tdm.clone()
    bad[3, 5] = -10.0 / float(c.min()) ** 2
    with pytest.raises(M.MatprobeError) as e:
        P.velocity_update(tc, bad)
    assert e.value.code == -5
    assert torch.equal(tc, before)
