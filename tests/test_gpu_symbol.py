"""Parity of the probing fit and of the fitted-inverse application (HIP, via the C ABI)."""
import numpy as np
import pytest

import fixtures as F
from oracle import symbol as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    return M


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _problem(M, w):
    P = M.Problem.from_spec(w)
    return P


@pytest.mark.parametrize("dtype,shape", [("f64", (32, 64)), ("f32", (64, 128)), ("f64", (128, 16))])
def test_apply_Hinv_matches_oracle(dtype, shape):
    M = _gpu()
    nz, nx = shape
    w = F.tiny(n=8, nr=8, dtype=dtype).with_(nx=nx, nz=nz)
    P = _problem(M, w)
    leg = [(0, 0), (1, 0), (2, 1), (0, 3)]
    qs = (0, 1, 2, 3)
    B = M.Basis(leg, qs, 2)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(B.p)
    img = F.normal_field(shape, 11)
    got = M.apply_Hinv(P, B, c, torch.from_numpy(img)).cpu().numpy()
    ref = S.apply_Hinv(c, img, w.h, leg, qs)
    assert rel(got, ref) <= (1e-13 if dtype == "f64" else 1e-6)


def test_single_multiplier_terms():
    """B_(P0,q) alone: the FFT, the |k| table and the normalisation of each power."""
    M = _gpu()
    w = F.tiny(n=8, nr=8, dtype="f64").with_(nx=64, nz=32)
    P = _problem(M, w)
    img = F.normal_field((32, 64), 12)
    for q in range(4):
        B = M.Basis([(0, 0)], (q,), 2)
        got = M.apply_Hinv(P, B, np.array([1.0]), torch.from_numpy(img)).cpu().numpy()
        ref = S.apply_basis(img, w.h, [(0, 0)], (q,))[0]
        assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("ntrial", [1, 2])
def test_probe_fit_exact_recovery(ntrial):
    """y = sum_i c_i B_i x exactly -> the GPU fit returns c to 1e-10 (Sec. 1.4)."""
    M = _gpu()
    w = F.tiny(n=8, nr=8, dtype="f64").with_(nx=128, nz=64)
    P = _problem(M, w)
    leg = [(a, 0) for a in range(5)]
    qs = (0, 1, 2, 3)
    B = M.Basis(leg, qs, 2)
    rng = np.random.default_rng(9)
    ctrue = rng.standard_normal(B.p)
    xs = [F.normal_field((64, 128), 40 + t).astype(np.float64) for t in range(ntrial)]
    ys = [S.apply_Hinv(ctrue, x, w.h, leg, qs) for x in xs]
    c, relres = M.probe_fit(P, B, [torch.from_numpy(y) for y in ys], [torch.from_numpy(x) for x in xs])
    assert np.max(np.abs(c - ctrue)) <= 1e-10 * np.max(np.abs(ctrue))
    assert relres < 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_probe_fit_matches_oracle_least_squares(dtype):
    M = _gpu()
    w = F.tiny(n=8, nr=8, dtype=dtype).with_(nx=64, nz=64)
    P = _problem(M, w)
    leg = [(0, 0), (1, 0), (2, 0)]
    qs = (0, 1, 2, 3)
    B = M.Basis(leg, qs, 2)
    xs = [F.normal_field((64, 64), 60 + t) for t in range(2)]
    ys = [F.normal_field((64, 64), 70 + t) for t in range(2)]
    c, relres = M.probe_fit(P, B, [torch.from_numpy(y) for y in ys], [torch.from_numpy(x) for x in xs])
    cref, rref, _ = S.fit([y.astype(np.float64) for y in ys], [x.astype(np.float64) for x in xs], w.h, leg, qs)
    assert rel(c, cref) <= 1e-10
    assert abs(relres - rref) <= 1e-10 * rref


def test_probe_fit_rank_deficient():
    """A duplicated column: the fit flags the system (code -5) and, with strict=False,
    returns the minimum-norm least-squares coefficients (numpy's lstsq on the stacked
    columns; the duplicate columns share the equilibration scale, so the minimum in the
    equilibrated variables is the plain minimum norm) and their residual."""
    M = _gpu()
    w = F.tiny(n=8, nr=8, dtype="f64").with_(nx=32, nz=32)
    P = _problem(M, w)
    x = F.normal_field((32, 32), 80).astype(np.float64)
    y = F.normal_field((32, 32), 81).astype(np.float64)
    for legs in ([(0, 0), (0, 0)], [(0, 0), (1, 0), (0, 0)]):
        B = M.Basis(legs, (0,), 2)
        with pytest.raises(M.MatprobeError) as e:
            M.probe_fit(P, B, [torch.from_numpy(y)], [torch.from_numpy(x)])
        assert e.value.code == -5
        c, relres, deficient = M.probe_fit(P, B, [torch.from_numpy(y)], [torch.from_numpy(x)], strict=False)
        assert deficient
        zt = (np.arange(32) * 2 + 1) / 32.0 - 1.0          # cell centres of the depth axis
        cols = [x * (zt[:, None] if a == 1 else 1.0) for a, _ in legs]
        A = np.stack([col.ravel() for col in cols], axis=1)
        cref = np.linalg.lstsq(A, y.ravel(), rcond=1e-10)[0]
        assert rel(np.asarray(c), cref) <= 1e-10
        rref = np.linalg.norm(A @ cref - y.ravel()) / np.linalg.norm(y)
        assert abs(relres - rref) <= 1e-8


def test_non_power_of_two_rejected():
    M = _gpu()
    w = F.tiny(n=8, nr=8, dtype="f64").with_(nx=48, nz=32)
    P = _problem(M, w)
    B = M.Basis([(0, 0)], (0,), 2)
    with pytest.raises(M.MatprobeError) as e:
        M.apply_Hinv(P, B, np.array([1.0]), torch.zeros(32, 48, dtype=torch.float64))
    assert e.value.code == -6


# ---- the paper's expansion: Fourier modes x angular harmonics x rational Chebyshev ----

MODES2 = [(0, 0, 0), (1, 0, 0), (0, 2, 1), (1, 1, 1), (2, 3, 0)]          # (m_z, m_x, phase)
MULTS2 = [(0, 0), (1, 1), (2, 0), (3, 2), (4, 1), (6, 3)]                 # (angle, TL degree)
MODES3 = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 2, 1)]                        # (m_z, m_y, m_x, phase)
MULTS3 = [(0, 0), (1, 1), (3, 0), (6, 2), (8, 1)]


def _cube_pow2(dtype, nx=16, ny=8, nz=8):
    from fixtures.configs import Workload
    src = np.array([[1, 1, 0]], np.int32)
    rec = np.array([[2, 2, 0], [5, 3, 1]], np.int32)
    return Workload(name="cube_p2", ndim=3, nx=nx, ny=ny, nz=nz, h=12.5, nb=4, dt=1.0e-3, nt=10,
                    f_peak=15.0, src=src, rec=rec, dtype=dtype, snap="full", ckpt_every=0,
                    medium=dict(kind="smooth_random", cmin=1500.0, cmax=3500.0, corr=60.0, seed=41))


@pytest.mark.parametrize("dtype,order", [("f64", 1), ("f64", -1), ("f64", 0), ("f64", 2), ("f32", 1), ("f32", -1)])
def test_paper_basis_apply_Hinv_matches_oracle_2d(dtype, order):
    M = _gpu()
    shape = (32, 64)
    w = F.tiny(n=8, nr=8, dtype=dtype).with_(nx=shape[1], nz=shape[0])
    P = _problem(M, w)
    B = M.Basis.fourier_angular(MODES2, MULTS2, 2, order=order, tl_scale=0.5)
    c = np.random.default_rng(21).standard_normal(B.p)
    img = F.normal_field(shape, 13)
    got = M.apply_Hinv(P, B, c, torch.from_numpy(img)).cpu().numpy()
    ref = np.tensordot(c, S.apply_paper_basis(img.astype(np.float64), w.h, MODES2, MULTS2, order, 0.5), axes=1)
    assert rel(got, ref) <= (1e-12 if dtype == "f64" else 2e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_paper_basis_apply_Hinv_matches_oracle_3d(dtype):
    M = _gpu()
    w = _cube_pow2(dtype)
    P = _problem(M, w)
    B = M.Basis.fourier_angular(MODES3, MULTS3, 3, order=1, tl_scale=0.75)
    c = np.random.default_rng(22).standard_normal(B.p)
    img = F.normal_field(w.model_shape, 14)
    got = M.apply_Hinv(P, B, c, torch.from_numpy(img)).cpu().numpy()
    ref = np.tensordot(c, S.apply_paper_basis(img.astype(np.float64), w.h, MODES3, MULTS3, 1, 0.75), axes=1)
    assert rel(got, ref) <= (1e-12 if dtype == "f64" else 2e-6)


@pytest.mark.parametrize("ndim", [2, 3])
def test_paper_basis_fit_exact_recovery(ndim):
    M = _gpu()
    if ndim == 2:
        w = F.tiny(n=8, nr=8, dtype="f64").with_(nx=64, nz=32)
        modes, mults = MODES2[:4], MULTS2[:4]
    else:
        w = _cube_pow2("f64")
        modes, mults = MODES3, MULTS3[:4]
    P = _problem(M, w)
    B = M.Basis.fourier_angular(modes, mults, ndim, order=1, tl_scale=0.5)
    ctrue = np.random.default_rng(23).standard_normal(B.p)
    xs = [F.normal_field(w.model_shape, 90 + t).astype(np.float64) for t in range(2)]
    ys = [np.tensordot(ctrue, S.apply_paper_basis(x, w.h, modes, mults, 1, 0.5), axes=1) for x in xs]
    c, relres = M.probe_fit(P, B, [torch.from_numpy(y) for y in ys], [torch.from_numpy(x) for x in xs])
    assert np.max(np.abs(c - ctrue)) <= 1e-10 * np.max(np.abs(ctrue))
    assert relres < 1e-10


def test_paper_basis_fit_matches_oracle_least_squares():
    M = _gpu()
    w = F.tiny(n=8, nr=8, dtype="f64").with_(nx=64, nz=64)
    P = _problem(M, w)
    modes, mults = MODES2[:3], MULTS2[:4]
    B = M.Basis.fourier_angular(modes, mults, 2, order=-1, tl_scale=0.5)
    xs = [F.normal_field((64, 64), 100 + t) for t in range(2)]
    ys = [F.normal_field((64, 64), 110 + t) for t in range(2)]
    c, relres = M.probe_fit(P, B, [torch.from_numpy(y) for y in ys], [torch.from_numpy(x) for x in xs])
    cref, rref, _ = S.fit_with(lambda v: S.apply_paper_basis(v, w.h, modes, mults, -1, 0.5),
                               [y.astype(np.float64) for y in ys], [x.astype(np.float64) for x in xs])
    assert rel(c, cref) <= 1e-10
    assert abs(relres - rref) <= 1e-10 * rref
