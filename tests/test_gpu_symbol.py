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


# ---- the 256^3 workload's basis: Legendre P_i(z~) P_j(y~) P_k(x~), i + j + k <= 2, times rho^0..3 ----

C5LEG = F.c5().legendre          # 10 position factors (numpy axis order z, y, x)
C5QS = F.c5().qs                 # (0, 1, 2, 3): p = 40


def _cube_problem(M, n, dtype):
    return M.Problem.from_spec(F.tiny(ndim=3, n=n, nb=4, nt=10, ns=1, nr=2, dtype=dtype).with_(h=12.5))


@pytest.mark.parametrize("n", [32, 64])
def test_c5_basis_fit_exact_recovery_and_least_squares(n):
    """The 40-term 3D basis: y = sum c_i B_i x (oracle) gives c back to 1e-10 (FP64,
    two trials); on unrelated FP32 fields the fit matches the oracle's Householder
    least squares to 1e-10."""
    M = _gpu()
    h = 12.5
    assert len(C5LEG) == 10 and len(C5QS) * len(C5LEG) == 40
    P = _cube_problem(M, n, "f64")
    B = M.Basis(C5LEG, C5QS, 3)
    rng = np.random.default_rng(90 + n)
    ctrue = rng.standard_normal(B.p)
    xs = [F.normal_field((n, n, n), 300 + t).astype(np.float64) for t in range(2)]
    ys = [S.apply_Hinv(ctrue, x, h, C5LEG, C5QS) for x in xs]
    c, relres = M.probe_fit(P, B, [torch.from_numpy(y) for y in ys], [torch.from_numpy(x) for x in xs])
    assert np.max(np.abs(c - ctrue)) <= 1e-10 * np.max(np.abs(ctrue))
    assert relres < 1e-10
    P32 = _cube_problem(M, n, "f32")
    xs = [F.normal_field((n, n, n), 310 + t) for t in range(2)]
    ys = [F.normal_field((n, n, n), 320 + t) for t in range(2)]
    c, relres = M.probe_fit(P32, B, [torch.from_numpy(y) for y in ys], [torch.from_numpy(x) for x in xs])
    cref, rref, _ = S.fit([y.astype(np.float64) for y in ys], [x.astype(np.float64) for x in xs], h, C5LEG, C5QS)
    assert rel(c, cref) <= 1e-10
    assert abs(relres - rref) <= 1e-10 * rref


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c5_basis_apply_Hinv_matches_oracle_64(dtype):
    M = _gpu()
    P = _cube_problem(M, 64, dtype)
    B = M.Basis(C5LEG, C5QS, 3)
    c = np.random.default_rng(95).standard_normal(B.p)
    img = F.normal_field((64, 64, 64), 330)
    got = M.apply_Hinv(P, B, c, torch.from_numpy(img)).cpu().numpy()
    ref = S.apply_Hinv(c, img, 12.5, C5LEG, C5QS)
    assert rel(got, ref) <= (1e-13 if dtype == "f64" else 1e-6)


def _plane_waves(n, h, waves):
    """sum_w a_w cos(k_w . x + phi_w) on the n^3 model grid, and each wave's rho = |k| h / pi.

    waves: (m_z, m_y, m_x, a, phi) with integer frequency indices, so each term is a
    grid eigenfunction of every Fourier multiplier: B_(a,q) cos = P_a(x~) rho^q cos.
    """
    idx = np.arange(n, dtype=np.float64)
    rho = S.rho((n, n, n), h)
    out, terms = np.zeros((n, n, n)), []
    for mz, my, mx, a, phi in waves:
        th = (2 * np.pi / n) * (mz * idx[:, None, None] + my * idx[None, :, None] + mx * idx[None, None, :]) + phi
        term = a * np.cos(th)
        r = rho[mz % n, my % n, mx % n]
        terms.append((term, r))
        out += term
    return out, terms


def _closed_form(c, terms, n):
    """sum_(a,q) c_(a,q) P_a(x~) rho_w^q cos_w for each plane-wave term (no FFT)."""
    out = np.zeros((n, n, n))
    cc = np.asarray(c).reshape(len(C5LEG), len(C5QS))
    for ia, a in enumerate(C5LEG):
        s = np.zeros((n, n, n))
        for term, r in terms:
            s += sum(cc[ia, iq] * r ** q for iq, q in enumerate(C5QS)) * term
        out += S.position_factor(a, (n, n, n)) * s
    return out


def test_c5_apply_Hinv_full_size_plane_waves():
    """apply_Hinv at the workload's 256^3 (FP32, 3D FFT multipliers): plane waves are
    eigenfunctions of every multiplier, so the output has a closed form."""
    M = _gpu()
    n = 256
    P = _cube_problem(M, n, "f32")
    B = M.Basis(C5LEG, C5QS, 3)
    c = np.random.default_rng(97).standard_normal(B.p)
    img, terms = _plane_waves(n, 12.5, [(3, -7, 20, 1.0, 0.3), (-40, 11, 5, 0.5, 1.1), (90, 64, -100, 0.25, 2.0)])
    got = M.apply_Hinv(P, B, c, torch.from_numpy(img.astype(np.float32))).cpu().numpy()
    assert rel(got, _closed_form(c, terms, n)) <= 1e-6


def test_c5_fit_full_size_exact_recovery():
    """The fit at the workload's size: 4 trials of 256^3 (67 M stacked rows, p = 40),
    FP64.  Each trial is a sum of plane waves of distinct |k|; y_t = sum c_i B_i x_t in
    closed form; the fit returns c to 1e-10."""
    M = _gpu()
    n = 256
    P = _cube_problem(M, n, "f64")
    B = M.Basis(C5LEG, C5QS, 3)
    ctrue = np.random.default_rng(98).standard_normal(B.p)
    rng = np.random.default_rng(99)
    xs, ys = [], []
    for t in range(4):
        waves = []
        for j in range(6):
            m = rng.integers(-100, 101, size=3)
            waves.append((int(m[0]), int(m[1]), int(m[2]), float(rng.uniform(0.5, 1.0)), float(rng.uniform(0, 6.28))))
        x, terms = _plane_waves(n, 12.5, waves)
        xs.append(torch.from_numpy(x))
        ys.append(torch.from_numpy(_closed_form(ctrue, terms, n)))
    c, relres = M.probe_fit(P, B, ys, xs)
    print(f"256^3 fit, 4 trials, p = 40: max |c - c_true| / max |c_true| = "
          f"{np.max(np.abs(c - ctrue)) / np.max(np.abs(ctrue)):.2e}, relres {relres:.2e}")
    assert np.max(np.abs(c - ctrue)) <= 1e-10 * np.max(np.abs(ctrue))
    assert relres < 1e-10
