"""Pins of the oracle's probing basis, fit and fitted-inverse application."""
import numpy as np
import pytest

import fixtures as F
from oracle import Problem
from oracle import symbol as S
from oracle.dense import basis_matrices, dense_H


def test_legendre_matches_library_and_orthogonality():
    t = np.linspace(-1, 1, 101)
    for n in range(7):
        ref = np.polynomial.legendre.legval(t, [0] * n + [1])
        np.testing.assert_allclose(S.legendre(n, t), ref, rtol=0, atol=1e-14)
    # Gauss-Legendre quadrature: int P_a P_b = 2/(2a+1) delta_ab
    x, wq = np.polynomial.legendre.leggauss(12)
    for a in range(5):
        for b in range(5):
            v = np.sum(wq * S.legendre(a, x) * S.legendre(b, x))
            assert abs(v - (2.0 / (2 * a + 1) if a == b else 0.0)) < 1e-13


def test_cell_centres():
    np.testing.assert_allclose(S.cell_centres(4), [-0.75, -0.25, 0.25, 0.75], atol=0)


def test_rho_is_one_at_nyquist_and_zero_at_dc():
    r = S.rho((8, 16), 10.0)
    assert r[0, 0] == 0.0
    assert abs(r[4, 0] - 1.0) < 1e-15 and abs(r[0, 8] - 1.0) < 1e-15
    assert abs(r[4, 8] - np.sqrt(2.0)) < 1e-15


def test_fft_against_brute_force_dft():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((8, 8))
    n = 8
    W = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    dft = W @ v @ W.T
    np.testing.assert_allclose(np.fft.fftn(v), dft, atol=1e-12)


def test_identity_and_pointwise_and_multiplier_eigenfunctions():
    shape = (16, 32)
    h = 5.0
    rng = np.random.default_rng(1)
    v = rng.standard_normal(shape)
    leg = [(0, 0), (1, 0), (2, 1)]
    qs = (0, 1, 2, 3)
    Bv = S.apply_basis(v, h, leg, qs)
    # B_(P0, 0) is the identity
    np.testing.assert_allclose(Bv[0], v, atol=1e-13)
    # B_(a, 0) is pointwise multiplication by P_a
    pz = S.legendre(2, S.cell_centres(16))[:, None] * S.legendre(1, S.cell_centres(32))[None, :]
    np.testing.assert_allclose(Bv[8], pz * v, atol=1e-13)
    # B_(P0, q) cos(k.x) = rho(k)^q cos(k.x) for grid wavenumbers
    jz, jx = 3, 5
    z = np.arange(16)[:, None]
    x = np.arange(32)[None, :]
    cosk = np.cos(2 * np.pi * (jz * z / 16 + jx * x / 32))
    rk = 2.0 * np.sqrt((jz / 16) ** 2 + (jx / 32) ** 2)
    Bc = S.apply_basis(cosk, h, [(0, 0)], qs)
    for q in qs:
        np.testing.assert_allclose(Bc[q], rk ** q * cosk, atol=1e-12)


def test_apply_Hinv_is_linear_combination():
    shape = (16, 16)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(shape)
    leg = [(0, 0), (1, 0)]
    qs = (0, 1, 2)
    c = rng.standard_normal(6)
    out = S.apply_Hinv(c, v, 10.0, leg, qs)
    Bv = S.apply_basis(v, 10.0, leg, qs)
    np.testing.assert_allclose(out, sum(c[i] * Bv[i] for i in range(6)), atol=1e-12)
    # linear in img
    v2 = rng.standard_normal(shape)
    np.testing.assert_allclose(S.apply_Hinv(c, v + 2 * v2, 10.0, leg, qs),
                               out + 2 * S.apply_Hinv(c, v2, 10.0, leg, qs), atol=1e-12)


@pytest.mark.parametrize("ntrial", [1, 2])
def test_fit_recovers_coefficients_exactly(ntrial):
    """If y = sum_i c_i B_i x exactly, the fit returns c (Sec. 1.4, exact expansion)."""
    shape = (32, 64)
    h = 10.0
    leg = [(a, 0) for a in range(5)]
    qs = (0, 1, 2, 3)
    rng = np.random.default_rng(3)
    ctrue = rng.standard_normal(len(leg) * len(qs))
    xs = [F.normal_field(shape, 30 + t).astype(np.float64) for t in range(ntrial)]
    ys = [S.apply_Hinv(ctrue, x, h, leg, qs) for x in xs]
    c, relres, deficient = S.fit(ys, xs, h, leg, qs)
    assert not deficient
    assert np.max(np.abs(c - ctrue)) <= 1e-10 * np.max(np.abs(ctrue))
    assert relres < 1e-12


def test_fit_rank_deficient_flagged():
    shape = (16, 16)
    x = F.normal_field(shape, 40).astype(np.float64)
    y = F.normal_field(shape, 41).astype(np.float64)
    # the same column twice -> exactly rank deficient
    c, relres, deficient = S.fit([y], [x], 10.0, [(0, 0), (0, 0)], (0,))
    assert deficient
    assert abs(c[0] - c[1]) < 1e-12


def test_fit_normal_equations_agree_with_qr():
    shape = (16, 32)
    leg = [(0, 0), (1, 0)]
    qs = (0, 1, 2)
    x = F.normal_field(shape, 42).astype(np.float64)
    y = F.normal_field(shape, 43).astype(np.float64)
    c, _, _ = S.fit([y], [x], 10.0, leg, qs)
    M, r = S.gram([x], [y], 10.0, leg, qs)
    np.testing.assert_allclose(np.linalg.solve(M, r), c, rtol=1e-9)


@pytest.fixture(scope="module")
def tinyH():
    w = F.tiny(n=16, nb=8, nt=200, ns=2, nr=16)
    P = Problem(w, F.medium(w))
    return P, dense_H(P)


def test_dense_H_symmetric_psd_and_matches_apply_H(tinyH):
    P, H = tinyH
    assert np.max(np.abs(H - H.T)) <= 1e-12 * np.max(np.abs(H))
    ev = np.linalg.eigvalsh(H)
    assert ev[0] >= -1e-12 * ev[-1]
    v = F.normal_field(P.w.model_shape, 50).astype(np.float64)
    np.testing.assert_allclose(P.apply_H(v).ravel(), H @ v.ravel(), rtol=0,
                               atol=1e-12 * np.max(np.abs(H @ v.ravel())))
    # epsilon-rank profile in the manner of the paper's Sec. 2.1 table (not comparable)
    sv = ev[::-1] / ev[-1]
    ranks = [int(np.sum(sv > e)) for e in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)]
    assert ranks == sorted(ranks) and ranks[-1] <= H.shape[0]


def test_expected_gram_is_trace_formula(tinyH):
    """E M_ij = Tr(H B_i^T B_j H) for y ~ N(0, I), x = H y (Sec. 1.4, Sec. 3.1)."""
    P, H = tinyH
    shape = P.w.model_shape
    leg = [(0, 0), (1, 0)]
    qs = (0, 1)
    B = basis_matrices(shape, P.h, leg, qs)
    p = B.shape[0]
    expect = np.array([[np.trace(H @ B[i].T @ B[j] @ H) for j in range(p)] for i in range(p)])
    K = 2000
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((K, H.shape[0]))
    X = Y @ H                                  # rows x_k = H y_k (H symmetric)
    BX = np.einsum("pij,kj->kpi", B, X)        # (K, p, n)
    Ms = np.einsum("kpi,kqi->kpq", BX, BX)
    mean = Ms.mean(axis=0)
    se = Ms.std(axis=0, ddof=1) / np.sqrt(K)
    assert np.all(np.abs(mean - expect) <= 4 * se + 1e-12 * np.abs(expect).max())
    # and the oracle's Gram routine gives the same M for one sample
    M1, _ = S.gram([X[0].reshape(shape)], [Y[0].reshape(shape)], P.h, leg, qs)
    np.testing.assert_allclose(M1, Ms[0], rtol=1e-10)


# ---- the paper's expansion (Fourier modes x angular harmonics x rational Chebyshev) ----

def test_rational_chebyshev_against_library():
    r = np.concatenate([np.linspace(0.0, 2.0, 41), [10.0, 1e3]])
    for L in (0.25, 0.5, 1.0):
        t = (r - L) / (r + L)
        for n in range(7):
            np.testing.assert_allclose(S.rational_chebyshev(n, r, L),
                                       np.polynomial.chebyshev.chebval(t, [0] * n + [1]), atol=1e-13)
            # TL_n(0) = T_n(-1) = (-1)^n, TL_n(L) = T_n(0) = cos(n pi / 2)
            assert abs(S.rational_chebyshev(n, 0.0, L) - (-1.0) ** n) < 1e-14
            assert abs(S.rational_chebyshev(n, L, L) - np.cos(n * np.pi / 2)) < 1e-14


def test_angular_2d_is_chebyshev_in_the_direction_cosine():
    shape, h = (8, 16), 10.0
    kz, kx = S.wavevector(shape, h)
    kn = np.hypot(kx, kz)
    c = np.where(kn > 0, kx / np.where(kn > 0, kn, 1), 0.0)
    s = np.where(kn > 0, kz / np.where(kn > 0, kn, 1), 0.0)
    np.testing.assert_allclose(S.angular(0, shape, h), 1.0)
    for j in range(1, 4):
        Tj = np.polynomial.chebyshev.chebval(c, [0] * j + [1])
        Uj1 = np.polynomial.chebyshev.chebval(c, np.polynomial.chebyshev.chebder([0] * j + [1])) / j
        np.testing.assert_allclose(S.angular(2 * j - 1, shape, h), np.where(kn > 0, Tj, 0.0), atol=1e-13)
        np.testing.assert_allclose(S.angular(2 * j, shape, h), np.where(kn > 0, s * Uj1, 0.0), atol=1e-13)


def test_angular_3d_spans_the_spherical_harmonics():
    from scipy.special import sph_harm_y
    shape, h = (6, 8, 10), 12.5
    kz, ky, kx = S.wavevector(shape, h)
    kn = np.sqrt(kx * kx + ky * ky + kz * kz)
    m = kn > 0
    pol = np.arccos(np.clip(kz[m] / kn[m], -1, 1))
    azi = np.arctan2(ky[m], kx[m])
    ours = {0: [0], 1: [1, 2, 3], 2: [4, 5, 6, 7, 8]}
    for l, idx in ours.items():
        ref = []
        for mm in range(-l, l + 1):
            y = sph_harm_y(l, mm, pol, azi)
            ref += [y.real, y.imag]
        R = np.stack(ref, 1)
        Ours = np.stack([S.angular(i, shape, h)[m] for i in idx], 1)
        # each of ours lies in the span of the library's degree-l harmonics, and they span it
        coef, *_ = np.linalg.lstsq(R, Ours, rcond=None)
        assert np.linalg.norm(R @ coef - Ours) <= 1e-10 * np.linalg.norm(Ours)
        assert np.linalg.matrix_rank(Ours, tol=1e-8) == 2 * l + 1


def test_fourier_factor_is_a_dct_ii_mode():
    from scipy.fft import dct
    n = 16
    rng = np.random.default_rng(3)
    v = rng.standard_normal(n)
    y = dct(v, type=2)
    for mm in range(n // 2):
        got = np.sum(v * S.fourier_factor((mm, 0), (n,)))
        assert abs(got - (-1) ** mm * y[2 * mm] / 2) < 1e-12
    # sin modes: sin(pi m x~) at the cell centres against the definition of x~
    np.testing.assert_allclose(S.fourier_factor((3, 1), (n,)), np.sin(3 * np.pi * (np.arange(n) + 0.5) * 2 / n - 3 * np.pi),
                               atol=1e-13)


def test_paper_basis_plane_wave_response():
    """B_(const, mult) cos(k.x) = (m(k) + m(-k))/2 cos(k.x), m from the library forms."""
    shape, h, L = (16, 32), 5.0, 0.5
    jz, jx = 3, 5
    z = np.arange(shape[0])[:, None]
    x = np.arange(shape[1])[None, :]
    wave = np.cos(2 * np.pi * (jz * z / shape[0] + jx * x / shape[1]))
    kx, kz = 2 * np.pi * jx / (shape[1] * h), 2 * np.pi * jz / (shape[0] * h)
    r = np.hypot(kx, kz) * h / np.pi
    th = np.arctan2(kz, kx)
    for (a, q2), order in [((0, 2), 1), ((1, 0), 1), ((2, 3), -1), ((4, 1), 0), ((3, 2), 1)]:
        tl = np.polynomial.chebyshev.chebval((r - L) / (r + L), [0] * q2 + [1])
        def ang(t):
            if a == 0:
                return 1.0
            j = (a + 1) // 2
            return np.cos(j * t) if a % 2 else np.sin(j * t)
        mk = ang(th) * tl * r ** order
        mmk = ang(th + np.pi) * tl * r ** order
        Bv = S.apply_paper_basis(wave, h, [(0, 0, 0)], [(a, q2)], order, L)[0]
        np.testing.assert_allclose(Bv, 0.5 * (mk + mmk) * wave, atol=1e-12)


@pytest.mark.parametrize("ndim", [2, 3])
def test_paper_basis_fit_recovers_coefficients(ndim):
    rng = np.random.default_rng(11 + ndim)
    shape = (8, 16) if ndim == 2 else (4, 8, 8)
    h, L, order = 10.0, 0.5, 1
    modes = [(0,) * ndim + (0,), (1,) + (0,) * (ndim - 1) + (0,), (0,) * (ndim - 1) + (1, 1)]
    mults = [(0, 0), (1, 1), (2, 0), (0, 2)] if ndim == 2 else [(0, 0), (3, 1), (6, 0), (0, 2)]
    c_true = rng.standard_normal(len(modes) * len(mults))
    xs = [rng.standard_normal(shape) for _ in range(2)]
    ys = [np.tensordot(c_true, S.apply_paper_basis(x, h, modes, mults, order, L), axes=1) for x in xs]
    c, relres, deficient = S.fit_with(lambda v: S.apply_paper_basis(v, h, modes, mults, order, L), ys, xs)
    assert not deficient and relres < 1e-12
    np.testing.assert_allclose(c, c_true, atol=1e-9)
