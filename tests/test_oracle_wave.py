"""Pins of the FP64 oracle's wave operators against what the mathematics fixes.

Each pin is chosen so that a plausible slip in the oracle (a wrong stencil
weight, a dropped factor in the leapfrog, a wrong source scaling or time
alignment, a sign error in the Born source, an off-by-one in the adjoint)
fails at least one of them.
"""
import numpy as np
import pytest

import fixtures as F
from fixtures.configs import Workload
from oracle import FD8, Problem, cfl_limit, laplacian, ricker
from oracle.green import green2d, green3d


# ---------------------------------------------------------------- stencil --

@pytest.mark.parametrize("k", range(0, 11))
def test_fd8_exact_on_polynomials_up_to_degree_9(k):
    """8th-order central second difference is exact for x^k, k <= 9, and not for k = 10."""
    x = np.arange(-10, 11, dtype=np.float64) + 1.0      # point index 10 is x = 1
    lap = laplacian(x ** k, 1.0, 1)
    exact = k * (k - 1) * 1.0 ** max(k - 2, 0) if k >= 2 else 0.0
    if k <= 9:
        assert abs(lap[10] - exact) <= 1e-9 * max(1.0, abs(exact))
    else:
        assert abs(lap[10] - exact) > 1e-3


def test_fd8_2d_sums_axes_and_scales_with_h():
    h = 2.5
    z = (np.arange(21) - 10.0) * h
    x = (np.arange(23) - 11.0) * h
    Z, X = np.meshgrid(z, x, indexing="ij")
    u = Z ** 3 * X ** 2 + 0.5 * X ** 4
    lap = laplacian(u, h, 2)
    exact = 6 * Z * X ** 2 + 2 * Z ** 3 + 6 * X ** 2
    core = (slice(4, -4), slice(4, -4))
    np.testing.assert_allclose(lap[core], exact[core], rtol=1e-10, atol=1e-8)


def test_fd8_nyquist_symbol():
    """Symbol at the Nyquist wavenumber is -2048/315 h^-2 per axis (closed form)."""
    h = 3.0
    n = 40
    u = (-1.0) ** np.arange(n)
    lap = laplacian(u, h, 1)
    assert abs(lap[n // 2] / u[n // 2] - (-2048.0 / 315.0) / h ** 2) < 1e-12
    assert abs(FD8[0] + 2 * sum(FD8[j] * (-1) ** j for j in range(1, 5)) + 2048 / 315) < 1e-14


def test_laplacian_is_symmetric_with_zero_exterior():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((13, 17))
    b = rng.standard_normal((13, 17))
    lhs = np.sum(laplacian(a, 1.7, 2) * b)
    rhs = np.sum(a * laplacian(b, 1.7, 2))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------- wavelet --

def test_ricker_shape():
    f = 12.0
    t0 = 1.0 / f
    dt = t0 / 1000.0
    w = ricker(f, t0, dt, 3000)
    n0 = 1000
    assert abs(w[n0] - 1.0) < 1e-12
    assert abs(w.argmax() - n0) <= 1
    zc = 1.0 / (np.sqrt(2.0) * np.pi * f)     # zero crossings at t0 +- zc
    for t in (t0 - zc, t0 + zc):
        val = (1 - 2 * (np.pi * f * (t - t0)) ** 2) * np.exp(-(np.pi * f * (t - t0)) ** 2)
        assert abs(val) < 1e-14
        assert abs(ricker(f, t0 - t, 1.0, 1)[0]) < 1e-12
    wl = ricker(f, 4.0 / f, dt, 8000)                 # zero mean over a long window
    assert abs(np.sum(wl) * dt) < 1e-12


# ---------------------------------------------------------- time stepping --

def _free_problem(n=24, nb=0, c=2000.0, h=10.0, courant=0.4, nt=400):
    dt = courant * h / c
    w = Workload(name="free", ndim=2, nx=n, nz=n, h=h, nb=nb, dt=dt, nt=nt,
                 f_peak=0.25 / dt, src=np.array([[n // 2, n // 2]], np.int32),
                 rec=np.array([[n // 3, n // 3]], np.int32),
                 medium=dict(kind="constant", c=c))
    return Problem(w, F.medium(w))


@pytest.mark.parametrize("factor,blows", [(0.97, False), (1.03, True)])
def test_cfl_limit(factor, blows):
    """The undamped leapfrog is stable just below c dt/h = 2/sqrt(2*2048/315), unstable above."""
    P = _free_problem(courant=factor * cfl_limit(2), nt=600)
    snaps = {}
    P.background(0, keep_g=False, snapshots=snaps)
    peak_early = np.max(np.abs(snaps[100]))
    peak_late = np.max(np.abs(snaps[600]))
    if blows:
        assert peak_late > 1e6 * peak_early
    else:
        assert peak_late < 10 * peak_early
    assert abs(cfl_limit(2) - 0.5546) < 1e-4 and abs(cfl_limit(3) - 0.4529) < 1e-4


def _energy(P, u_next, u):
    du = u_next - u
    return np.sum(du * du / P.kappa) - np.sum(u_next * laplacian(u, P.h, P.nd))


def test_leapfrog_conserves_discrete_energy_without_damping():
    """With eta = 0 and no source, E = <(u+ - u)^2 / kappa> - <u+, L u> is invariant."""
    P = _free_problem(nb=0, nt=300)
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(P.c_pad.shape)
    snaps = {-1: u0, 0: u0 + 0.01 * rng.standard_normal(P.c_pad.shape)}
    P.background(0, keep_g=False, snapshots=snaps, source=False)
    e = [_energy(P, snaps[n + 1], snaps[n]) for n in range(0, 300, 10)]
    assert np.max(np.abs(np.array(e) - e[0])) < 1e-10 * abs(e[0])


def test_sponge_dissipates_energy():
    P = _free_problem(n=24, nb=10, nt=300)
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal(P.c_pad.shape)
    snaps = {-1: u0, 0: u0}
    P.background(0, keep_g=False, snapshots=snaps, source=False)
    e = np.array([_energy(P, snaps[n + 1], snaps[n]) for n in range(0, 300)])
    assert np.all(np.diff(e) <= 1e-9 * e[0])
    assert e[-1] < 0.5 * e[0]
    # no damping inside the model region
    ms = P.model_slice
    assert np.all(P.a[ms] == 1.0) and np.all(P.b[ms] == 1.0)


# ---------------------------------------------- closed-form Green's function --

def _green_run(nd, dt, f, off, n, nb, c=2000.0, h=10.0, tmax=0.4):
    mid = n // 2
    src = np.array([[mid] * nd], np.int32)
    rec = np.array([[mid + off] + [mid] * (nd - 1)], np.int32)
    nt = int(round(tmax / dt))
    w = Workload(name="green", ndim=nd, nx=n, nz=n, ny=(n if nd == 3 else 1), h=h,
                 nb=nb, dt=dt, nt=nt, f_peak=f, src=src, rec=rec,
                 medium=dict(kind="constant", c=c))
    P = Problem(w, F.medium(w))
    _, tr = P.background(0, keep_g=False)
    t = (np.arange(nt) + 1) * dt           # trace n holds u^{n+1} <-> t_{n+1}

    def wav(tt):
        tt = np.asarray(tt, dtype=np.float64)
        a = (np.pi * f * (tt - 1.0 / f)) ** 2
        return np.where(tt >= 0.0, (1 - 2 * a) * np.exp(-a), 0.0)

    exact = (green2d if nd == 2 else green3d)(wav, off * h, c, t)
    return np.linalg.norm(tr[:, 0] - exact) / np.linalg.norm(exact)


def test_green_2d_second_order_in_time():
    e1 = _green_run(2, 2e-3, 10.0, 20, 121, 10)
    e2 = _green_run(2, 1e-3, 10.0, 20, 121, 10)
    assert e2 < 3e-3
    assert 3.5 < e1 / e2 < 4.5


def test_green_3d_second_order_in_time():
    e1 = _green_run(3, 2e-3, 15.0, 8, 41, 12, tmax=0.2)
    e2 = _green_run(3, 1e-3, 15.0, 8, 41, 12, tmax=0.2)
    assert e2 < 5e-3
    assert 3.5 < e1 / e2 < 4.5


# -------------------------------------------------------- Born and adjoint --

@pytest.fixture(scope="module")
def small():
    w = F.tiny(n=20, nb=8, nt=220, ns=2, nr=10, kind="smooth_random")
    c = F.medium(w)
    return Problem(w, c)


def test_born_is_the_jacobian_of_modelling(small):
    """(F[m0 + e dm] - F[m0 - e dm]) / 2e -> F dm with an O(e^2) error (Sec. 1.1, Sec. 2)."""
    P = small
    dm = F.normal_field(P.w.model_shape, 5).astype(np.float64)
    m0 = 1.0 / P.c_pad ** 2
    dm = dm * 0.02 * float(np.mean(m0))
    born = P.apply_F(dm)
    errs = []
    for eps in (1.0, 0.5, 0.25):
        plus = P.model_data(m0 + eps * P.extend(dm))
        minus = P.model_data(m0 - eps * P.extend(dm))
        fd = (plus - minus) / (2 * eps)
        errs.append(np.linalg.norm(fd - born) / np.linalg.norm(born))
    assert errs[-1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_born_sign_against_nonlinear_first_order(small):
    P = small
    dm = np.zeros(P.w.model_shape)
    dm[10, 10] = 1e-3 * float(np.mean(1.0 / P.c_pad ** 2))
    m0 = 1.0 / P.c_pad ** 2
    lin = P.apply_F(dm)
    non = P.model_data(m0 + P.extend(dm)) - P.model_data(m0)
    assert np.sum(lin * non) > 0.99 * np.linalg.norm(lin) * np.linalg.norm(non)


def test_dot_product_adjoint(small):
    """<F m, d> = <m, F* d> to rounding (FP64)."""
    P = small
    m = F.normal_field(P.w.model_shape, 7).astype(np.float64)
    d = F.normal_field((len(P.src), P.nt, len(P.rec[0])), 8).astype(np.float64)
    lhs = np.sum(P.apply_F(m) * d)
    rhs = np.sum(m * P.apply_Fadj(d))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_adjoint_index_check_single_step():
    """Nt = 1: nu^1 = a kappa R^T d^0 and F* d = -g^0 nu^1."""
    w = F.tiny(n=12, nb=4, nt=1, ns=1, nr=3)
    P = Problem(w, F.medium(w))
    d = np.array([[[1.0, -2.0, 0.5]]])
    g, _ = P.background(0)
    img = P.apply_Fadj(d)
    inj = np.zeros(P.c_pad.shape)
    np.add.at(inj, P.rec, d[0, 0])
    expect = -g[0] * P.restrict(P.a * P.kappa * inj)
    np.testing.assert_allclose(img, expect, rtol=1e-14, atol=0)


def test_H_symmetric_psd_and_shot_additive(small):
    P = small
    a = F.normal_field(P.w.model_shape, 11).astype(np.float64)
    b = F.normal_field(P.w.model_shape, 12).astype(np.float64)
    Ha = P.apply_H(a)
    Hb = P.apply_H(b)
    assert abs(np.sum(Ha * b) - np.sum(a * Hb)) <= 1e-13 * abs(np.sum(Ha * b))
    assert np.sum(Ha * a) > 0
    parts = [P.apply_H(a, shots=[s]) for s in range(len(P.src))]
    np.testing.assert_allclose(sum(parts), Ha, rtol=1e-13, atol=1e-13 * np.max(np.abs(Ha)))
    # batch axis gives the same as one at a time
    both = P.apply_H(np.stack([a, b]))
    np.testing.assert_allclose(both[1], Hb, rtol=1e-13, atol=1e-13 * np.max(np.abs(Hb)))


def test_fused_H_equals_adjoint_of_born_data(small):
    P = small
    a = F.normal_field(P.w.model_shape, 13).astype(np.float64)
    np.testing.assert_allclose(P.apply_Fadj(P.apply_F(a)), P.apply_H(a), rtol=1e-12,
                               atol=1e-12 * np.max(np.abs(P.apply_H(a))))
