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


def _adjoint_by_parts(P, s, d, shift=0):
    """The image of shot s summed by parts in time: -sum_k u^{k-shift} c^2 (L nu^{k+1} + R^T d^{k-1}).

    The GPU path images in this form when it recomputes the background from
    checkpoints (the rounding of a stored level then enters without the
    Laplacian).  u^k are the oracle's own background levels, nu the adjoint
    recurrence; shift=1 plants an off-by-one in the level index.
    """
    snaps = {}
    P.background(s, keep_g=False, snapshots=snaps)
    snaps[-1] = np.zeros(P.c_pad.shape)
    nu1 = np.zeros(P.c_pad.shape)
    nu2 = np.zeros(P.c_pad.shape)
    img = np.zeros(P.w.model_shape)
    for k in range(P.nt, 0, -1):
        lam = laplacian(nu1, P.h, P.nd)
        np.add.at(lam, P.rec, d[k - 1])
        nu = P.a * (2.0 * nu1 + P.kappa * lam) - P.b * nu2
        img -= P.restrict(snaps[k - shift] * P.csq * lam)
        nu2, nu1 = nu1, nu
    return img


def test_adjoint_summed_by_parts_equals_the_transpose(small):
    """-sum_k g^{k-1} nu^k = -sum_k u^k c^2 (L nu^{k+1} + R^T d^{k-1}) on the model grid.

    Summation by parts of the second difference u^{k} - 2u^{k-1} + u^{k-2} = dt^2 g^{k-1}
    (the model grid carries no damping), with u^0 = u^{-1} = 0 and nu^{nt+1} =
    nu^{nt+2} = 0, turns one form into the other; a level index off by one fails.
    """
    P = small
    d = F.normal_field((len(P.src), P.nt, len(P.rec[0])), 23).astype(np.float64)
    for s in range(len(P.src)):
        g, _ = P.background(s)
        ref = P.adjoint(s, d[s], g)
        byparts = _adjoint_by_parts(P, s, d[s])
        assert np.linalg.norm(byparts - ref) <= 1e-12 * np.linalg.norm(ref)
        off = _adjoint_by_parts(P, s, d[s], shift=1)
        assert np.linalg.norm(off - ref) > 1e-2 * np.linalg.norm(ref)


# ------------------------------------------------------- absorbing layer --
#
# The layer is defined (a reading: the paper names a PML of width .15N) as a
# damping term eta u_t with eta = eta_max (d / nb)^2 at distance d cells into
# the layer, eta_max = 3 c_max ln(1/R) / (2 nb h), c_max the background's
# maximum.  Two pins tie the oracle's time stepping to that definition through
# what the damped wave equation u_tt + eta u_t = c^2 Lap u fixes: an exact
# discrete energy balance and the WKB attenuation of a plane-wave pulse.

def _stated_eta(P, R):
    """eta on the propagation grid from the definition above (not from the oracle)."""
    nb, h = P.nb, P.h
    eta_max = 3.0 * float(np.max(P.c_model)) * np.log(1.0 / R) / (2.0 * nb * h)
    eta = np.zeros(P.c_pad.shape)
    for ax, n in enumerate(P.w.model_shape):
        i = np.arange(n + 2 * nb)
        d = np.where(i < nb, nb - i, np.where(i >= n + nb, i - (n + nb - 1), 0))
        eta = eta + (eta_max * (d / nb) ** 2).reshape([-1 if k == ax else 1 for k in range(P.nd)])
    return eta


def _plant_eta_scale(P, scale):
    """Plant a mistake in the oracle object: its damping profile times ``scale``."""
    eta = P.eta * scale
    P.a = 1.0 / (1.0 + eta * P.dt / 2.0)
    P.b = (1.0 - eta * P.dt / 2.0) * P.a


def _energy_balance_error(P, R, nt=120):
    """max over steps of |E(n+1/2) - E(n-1/2) + dt/2 sum eta (u+ - u-)^2 / kappa| / E0.

    For u+ = a (2u + kappa L u) - b u- with a = 1/(1 + eta dt/2),
    b = (1 - eta dt/2) a, multiplying the scheme by (u+ - u-)/kappa and summing
    (L symmetric) gives E(n+1/2) - E(n-1/2) = -(dt/2) sum eta (u+ - u-)^2 / kappa
    with E(n+1/2) = sum (u+ - u)^2 / kappa - sum u+ L u, exactly.
    """
    rng = np.random.default_rng(17)
    u0 = rng.standard_normal(P.c_pad.shape)
    snaps = {-1: u0, 0: u0 + 0.05 * rng.standard_normal(P.c_pad.shape)}
    P.nt = nt
    P.background(0, keep_g=False, snapshots=snaps, source=False)
    eta = _stated_eta(P, R)
    e = [_energy(P, snaps[n + 1], snaps[n]) for n in range(-1, nt)]     # E(n + 1/2)
    worst = 0.0
    for n in range(0, nt):
        drop = 0.5 * P.dt * np.sum(eta * (snaps[n + 1] - snaps[n - 1]) ** 2 / P.kappa)
        worst = max(worst, abs(e[n + 1] - e[n] + drop))
    return worst / abs(e[0])


@pytest.mark.parametrize("nb,R", [(8, 1e-3), (12, 1e-2)])
def test_sponge_exact_discrete_energy_balance(nb, R):
    """Energy lost per step = (dt/2) sum eta (u+ - u-)^2 / kappa with the stated eta.

    A smooth random medium makes c_max (which sets eta_max) differ from the
    local c in kappa; a wrong eta_max, profile exponent, distance origin or
    damping form (a, b) breaks the identity far above rounding.
    """
    w = F.tiny(n=20, nb=nb, nt=120, ns=1, nr=2, kind="smooth_random").with_(sponge_R=R)
    P = Problem(w, F.medium(w))
    assert _energy_balance_error(P, R) < 1e-11
    _plant_eta_scale(P, 1.5)
    assert _energy_balance_error(P, R) > 1e-4


def _plane_wave_round_trip(nb, R, eta_scale=1.0, kh=1.0, courant=0.2, nx=240, nz=100,
                           c=2000.0, h=10.0):
    """Ratio of the reflected to the incident L2 norm of a downgoing plane pulse.

    The pulse (carrier kh, Gaussian envelope of 8 cells) starts 30 cells below
    the top of the model, is recorded 50 cells deep, crosses the bottom layer,
    reflects from the zero exterior and comes back.  The model is wide enough
    that nothing from the side layers reaches the recording column in time, so
    the column sees the 1D problem.
    """
    dt = courant * h / c
    z0, zr = 30, 50
    dist = (nz - zr) + nb + 1                      # recording depth to the first exterior cell
    nt = int(((2 * dist + 40) * h / c) / dt)
    w = Workload(name="sponge", ndim=2, nx=nx, nz=nz, h=h, nb=nb, dt=dt, nt=nt, f_peak=10.0,
                 src=np.array([[nx // 2, 0]], np.int32), rec=np.array([[nx // 2, zr]], np.int32),
                 medium=dict(kind="constant", c=c), sponge_R=R)
    P = Problem(w, F.medium(w))
    if eta_scale != 1.0:
        _plant_eta_scale(P, eta_scale)
    zz = np.arange(nz + 2 * nb) - nb - float(z0)

    def pulse(shift):
        s = zz - shift
        return np.repeat((np.exp(-0.5 * (s / 8.0) ** 2) * np.cos(kh * s))[:, None],
                         P.c_pad.shape[1], axis=1)

    snaps = {-1: pulse(-c * dt / h), 0: pulse(0.0)}      # moving down at speed c
    _, tr = P.background(0, keep_g=False, snapshots=snaps, source=False)
    t = (np.arange(nt) + 1) * dt
    split = ((zr - z0) + dist) * h / c                 # between the two passes
    tr = tr[:, 0]
    return np.linalg.norm(tr[t >= split]) / np.linalg.norm(tr[t < split])


def _local_decay(eta, kh, courant, c, h):
    """Im k h of the damped scheme's plane wave at the pulse's frequency, for each eta.

    Discrete dispersion relation of u+ = a(2u + kappa L u) - b u- for
    u = exp(i(k x - w t)): -(4/dt^2) sin^2(w dt/2) - i eta sin(w dt)/dt = c^2 sigma(k),
    sigma(k) = h^-2 (w0 + 2 sum_j w_j cos(j k h)), solved for complex k by Newton.
    """
    dt = courant * h / c
    jj = np.arange(1, 5)

    def sig(k):
        return (FD8[0] + 2 * np.sum(FD8[1:] * np.cos(jj * k * h))) / h ** 2

    def dsig(k):
        return -2 * np.sum(FD8[1:] * jj * h * np.sin(jj * k * h)) / h ** 2

    k0 = kh / h
    om = 2.0 / dt * np.arcsin(np.sqrt(-c * c * sig(k0) * dt * dt / 4.0))
    out = []
    for e in np.atleast_1d(eta):
        rhs = -(4.0 / dt ** 2) * np.sin(om * dt / 2) ** 2 - 1j * e * np.sin(om * dt) / dt
        k = complex(k0)
        for _ in range(60):
            k = k - (c * c * sig(k) - rhs) / (c * c * dsig(k))
        out.append(k.imag * h)
    return np.array(out)


@pytest.mark.parametrize("nb", [20, 40])
def test_sponge_wkb_round_trip_attenuation(nb):
    """Round trip through the layer attenuates as exp(-2 sum_d Im k_d h) (WKB).

    Im k_d is the local decay of the damped scheme at each layer cell
    d = 1..nb; for eta << omega it is eta_d / (2c), so the exponent is close to
    sum_d eta_d h / c.  The zero exterior acts as the reflecting wall somewhere
    in the first exterior cell, whose share is not fixed by WKB: the measured
    exponent (relative to the same run with R = 1, i.e. no damping, which
    measures the wall's own reflection) must lie between the sum over the
    layer's cells and that sum plus one exterior cell's round trip.  Measured:
    the wall sits 0.40 of a cell out for both widths.  A damping 1.5 times too
    strong, or a linear or cubic profile, falls far outside.
    """
    R, c, h, kh, courant = 1e-3, 2000.0, 10.0, 1.0, 0.2
    eta_max = 3.0 * c * np.log(1.0 / R) / (2.0 * nb * h)
    d = np.arange(1, nb + 2)
    decay = _local_decay(eta_max * (d / nb) ** 2, kh, courant, c, h)
    lo = 2.0 * np.sum(decay[:nb])
    hi = lo + 2.0 * decay[nb]
    wall = _plane_wave_round_trip(nb, 1.0)
    assert abs(wall - 1.0) < 1e-3                      # undamped: the wall reflects all
    got = -np.log(_plane_wave_round_trip(nb, R) / wall)
    assert lo <= got <= hi, (lo, got, hi)
    # the simple WKB estimate sum eta h / c is within 5 % of the measured exponent
    simple = np.sum(eta_max * (d[:nb] / nb) ** 2) * h / c
    assert abs(got / simple - 1.0) < 0.05
    planted = -np.log(_plane_wave_round_trip(nb, R, eta_scale=1.5) / wall)
    assert planted > hi + 0.5
