"""Pins of the curvelet and illumination oracle (Sec. 1.5, Sec. 2) against closed forms,
textbook ray geometry and an independent integrator."""
import numpy as np
import pytest

from oracle import curvelet as C

SHAPES = [(32, 64), (64, 64), (128, 32)]


def test_smooth_step():
    t = np.linspace(-0.5, 1.5, 201)
    np.testing.assert_allclose(C.smooth_step(t) + C.smooth_step(1 - t), 1.0, atol=1e-15)
    assert C.smooth_step(0.0) == 0.0 and C.smooth_step(1.0) == 1.0
    # flat ends: the first three derivatives vanish at 0 and 1
    e = 1e-3
    assert C.smooth_step(e) < 40 * e ** 4 and 1 - C.smooth_step(1 - e) < 40 * e ** 4


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("J,A1", [(2, 4), (3, 8), (4, 4)])
def test_windows_partition_unity(shape, J, A1):
    U = C.windows(*shape, J, A1)
    assert U.shape[0] == len(C.wedges(J, A1)) == 1 + sum(C.directions(j, A1) for j in range(1, J))
    np.testing.assert_allclose(np.sum(U ** 2, axis=0), 1.0, atol=1e-13)
    assert U.min() >= 0.0


@pytest.mark.parametrize("shape", SHAPES)
def test_tight_frame_reconstruction(shape):
    rng = np.random.default_rng(3)
    f = rng.standard_normal(shape)
    U = C.windows(*shape, 4, 8)
    coef = C.analysis(f, U)
    np.testing.assert_allclose(C.synthesis(coef, U), f, atol=1e-12)
    # Parseval for the undecimated frame: sum_w ||C_w||^2 = ||f||^2
    assert abs(np.sum(coef ** 2) - np.sum(f ** 2)) <= 1e-11 * np.sum(f ** 2)


def test_windows_even_and_atoms_real():
    nz, nx = 32, 64
    U = C.windows(nz, nx, 3, 8)
    flip = U[:, (-np.arange(nz)) % nz][:, :, (-np.arange(nx)) % nx]
    np.testing.assert_allclose(U, flip, atol=1e-15)
    atoms = np.fft.ifft2(U)
    assert np.max(np.abs(atoms.imag)) < 1e-15


def test_plane_wave_coefficients():
    """f = cos(2 pi (a x/nx + b z/nz)) has only the bins +-(b, a): C_w = U_w(b, a) f exactly."""
    nz, nx, a, b = 64, 64, 9, -5
    z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    f = np.cos(2 * np.pi * (a * x / nx + b * z / nz))
    U = C.windows(nz, nx, 4, 8)
    coef = C.analysis(f, U)
    for w in range(U.shape[0]):
        np.testing.assert_allclose(coef[w], U[w, b % nz, a % nx] * f, atol=1e-13)


def test_angular_window_centres_and_direction():
    for A in (4, 8, 16):
        for l in range(A):
            th = (l + 0.5) * np.pi / A
            assert abs(C.angular_window(th, l, A) - 1.0) < 1e-15
            assert C.angular_window(th, (l + 2) % A, A) == 0.0 if A > 3 else True
    # a plane wave's energy sits in the wedge whose direction is the wavevector's
    nz, nx = 64, 64
    U = C.windows(nz, nx, 4, 8)
    ws = C.wedges(4, 8)
    b, a = 12, 12   # 45 degrees, radius 12/32 * sqrt(2)
    energies = U[:, b, a] ** 2
    j, l, A = ws[int(np.argmax(energies))]
    assert j >= 1 and abs((l + 0.5) * np.pi / A - np.pi / 4) <= np.pi / A


def test_atom_norms_parseval():
    U = C.windows(32, 64, 3, 4)
    atoms = np.real(np.fft.ifft2(U))
    np.testing.assert_allclose(C.atom_norms(U), np.sqrt(np.sum(atoms ** 2, axis=(1, 2))), rtol=1e-13)


def test_trial_is_the_masked_synthesis():
    """The trial's coefficients are sigma ||phi_w|| z on the mask: analysing the atoms' span
    gives back the masked synthesis; a zero mask gives zero."""
    nz, nx = 32, 32
    U = C.windows(nz, nx, 3, 4)
    rng = np.random.default_rng(5)
    z = rng.standard_normal(U.shape)
    mask = (rng.random(U.shape) < 0.5).astype(np.uint8)
    y = C.trial(z, U, mask, sigma=2.0)
    ref = C.synthesis(2.0 * C.atom_norms(U)[:, None, None] * z * mask, U)
    np.testing.assert_allclose(y, ref, atol=1e-13)
    assert np.all(C.trial(z, U, np.zeros_like(mask)) == 0.0)


# ---- rays ----

def test_rays_straight_in_a_uniform_medium():
    h = 10.0
    med = C.Medium(np.full((40, 60), 2000.0), h)
    th = np.linspace(-1.2, 1.2, 9)
    dx, dz = np.sin(th), -np.cos(th)
    x0, z0 = np.full(9, 300.0), np.full(9, 350.0)
    ok, xc = C.trace_to_depth(med, x0, z0, dx, dz, 0.0)
    exp = x0 + z0 * np.tan(th)
    inside = (exp >= 0) & (exp <= 590.0)
    assert np.array_equal(ok, inside)
    np.testing.assert_allclose(xc[ok], exp[ok], atol=1e-9)


def test_rays_circular_arcs_in_a_linear_gradient():
    """c = c0 + g z: rays are circular arcs.  Snell's law keeps q = sin(phi)/c, phi from the
    upward vertical, and integrating dx = tan(phi) |dz| from the surface (c0) to z0 gives
    x_s - x0 = (sqrt(1 - q^2 c0^2) - sqrt(1 - q^2 c(z0)^2)) / (q g)."""
    h, c0, g = 10.0, 1500.0, 0.8
    nz, nx = 64, 128
    zz = np.arange(nz)[:, None] * h
    c = np.broadcast_to(c0 + g * zz, (nz, nx)).copy()
    med = C.Medium(c, h)
    phi = np.array([-0.9, -0.5, -0.2, 0.1, 0.4, 0.7])   # from the upward vertical
    x0, z0 = np.full(6, 640.0), np.full(6, 600.0)
    ok, xc = C.trace_to_depth(med, x0, z0, np.sin(phi), -np.cos(phi), 0.0, rtol=1e-6)
    q = np.sin(phi) / (c0 + g * z0)
    exp = x0 + (np.sqrt(1 - (q * c0) ** 2) - np.sqrt(1 - (q * (c0 + g * z0)) ** 2)) / (q * g)
    assert ok.all()
    np.testing.assert_allclose(xc, exp, atol=1e-3 * h)


def test_rays_against_an_independent_integrator():
    """A smooth random medium: the crossing points agree with scipy's RK45 (dense output,
    tight tolerances) to within the step control's position tolerance."""
    from scipy.integrate import solve_ivp
    h = 10.0
    rng = np.random.default_rng(7)
    from scipy.ndimage import gaussian_filter
    c = 2000.0 + 300.0 * gaussian_filter(rng.standard_normal((48, 64)), 6.0) / 0.05
    c = np.clip(c, 1500.0, 2600.0)
    med = C.Medium(c, h)
    phi = np.array([-0.6, -0.3, 0.0, 0.25, 0.5])
    x0, z0 = np.full(5, 320.0), np.full(5, 420.0)
    ok, xc = C.trace_to_depth(med, x0, z0, np.sin(phi), -np.cos(phi), 0.0, rtol=1e-6)
    for i in range(5):
        cc = med.eval(np.array([x0[i]]), np.array([z0[i]]))[0][0]
        y0 = [x0[i], z0[i], np.sin(phi[i]) / cc, -np.cos(phi[i]) / cc]

        def rhs(t, y):
            return C.ray_rhs(med, np.asarray(y)[:, None])[:, 0]

        ev = lambda t, y: y[1]
        ev.terminal, ev.direction = True, -1
        sol = solve_ivp(rhs, (0, 5.0), y0, method="RK45", rtol=1e-10, atol=1e-9, events=ev)
        assert sol.t_events[0].size == 1
        x_ref = sol.y_events[0][0][0]
        # scipy's ray is not confined to the box; ours stops where it leaves it
        assert ok[i] == (0.0 <= x_ref <= (64 - 1) * h)
        if ok[i]:
            assert abs(xc[i] - x_ref) < 0.01 * h
    assert ok.sum() >= 3


def test_uniform_visibility_matches_straight_lines():
    """In a uniform medium the traced mask is the straight-line fan of Sec. 2, and a node
    whose normal-incidence point lies well inside a shared source/receiver spread is
    visible while one whose rays all leave the spread is not."""
    h, nz, nx = 10.0, 32, 64
    src = np.array([[20, 0], [40, 0]])
    rec = np.stack([np.arange(16, 49), np.zeros(33, int)], 1)
    J, A1, stride, nfan = 3, 8, 4, 6
    traced = C.visibility(np.full((nz, nx), 1800.0), h, src, rec, J, A1, stride, nfan)
    closed = C.straight_visibility(h, nz, nx, src, rec, J, A1, stride, nfan)
    assert np.array_equal(traced, closed)
    dirs = C.direction_set(J, A1)
    zi, xi = C.mask_nodes(nz, stride), C.mask_nodes(nx, stride)
    # node under the spread's centre, normal near vertical (theta near pi/2): visible
    a, b = 5, int(np.argmin(np.abs(xi - 30)))
    d = int(np.argmin([abs((l + 0.5) * np.pi / A - np.pi / 2) for A, l in dirs]))
    assert closed[d, a, b]
    # node at the left edge, normal tilted further left: every ray pair misses the spread
    b = 0
    d = int(np.argmin([abs((l + 0.5) * np.pi / A - 0.2) for A, l in dirs]))   # normal up-left
    assert not closed[d, a, b]


def test_expand_mask_layout():
    vis = np.zeros((len(C.direction_set(3, 4)), 2, 3), dtype=bool)
    vis[1, 0, 2] = True
    m = C.expand_mask(vis, 3, 4, 8, 12, 4)
    assert m.shape == (len(C.wedges(3, 4)), 8, 12)
    # wedge (1, 1) uses direction (4, 1); the lowpass any of band 1
    w = C.wedges(3, 4).index((1, 1, 4))
    assert m[w, :4, 8:].all() and m[w].sum() == 16
    assert m[0, :4, 8:].all() and m[0].sum() == 16
