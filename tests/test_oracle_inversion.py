"""Pins of the oracle's inversion solvers and Krylov trial pairs on small dense SPD systems."""
import numpy as np

from oracle import inversion as I


def _spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def test_conjugate_gradient_solves_in_n_steps():
    A = _spd(12, 1)
    b = np.random.default_rng(2).standard_normal(12)
    x, norms = I.conjugate_gradient(lambda v: A @ v, b, 12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)
    assert norms[-1] < 1e-6 * norms[0]


def test_exact_preconditioner_converges_in_one_step():
    A = _spd(10, 3)
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(4).standard_normal(10)
    x, norms = I.conjugate_gradient(lambda v: A @ v, b, 1, precond=lambda v: Ainv @ v)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-10)


def test_steepest_descent_decreases_the_energy_and_converges():
    A = _spd(8, 5, cond=10.0)
    b = np.random.default_rng(6).standard_normal(8)
    f = lambda x: 0.5 * x @ A @ x - b @ x
    xs = [I.steepest_descent(lambda v: A @ v, b, k) for k in range(0, 40, 5)]
    energies = [f(x) for x in xs]
    assert all(e2 <= e1 + 1e-12 for e1, e2 in zip(energies, energies[1:]))
    # linear rate bound of steepest descent: ((kappa-1)/(kappa+1))^k in the energy norm
    x200 = I.steepest_descent(lambda v: A @ v, b, 200)
    np.testing.assert_allclose(x200, np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)


def test_krylov_pairs_and_relative_mse():
    A = _spd(6, 7)
    b = np.arange(6.0)
    pairs = I.krylov_pairs(lambda v: A @ v, b, 3)
    np.testing.assert_allclose(pairs[0][0], b)
    np.testing.assert_allclose(pairs[2][1], A @ A @ A @ b)
    np.testing.assert_allclose(pairs[1][0], pairs[0][1])
    assert I.relative_mse(2 * b, b) == 1.0
    assert I.relative_mse(b, b) == 0.0
    # a ratio of norms, not of squared norms: an error of half the reference's norm is 0.5
    e = np.zeros(6)
    e[0] = 0.5 * np.linalg.norm(b)
    assert abs(I.relative_mse(b + e, b) - 0.5) < 1e-15


# ---- Gauss-Newton on the wave-equation problem (Sec. 1.1), tiny grid ----

def _tiny_wave():
    import fixtures as F
    from oracle import Problem
    w = F.tiny(n=16, nr=16, nt=120, ns=2, dtype="f64", kind="smooth")
    c = F.medium(w)
    return w, c, (lambda cc: Problem(w, cc))


def _blob(w, c, amp, zc=0.35, xc=0.5, width=2.0):
    nz, nx = w.model_shape
    z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    m0 = 1.0 / np.asarray(c, np.float64) ** 2
    return amp * float(np.mean(m0)) * np.exp(-((z - zc * nz) ** 2 + (x - xc * nx) ** 2) / (2 * width ** 2))


def test_migrated_residual_is_minus_the_gradient_of_the_misfit():
    """b = F*(d - F[m0]) = -dJ/dm: a central difference of J along a direction v on the
    model grid (damping and the layer's velocity held, as in the Born map) matches -b.v:
    the sign and the pairing of modelling, Born and migration."""
    w, c0, at = _tiny_wave()
    P = at(c0)
    m_pad = 1.0 / P.c_pad ** 2
    d_obs = P.model_data(m_pad + P.extend(_blob(w, c0, 0.05)))
    r, J0 = I.misfit(P, c0, d_obs)
    b = P.apply_Fadj(r)
    v = _blob(w, c0, 1.0, zc=0.45, xc=0.4, width=2.5)
    eps = 1e-3
    Jp = 0.5 * np.sum((d_obs - P.model_data(m_pad + eps * P.extend(v))) ** 2)
    Jm = 0.5 * np.sum((d_obs - P.model_data(m_pad - eps * P.extend(v))) ** 2)
    fd = (Jp - Jm) / (2 * eps)
    assert J0 > 0
    assert abs(fd + float(np.sum(b * v))) <= 1e-4 * abs(fd)


def test_gauss_newton_step_is_zero_on_exact_data():
    w, c0, at = _tiny_wave()
    P = at(c0)
    d_obs = P.model_data(1.0 / P.c_pad ** 2)
    cs, Js = I.gauss_newton(at, c0, d_obs, 1, 3)
    assert Js[0] == 0.0
    # dm = 0 exactly; c -> (c^-2)^(-1/2) only rounds
    np.testing.assert_allclose(cs[1], c0, rtol=4e-16, atol=0)
    assert Js[1] <= 1e-24 * float(np.sum(d_obs ** 2))


def test_gauss_newton_lowers_the_misfit():
    """A weak, smooth perturbation: each Gauss-Newton step (three CG iterations) lowers J."""
    w, c0, at = _tiny_wave()
    m_true = 1.0 / c0 ** 2 + _blob(w, c0, 0.03)
    P = at(1.0 / np.sqrt(m_true))
    d_obs = P.model_data(1.0 / P.c_pad ** 2)
    cs, Js = I.gauss_newton(at, c0, d_obs, 2, 3)
    assert Js[1] < 0.5 * Js[0] and Js[2] < Js[1], Js
    err = [np.linalg.norm(1.0 / c ** 2 - m_true) for c in cs]
    assert err[2] < err[1] < err[0]


def test_gauss_newton_without_inner_iterations_applies_the_preconditioner():
    """inner = 0: the step is the preconditioner applied to the migrated residual; with
    three CG iterations as that preconditioner the iterates are those of inner = 3."""
    w, c0, at = _tiny_wave()
    P = at(1.0 / np.sqrt(1.0 / c0 ** 2 + _blob(w, c0, 0.03)))
    d_obs = P.model_data(1.0 / P.c_pad ** 2)
    cs3, Js3 = I.gauss_newton(at, c0, d_obs, 1, 3)
    cs0, Js0 = I.gauss_newton(at, c0, d_obs, 1, 0,
                              precond_at=lambda Q, b: (lambda v: I.conjugate_gradient(Q.apply_H, v, 3)[0]))
    np.testing.assert_array_equal(cs0[1], cs3[1])
    assert Js0 == Js3


def test_gauss_newton_line_search_step():
    """inner = 0 with line_search: the step minimises the quadratic model along the
    preconditioned direction; with the identity as preconditioner that is one exact
    steepest-descent step on H dm = b."""
    w, c0, at = _tiny_wave()
    P = at(1.0 / np.sqrt(1.0 / c0 ** 2 + _blob(w, c0, 0.03)))
    d_obs = P.model_data(1.0 / P.c_pad ** 2)
    c0 = c0.astype(np.float64)
    cs, _ = I.gauss_newton(at, c0, d_obs, 1, 0, precond_at=lambda Q, b: (lambda v: v), line_search=True)
    Q = at(c0)
    b = Q.apply_Fadj(I.misfit(Q, c0, d_obs)[0])
    dm = I.steepest_descent(Q.apply_H, b, 1)
    np.testing.assert_allclose(1.0 / cs[1] ** 2 - 1.0 / c0 ** 2, dm, rtol=1e-9, atol=1e-9 * np.abs(dm).max())
