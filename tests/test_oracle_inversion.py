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
