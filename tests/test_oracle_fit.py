"""Pins of the oracle's fitting loops: SplitMix64 against its published test
vector; the particle swarm on a concave quadratic (finds the maximum, keeps
every particle in the box, never loses its best); L-BFGS on a quadratic (the
solution of the linear system), on Rosenbrock's function (its minimum, and
SciPy's L-BFGS-B) and against an active bound."""
import numpy as np
from scipy.optimize import minimize

import oracle as O


def test_splitmix64_published_vector():
    # the first five outputs of the reference generator seeded with 1234567
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
              16408922859458223821]
    assert [O.splitmix64(1234567, i) for i in range(5)] == expect


def test_uniform_range_and_moments():
    u = np.array([O.uniform(99, i) for i in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1.0 / 12.0) < 0.005


def test_pso_finds_the_maximum_of_a_quadratic_and_stays_in_the_box():
    c = np.array([0.3, -1.2, 2.5])
    lo, hi = np.array([-2.0, -2.0, 0.0]), np.array([2.0, 1.0, 3.0])
    seen = []

    def f(x):
        seen.append(x.copy())
        return -np.sum((x - c) ** 2, axis=1)

    best, fbest, hist = O.pso(f, lo, hi, N=30, n_iter=120, seed=7)
    np.testing.assert_allclose(best, c, atol=1e-4)
    assert np.all(np.diff(hist) >= 0.0)
    allx = np.concatenate(seen)
    assert np.all(allx >= lo) and np.all(allx <= hi)


def test_pso_maximum_on_the_bound():
    best, _, _ = O.pso(lambda x: x[:, 0] + x[:, 1], [0.0, 0.0], [1.0, 2.0], N=10, n_iter=40, seed=3)
    np.testing.assert_allclose(best, [1.0, 2.0], atol=1e-12)


def test_lbfgs_solves_a_quadratic():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    A = Q @ np.diag(np.logspace(0, 2, 6)) @ Q.T
    b = rng.normal(size=6)
    F = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    x, fx, it = O.lbfgs(F, np.zeros(6), np.full(6, -1e3), np.full(6, 1e3), ftol=0.0, gtol=1e-10)
    # it stops once F no longer changes in double precision, which fixes x to ~sqrt(eps)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-7, atol=1e-7)
    assert it <= 40


def test_lbfgs_rosenbrock_minimum_and_scipy():
    def F(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
        return f, g

    x, fx, it = O.lbfgs(F, [-1.2, 1.0], [-5, -5], [5, 5], max_iter=500, ftol=0.0, gtol=1e-9)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-7)
    ref = minimize(lambda z: F(z)[0], [-1.2, 1.0], jac=lambda z: F(z)[1], method="L-BFGS-B",
                   options={"gtol": 1e-12, "ftol": 0.0, "maxiter": 1000})
    np.testing.assert_allclose(x, ref.x, atol=1e-5)


def test_lbfgs_active_bound():
    F = lambda x: ((x[0] - 2.0) ** 2 + (x[1] + 0.5) ** 2, np.array([2 * (x[0] - 2.0), 2 * (x[1] + 0.5)]))
    x, fx, _ = O.lbfgs(F, [0.2, 0.3], [0.0, -1.0], [1.0, 1.0])
    np.testing.assert_allclose(x, [1.0, -0.5], atol=1e-9)


def test_lbfgs_holds_fixed_coordinates():
    # a coupled quadratic with coordinate 2 fixed (equal bounds): the free
    # coordinates solve the reduced system
    rng = np.random.default_rng(4)
    M = rng.normal(size=(5, 5))
    A = M @ M.T + 5 * np.eye(5)
    b = rng.normal(size=5)
    F = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    lo, hi = np.full(5, -1e3), np.full(5, 1e3)
    lo[2] = hi[2] = 0.7
    x, _, _ = O.lbfgs(F, np.zeros(5), lo, hi, ftol=0.0, gtol=1e-10)
    keep = [0, 1, 3, 4]
    expect = np.linalg.solve(A[np.ix_(keep, keep)], b[keep] - A[keep, 2] * 0.7)
    assert x[2] == 0.7
    np.testing.assert_allclose(x[keep], expect, rtol=1e-7, atol=1e-7)
