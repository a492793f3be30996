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


# ---- one swarm step worked by hand -----------------------------------------
# The random numbers come from the published SplitMix64 vector (seed 1234567,
# outputs 0..4).  SplitMix64 advances its state by 0x9E3779B97F4A7C15 per
# output, so output i of seed s is output i - j of seed s + j*0x9E3779B97F4A7C15
# (mod 2^64): shifting the seed places the published outputs at any counter.
_PUB = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
        16408922859458223821]
_GAMMA = 0x9E3779B97F4A7C15


def _seed_for(counter):
    """A seed whose counter `counter` draws published output 0."""
    return (1234567 - counter * _GAMMA) % (1 << 64)


def test_pso_move_one_step_by_hand():
    # N = 1 particle, P = 1 dimension, step t = 1: the update draws counters
    # ((t N + p) P + d) 2 + k = 2 and 3, i.e. published outputs 2 and 3:
    #   r0 = (9817491932198370423 >> 11) / 2^53 = 4793697232518735 / 2^53
    #   r1 = (4593380528125082431 >> 11) / 2^53 = 2242861585998575 / 2^53
    # with w = 0.5, c1 = 2, c2 = 0.25, x = 1, v = 0.5, pbest = 3, gbest = -1:
    #   v' = 0.5*0.5 + 2 r0 (3 - 1) + 0.25 r1 (-1 - 1) = 0.25 + 4 r0 - 0.5 r1
    #      = 2.254325387558531...,   x' = 1 + v' = 3.254325387558531...
    r0 = 4793697232518735 / 2 ** 53
    r1 = 2242861585998575 / 2 ** 53
    assert abs(r0 - 0.5322073040624192) < 1e-16 and abs(r1 - 0.24900765738229136) < 1e-16
    args = dict(lo=np.array([-10.0]), hi=np.array([10.0]), seed=1234567, w=0.5, c1=2.0, c2=0.25)
    x, v = O.pso_move(1, np.array([[1.0]]), np.array([[0.5]]), np.array([[3.0]]), np.array([-1.0]), **args)
    assert abs(v[0, 0] - 2.254325387558531) < 1e-15
    assert abs(x[0, 0] - 3.254325387558531) < 1e-15
    # the same move beyond the upper bound stops on it with zero velocity
    x, v = O.pso_move(1, np.array([[1.0]]), np.array([[0.5]]), np.array([[3.0]]), np.array([-1.0]),
                      **{**args, "hi": np.array([2.0])})
    assert x[0, 0] == 2.0 and v[0, 0] == 0.0
    # and below the lower bound: v' = 0.25 + 2 r0 (-4) + 0.25 r1 (-6) = -4.38... -> x' = -3.38...
    x, v = O.pso_move(1, np.array([[1.0]]), np.array([[0.5]]), np.array([[-3.0]]), np.array([-5.0]),
                      **{**args, "lo": np.array([-2.0])})
    assert x[0, 0] == -2.0 and v[0, 0] == 0.0
    x, v = O.pso_move(1, np.array([[1.0]]), np.array([[0.5]]), np.array([[-3.0]]), np.array([-5.0]), **args)
    assert abs(v[0, 0] - (0.25 - 8 * r0 - 1.5 * r1)) < 1e-15 and abs(x[0, 0] - (1.25 - 8 * r0 - 1.5 * r1)) < 1e-15


def test_pso_move_counters_of_every_particle_and_dimension():
    # N = 2, P = 2, t = 1: element (p, d) draws counters ((2 + p) 2 + d) 2 + {0, 1}
    # = 8 + 4p + 2d + {0, 1}.  Two seeds put the published outputs 0..3 at
    # counters 8..11 (elements (0, 0), (0, 1)) and 12..15 ((1, 0), (1, 1)).
    u = [(o >> 11) / 2 ** 53 for o in _PUB]
    x0 = np.array([[0.2, -0.7], [1.1, 0.4]])
    v0 = np.array([[0.3, -0.1], [0.0, 0.25]])
    pb = np.array([[0.9, -0.2], [1.5, -0.6]])
    gb = np.array([-0.4, 0.8])
    w, c1, c2 = 0.7, 1.3, 1.9
    lo, hi = np.full(2, -50.0), np.full(2, 50.0)
    for seed, elems in ((_seed_for(8), [(0, 0), (0, 1)]), (_seed_for(12), [(1, 0), (1, 1)])):
        x, v = O.pso_move(1, x0, v0, pb, gb, lo, hi, seed, w, c1, c2)
        for j, (p, d) in enumerate(elems):
            r0, r1 = u[2 * j], u[2 * j + 1]
            ev = w * v0[p, d] + c1 * r0 * (pb[p, d] - x0[p, d]) + c2 * r1 * (gb[d] - x0[p, d])
            assert abs(v[p, d] - ev) < 1e-15 and abs(x[p, d] - (x0[p, d] + ev)) < 1e-15
