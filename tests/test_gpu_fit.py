"""GPU checks of the fitting loops (jt_pso, jt_lbfgs) against the oracle:
the initial swarm's best particle and value, the swarm's invariants and its
convergence on noise-free data, and L-BFGS chains against the oracle's L-BFGS
on the oracle's objective from the same starts."""
import copy

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2606_01547_amd import Context
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = Context(0)
    yield c
    c.close()


def _problem(npix=36):
    sc = W.config1_scene(draw=2)
    sc.grid = W.Grid(nx=npix, ny=npix, pixel_scale=0.06, supersample=1)
    d = O.simulate_image(sc).astype(np.float32)
    w = np.full(d.shape, 1.0 / 0.01 ** 2, dtype=np.float32)
    truth = O.macro_vector(sc.lens, sc.source, sc.lens_light)
    lo, hi = truth.copy(), truth.copy()
    free = [0, 1, 2, 3, 4, 7, 12, 13]          # theta_E, q, phi, centre, source amp and centre
    width = np.array([0.1, 0.08, 0.2, 0.03, 0.03, 0, 0, 2.0, 0, 0, 0, 0, 0.05, 0.05])
    lo[free] = truth[free] - width[free]
    hi[free] = truth[free] + width[free]
    hi[1] = min(hi[1], 1.0)
    return sc, d, w, truth, lo, hi


def _scene_at(sc, x):
    s = copy.deepcopy(sc)
    s.lens.sie = W.SIE(*x[:5])
    s.lens.shear = W.Shear(*x[5:7])
    s.source = [W.Sersic(*x[7:14])]
    return s


def _oracle_logL(sc, x, d, w):
    m = O.simulate_image(_scene_at(sc, x))
    return -0.5 * float(np.sum(w.astype(np.float64) * (m - d) ** 2))


def test_initial_swarm_best_matches_the_oracle(ctx):
    sc, d, w, truth, lo, hi = _problem()
    best, bl, _ = ctx.pso(sc.grid, 1, 0, lo, hi, d, w, psf=sc.psf, n_particles=24, n_iterations=0, seed=5)
    x0, _ = O.pso_start(24, lo, hi, 5)
    ll = np.array([_oracle_logL(sc, x, d, w) for x in x0])
    order = np.argsort(ll)[::-1]
    assert ll[order[0]] - ll[order[1]] > 1e-3 * abs(ll[order[0]])     # a clear winner for this seed
    np.testing.assert_array_equal(best, x0[order[0]])
    assert abs(bl - ll[order[0]]) <= 1e-4 * abs(ll[order[0]])


def test_swarm_invariants_and_convergence(ctx):
    sc, d, w, truth, lo, hi = _problem()
    best, bl, hist = ctx.pso(sc.grid, 1, 0, lo, hi, d, w, psf=sc.psf, n_particles=96, n_iterations=120, seed=9)
    assert np.all(np.diff(hist) >= 0.0) and hist[-1] == bl
    assert np.all(best >= lo) and np.all(best <= hi)
    # the swarm's best value is the library's own likelihood at that point
    ll_again = ctx.lbfgs(sc.grid, 1, 0, lo, hi, d, w, best, psf=sc.psf, max_iter=0)[1][0]
    assert abs(ll_again - bl) <= 1e-9 * abs(bl)
    # noise-free data: the swarm closes in on the truth (the oracle's own swarm
    # with this seed ends within 0.2% of the box of every free parameter)
    assert np.all(np.abs(best - truth) <= 0.01 * (hi - lo) + 1e-12)
    assert _oracle_logL(sc, best, d, w) >= -20.0


def test_lbfgs_chains_match_the_oracle(ctx):
    sc, d, w, truth, lo, hi = _problem(npix=30)
    rng = np.random.default_rng(1)
    starts = truth + (hi - lo) * rng.uniform(-0.25, 0.25, (3, truth.size))
    x, ll, its = ctx.lbfgs(sc.grid, 1, 0, lo, hi, d, w, starts, psf=sc.psf, max_iter=150)

    def F(v):
        l, g, _ = O.chi2_gradient(_scene_at(sc, v), d, w)
        return -l, -g

    for c in range(3):
        xo, fo, _ = O.lbfgs(F, starts[c], lo, hi, max_iter=150)
        scale = np.maximum(hi - lo, 1e-12)
        assert np.max(np.abs(x[c] - xo) / scale) <= 1e-3, (x[c], xo)
        assert abs(ll[c] + fo) <= 1e-3 * max(1.0, abs(fo)) + 1e-2
        assert its[c] >= 1
