"""Fitting loops (oracle, FP64).  Test infrastructure only.

The paper keeps lenstronomy's particle swarm optimiser and adds L-BFGS on
automatic-differentiation gradients (section "Improvements over lenstronomy
in lens modelling").  It fixes neither algorithm's constants; the readings:

Random numbers: u(seed, i) = (the (i+1)-th output of SplitMix64 seeded with
`seed`) >> 11, times 2^-53, in [0, 1).  SplitMix64 (Steele, Lea & Flood 2014)
advances its state by 0x9E3779B97F4A7C15 and mixes it, so output i depends
only on seed + (i+1) * 0x9E3779B97F4A7C15: a counter-based generator.

PSO (Kennedy & Eberhart 1995, with the inertia weight of Shi & Eberhart
1998), maximising f over the box [lo, hi] with N particles in P dimensions:
  start  x = lo + u (hi - lo), u = u(seed, p P + d); v = 0; personal bests
         are the start points; the swarm best is the first particle with the
         largest value;
  step t = 1, 2, ...:  with r_k = u(seed, ((t N + p) P + d) 2 + k), k = 0, 1,
         v <- w v + c1 r_0 (pbest - x) + c2 r_1 (gbest - x);  x <- x + v;
         a coordinate outside the box is set to the bound and its velocity to
         zero; then f at every particle; a personal best moves when its new
         value is strictly larger (NaN counts as -inf); the swarm best is the
         first particle with the largest personal best.

L-BFGS (Nocedal 1980; Liu & Nocedal 1989), minimising F = -f from x0 in the
box: a coordinate on a bound whose gradient points out of the box is held
(also every coordinate with equal bounds); on the free coordinates the
direction is -H g by the two-loop recursion over the last m pairs (s, y)
with H0 = (s.y / y.y) I from the newest pair (the steepest-descent direction
scaled to unit length when there is none, or when the direction does not
descend, which also clears the pairs); the step starts at 1 and is
halved until the projected trial point x_t = clamp(x + a d) satisfies
F(x_t) <= F(x) + 1e-4 g.(x_t - x) (at most 40 halvings, else the run
stops); a pair is kept when s.y > 1e-12 |s| |y|; the run stops after
max_iter accepted steps, when |F - F_t| <= ftol max(1, |F|), or when the
largest component of the projected gradient is at most gtol.
"""
import numpy as np

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed, i):
    """The (i+1)-th SplitMix64 output of the stream seeded with `seed`."""
    z = (int(seed) + (int(i) + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform(seed, i):
    return (splitmix64(seed, i) >> 11) * (1.0 / 9007199254740992.0)


def pso_start(N, lo, hi, seed):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    P = lo.size
    x = np.empty((N, P))
    for p in range(N):
        for d in range(P):
            x[p, d] = lo[d] + uniform(seed, p * P + d) * (hi[d] - lo[d])
    return x, np.zeros((N, P))


def pso_move(t, x, v, pbest, gbest, lo, hi, seed, w, c1, c2):
    """One velocity/position update (step t >= 1) of every particle."""
    N, P = x.shape
    x = x.copy()
    v = v.copy()
    for p in range(N):
        for d in range(P):
            r0 = uniform(seed, ((t * N + p) * P + d) * 2)
            r1 = uniform(seed, ((t * N + p) * P + d) * 2 + 1)
            vv = w * v[p, d] + c1 * r0 * (pbest[p, d] - x[p, d]) + c2 * r1 * (gbest[d] - x[p, d])
            xx = x[p, d] + vv
            if xx < lo[d]:
                xx, vv = lo[d], 0.0
            elif xx > hi[d]:
                xx, vv = hi[d], 0.0
            x[p, d] = xx
            v[p, d] = vv
    return x, v


def pso_bests(x, f, pbest, pbest_f):
    """Personal bests after the values f at x; the swarm best."""
    pbest = pbest.copy()
    pbest_f = pbest_f.copy()
    f = np.where(np.isnan(f), -np.inf, f)          # an undefined value never wins
    better = f > pbest_f
    pbest[better] = x[better]
    pbest_f[better] = f[better]
    g = int(np.argmax(pbest_f))
    return pbest, pbest_f, pbest[g].copy(), float(pbest_f[g])


def pso(f, lo, hi, N, n_iter, seed, w=0.7298, c1=1.49618, c2=1.49618):
    """Maximise f (a function of an [N, P] array returning [N] values).
    Returns the swarm best, its value and the best value after each step."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    x, v = pso_start(N, lo, hi, seed)
    fx = np.asarray(f(x), dtype=np.float64)
    pbest, pbest_f, gbest, gbest_f = pso_bests(x, fx, x.copy(), np.full(N, -np.inf))
    hist = []
    for t in range(1, n_iter + 1):
        x, v = pso_move(t, x, v, pbest, gbest, lo, hi, seed, w, c1, c2)
        fx = np.asarray(f(x), dtype=np.float64)
        pbest, pbest_f, gbest, gbest_f = pso_bests(x, fx, pbest, pbest_f)
        hist.append(gbest_f)
    return gbest, gbest_f, np.array(hist)


def lbfgs(F, x0, lo, hi, m=10, max_iter=200, ftol=1e-12, gtol=1e-10):
    """Minimise F (returning value and gradient) in the box [lo, hi].
    Returns x, F(x) and the number of accepted steps."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    x = np.clip(np.asarray(x0, dtype=np.float64), lo, hi)
    fx, g = F(x)
    S, Y = [], []
    it = 0
    while it < max_iter:
        # coordinates on a bound whose gradient points out of the box stay
        # put; the recursion runs on the free ones
        free = ~(((x <= lo) & (g > 0)) | ((x >= hi) & (g < 0)))
        gf = np.where(free, g, 0.0)
        if np.max(np.abs(gf)) <= gtol:
            break
        Sf = [np.where(free, s, 0.0) for s in S]
        Yf = [np.where(free, y, 0.0) for y in Y]
        q = gf.copy()
        alphas = []
        for s, y in zip(reversed(Sf), reversed(Yf)):
            a = (s @ q) / (y @ s)
            q = q - a * y
            alphas.append(a)
        if Sf:
            q = q * ((Sf[-1] @ Yf[-1]) / (Yf[-1] @ Yf[-1]))
        else:
            q = q / np.linalg.norm(gf)
        for (s, y), a in zip(zip(Sf, Yf), reversed(alphas)):
            b = (y @ q) / (y @ s)
            q = q + s * (a - b)
        d = -q
        if not (g @ d < 0.0):
            S, Y = [], []
            d = -gf / np.linalg.norm(gf)
        step = 1.0
        for _ in range(41):
            xt = np.clip(x + step * d, lo, hi)
            ft, gt = F(xt)
            if ft <= fx + 1e-4 * (g @ (xt - x)):
                break
            step *= 0.5
        else:
            break
        s = xt - x
        y = gt - g
        if s @ y > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        it += 1
        done = abs(fx - ft) <= ftol * max(1.0, abs(fx))
        x, fx, g = xt, ft, gt
        if done:
            break
    return x, fx, it
