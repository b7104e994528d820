"""Oracle, parareal level: slice schedule, quantile iterator, matching, the
generic parareal iteration and the micro-macro driver.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Follows Sec. 3.1 (classical parareal, eq. (sequential)), Sec. 3.2.3-3.2.4
(generic and zeroth micro-macro iterations, eq. (mm_sequential) and
eq. (mm_match)), Sec. 3.3.3 (exactness), Sec. 4.4 (quantile iterator
eq. (quantile_reconstruction) and its monotonicity repair) and Sec. 5.1
(matching preserving the fast marginal, eq. (transformation)).
"""
import math

import numpy as np

from . import coarse as _coarse
from . import particles as _particles
from . import restrict as _restrict


# --------------------------------------------------------------------------
# Slice schedule.  The paper splits [0, T] into equal slices (Sec. 3.1).
# Reading: S = round(T/dt) fine steps of dt_eff = T/S; slice n covers the
# global steps [floor(n S / K), floor((n+1) S / K)).
# --------------------------------------------------------------------------
def total_steps(T, dt):
    S = int(round(T / dt))
    return S, T / S


def slice_bounds(S, K):
    return [(n * S) // K for n in range(K + 1)]


# --------------------------------------------------------------------------
# Quantile iterator (Sec. 4.4) on fixed levels p_j = j/Q.
# --------------------------------------------------------------------------
def pava(v):
    """Pool-adjacent-violators with equal weights: the non-decreasing
    sequence closest to v in least squares.  Adjacent violating values are
    replaced by their average, repeatedly, which is the paper's repair of a
    non-monotone quantile function; identity on non-decreasing input."""
    sums, counts = [], []
    for x in v:
        s, c = float(x), 1
        while sums and sums[-1] / counts[-1] > s / c:
            s += sums.pop()
            c += counts.pop()
        sums.append(s)
        counts.append(c)
    out = []
    for s, c in zip(sums, counts):
        out.extend([s / c] * c)
    return np.array(out)


def j_quantile(q_c_next, q_f, q_c_star):
    """q = q_f + (q_c^{n+1} - q_c^*), then made non-decreasing.  With
    q_c^{n+1} == q_c^* the result is q_f bitwise (eq. (iterator_property))."""
    q_c_next, q_f, q_c_star = (np.asarray(v, dtype=np.float64) for v in (q_c_next, q_f, q_c_star))
    return pava(q_f + (q_c_next - q_c_star))


# --------------------------------------------------------------------------
# Matching preserving the fast marginal (Sec. 5.1), quantile add/subtract form.
# --------------------------------------------------------------------------
def match_quantiles(x_prior, rank, q_target, q_prior):
    """X = Xbar + delta(u), u = (rank + 1/2)/P the prior's mid-rank cdf value,
    delta the piecewise-linear interpolant of q_target - q_prior on the knots
    p_j = j/Q.  The fast variables and the weights are unchanged.  With
    q_target == q_prior the ensemble is returned bitwise (eq. (projection))."""
    x_prior = np.asarray(x_prior, dtype=np.float64)
    N = x_prior.shape[0]
    Q = len(q_target) - 1
    d = np.asarray(q_target, dtype=np.float64) - np.asarray(q_prior, dtype=np.float64)
    u = (np.asarray(rank, dtype=np.float64) + 0.5) / N
    uq = u * Q
    j = np.minimum(np.floor(uq), Q - 1).astype(np.int64)
    w = uq - j
    delta = (1.0 - w) * d[j] + w * d[j + 1]
    return x_prior + delta


# --------------------------------------------------------------------------
# Generic parareal iteration (Sec. 3.1 and Sec. 3.2.3-3.2.4), parameterised by
# the propagators and coupling operators so that the same code runs the
# classical scalar method and the micro-macro method.
#   fine(n, u)       : fine propagator over slice n       (micro state)
#   coarse(n, rho)   : coarse propagator over slice n     (macro state)
#   restrict(u)      : micro -> macro
#   match(rho, u*)   : macro -> micro given a prior (with timed_match,
#                      match(rho, u*, n) for the time point n it produces)
#   jump(c, f, cs)   : the iterator J
# --------------------------------------------------------------------------
class Parareal:
    def __init__(self, u0, n_slices, fine, coarse, restrict, match, jump, reuse_coarse=False,
                 timed_match=False):
        self.K = n_slices
        self.fine, self.coarse, self.restrict, self.jump = fine, coarse, restrict, jump
        self.match = match if timed_match else (lambda rho, prior, n: match(rho, prior))
        self.reuse = reuse_coarse
        self.k = 0
        # zeroth iteration: a coarse pass from R(u0), matched against u0
        r0 = restrict(u0)
        rho = [r0]
        for n in range(self.K):
            rho.append(coarse(n, rho[n]))
        self.rho = rho
        self.u = [u0] + [self.match(rho[n], u0, n) for n in range(1, self.K + 1)]

    def iterate(self):
        K = self.K
        # parallel phase: fine and coarse propagation of every slice
        ubar = [None] + [self.fine(n, self.u[n]) for n in range(K)]
        rho_f = [None] + [self.restrict(ubar[n + 1]) for n in range(K)]
        if self.reuse:
            rho_cs = [None] + [self.coarse(n, self.rho[n]) for n in range(K)]
        else:
            rho_cs = [None] + [self.coarse(n, self.restrict(self.u[n])) for n in range(K)]
        # serial phase
        rho_new = [self.rho[0]]
        for n in range(K):
            rho_new.append(self.jump(self.coarse(n, rho_new[n]), rho_f[n + 1], rho_cs[n + 1]))
        # matching with the fine results as priors
        self.u = [self.u[0]] + [self.match(rho_new[n + 1], ubar[n + 1], n + 1) for n in range(K)]
        self.rho = rho_new
        self.k += 1


# --------------------------------------------------------------------------
# Micro-macro instance: ensemble of the slow-fast SDE, finite-volume coarse
# model on the slow variable, quantile iterator, fast-marginal matching.
# --------------------------------------------------------------------------
class Ensemble:
    """Micro state: slow x[P], fast y[d][P], the prior's ranks and knots
    cached on first restriction."""

    def __init__(self, x, y):
        self.x, self.y = x, y
        self._r = None

    def restricted(self, n_q):
        if self._r is None:
            q, rank, _, _ = _restrict.restrict(self.x, n_q)
            self._r = (q, rank)
        return self._r


def micmac_parareal(sde, seed, inst, n_particles, T, dt, n_slices, grid, n_q, reuse_coarse=False):
    """Builds the micro-macro parareal iteration at k = 0.  Returns
    (Parareal, helpers) where helpers holds the schedule and propagators."""
    S, dt_eff = total_steps(T, dt)
    bounds = slice_bounds(S, n_slices)
    prop = _coarse.Propagator(grid, sde)
    taus = {}
    for n in range(n_slices):
        L = bounds[n + 1] - bounds[n]
        if L not in taus:
            taus[L] = prop.expm(L * dt_eff)
    E = [taus[bounds[n + 1] - bounds[n]] for n in range(n_slices)]
    x0, y0 = _particles.init_ensemble(sde, seed, inst, n_particles)

    def fine(n, u):
        x, y = _particles.em_propagate(sde, seed, inst, u.x, u.y, bounds[n], bounds[n + 1], dt_eff)
        return Ensemble(x, y)

    def coarse(n, q):
        return _coarse.coarse_step(q, E[n], grid)[0]

    def restrict(u):
        return u.restricted(n_q)[0]

    def match(q, prior):
        q_prior, rank = prior.restricted(n_q)
        return Ensemble(match_quantiles(prior.x, rank, q, q_prior), prior.y)

    pr = Parareal(Ensemble(x0, y0), n_slices, fine, coarse, restrict, match, j_quantile,
                  reuse_coarse=reuse_coarse)
    helpers = dict(S=S, dt=dt_eff, bounds=bounds, E=E, x0=x0, y0=y0, fine=fine, restrict=restrict)
    return pr, helpers


def sequential_reference(helpers, n_slices, n_q):
    """The fine propagator run serially from the initial ensemble:
    states F^n X0, n = 0..K, and their knots."""
    u = Ensemble(helpers["x0"], helpers["y0"])
    states = [u]
    for n in range(n_slices):
        u = helpers["fine"](n, u)
        states.append(u)
    return states, [s.restricted(n_q)[0] for s in states]


def quantile_error(q, q_ref):
    """RMS over the knots of the difference of two knot vectors."""
    q, q_ref = np.asarray(q), np.asarray(q_ref)
    return math.sqrt(float(np.mean((q - q_ref) ** 2)))
