"""Oracle, histogram-state micro-macro parareal: the macroscopic state is the
vector of cell masses of the slow variable (eq. (integral), eq. (binning)),
iterated by the additive, multiplicative, rotation or quantile iterator
(Sec. 4.1-4.4) and coupled to the ensemble by the fast-marginal matching on
piecewise-linear cdfs (Sec. 5.1) or by the conditional matching with
reweighting, optionally followed by stratified resampling (Sec. 5.2).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Readings where the paper is silent (each listed in the design notes):
  H1 binning: cell index floor((x - x_lo) I / (x_hi - x_lo)) clamped to the
     grid (as for the quantile restriction); the mass of a cell is the exact
     sum of its weights rounded once (math.fsum); equal weights are the
     double nearest 1/P.
  H2 the cdf at the edges is the left-to-right running sum of the masses.
  H3 quantile of a histogram at level p: the set {x : c(x) = p} of the
     piecewise-linear cdf eq. (discr_cdf) is an interval [L, R]; q(p) is its
     midpoint inside (0, M), R at p = 0 and L at p = M (M the total mass),
     the support rules of Sec. 4.4; levels beyond M are taken at M.
  H4 quantile iterator: q = q_f + (q_c^{n+1} - q_c^*) at the union of the
     three cdfs' edge levels, pool-adjacent-violators, then the cdf at each
     edge is inf{p : q(p) >= x_i} on the piecewise-linear q; the mass left of
     the grid or right of it goes to the end cells.
  H5 additive: rho_f + (rho_c^{n+1} - rho_c^*); negative cells set to 0 and,
     only then, the result scaled to the mass of rho_f.
  H6 multiplicative: rho_f (rho_c^{n+1} / rho_c^*) where rho_c^* > 0, else 0,
     scaled to the mass of rho_f.
  H7 rotation: the paper's closed form with the inner products taken as
     sum_i sqrt(a_i b_i); no rescaling.
  H8 fast-marginal matching: X = q(cbar(Xbar)) with cbar the prior's
     piecewise-linear cdf (a particle outside the grid is clamped to its end
     cell) and q the target's quantile function of H3.  The paper's inverse
     divides by the prior mass (an open note of the authors); the inverse of
     the target cdf needs the target mass.
  H9 reweighting: cells with target mass but no prior particle hand half
     of it to the nearest supported cell on each side (all of it when only
     one side has one), in increasing cell order; W = Wbar (rho'_i / rhobar_i).
  H10 stratified resampling: weights in fixed point Q(W) = floor(W 2^64);
     with T the total, slot j takes the particle p with
     C_{p-1} <= U_j < C_p, U_j = floor(j T / P) + floor(k_j T / (P 2^32)),
     C the running sums of Q(W); k_j is the first Philox word of block
     (tag 4, m = 0, p = j, pair = slice, instance) for random u_j, 2^31 for
     the deterministic choice u_j = 1/2.  Equal weights give the identity.
"""
import math

import numpy as np

from . import chem as _chem
from . import coarse as _coarse
from . import iterate as _iterate
from . import particles as _particles

J_ADD, J_MULT, J_ROT, J_QUANTILE = 0, 1, 2, 3
M_MARGINAL, M_REWEIGHT, M_RESAMPLE, M_RESAMPLE_DET = 0, 1, 2, 3
TAG_RESAMPLE = 4
FIX = 2.0 ** 64


# --------------------------------------------------------------------------
# Restriction (eq. (binning)) and the cdf at the edges (eq. (discr_cdf)).
# --------------------------------------------------------------------------
def cell_index(x, grid):
    x = np.asarray(x, dtype=np.float64)
    inv_h = grid.n / (grid.hi - grid.lo)
    c = np.floor((x - grid.lo) * inv_h)
    return np.clip(c, 0, grid.n - 1).astype(np.int64)


def equal_weights(n):
    return np.full(n, 1.0 / n)


def hist_restrict(x, w, grid):
    """rho_i = the weights of the particles in cell i, summed exactly and
    rounded once (H1)."""
    idx = cell_index(x, grid)
    w = np.asarray(w, dtype=np.float64)
    order = np.argsort(idx, kind="stable")
    idx_s, w_s = idx[order], w[order]
    bounds = np.searchsorted(idx_s, np.arange(grid.n + 1), side="left")
    return np.array([math.fsum(w_s[bounds[i]:bounds[i + 1]].tolist()) for i in range(grid.n)])


def cdf_edges(rho):
    """c_0 = 0, c_{i+1} = c_i + rho_i (H2)."""
    c = np.zeros(len(rho) + 1)
    for i in range(len(rho)):
        c[i + 1] = c[i] + rho[i]
    return c


def quantile_at(rho, c, grid, p):
    """q(p) of the histogram rho with edge cdf c (H3)."""
    I = grid.n
    e = grid.edges
    M = c[I]
    p = min(max(p, 0.0), M)
    a = int(np.searchsorted(c, p, side="left"))       # first edge with c_a >= p
    b = int(np.searchsorted(c, p, side="right")) - 1  # last edge with c_b <= p
    if a == 0:
        L = e[0]
    else:
        t = min(max((p - c[a - 1]) / rho[a - 1], 0.0), 1.0)
        L = e[a - 1] + t * grid.h
    if b == I:
        R = e[I]
    else:
        t = min(max((p - c[b]) / rho[b], 0.0), 1.0)
        R = e[b] + t * grid.h
    if p == 0.0:
        return R
    if p == M:
        return L
    return 0.5 * (L + R)


# --------------------------------------------------------------------------
# Iterators J(rho_c^{n+1}, rho_f^*, rho_c^*) (Sec. 4).
# --------------------------------------------------------------------------
def _sum(v):
    s = 0.0
    for a in v:
        s += a
    return s


def _scaled(r, rf):
    """r scaled to the mass of rf; a result without mass leaves rf."""
    s = _sum(r)
    if s == 0.0:
        return rf.copy()
    return r * (_sum(rf) / s)


def j_add(rc, rf, rcs):
    r = rf + (rc - rcs)
    if np.any(r < 0.0):
        r = _scaled(np.maximum(r, 0.0), rf)
    return r


def j_mult(rc, rf, rcs):
    r = np.zeros_like(rf)
    pos = rcs > 0.0
    r[pos] = rf[pos] * (rc[pos] / rcs[pos])
    return _scaled(r, rf)


def j_rot(rc, rf, rcs):
    u = _sum(np.sqrt(rf * rcs))
    v = _sum(np.sqrt(rf * rc))
    w = _sum(np.sqrt(rcs * rc))
    a = (u + 2.0 * u * w - v) / (1.0 + w)
    b = (u + v) / (1.0 + w)
    s = a * np.sqrt(rc) + np.sqrt(rf) - b * np.sqrt(rcs)
    return s * s


def j_quantile(rc, rf, rcs, grid):
    cc, cf, ccs = cdf_edges(rc), cdf_edges(rf), cdf_edges(rcs)
    levels = np.unique(np.concatenate([cc, cf, ccs]))
    qt = np.array([quantile_at(rf, cf, grid, p) + (quantile_at(rc, cc, grid, p) - quantile_at(rcs, ccs, grid, p))
                   for p in levels])
    qt = _iterate.pava(qt)
    I = grid.n
    ct = np.empty(I + 1)
    for i in range(I + 1):
        x = grid.edges[i]
        j = int(np.searchsorted(qt, x, side="left"))  # first j with qt_j >= x
        if j == 0:
            ct[i] = 0.0
        elif j == len(qt):
            ct[i] = levels[-1]
        else:
            t = (x - qt[j - 1]) / (qt[j] - qt[j - 1])
            ct[i] = levels[j - 1] + t * (levels[j] - levels[j - 1])
    ct[0] = 0.0
    ct[I] = levels[-1]
    return np.array([ct[i + 1] - ct[i] for i in range(I)])


def jump(kind, rc, rf, rcs, grid):
    rc, rf, rcs = (np.asarray(v, dtype=np.float64) for v in (rc, rf, rcs))
    if kind == J_ADD:
        return j_add(rc, rf, rcs)
    if kind == J_MULT:
        return j_mult(rc, rf, rcs)
    if kind == J_ROT:
        return j_rot(rc, rf, rcs)
    return j_quantile(rc, rf, rcs, grid)


# --------------------------------------------------------------------------
# Matchings (Sec. 5).
# --------------------------------------------------------------------------
def match_marginal(rho_t, rho_p, x, grid):
    """X = q_t(cbar(Xbar)) (eq. (transformation), H8)."""
    c_p, c_t = cdf_edges(rho_p), cdf_edges(rho_t)
    idx = cell_index(x, grid)
    out = np.empty(len(x))
    for k, (xv, i) in enumerate(zip(np.asarray(x, dtype=np.float64), idx)):
        t = min(max((xv - grid.edges[i]) / grid.h, 0.0), 1.0)
        cbar = c_p[i] + t * rho_p[i]
        out[k] = quantile_at(rho_t, c_t, grid, cbar)
    return out


def move_unsupported(rho_t, rho_p):
    """H9: the target mass of cells without prior particles, handed to the
    nearest supported cells."""
    I = len(rho_t)
    sup = np.nonzero(rho_p > 0.0)[0]
    r = np.where(rho_p > 0.0, rho_t, 0.0)
    for i in range(I):
        if rho_p[i] > 0.0 or rho_t[i] == 0.0:
            continue
        k = int(np.searchsorted(sup, i))
        left = sup[k - 1] if k > 0 else None
        right = sup[k] if k < len(sup) else None
        if left is not None and right is not None:
            half = 0.5 * rho_t[i]
            r[left] += half
            r[right] += half
        elif left is not None:
            r[left] += rho_t[i]
        else:
            r[right] += rho_t[i]
    return r


def reweight(rho_t, rho_p, x, w, grid):
    r = move_unsupported(np.asarray(rho_t, dtype=np.float64), np.asarray(rho_p, dtype=np.float64))
    ratio = np.zeros(grid.n)
    pos = rho_p > 0.0
    ratio[pos] = r[pos] / rho_p[pos]
    return np.asarray(w, dtype=np.float64) * ratio[cell_index(x, grid)]


def fixed_weights(w):
    """Q(W) = floor(W 2^64), capped at 2^64 - 1 (H10)."""
    out = []
    for v in np.asarray(w, dtype=np.float64):
        q = int(math.floor(float(v) * FIX))
        out.append(min(max(q, 0), 2 ** 64 - 1))
    return out


def resample_slots(w, seed, inst, slice_id, deterministic):
    """Particle index of every slot j of the stratified resampling (H10)."""
    P = len(w)
    q = fixed_weights(w)
    C = [0] * (P + 1)
    for p in range(P):
        C[p + 1] = C[p] + q[p]
    T = C[P]
    if deterministic:
        k = [2 ** 31] * P
    else:
        blocks = _particles.blocks(seed, inst, TAG_RESAMPLE, 0, 0, P, j=slice_id)
        k = [int(b[0]) for b in blocks]
    out = np.empty(P, dtype=np.int64)
    p = 0
    for j in range(P):
        U = (j * T) // P + (k[j] * T) // (P << 32)
        while p < P - 1 and C[p + 1] <= U:
            p += 1
        out[j] = p
    return out


def match(kind, rho_t, rho_p, ens, grid, seed=0, inst=0, slice_id=0):
    """Posterior ensemble (x, y, w) for target rho_t, prior ensemble ens
    (whose restriction is rho_p)."""
    x, y, w = ens
    if kind == M_MARGINAL:
        return match_marginal(rho_t, rho_p, x, grid), y, w
    wn = reweight(rho_t, rho_p, x, w, grid)
    if kind == M_REWEIGHT:
        return x, y, wn
    slots = resample_slots(wn, seed, inst, slice_id, kind == M_RESAMPLE_DET)
    P = len(x)
    return x[slots], y[..., slots], equal_weights(P)


# --------------------------------------------------------------------------
# Driver.
# --------------------------------------------------------------------------
class HistEnsemble:
    def __init__(self, x, y, w):
        self.x, self.y, self.w = x, y, w
        self._rho = None

    def rho(self, grid):
        if self._rho is None:
            self._rho = hist_restrict(self.x, self.w, grid)
        return self._rho


def _model(model):
    """(initial ensemble, Euler-Maruyama, coarse propagator class) of the
    double-well model (an oracle.particles.Sde) or of the chemical-reaction
    model (an oracle.chem.Chem)."""
    if isinstance(model, _chem.Chem):
        return ((lambda s, i, n: _chem.init_ensemble(model, s, i, n)),
                (lambda s, i, x, y, a, b, dt: _chem.em_propagate(model, s, i, x, y, a, b, dt)),
                (lambda g: _chem.Propagator(g, model)))
    return ((lambda s, i, n: _particles.init_ensemble(model, s, i, n)),
            (lambda s, i, x, y, a, b, dt: _particles.em_propagate(model, s, i, x, y, a, b, dt)),
            (lambda g: _coarse.Propagator(g, model)))


def micmac_parareal_hist(sde, seed, inst, n_particles, T, dt, n_slices, grid, iterator, matching):
    """The histogram-state micro-macro parareal iteration at k = 0 (the
    generic driver of iterate.Parareal with these operators), for either
    model (`sde` an oracle.particles.Sde or an oracle.chem.Chem).  The
    resampling draws its stratified numbers per time point n of the state it
    produces."""
    init, propagate, propagator = _model(sde)
    S, dt_eff = _iterate.total_steps(T, dt)
    bounds = _iterate.slice_bounds(S, n_slices)
    prop = propagator(grid)
    taus = {}
    for n in range(n_slices):
        L = bounds[n + 1] - bounds[n]
        if L not in taus:
            taus[L] = prop.expm(L * dt_eff)
    E = [taus[bounds[n + 1] - bounds[n]] for n in range(n_slices)]
    x0, y0 = init(seed, inst, n_particles)
    w0 = equal_weights(n_particles)

    def fine(n, u):
        x, y = propagate(seed, inst, u.x, u.y, bounds[n], bounds[n + 1], dt_eff)
        return HistEnsemble(x, y, u.w)

    def coarse(n, rho):
        return np.maximum(E[n] @ rho, 0.0)

    def restrict(u):
        return u.rho(grid)

    def match_op(rho, prior, n):
        x, y, w = match(matching, rho, prior.rho(grid), (prior.x, prior.y, prior.w), grid, seed, inst, n)
        return HistEnsemble(x, y, w)

    def jump_op(rc, rf, rcs):
        return jump(iterator, rc, rf, rcs, grid)

    pr = _iterate.Parareal(HistEnsemble(x0, y0, w0), n_slices, fine, coarse, restrict, match_op, jump_op,
                           timed_match=True)
    helpers = dict(S=S, dt=dt_eff, bounds=bounds, E=E, x0=x0, y0=y0, w0=w0, fine=fine)
    return pr, helpers


def sequential_reference_hist(helpers, n_slices, grid):
    u = HistEnsemble(helpers["x0"], helpers["y0"], helpers["w0"])
    states = [u]
    for n in range(n_slices):
        u = helpers["fine"](n, u)
        states.append(u)
    return states, [s.rho(grid) for s in states]


def hist_error(rho, rho_ref):
    """L2 error of two histograms (the error measure of Sec. 6)."""
    d = np.asarray(rho) - np.asarray(rho_ref)
    return math.sqrt(float(np.sum(d * d)))


def serial_hist(model, seed, inst, n_particles, T, dt, n_slices, grid):
    """Histograms at the slice ends t_n of a serial fine run of n_particles
    (the reference of the paper's error plots uses ten times the parareal
    ensemble size, Sec. 6)."""
    init, propagate, _ = _model(model)
    S, dt_eff = _iterate.total_steps(T, dt)
    bounds = _iterate.slice_bounds(S, n_slices)
    x, y = init(seed, inst, n_particles)
    w = equal_weights(n_particles)
    out = [hist_restrict(x, w, grid)]
    for n in range(n_slices):
        x, y = propagate(seed, inst, x, y, bounds[n], bounds[n + 1], dt_eff)
        out.append(hist_restrict(x, w, grid))
    return np.array(out)
