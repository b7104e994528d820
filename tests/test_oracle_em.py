"""Pins for the oracle's Euler-Maruyama ensemble (Sec. 2.1.3 eq. (EMx)/(EMy)):
the exact moment recursion of the scheme in the linear (OU) case, the Gibbs
marginal exp(-beta V) at long times for the reversible coupling lambda = 1,
the initial law, slice concatenation, and the pathwise tangents against
common-random-number finite differences."""
import numpy as np
import scipy.stats as st

from oracle import particles as P
from oracle import coarse as C


def test_initial_law(oracle_lib):
    n = 200_000
    s = P.Sde(beta=2.0)
    x, y = P.init_ensemble(s, 0, 0, n)
    cov = np.cov(np.vstack([x, y[0]]))
    ref = np.array([[0.25, 0.25], [0.25, 0.25 + 1 / s.beta]])
    se = np.sqrt((ref ** 2 + np.outer(np.diag(ref), np.diag(ref))) / n)  # sd of sample covariances
    assert np.all(np.abs(cov - ref) < 5 * se)
    assert abs(x.mean()) < 5 * 0.5 / np.sqrt(n)


def _ou_moments(lam, eps, beta, c1, dt, steps, m0, S0):
    """Exact mean/covariance recursion of the EM scheme for the linear case
    c3 = 0: z_{t+1} = M z_t + noise, M = I + dt A, noise cov dt B."""
    A = np.array([[-(c1 + lam), lam], [1 / eps, -1 / eps]])
    M = np.eye(2) + dt * A
    B = np.diag([2 / beta, 2 / (beta * eps)])
    m, S = m0.copy(), S0.copy()
    for _ in range(steps):
        m = M @ m
        S = M @ S @ M.T + dt * B
    return m, S


def test_ou_closed_form(oracle_lib):
    n, steps, dt = 200_000, 300, 2e-3
    s = P.Sde(lam=0.7, eps=0.05, beta=1.5, c3=0.0, c1=1.0)
    x0, y0 = P.init_ensemble(s, 3, 0, n)
    x0 = x0 + 0.8  # non-zero mean start
    y0 = y0 + 0.8
    x, y = P.em_propagate(s, 3, 0, x0, y0, 0, steps, dt)
    m0 = np.array([0.8, 0.8])
    S0 = np.array([[0.25, 0.25], [0.25, 0.25 + 1 / s.beta]])
    m, S = _ou_moments(s.lam, s.eps, s.beta, s.c1, dt, steps, m0, S0)
    z = np.vstack([x, y[0]])
    assert np.all(np.abs(z.mean(1) - m) < 5 * np.sqrt(np.diag(S) / n))
    cov = np.cov(z)
    se = np.sqrt((S ** 2 + np.outer(np.diag(S), np.diag(S))) / n)
    assert np.all(np.abs(cov - S) < 5 * se)
    # marginal law of X is Gaussian with that mean/variance
    ks = st.kstest(x, "norm", args=(m[0], np.sqrt(S[0, 0]))).statistic
    assert ks < 1.63 / np.sqrt(n)


def test_ou_catches_sign_error(oracle_lib):
    """The recursion above separates the coupling sign: flipping lambda's
    sign in the closed form is rejected by the same sample."""
    n, steps, dt = 100_000, 300, 2e-3
    s = P.Sde(lam=0.7, eps=0.05, beta=1.5, c3=0.0, c1=1.0)
    x0, y0 = P.init_ensemble(s, 3, 0, n)
    x, y = P.em_propagate(s, 3, 0, x0 + 0.8, y0 + 0.8, 0, steps, dt)
    S0 = np.array([[0.25, 0.25], [0.25, 0.25 + 1 / s.beta]])
    m_bad, S_bad = _ou_moments(-s.lam, s.eps, s.beta, s.c1, dt, steps, np.array([0.8, 0.8]), S0)
    assert abs(x.mean() - m_bad[0]) > 5 * np.sqrt(S_bad[0, 0] / n) or abs(x.var() - S_bad[0, 0]) > 0.01


def test_gibbs_marginal_long_time(oracle_lib):
    """lambda = 1: H(x,y) = V(x) + (x-y)^2/2 is a potential for the full
    system, so the X-marginal of the invariant law is exp(-beta V)/Z for
    every eps; after a long run the empirical cdf matches it (KS) up to the
    O(dt) bias of the scheme."""
    n, dt, T = 20_000, 2e-3, 8.0
    s = P.Sde(lam=1.0, eps=0.1, beta=2.0)
    x0, y0 = P.init_ensemble(s, 11, 0, n)
    x, _ = P.em_propagate(s, 11, 0, x0, y0, 0, int(T / dt), dt)
    grid = np.linspace(-4, 4, 40001)
    V = grid ** 4 / 4 - grid ** 2 / 2
    w = np.exp(-s.beta * V)
    cdf = np.concatenate([[0], np.cumsum(0.5 * (w[1:] + w[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    xs = np.sort(x)
    F = np.interp(xs, grid, cdf)
    emp_hi = np.arange(1, n + 1) / n
    emp_lo = np.arange(0, n) / n
    ks = max(np.max(emp_hi - F), np.max(F - emp_lo))
    assert ks < 1.63 / np.sqrt(n) + 0.01


def test_slices_concatenate_bitwise(oracle_lib):
    s = P.Sde()
    x0, y0 = P.init_ensemble(s, 0, 0, 3000)
    xa, ya = P.em_propagate(s, 0, 0, x0, y0, 0, 250, 1e-3)
    x1, y1 = P.em_propagate(s, 0, 0, x0, y0, 0, 100, 1e-3)
    x2, y2 = P.em_propagate(s, 0, 0, x1, y1, 100, 250, 1e-3)
    assert np.array_equal(xa, x2) and np.array_equal(ya, y2)


def test_particle_subset_is_exact(oracle_lib):
    """Counter-based noise: propagating particles [p0, p0+m) alone gives the
    same numbers as inside the full ensemble."""
    s = P.Sde()
    x0, y0 = P.init_ensemble(s, 0, 0, 1000)
    xa, ya = P.em_propagate(s, 0, 0, x0, y0, 0, 50, 1e-3)
    xb, yb = P.em_propagate(s, 0, 0, x0[300:400], y0[:, 300:400], 0, 50, 1e-3, p0=300)
    assert np.array_equal(xa[300:400], xb) and np.array_equal(ya[:, 300:400], yb)


def test_high_dimensional_fast_part(oracle_lib):
    """d = 32: with eps -> small the fast block relaxes to Y_i ~ N(a_i X, 1/beta)."""
    d, n = 32, 20_000
    a = P.coupling(0, 0, d)
    s = P.Sde(lam=1.0, eps=0.01, beta=2.0, d=d, a=a)
    x0, y0 = P.init_ensemble(s, 0, 0, n)
    x, y = P.em_propagate(s, 0, 0, x0, y0, 0, 200, 1e-4)
    r = y - a[:, None] * x[None, :]
    assert np.all(np.abs(r.mean(1)) < 0.03)
    assert np.all(np.abs(r.var(1) - 1 / s.beta) < 0.05)


def test_tangent_matches_crn_finite_differences(oracle_lib):
    """Forward-mode tangents w.r.t. (lambda, eps, beta, c3) against central
    differences with common random numbers (same seed, same counters)."""
    n, steps, dt, h = 64, 400, 1e-3, 1e-6
    base = dict(lam=1.0, eps=0.1, beta=2.0, c3=1.0, c1=-1.0)
    s = P.Sde(**base)
    x, y, dx, dy = P.em_tangent(s, 0, 0, n, steps, dt)
    x_ref, y_ref = P.em_propagate(s, 0, 0, *P.init_ensemble(s, 0, 0, n), 0, steps, dt)
    assert np.array_equal(x, x_ref) and np.array_equal(y, y_ref[0])
    for k, name in enumerate(("lam", "eps", "beta", "c3")):
        vals = []
        for sgn in (+1, -1):
            p = dict(base)
            p[name] += sgn * h
            sp = P.Sde(**p)
            xp, yp = P.em_propagate(sp, 0, 0, *P.init_ensemble(sp, 0, 0, n), 0, steps, dt)
            vals.append((xp, yp[0]))
        fdx = (vals[0][0] - vals[1][0]) / (2 * h)
        fdy = (vals[0][1] - vals[1][1]) / (2 * h)
        scale = np.abs(fdx).max() + 1e-12
        assert np.abs(dx[k] - fdx).max() < 1e-5 * scale + 1e-8, name
        assert np.abs(dy[k] - fdy).max() < 1e-5 * (np.abs(fdy).max() + 1e-12) + 1e-8, name


def test_effective_potential_cases():
    s = P.Sde(lam=0.3, c3=1.0, c1=-1.0)
    V = C.effective_potential(s)
    assert abs(V(2.0) - (4.0 - 2.0)) < 1e-15  # a = 1: coupling averages out
    s2 = P.Sde(lam=0.5, c3=1.0, c1=-1.0, d=2, a=np.array([0.5, 1.0]))
    V2 = C.effective_potential(s2)
    # abar = 0.75: extra lambda (1 - abar) x^2 / 2 = 0.0625 x^2
    assert abs(V2(2.0) - (4.0 - 2.0 + 0.25)) < 1e-15


def test_f32_noise_pure_diffusion_increments(oracle_lib):
    """With every drift coefficient zero (c3 = c1 = lambda = 0, Y started at
    X with a = 1) one step moves X by sqrt(2 dt/beta) z0 and Y by
    sqrt(2 dt/(beta eps)) z1, z from the single-precision propagator's normals
    of the block (tag 0, step m, particle p, pair 0); pair 1 drives Y_2."""
    n, m, dt = 64, 37, 1e-3
    for d in (1, 2):
        s = P.Sde(lam=0.0, eps=0.05, beta=2.0, c3=0.0, c1=0.0, d=d)
        x0 = np.linspace(-1.0, 1.0, n)
        y0 = np.tile(x0, (d, 1))
        x, y = P.em_propagate(s, 5, 2, x0, y0, m, m + 1, dt, p0=11, f32_noise=True)
        z0, z1 = P.box_muller_f32(P.blocks(5, 2, 0, m, 11, n, j=0))
        assert np.abs((x - x0) / np.sqrt(2 * dt / s.beta) - z0).max() < 1e-9
        assert np.abs((y[0] - y0[0]) / np.sqrt(2 * dt / (s.beta * s.eps)) - z1).max() < 1e-9
        if d == 2:
            w0, _ = P.box_muller_f32(P.blocks(5, 2, 0, m, 11, n, j=1))
            assert np.abs((y[1] - y0[1]) / np.sqrt(2 * dt / (s.beta * s.eps)) - w0).max() < 1e-9
        # the double-precision normals are other numbers
        xd, _ = P.em_propagate(s, 5, 2, x0, y0, m, m + 1, dt, p0=11)
        assert np.abs(xd - x).max() > 1e-10


def test_f32_noise_ou_closed_form(oracle_lib):
    """The single-precision propagator's normals drive the scheme with the
    exact moment recursion of the linear case, as the double ones do."""
    n, steps, dt = 200_000, 300, 2e-3
    s = P.Sde(lam=0.7, eps=0.05, beta=1.5, c3=0.0, c1=1.0)
    x0, y0 = P.init_ensemble(s, 3, 0, n)
    x, y = P.em_propagate(s, 3, 0, x0 + 0.8, y0 + 0.8, 0, steps, dt, f32_noise=True)
    m0 = np.array([0.8, 0.8])
    S0 = np.array([[0.25, 0.25], [0.25, 0.25 + 1 / s.beta]])
    m, S = _ou_moments(s.lam, s.eps, s.beta, s.c1, dt, steps, m0, S0)
    z = np.vstack([x, y[0]])
    assert np.all(np.abs(z.mean(1) - m) < 5 * np.sqrt(np.diag(S) / n))
    cov = np.cov(z)
    se = np.sqrt((S ** 2 + np.outer(np.diag(S), np.diag(S))) / n)
    assert np.all(np.abs(cov - S) < 5 * se)
    assert st.kstest(x, "norm", args=(m[0], np.sqrt(S[0, 0]))).statistic < 1.63 / np.sqrt(n)
