"""Pins for the oracle's coarse propagator (Sec. 2.2.2: finite volumes in the
rho/rho_inf form, exact exponential in time) and the knot/mass conversions
(Sec. 4.4, eq. (discr_cdf), support-end and flat-part rules)."""
import numpy as np

from oracle import coarse as C
from oracle import particles as P


def _setup(I=200, **kw):
    s = P.Sde(**kw) if kw else P.Sde()
    g = C.Grid(I)
    return s, g, C.Propagator(g, s)


def test_generator_conserves_mass_and_gibbs():
    s, g, pr = _setup()
    A = pr.A
    col = np.abs(A).sum(0)
    assert np.all(np.abs(A.sum(0)) <= 1e-14 * col)  # columns sum to zero: mass
    assert np.all(np.abs(A @ pr.g) <= 1e-13 * (np.abs(A) @ pr.g + 1e-300))  # discrete Gibbs is a null vector
    off = A - np.diag(np.diag(A))
    assert np.all(off >= 0) and np.count_nonzero(np.triu(off, 2)) == 0 and np.count_nonzero(np.tril(off, -2)) == 0


def test_exponential_properties():
    s, g, pr = _setup(I=256)
    E1, E2, E3 = pr.expm(0.05), pr.expm(0.11), pr.expm(0.16)
    for E in (E1, E2, E3):
        assert np.all(E >= -1e-15)
        assert np.abs(E.sum(0) - 1).max() < 1e-12
        assert np.abs(E @ pr.g - pr.g).max() < 1e-12 * pr.g.max()
    assert np.abs(E1 @ E2 - E3).max() < 1e-12  # semigroup
    Einf = pr.expm(200.0)
    rho = np.zeros(g.n)
    rho[17] = 1.0
    assert np.abs(Einf @ rho - pr.g / pr.g.sum()).max() < 1e-10


def test_exponential_against_eigendecomposition():
    """Second route to exp(A tau) on a well-conditioned grid."""
    s, g, pr = _setup(I=64, beta=0.5)
    for tau in (0.01, 0.3, 2.0):
        assert np.abs(pr.expm(tau) - pr.expm_eig(tau)).max() < 1e-12


def _gauss_masses(grid, m, v):
    from scipy.stats import norm
    c = norm.cdf(grid.edges, loc=m, scale=np.sqrt(v))
    return np.diff(c)


def test_ou_coarse_model_second_order():
    """c3 = 0, c1 = 1: the coarse model is dZ = -Z dt + sqrt(2/beta) dW, whose
    Gaussian law keeps mean m0 e^-t and variance v0 e^-2t + (1-e^-2t)/beta.
    The finite-volume error is O(h^2): halving h divides it by about 4."""
    m0, v0, t, beta = 1.0, 0.3, 0.7, 2.0
    mt = m0 * np.exp(-t)
    vt = v0 * np.exp(-2 * t) + (1 - np.exp(-2 * t)) / beta
    errs = []
    for I in (60, 120, 240):
        s = P.Sde(beta=beta, c3=0.0, c1=1.0)
        grid = C.Grid(I, -7.0, 7.0)
        pr = C.Propagator(grid, s)
        rho = pr.expm(t) @ _gauss_masses(grid, m0, v0)
        ref = _gauss_masses(grid, mt, vt)
        errs.append(np.abs(rho - ref).sum())
    assert errs[0] / errs[1] > 3.2 and errs[1] / errs[2] > 3.2, errs
    assert errs[2] < 1e-3


def test_cdf_and_masses_basic():
    g = C.Grid(10, 0.0, 10.0)
    q = np.linspace(2.0, 6.0, 5)  # uniform on [2, 6]
    rho = C.knots_to_masses(q, g)
    assert abs(rho.sum() - 1) < 1e-15
    ref = np.array([0, 0, .25, .25, .25, .25, 0, 0, 0, 0])
    assert np.abs(rho - ref).max() < 1e-15
    # atoms: two coincident knots carry mass 1/Q; c(x) is P(X < x)
    q2 = np.array([1.0, 3.0, 3.0, 5.0])
    assert C.cdf_at(q2, 3.0) == 1 / 3
    assert abs(C.cdf_at(q2, np.nextafter(3.0, 4)) - 2 / 3) < 1e-12
    assert C.cdf_at(q2, 1.0) == 0.0 and C.cdf_at(q2, 5.0) == 1.0 and C.cdf_at(q2, 5.1) == 1.0


def test_cdf_brute_force_sampling():
    """c(x) against dense sampling of the piecewise-linear law (inverse
    transform of evenly spread levels)."""
    rng = np.random.default_rng(3)
    q = np.sort(rng.uniform(-2, 2, 11))
    Q = len(q) - 1
    u = (np.arange(2_000_000) + 0.5) / 2_000_000
    j = np.minimum(np.floor(u * Q).astype(int), Q - 1)
    samples = q[j] + (u * Q - j) * (q[j + 1] - q[j])
    for x in np.linspace(-2.5, 2.5, 41):
        assert abs(C.cdf_at(q, x) - np.mean(samples < x)) < 2e-6


def test_masses_to_knots_roundtrip_on_edges():
    g = C.Grid(20, -3.0, 3.0)
    idx = np.array([0, 3, 4, 7, 8, 9, 12, 15, 16, 20])  # knots on edges, ends on the grid ends
    q = g.edges[idx]
    rho = C.knots_to_masses(q, g)
    q2 = C.masses_to_knots(rho, g, len(q) - 1)
    assert np.abs(q2 - q).max() < 1e-15


def test_masses_to_knots_flat_midpoint():
    g = C.Grid(10, 0.0, 10.0)
    rho = np.array([0.25, 0.25, 0, 0, 0, 0.25, 0.25, 0, 0, 0])  # flat cdf on [2, 5] at level 1/2
    q = C.masses_to_knots(rho, g, 4)  # levels 0, .25, .5, .75, 1
    assert list(q) == [0.0, 1.0, 3.5, 6.0, 10.0]


def test_masses_to_knots_interpolates_linear_cdf():
    g = C.Grid(4, 0.0, 4.0)
    rho = np.array([0.1, 0.2, 0.3, 0.4])
    q = C.masses_to_knots(rho, g, 10)
    C_edges = np.concatenate([[0], np.cumsum(rho)])
    ref = np.interp(np.arange(11) / 10, C_edges, g.edges)
    ref[0], ref[-1] = 0.0, 4.0
    assert np.abs(q - ref).max() < 1e-14


def test_coarse_step_long_time_reaches_gibbs():
    s, g, pr = _setup(I=300)
    q0 = np.linspace(-0.5, 0.5, 101)
    qT, rho = C.coarse_step(q0, pr.expm(60.0), g)
    ref = C.masses_to_knots(pr.g / pr.g.sum(), g, 100)
    assert abs(rho.sum() - 1) < 1e-10  # 60 time units: many squarings
    assert np.abs(qT - ref).max() < 1e-8
