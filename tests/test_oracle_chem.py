"""Pins of the chemical-reaction oracle (Sec. 2.1.2, Sec. 2.2.1, Sec. 2.2.2,
Sec. 6): the Euler-Maruyama loop against the reaction network it stands for,
the exact moment recursion of the scheme in the linear case, the stationary
identities of the fast law, the closed-form moment equations of the coarse
model, and the exactness of the histogram-state parareal iteration."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sl
import scipy.stats as st

from oracle import chem as C
from oracle import coarse as OC
from oracle import histogram as H

# The reaction network behind D and E: (change of X, change of Y, propensity).
REACTIONS = [
    (0, +1, lambda k, x, y: k[0]),
    (0, -1, lambda k, x, y: k[1] * y),
    (0, +1, lambda k, x, y: k[2] * y * (y - 1.0)),
    (0, -1, lambda k, x, y: k[3] * y * (y - 1.0) * (y - 2.0)),
    (+1, 0, lambda k, x, y: k[4] * y),
    (-1, 0, lambda k, x, y: k[5] * x),
]


def _langevin(k, x, y):
    """Chemical-Langevin drift and half variance rate of (X, Y) built from the
    reaction list, independently of the oracle's formulas."""
    bx = sum(nx * a(k, x, y) for nx, ny, a in REACTIONS)
    by = sum(ny * a(k, x, y) for nx, ny, a in REACTIONS)
    dx = 0.5 * sum(nx * nx * a(k, x, y) for nx, ny, a in REACTIONS)
    ey = 0.5 * sum(ny * ny * a(k, x, y) for nx, ny, a in REACTIONS)
    return bx, by, dx, ey


def test_fast_coefficients_are_the_reaction_network():
    c = C.Chem()
    y = np.linspace(0.0, 900.0, 37)
    bx, by, dx, ey = _langevin(c.k, 0.0 * y, y)
    assert np.allclose(C.fast_drift(c, y), by, rtol=1e-13, atol=1e-10)
    assert np.allclose(C.fast_diffusion(c, y), ey, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("x0,y0", [(150.0, 120.0), (80.0, 380.0)])
def test_one_em_step_has_the_network_drift_and_variance(oracle_lib, x0, y0):
    """From a fixed state, one Euler-Maruyama step of many particles: the
    increments' means and variances are (dt/tau_x) b_x, (dt/eps) b_y and
    2 D dt/tau_x, 2 E dt/eps of the reaction network, within 5 sigma."""
    c = C.Chem()
    n, dt = 200_000, 1e-3
    x = np.full(n, x0)
    y = np.full((1, n), y0)
    x1, y1 = C.em_propagate(c, 7, 3, x, y, 11, 12, dt)
    bx, by, dx, ey = _langevin(c.k, x0, y0)
    ax, ay = dt / c.tau_x, dt / c.eps
    for inc, drift, var in ((x1 - x0, ax * bx, 2.0 * dx * ax), (y1[0] - y0, ay * by, 2.0 * ey * ay)):
        assert abs(inc.mean() - drift) < 5.0 * math.sqrt(var / n)
        assert abs(inc.var() - var) < 5.0 * var * math.sqrt(2.0 / n)
    assert abs(np.corrcoef(x1, y1[0])[0, 1]) < 5.0 / math.sqrt(n)


def test_reading_of_k3_makes_the_fast_variable_bistable():
    def roots(k3):
        k0, k1, k2 = C.K_DEFAULT[:3]
        # b(y) = k0 - k1 y + k2 (y^2 - y) - k3 (y^3 - 3y^2 + 2y)
        r = np.roots([-k3, k2 + 3 * k3, -k1 - k2 - 2 * k3, k0])
        return np.sort(r.real[np.abs(r.imag) < 1e-9])
    r = roots(C.K_DEFAULT[3])
    assert len(r) == 3 and abs(r[0] - 104.6) < 0.5 and abs(r[1] - 210.9) < 0.5 and abs(r[2] - 408.2) < 0.5
    c = C.Chem()
    # stable, unstable, stable: b changes sign from + to -, - to +, + to -
    s = np.sign(C.fast_drift(c, np.array([r[0] - 1, r[0] + 1, r[1] - 1, r[1] + 1, r[2] - 1, r[2] + 1])))
    assert list(s) == [1, -1, -1, 1, 1, -1]
    assert len(roots(0.666e-6)) == 1  # the printed value: one state, near 7000
    assert roots(0.666e-6)[0] > 6000


def test_lognormal_initial_law(oracle_lib):
    c = C.Chem(x0=(100.0, 20.0), y0=(50.0, 5.0))
    n = 200_000
    x, y = C.init_ensemble(c, 3, 1, n)
    for v, (m, s) in ((x, c.x0), (y[0], c.y0)):
        assert abs(v.mean() - m) < 5.0 * s / math.sqrt(n)
        assert abs(v.std() - s) < 5.0 * s * 0.02  # sd of the sample sd of a lognormal, generously
        s2 = math.log(1.0 + (s / m) ** 2)
        ks = st.kstest(np.log(v), "norm", args=(math.log(m) - 0.5 * s2, math.sqrt(s2)))
        assert ks.pvalue > 1e-3
    assert abs(np.corrcoef(x, y[0])[0, 1]) < 5.0 / math.sqrt(n)
    xs, ys = C.init_ensemble(c, 3, 1, 1000)
    assert np.array_equal(xs, x[:1000]) and np.array_equal(ys[0], y[0, :1000])


def test_linear_network_follows_the_exact_moment_recursion(oracle_lib):
    """Without the autocatalytic reactions (k2 = k3 = 0) drift and squared
    diffusion are affine, so the first and second moments of the
    Euler-Maruyama scheme obey a closed linear recursion (no O(dt) bias).
    The recursion is started from the sample moments of the initial ensemble
    and compared at the end within 5 sigma."""
    k = (60.0, 1.0, 0.0, 0.0, 0.833, 1.0)
    c = C.Chem(k=k)
    n, dt, steps = 100_000, 1e-3, 2000
    x, y = C.init_ensemble(c, 5, 0, n)
    m = np.array([x.mean(), y[0].mean(), (x * x).mean(), (x * y[0]).mean(), (y[0] * y[0]).mean()])
    al, ga = dt / c.tau_x, dt / c.eps
    k0, k1, _, _, k4, k5 = k
    p, q = 1.0 - al * k5, al * k4      # X~ = p X + q Y
    r, s = 1.0 - ga * k1, ga * k0      # Y~ = r Y + s
    for _ in range(steps):
        EX, EY, EXX, EXY, EYY = m
        m = np.array([
            p * EX + q * EY,
            r * EY + s,
            p * p * EXX + 2 * p * q * EXY + q * q * EYY + al * (k4 * EY + k5 * EX),
            p * r * EXY + p * s * EX + q * r * EYY + q * s * EY,
            r * r * EYY + 2 * r * s * EY + s * s + ga * (k0 + k1 * EY),
        ])
    x1, y1 = C.em_propagate(c, 5, 0, x, y, 0, steps, dt)
    got = np.array([x1.mean(), y1[0].mean(), (x1 * x1).mean(), (x1 * y1[0]).mean(), (y1[0] * y1[0]).mean()])
    sd = np.array([x1.std(), y1[0].std(), (x1 * x1).std(), (x1 * y1[0]).std(), (y1[0] * y1[0]).std()])
    assert np.all(np.abs(got - m) < 5.0 * sd / math.sqrt(n)), (got, m)
    # a sign slip in the slow decay would move the mean by far more
    assert abs(m[0] - x.mean()) > 10.0 * sd[0] / math.sqrt(n)


def test_fast_mean_closed_form_and_stationarity():
    # linear drift: the stationary mean is the root k0/k1 and the variance
    # (k0 + k1 ybar)/(2 k1), whatever the (affine) diffusion
    c = C.Chem(k=(60.0, 1.0, 0.0, 0.0, 0.833, 1.0))
    y, phi = C.fast_density(c)
    w = np.full(len(y), y[1] - y[0])
    w[0] = w[-1] = 0.5 * w[1]
    Z = np.sum(w * phi)
    mean = np.sum(w * phi * y) / Z
    var = np.sum(w * phi * (y - mean) ** 2) / Z
    assert abs(C.mean_fast(c) - 60.0) < 1e-6 and abs(mean - 60.0) < 1e-6
    assert abs(var - 60.0) < 1e-5
    # bistable default: E[b(Y)] = 0 under phi (zero flux at both ends)
    c = C.Chem()
    y, phi = C.fast_density(c)
    b = C.fast_drift(c, y)
    assert abs(np.sum(w * phi * b) / np.sum(w * phi * np.abs(b))) < 1e-8
    yb = C.mean_fast(c)
    assert 150.0 < yb < 350.0  # between the two wells, mass in both
    # the trapezoidal value against adaptive quadrature of the same density
    dens = lambda s: math.exp(si.quad(lambda u: C.fast_drift(c, u) / C.fast_diffusion(c, u), 0.0, s,
                                      limit=200)[0] - 40.0) / C.fast_diffusion(c, s)
    # the log density peaks near 40 on [0, 1000]; 40 keeps exp() in range
    num = si.quad(lambda s: s * dens(s), 0.0, 1000.0, limit=400, points=[100.0, 211.0, 400.0])[0]
    den = si.quad(dens, 0.0, 1000.0, limit=400, points=[100.0, 211.0, 400.0])[0]
    assert abs(num / den - yb) < 1e-5


def test_rho_inf_ratios_match_the_closed_form():
    """For the linear effective drift and diffusion the integral in rho_inf
    has a closed form: log rho_inf = (4A/k5 - 1) log(A + k5 x) - 2x + const,
    A = k4 ybar."""
    c = C.Chem()
    yb = 250.0
    A, k5 = c.k[4] * yb, c.k[5]
    for xa, xb in [(0.0, 0.5), (10.0, 10.5), (208.0, 207.5), (599.5, 600.0)]:
        exact = (4 * A / k5 - 1) * math.log1p(k5 * (xa - xb) / (A + k5 * xb)) - 2.0 * (xa - xb)
        assert abs(C.log_rho_inf_ratio(c, yb, xa, xb) - exact) < 1e-12


def _lognormal_cells(grid, m, s):
    s2 = math.log(1.0 + (s / m) ** 2)
    cdf = st.lognorm.cdf(grid.edges, math.sqrt(s2), scale=math.exp(math.log(m) - 0.5 * s2))
    rho = np.diff(cdf)
    rho[0] += cdf[0]
    rho[-1] += 1.0 - cdf[-1]
    return rho


def _coarse_moments(I, tau):
    c = C.Chem()
    yb = C.mean_fast(c)
    g = OC.Grid(I, 0.0, 600.0)
    A, gv = C.fv_generator(g, c, yb)
    E = sl.expm(A * tau)
    r = E @ _lognormal_cells(g, 100.0, 20.0)
    mean = np.sum(g.mids * r)
    var = np.sum((g.mids - mean) ** 2 * r) + g.h ** 2 / 12.0
    return c, yb, A, gv, mean, var


def test_coarse_generator_structure_and_moment_equations():
    """The coarse model has an affine drift and diffusion, so its mean and
    variance obey closed ODEs: m' = (A - k5 m)/tau_x and
    v' = (A + k5 m - 2 k5 v)/tau_x (A = k4 ybar).  The finite-volume solution
    tracks them to second order in h."""
    tau = 10.0
    errs = []
    for I in (300, 600):
        c, yb, A, gv, mean, var = _coarse_moments(I, tau)
        assert np.abs(A.sum(axis=0)).max() < 1e-12 * np.abs(A).max()
        assert np.abs(A @ gv).max() < 1e-11 * np.abs(A).max()
        off = A - np.diag(np.diag(A))
        assert off.min() >= 0.0
        Aa, k5 = c.k[4] * yb, c.k[5]
        m0, v0 = 100.0, 400.0
        sol = si.solve_ivp(lambda t, u: [(Aa - k5 * u[0]) / c.tau_x, (Aa + k5 * u[0] - 2 * k5 * u[1]) / c.tau_x],
                           (0.0, tau), [m0, v0], rtol=1e-12, atol=1e-12)
        m_ex, v_ex = sol.y[0, -1], sol.y[1, -1]
        errs.append((abs(mean - m_ex), abs(var - v_ex)))
    (em1, ev1), (em2, ev2) = errs
    assert em2 < 1.0 and ev2 < 8.0, errs  # h = 1: about 0.5 and 4 (second order, large constant)
    assert em1 / max(em2, 1e-12) > 3.0 or em2 < 1e-6, errs
    assert ev1 / max(ev2, 1e-12) > 3.0 or ev2 < 1e-6, errs


def test_slices_concatenate_bitwise(oracle_lib):
    c = C.Chem()
    x, y = C.init_ensemble(c, 9, 2, 500)
    xa, ya = C.em_propagate(c, 9, 2, x, y, 0, 300, 1e-3)
    xb, yb = C.em_propagate(c, 9, 2, x, y, 0, 120, 1e-3)
    xb, yb = C.em_propagate(c, 9, 2, xb, yb, 120, 300, 1e-3)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    xs, ys = C.em_propagate(c, 9, 2, x[100:200], y[:, 100:200], 0, 300, 1e-3, p0=100)
    assert np.array_equal(xs, xa[100:200])


@pytest.mark.parametrize("it,mt", [(H.J_ADD, H.M_RESAMPLE), (H.J_MULT, H.M_REWEIGHT), (H.J_QUANTILE, H.M_RESAMPLE),
                                   (H.J_ROT, H.M_MARGINAL)])
def test_chem_hist_parareal_exactness(oracle_lib, it, mt):
    """After N iterations the histogram-state iteration on the chemical model
    reproduces the serial fine run (Sec. 3.3.3): its states bitwise for the
    additive and multiplicative iterators with conditional matching, its
    histograms to rounding otherwise.  The grid (20 cells on [0, 600]) keeps
    the fine histograms free of empty interior cells, across which the
    union-of-levels quantile iterator moves mass (its iterator property needs
    gap-free histograms)."""
    c = C.Chem()
    g = OC.Grid(20, 0.0, 600.0)
    K = 3
    pr, hp = H.micmac_parareal_hist(c, 4, 0, 2000, 3.0, 1e-2, K, g, it, mt)
    states, ref = H.sequential_reference_hist(hp, K, g)
    for k in range(K):
        pr.iterate()
    assert max(H.hist_error(pr.u[n].rho(g), ref[n]) for n in range(K + 1)) < 1e-14
    if it in (H.J_ADD, H.J_MULT) and mt != H.M_MARGINAL:
        for n in range(K + 1):
            assert np.array_equal(pr.u[n].x, states[n].x)
    # the serial reference helper is the same run
    sh = H.serial_hist(c, 4, 0, 2000, 3.0, 1e-2, K, g)
    assert np.array_equal(sh, np.array(ref))
