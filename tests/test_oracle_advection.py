"""Pins of the linear-advection oracle (Sec. 6, the linear advection case):
closed-form moments of the advection-diffusion equation, the structure of
the generator, exactness of the deterministic parareal after N iterations,
and the paper's observation that the quantile iterator corrects an error in
the advection speed almost perfectly."""
import numpy as np
import pytest

from oracle import advection as AD
from oracle import coarse as OC
from oracle import histogram as H


def test_generator_structure():
    g = OC.Grid(200, -8.0, 8.0)
    A, gv = AD.fv_generator(g, AD.Advection(0.7, 1.3))
    assert np.abs(A.sum(axis=0)).max() < 1e-12 * np.abs(A).max()
    assert np.abs(A @ gv).max() < 1e-12 * np.abs(A).max()
    assert (A - np.diag(np.diag(A))).min() >= 0.0
    # rho_inf decreases like exp(-beta x / eps): the equilibrium piles up on the left
    assert np.all(np.diff(np.log(gv)) < 0.0)
    assert abs(np.log(gv[0] / gv[1]) - (1.3 / 0.7) * g.h) < 1e-12


@pytest.mark.parametrize("eps,beta", [(1.0, 1.0), (2.0, 2.0), (0.5, 1.0)])
def test_moments_follow_the_advection_diffusion_closed_form(eps, beta):
    """Drift -1/eps and diffusion 1/beta: the mean moves as m0 - t/eps and the
    variance grows as v0 + 2t/beta while the mass stays inside the grid;
    the finite-volume solution converges to them at second order in h."""
    t = 1.0
    errs = []
    for I in (400, 800):
        g = OC.Grid(I, -8.0, 8.0)
        r = AD.Propagator(g, AD.Advection(eps, beta)).expm(t) @ AD.gaussian_cells(g, 2.0, 0.5)
        m = np.sum(g.mids * r)
        v = np.sum((g.mids - m) ** 2 * r)
        errs.append((abs(m - (2.0 - t / eps)), abs(v - (0.25 + 2.0 * t / beta))))
        assert abs(r.sum() - 1.0) < 1e-11
    (m1, v1), (m2, v2) = errs
    assert m2 < 2e-4 and v2 < 2e-3, errs
    assert m1 / m2 > 3.0 and v1 / v2 > 3.0, errs


@pytest.mark.parametrize("it", [H.J_ADD, H.J_MULT, H.J_ROT, H.J_QUANTILE])
def test_parareal_is_exact_after_n_iterations(it):
    g = OC.Grid(160, -8.0, 8.0)
    rho0 = AD.gaussian_cells(g, 2.0, 0.5)
    pr, serial, _, _ = AD.fp_parareal(AD.Advection(), AD.Advection(1.0, 2.0), g, rho0, 1.0, 5, it)
    for k in range(5):
        pr.iterate()
        # the first k+1 time points are exact after k+1 iterations
        assert max(H.hist_error(pr.rho[n], serial[n]) for n in range(k + 2)) < 1e-12
    assert max(H.hist_error(pr.rho[n], serial[n]) for n in range(6)) < 1e-12


def test_quantile_iterator_corrects_an_advection_error():
    """A coarse model with the wrong advection speed (eps~ = 2): after one
    iteration the quantile iterator leaves less than 1% of the coarse error
    at T, the additive iterator more than 10% (Sec. 6, linear advection)."""
    g = OC.Grid(800, -8.0, 8.0)
    rho0 = AD.gaussian_cells(g, 2.0, 0.5)
    out = {}
    for it in (H.J_ADD, H.J_QUANTILE):
        pr, serial, _, _ = AD.fp_parareal(AD.Advection(), AD.Advection(2.0, 1.0), g, rho0, 1.0, 10, it)
        e0 = H.hist_error(pr.rho[10], serial[10])
        pr.iterate()
        out[it] = H.hist_error(pr.rho[10], serial[10]) / e0
    assert out[H.J_QUANTILE] < 0.01 and out[H.J_ADD] > 0.1, out
