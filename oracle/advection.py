"""Oracle, linear-advection study (Sec. 6, the linear advection case): a
deterministic parareal in which the fine and the coarse propagator both
advance the discretised one-dimensional Fokker-Planck equation eq. (FPz) of
Sec. 2.2.2 with the potential Fbar(x) = x/eps and the diffusion
Dbar = 1/beta, the coarse one with biased parameters (eps~, beta~).
Restriction and matching are the identity; the iterators of Sec. 4 act on
the cell masses.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Readings where the paper is silent (each listed in the design notes):
  A1 tau_x = 1; zero flux at the grid ends, as for the other coarse models.
  A2 the domain, grid, initial law, horizon and slices appear only in a
     figure: grid [-8, 8] with 800 cells, X0 ~ N(2, 1/4) as exact cell
     masses (the mass beyond the grid in the end cells), T = 1 in N = 10
     slices, eps = beta = 1 for the fine model (at T the law N(1, 9/4) has
     less than 2e-6 of its mass beyond either end).
  A3 the biased coarse models of the figure's rows, whose values are not
     printed: underdiffusive beta~ = 2, wrong advection speed eps~ = 2,
     overdiffusive beta~ = 1/2 (the other parameter unbiased).
  A4 both propagators apply the exact exponential of their generator once
     per slice and clip negative rounding residue to 0.
"""
import numpy as np
import scipy.linalg as _sla
import scipy.stats as _st

from . import histogram as _hist
from . import iterate as _iterate


class Advection:
    """Fbar(x) = x/eps, Dbar = 1/beta (tau_x = 1)."""

    def __init__(self, eps=1.0, beta=1.0):
        self.eps, self.beta = float(eps), float(beta)


def log_rho_inf_ratio(m, xa, xb):
    """log(rho_inf(xa)/rho_inf(xb)), rho_inf(x) = exp(-int_0^x Fbar'/Dbar ds)/Dbar
    (Sec. 2.2.2): Fbar'/Dbar = beta/eps is constant, so the integral over
    [xb, xa] is (beta/eps)(xa - xb)."""
    return -(m.beta / m.eps) * (xa - xb)


def fv_generator(grid, m):
    """Generator of the finite-volume scheme (Sec. 2.2.2, uniform grid):
      d rho_i/dt = a_{i+1} (rho_{i+1}/g_{i+1} - rho_i/g_i) - a_i (rho_i/g_i - rho_{i-1}/g_{i-1}),
    a_i = Dbar rho_inf(x_i)/h at interior edges, 0 at the ends, g_i = h rho_inf(m_i);
    each coefficient a_i/g_j from the ratio of rho_inf at neighbouring points.
    Also returns g (A g = 0) normalised to its largest entry."""
    I, h = grid.n, grid.h
    e, mid = grid.edges, grid.mids
    dbar = 1.0 / m.beta
    A = np.zeros((I, I))
    for i in range(1, I):
        base = dbar / (h * h)
        to_left = base * np.exp(log_rho_inf_ratio(m, e[i], mid[i - 1]))
        to_right = base * np.exp(log_rho_inf_ratio(m, e[i], mid[i]))
        A[i - 1, i - 1] -= to_left
        A[i, i - 1] += to_left
        A[i, i] -= to_right
        A[i - 1, i] += to_right
    logg = np.array([log_rho_inf_ratio(m, x, mid[0]) for x in mid])
    return A, np.exp(logg - logg.max())


class Propagator:
    def __init__(self, grid, m):
        self.A, self.g = fv_generator(grid, m)

    def expm(self, tau):
        return _sla.expm(self.A * tau)


def gaussian_cells(grid, mean, sd):
    """Cell masses of N(mean, sd^2), the mass beyond the grid in the end cells."""
    c = _st.norm.cdf(grid.edges, loc=mean, scale=sd)
    rho = np.diff(c)
    rho[0] += c[0]
    rho[-1] += 1.0 - c[-1]
    return rho


def fp_parareal(fine_model, coarse_model, grid, rho0, T, n_slices, iterator):
    """The generic parareal driver with F and C the exact slice exponentials of
    the fine and the coarse model, restriction and matching the identity."""
    tau = T / n_slices
    EF = Propagator(grid, fine_model).expm(tau)
    EC = Propagator(grid, coarse_model).expm(tau)

    def fine(n, u):
        return np.maximum(EF @ u, 0.0)

    def coarse(n, u):
        return np.maximum(EC @ u, 0.0)

    def jump(rc, rf, rcs):
        return _hist.jump(iterator, rc, rf, rcs, grid)

    pr = _iterate.Parareal(np.asarray(rho0, dtype=np.float64), n_slices, fine, coarse, lambda u: u,
                           lambda rho, prior: rho, jump)
    serial = [np.asarray(rho0, dtype=np.float64)]
    for n in range(n_slices):
        serial.append(fine(n, serial[-1]))
    return pr, serial, EF, EC
