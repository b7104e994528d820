"""Oracle, coarse propagator: finite volumes for the slow Fokker-Planck
equation, exact exponential in time, and the knot <-> cell-mass conversions.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Follows Sec. 2.2.1 (effective drift and diffusion, eq. (Fbar)/(Dbar); the
slow Fokker-Planck equation eq. (FPz)), Sec. 2.2.2 (finite volumes in the
rho/rho_inf form with central differences, and the matrix exponential as the
exact time integrator), and Sec. 4.4 (piecewise-linear cdf eq. (discr_cdf),
quantile function with the support-end and flat-part rules).
"""
import numpy as np
import scipy.linalg as _sla


class Grid:
    """Uniform grid x_i = x_lo + i h, i = 0..I, h = (x_hi - x_lo)/I."""

    def __init__(self, n_cells, x_lo=-3.0, x_hi=3.0):
        self.n = int(n_cells)
        self.lo = float(x_lo)
        self.hi = float(x_hi)
        self.h = (self.hi - self.lo) / self.n
        self.edges = np.array([self.lo + i * self.h for i in range(self.n + 1)])
        self.mids = np.array([self.lo + (i + 0.5) * self.h for i in range(self.n)])


def effective_potential(sde):
    """V with V' = the effective drift of eq. (Fbar).  For fixed x the fast
    law is Y_i ~ N(a_i x, 1/beta), so the average of
    dF/dx = c3 x^3 + c1 x + lambda (x - mean_i y_i) is
    c3 x^3 + c1 x + lambda (1 - abar) x."""
    c3, c1, lam, abar = sde.c3, sde.c1, sde.lam, sde.abar()
    k2 = c1 + lam * (1.0 - abar)
    return lambda x: c3 * x ** 4 / 4.0 + k2 * x ** 2 / 2.0


def fv_generator(grid, sde):
    """Generator A of d rho/dt = A rho for the cell masses rho_i, and the
    discrete equilibrium g (A g = 0).

    With tau_x = 1 and Dbar = 1/beta, rho_inf = exp(-beta V) (normalisation
    immaterial).  g_i = h rho_inf(m_i) and the edge coefficients are
    a_i = Dbar rho_inf(x_i)/h at interior edges, 0 at the two ends (zero flux,
    which conserves mass).  Then
      d rho_i/dt = a_{i+1} (rho_{i+1}/g_{i+1} - rho_i/g_i)
                 - a_i (rho_i/g_i - rho_{i-1}/g_{i-1}).
    """
    V = effective_potential(sde)
    I, h = grid.n, grid.h
    dbar = 1.0 / sde.beta
    g = h * np.exp(-sde.beta * V(grid.mids))
    a = np.zeros(I + 1)
    a[1:I] = dbar * np.exp(-sde.beta * V(grid.edges[1:I])) / h
    A = np.zeros((I, I))
    for i in range(I):
        A[i, i] = -(a[i] + a[i + 1]) / g[i]
        if i + 1 < I:
            A[i, i + 1] = a[i + 1] / g[i + 1]
        if i >= 1:
            A[i, i - 1] = a[i] / g[i - 1]
    return A, g, a


class Propagator:
    """E(tau) = exp(A tau), the exact time integrator of the semi-discrete
    system (Sec. 2.2.2), by the library matrix exponential (Pade
    scaling-and-squaring).  expm_eig is a second, independent route through
    the symmetric form G^-1/2 A G^1/2 (A = K G^-1 with K symmetric
    tridiagonal), used to pin the first on well-conditioned grids."""

    def __init__(self, grid, sde):
        A, g, a = fv_generator(grid, sde)
        self.A, self.g = A, g

    def expm(self, tau):
        return _sla.expm(self.A * tau)

    def expm_eig(self, tau):
        s = np.sqrt(self.g)
        S = self.A * s[None, :] / s[:, None]
        S = 0.5 * (S + S.T)
        w, U = np.linalg.eigh(S)
        Es = (U * np.exp(w * tau)[None, :]) @ U.T
        return Es * s[:, None] / s[None, :]


def cdf_at(q, x):
    """Piecewise-linear cdf through (q_j, j/Q), 0 left of q_0 and 1 right of
    q_Q; a repeated knot is a jump and c(x) = P(X < x)."""
    Q = len(q) - 1
    if x <= q[0]:
        return 0.0
    if x > q[Q]:
        return 1.0
    j = int(np.searchsorted(q, x, side="left")) - 1  # largest j with q_j < x
    t = (x - q[j]) / (q[j + 1] - q[j])
    return (j + t) / Q


def knots_to_masses(q, grid):
    """H: cell masses of the law with knots q: rho_i = c(x_{i+1}) - c(x_i) with
    the mass outside the grid put into the two end cells."""
    I = grid.n
    c = np.array([cdf_at(q, grid.edges[i]) for i in range(1, I)])
    rho = np.empty(I)
    rho[0] = c[0]
    for i in range(1, I - 1):
        rho[i] = c[i] - c[i - 1]
    rho[I - 1] = 1.0 - c[I - 2]
    return rho


def masses_to_knots(rho, grid, n_q):
    """Qf: knots at p_j = j/Q of the piecewise-linear cdf eq. (discr_cdf) of the
    cell masses rho (normalised by their total).  A level reached on a flat
    stretch of the cdf gives the midpoint of that stretch (Sec. 4.4); the end
    knots are the grid ends."""
    I = grid.n
    C = np.zeros(I + 1)
    for i in range(I):
        C[i + 1] = C[i] + rho[i]
    tot = C[I]
    e = grid.edges
    q = np.empty(n_q + 1)
    q[0] = e[0]
    q[n_q] = e[I]
    for j in range(1, n_q):
        ct = (j / n_q) * tot
        i1 = int(np.searchsorted(C, ct, side="left"))  # first i with C_i >= ct
        if C[i1] > ct:
            i = i1 - 1
            v = e[i] + (ct - C[i]) / rho[i] * grid.h
            q[j] = min(max(v, e[i]), e[i + 1])
        else:
            i2 = int(np.searchsorted(C, ct, side="right")) - 1  # last i with C_i <= ct
            q[j] = 0.5 * (e[i1] + e[i2])
    return q


def coarse_step(q, E, grid):
    """One coarse propagation of a knot vector: knots -> masses -> E masses
    (negative rounding residue clipped to 0) -> knots."""
    rho = knots_to_masses(q, grid)
    rho = np.maximum(E @ rho, 0.0)
    return masses_to_knots(rho, grid, len(q) - 1), rho
